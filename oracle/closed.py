"""Closed-form and quadrature solutions of the free-space pressure Poisson problem.

TEST INFRASTRUCTURE ONLY.  These give P = G * f (Appendix A, eq. greenConv with
G = (1/2pi) ln|x - x'|, eq. green2D) for sources whose convolution is known in
closed form, so that the direct sum of eq. greenSum can be checked against
something other than itself.

For a radially symmetric source f(r) the convolution reduces to the 1-D
integral P(r) = int_0^inf f(s) s ln(max(r, s)) ds (mean-value property of the
logarithm), which fixes the additive constant completely (no free constant:
the Green's function of eq. green2D is used as is).
"""

from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special

EULER_GAMMA = 0.5772156649015329
#: mean of ln r over the h x h square centred at the origin is ln h - KAPPA
KAPPA = 1.5 - math.pi / 4.0 + 0.5 * math.log(2.0)


def gaussian_pressure(r, sigma: float):
    """P(r) for f = exp(-r^2/sigma^2): sigma^2/4 [ln r^2 + E1(r^2/sigma^2)].

    The limit r -> 0 is sigma^2/4 (ln sigma^2 - gamma_Euler).  Far away P tends to
    (S/2pi) ln r with S = pi sigma^2, with no additive constant.
    """
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    small = r < 1e-300
    rs = np.where(small, 1.0, r)
    x = rs * rs / (sigma * sigma)
    out = sigma * sigma / 4.0 * (np.log(rs * rs) + special.exp1(x))
    return np.where(small, sigma * sigma / 4.0 * (math.log(sigma * sigma) - EULER_GAMMA), out)


def lamb_oseen_pressure(r, gamma: float, rc: float, rho: float = 1.0):
    """Pressure of one Lamb-Oseen vortex (u_theta = K (1 - e^{-r^2/rc^2}) / r, K = Gamma/2pi).

    dP/dr = rho u_theta^2 / r with P -> 0 at infinity gives
    P = -(rho K^2 / 2 rc^2) [ (1 - e^{-x})^2 / x + 2 E1(x) - 2 E1(2x) ],  x = r^2/rc^2,
    with P(0) = -rho K^2 ln 2 / rc^2.  Its Laplacian is the source
    2 rho (u_x v_y - u_y v_x) of the vortex.
    """
    K = gamma / (2.0 * math.pi)
    r = np.asarray(r, dtype=np.float64)
    x = r * r / (rc * rc)
    xs = np.where(x < 1e-300, 1.0, x)
    val = -(rho * K * K / (2.0 * rc * rc)) * (np.expm1(-xs) ** 2 / xs + 2.0 * special.exp1(xs) - 2.0 * special.exp1(2.0 * xs))
    return np.where(x < 1e-300, -rho * K * K * math.log(2.0) / (rc * rc), val)


def radial_shell_pressure(f_radial, r, R: float, epsabs: float = 1e-15, epsrel: float = 1e-13):
    """P(r) = int_0^R f(s) s ln(max(r, s)) ds for a radial source supported on s < R.

    Evaluated by adaptive quadrature (scipy.integrate.quad) split at s = r.
    """
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    out = np.empty_like(r)
    for k, rk in enumerate(r):
        inner_hi = min(rk, R)
        inner = 0.0
        if inner_hi > 0.0:
            inner = integrate.quad(lambda s: f_radial(s) * s, 0.0, inner_hi, epsabs=epsabs, epsrel=epsrel,
                                   limit=200)[0] * math.log(rk)
        outer = 0.0
        if rk < R:
            outer = integrate.quad(lambda s: f_radial(s) * s * math.log(s), rk, R, epsabs=epsabs, epsrel=epsrel,
                                   limit=200)[0]
        out[k] = inner + outer
    return out


def bump_source(s, R: float):
    """A C^3 compact radial source (1 - s^2/R^2)^4 on s < R, zero outside."""
    s = np.asarray(s, dtype=np.float64)
    return np.where(s < R, (1.0 - (s / R) ** 2) ** 4, 0.0)


def bump_total(R: float) -> float:
    """S = int f dA for ``bump_source``: 2 pi int_0^R (1-s^2/R^2)^4 s ds = pi R^2 / 5."""
    return math.pi * R * R / 5.0
