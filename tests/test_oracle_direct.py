"""Pins of the CPU direct-sum oracle against closed forms, invariants and brute force.

The oracle computes eq. greenSum of Appendix A with the kernel of eq. green2D.
Each test checks it against something other than itself: continuum solutions
of the Poisson equation (eq. greenConv), the far-field behaviour of eq.
pressTruncated, exact-arithmetic brute force, hand-computed fixtures and
symmetries of the kernel.
"""

import math
import os

import numpy as np
import pytest

from oracle import closed, direct
from workloads import generators as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _gauss(n, sigma=0.1):
    g = G.GridSpec(n, n, 1.0 / n)
    f = G.gaussian_source(g, sigma=sigma)
    x, y = G.grid_nodes(g)
    return g, f, x.ravel(), y.ravel()


def test_gaussian_closed_form_cellavg_converges():
    """Gaussian source: discrete sum vs sigma^2/4 [ln r^2 + E1(r^2/sigma^2)] (eq. greenConv).

    Pins the 1/2pi normalisation, the sign, the h^2 weighting and the self-cell rule:
    any of those wrong gives an O(1) error; right, the error falls ~4x per halving of h.
    """
    errs = []
    for n in (64, 128):
        g, f, tx, ty = _gauss(n)
        P = direct.direct_grid(f, g.h, tx, ty, self_mode=direct.SELF_CELLAVG)
        Pc = closed.gaussian_pressure(np.hypot(tx - 0.5, ty - 0.5), 0.1)
        errs.append(rel_l2(P, Pc))
    assert errs[0] < 3e-4
    assert errs[0] / errs[1] > 3.5


def test_gaussian_closed_form_skip():
    """SKIP drops the self cell, an O(h^2 ln h) term: about 4.7e-3 at 64^2."""
    g, f, tx, ty = _gauss(64)
    P = direct.direct_grid(f, g.h, tx, ty, self_mode=direct.SELF_SKIP)
    Pc = closed.gaussian_pressure(np.hypot(tx - 0.5, ty - 0.5), 0.1)
    e = rel_l2(P, Pc)
    assert 3e-3 < e < 6e-3


def test_gaussian_far_field():
    """Far from the source P -> (S/2pi) ln r with S = pi sigma^2 and no constant (eq. pressTruncated, first term)."""
    g, f, _, _ = _gauss(64)
    ang = np.linspace(0, 2 * math.pi, 13, endpoint=False)
    rad = np.array([3.0, 10.0, 100.0])
    tx = (0.5 + rad[:, None] * np.cos(ang)[None, :]).ravel()
    ty = (0.5 + rad[:, None] * np.sin(ang)[None, :]).ravel()
    P = direct.direct_grid(f, g.h, tx, ty)
    S = math.pi * 0.01
    Pfar = S / (2 * math.pi) * np.log(np.hypot(tx - 0.5, ty - 0.5))
    assert np.max(np.abs(P - Pfar) / np.abs(Pfar)) < 1e-9


def test_bump_shell_theorem():
    """Compact radial bump: discrete sum vs the 1-D shell-theorem quadrature, on and off the grid."""
    R = 0.3
    g = G.GridSpec(128, 128, 1.0 / 128)
    x, y = G.grid_nodes(g)
    f = closed.bump_source(np.hypot(x - 0.5, y - 0.5), R)
    rng = np.random.Generator(np.random.PCG64(11))
    tx = np.concatenate([x.ravel()[::61], rng.uniform(0, 1, 200), [0.5 + 0.45, 0.5, 2.0]])
    ty = np.concatenate([y.ravel()[::61], rng.uniform(0, 1, 200), [0.5, 0.5 - 0.41, -1.0]])
    P = direct.direct_grid(f, g.h, tx, ty, self_mode=direct.SELF_CELLAVG)
    Pq = closed.radial_shell_pressure(lambda s: float(closed.bump_source(s, R)), np.hypot(tx - 0.5, ty - 0.5), R)
    assert rel_l2(P, Pq) < 1e-4
    # outside the support the shell theorem is exact: (S/2pi) ln r, S = pi R^2 / 5
    far = np.hypot(tx - 0.5, ty - 0.5) > R + 0.05
    S = closed.bump_total(R)
    assert np.max(np.abs(P[far] - S / (2 * math.pi) * np.log(np.hypot(tx[far] - 0.5, ty[far] - 0.5)))) < 2e-6 * S


def _vortex_radial_source(gamma, rc):
    """Radial profile of the generator's vortex source (evaluated through the generator itself)."""
    def fr(s):
        x = np.array([[0.5 + s]])
        y = np.array([[0.5]])
        ux, uy, vx, vy = G.vortex_velocity_gradients(x, y, [(0.5, 0.5)], [gamma], [rc])
        return float(2.0 * (ux * vy - uy * vx)[0, 0])
    return fr


def test_lamb_oseen_closed_form_is_the_generator_source():
    """The Lamb-Oseen pressure closed form has the generator's source as its radial Laplacian.

    Shell-theorem quadrature of the generator's f (to r = 1e4 rc, tail below 1e-7) reproduces
    the closed form; this pins both the generator's gradient formulas and the closed form.
    """
    gamma, rc = 1.3, 0.02
    fr = _vortex_radial_source(gamma, rc)
    r = np.array([0.0, 0.3 * rc, rc, 2.5 * rc, 7 * rc, 30 * rc])
    Pq = closed.radial_shell_pressure(fr, r, 1e4 * rc, epsrel=1e-12)
    Pc = closed.lamb_oseen_pressure(r, gamma, rc)
    assert np.max(np.abs(Pq - Pc)) < 1e-6 * abs(Pc[0])


def test_lamb_oseen_disk_masked_grid():
    """Discrete sum of a disk-masked vortex source vs the shell-theorem quadrature of the same source."""
    gamma, rc, R = -0.8, 0.03, 0.45
    g = G.GridSpec(256, 256, 1.0 / 256)
    x, y = G.grid_nodes(g)
    ux, uy, vx, vy = G.vortex_velocity_gradients(x, y, [(0.5, 0.5)], [gamma], [rc])
    f = 2.0 * (ux * vy - uy * vx)
    f = np.where(np.hypot(x - 0.5, y - 0.5) < R, f, 0.0)
    sel = slice(None, None, 173)
    tx, ty = x.ravel()[sel], y.ravel()[sel]
    P = direct.direct_grid(f, g.h, tx, ty, self_mode=direct.SELF_CELLAVG)
    fr = _vortex_radial_source(gamma, rc)
    Pq = closed.radial_shell_pressure(lambda s: fr(s) if s < R else 0.0, np.hypot(tx - 0.5, ty - 0.5), R)
    assert rel_l2(P, Pq) < 2e-3


def test_tiny_brute_force_mpmath():
    """Random tiny problem vs a 50-digit evaluation of eq. greenSum: pins the FP64 rounding."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    rng = np.random.Generator(np.random.PCG64(7))
    n = 12
    f = rng.standard_normal((n, n))
    h = 1.0 / n
    tx = rng.uniform(-0.2, 1.2, 40)
    ty = rng.uniform(-0.2, 1.2, 40)
    P = direct.direct_grid(f, h, tx, ty)
    for k in range(tx.size):
        acc = mpmath.mpf(0)
        for j in range(n):
            for i in range(n):
                sx = mpmath.mpf(float((i + 0.5) * h))
                sy = mpmath.mpf(float((j + 0.5) * h))
                w = mpmath.mpf(float(f[j, i])) * mpmath.mpf(h) ** 2
                acc += w * mpmath.log(mpmath.sqrt((mpmath.mpf(tx[k]) - sx) ** 2 + (mpmath.mpf(ty[k]) - sy) ** 2))
        ref = float(acc / (2 * mpmath.pi))
        assert abs(P[k] - ref) <= 1e-14 * max(abs(ref), 1e-300) + 1e-16 * float(np.sum(np.abs(f)) * h * h)


def test_golden_hand_cases():
    """Hand-computed fixtures (tests/golden/direct_hand_cases.txt)."""
    path = os.path.join(GOLDEN, "direct_hand_cases.txt")
    cases = []
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                cases.append([float(v) for v in line.split()])
    assert cases
    for nx, ny, x0, y0, h, fvals_n, *rest in [(int(c[0]), int(c[1]), *c[2:5], int(c[5]), *c[6:]) for c in cases]:
        fvals = np.array(rest[:fvals_n]).reshape(ny, nx)
        tx, ty, self_mode, expect = rest[fvals_n:fvals_n + 4]
        P = direct.direct_grid(fvals, h, [tx], [ty], x0=x0, y0=y0, self_mode=int(self_mode))
        assert abs(P[0] - expect) <= 1e-15 * max(1.0, abs(expect)), (P[0], expect)


def test_linearity_and_superposition():
    """P[a f1 + b f2] = a P[f1] + b P[f2] (linearity of eq. greenSum, superposition of groups)."""
    rng = np.random.Generator(np.random.PCG64(3))
    g = G.GridSpec(48, 40, 1.0 / 48)
    f1 = rng.standard_normal((40, 48))
    f2 = rng.standard_normal((40, 48))
    tx = rng.uniform(0, 1, 300)
    ty = rng.uniform(0, 1, 300)
    a, b = 1.7, -0.3
    P = direct.direct_grid(a * f1 + b * f2, g.h, tx, ty)
    P12 = a * direct.direct_grid(f1, g.h, tx, ty) + b * direct.direct_grid(f2, g.h, tx, ty)
    scale = float(np.sum(np.abs(a * f1) + np.abs(b * f2)) * g.h**2)
    assert np.max(np.abs(P - P12)) < 1e-13 * scale


def test_rotation_reflection_and_translation():
    """G depends on |x - x'| only (eq. green2D): rotating/reflecting the grid permutes the result."""
    rng = np.random.Generator(np.random.PCG64(5))
    n = 32
    h = 1.0 / n
    f = rng.standard_normal((n, n))
    g = G.GridSpec(n, n, h)
    x, y = G.grid_nodes(g)
    tx, ty = x.ravel(), y.ravel()
    P = direct.direct_grid(f, h, tx, ty).reshape(n, n)
    # rotation by 90 degrees about the grid centre: node (i, j) -> (n-1-j, i)
    fr = np.rot90(f, k=1)  # fr[j', i'] with i' = ..., checked through the node map below
    Pr = direct.direct_grid(fr, h, tx, ty).reshape(n, n)
    scale = float(np.sum(np.abs(f)) * h * h)
    assert np.max(np.abs(np.rot90(P, k=1) - Pr)) < 1e-13 * scale
    # reflection x -> 1 - x
    Pm = direct.direct_grid(f[:, ::-1], h, tx, ty).reshape(n, n)
    assert np.max(np.abs(P[:, ::-1] - Pm)) < 1e-13 * scale
    # translation of sources and targets by the same amount
    Pt = direct.direct_grid(f, h, tx + 3.25, ty - 1.5, x0=3.25, y0=-1.5).reshape(n, n)
    assert np.max(np.abs(P - Pt)) < 1e-12 * scale


def test_scaling_law():
    """Scaling all lengths by lam: P' = lam^2 (P + ln(lam)/(2pi) * sum w) (w = f h^2 scales by lam^2)."""
    rng = np.random.Generator(np.random.PCG64(9))
    n = 24
    f = rng.standard_normal((n, n))
    h = 1.0 / n
    tx = rng.uniform(0, 1, 100)
    ty = rng.uniform(0, 1, 100)
    lam = 3.0
    P = direct.direct_grid(f, h, tx, ty)
    P2 = direct.direct_grid(f, lam * h, lam * tx, lam * ty)
    W = float(np.sum(f) * h * h)
    expect = lam**2 * (P + math.log(lam) / (2 * math.pi) * W)
    assert np.max(np.abs(P2 - expect)) < 1e-12 * lam**2 * float(np.sum(np.abs(f)) * h * h)


def test_self_modes_differ_by_the_cell_average():
    """At a grid-node target CELLAVG - SKIP = w (ln h - kappa) / 2pi for the coincident node."""
    rng = np.random.Generator(np.random.PCG64(2))
    n = 16
    h = 0.05
    f = rng.standard_normal((n, n))
    i, j = 5, 9
    tx = [(i + 0.5) * h]
    ty = [(j + 0.5) * h]
    Ps = direct.direct_grid(f, h, tx, ty, self_mode=0)
    Pc = direct.direct_grid(f, h, tx, ty, self_mode=1)
    expect = f[j, i] * h * h * (math.log(h) - closed.KAPPA) / (2 * math.pi)
    assert abs((Pc - Ps)[0] - expect) < 1e-15


def test_kappa_is_the_cell_mean_of_log_r():
    """kappa: mean of ln r over the unit square centred at the origin is -kappa (2-D quadrature)."""
    from scipy import integrate
    val, _ = integrate.dblquad(lambda y, x: 0.5 * math.log(x * x + y * y), 0.0, 0.5, 0.0, 0.5,
                               epsabs=1e-13, epsrel=1e-13)
    assert abs(4.0 * val - (-closed.KAPPA)) < 1e-10


def test_points_entry_matches_grid_entry():
    rng = np.random.Generator(np.random.PCG64(4))
    n = 20
    h = 0.037
    f = rng.standard_normal((n, n))
    g = G.GridSpec(n, n, h, 0.1, -0.2)
    x, y = G.grid_nodes(g)
    tx = np.concatenate([x.ravel()[::7], rng.uniform(0, 1, 50)])
    ty = np.concatenate([y.ravel()[::7], rng.uniform(-0.2, 0.6, 50)])
    Pg = direct.direct_grid(f, h, tx, ty, x0=0.1, y0=-0.2)
    Pp = direct.direct_points(x.ravel(), y.ravel(), (f * h * h).ravel(), tx, ty)
    assert np.max(np.abs(Pg - Pp)) < 1e-14 * float(np.sum(np.abs(f)) * h * h)


def test_points_tiny_brute_force_mpmath():
    """Scattered sources with their own weights (some zero, some coincident with targets) vs a
    50-digit evaluation of eq. greenSum with G(0) := 0: pins the points entry on its own."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    rng = np.random.Generator(np.random.PCG64(17))
    n = 60
    sx = rng.uniform(-1.0, 2.0, n)
    sy = rng.uniform(0.0, 0.5, n)
    w = rng.standard_normal(n) * rng.uniform(0.1, 3.0, n)
    w[::9] = 0.0
    tx = np.concatenate([sx[:10], rng.uniform(-1.5, 2.5, 20)])
    ty = np.concatenate([sy[:10], rng.uniform(-0.5, 1.0, 20)])
    P = direct.direct_points(sx, sy, w, tx, ty)
    for k in range(tx.size):
        acc = mpmath.mpf(0)
        for i in range(n):
            dx = mpmath.mpf(float(tx[k])) - mpmath.mpf(float(sx[i]))
            dy = mpmath.mpf(float(ty[k])) - mpmath.mpf(float(sy[i]))
            if dx == 0 and dy == 0:
                continue
            acc += mpmath.mpf(float(w[i])) * mpmath.log(mpmath.sqrt(dx * dx + dy * dy))
        ref = float(acc / (2 * mpmath.pi))
        assert abs(P[k] - ref) <= 1e-14 * max(abs(ref), 1e-300) + 1e-16 * float(np.sum(np.abs(w)))


def test_thread_count_does_not_change_bits():
    """Static schedule over targets and fixed source order: bitwise identical for 1 and N threads."""
    import subprocess
    import sys
    code = ("import numpy as np, sys; sys.path.insert(0, %r); from oracle import direct; "
            "rng=np.random.Generator(np.random.PCG64(1)); f=rng.standard_normal((40,40)); "
            "t=rng.uniform(0,1,(2,333)); print(direct.direct_grid(f,1/40,t[0],t[1]).tobytes().hex())"
            % os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    outs = []
    for nt in ("1", "5"):
        env = dict(os.environ, OMP_NUM_THREADS=nt)
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                                   check=True).stdout)
    assert outs[0] == outs[1]
