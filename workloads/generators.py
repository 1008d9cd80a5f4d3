"""Seeded generators for the synthetic pressure-Poisson workloads.

Every field is produced in FP64 with NumPy's PCG64 from a stated seed.  The
paper's own flow fields are not available, so these stand in for them at the
paper's scales:

* sources live on a uniform, cell-centred n x n grid over the unit square
  (node (i, j) at (x0 + (i + 1/2) h, y0 + (j + 1/2) h)), as in the uniform
  4096^2 cylinder runs of Sec. 3.1;
* the pressure source of the Poisson equation (Sec. 2.2, eq. PoissonFinal,
  fluid part) is f = -rho grad(u)^T : grad(u); for a divergence-free 2-D field
  this equals 2 rho (u_x v_y - u_y v_x), which is what ``vortex_source``
  assembles from an analytic superposition of Lamb-Oseen vortices;
* targets are grid nodes (the full-field evaluation of Sec. 3.3), points on a
  body surface (Sec. 2.3.1) or on a lifted surface moved outward along the
  normal by 2h (Sec. 2.3.2), with the fish half-width profile of eq. fishWidth.

Nothing here evaluates the Green's function or any expansion.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class GridSpec:
    """A cell-centred nx x ny grid: node (i, j) sits at (x0+(i+.5)h, y0+(j+.5)h).

    Field arrays are row-major with shape (ny, nx): ``f[j, i]`` belongs to
    node (i, j).
    """

    nx: int
    ny: int
    h: float
    x0: float = 0.0
    y0: float = 0.0


def grid_nodes(g: GridSpec) -> tuple[np.ndarray, np.ndarray]:
    """Node coordinates as two (ny, nx) FP64 arrays, computed as x0 + (i + 0.5) * h."""
    i = np.arange(g.nx, dtype=np.float64)
    j = np.arange(g.ny, dtype=np.float64)
    x = g.x0 + (i + 0.5) * g.h
    y = g.y0 + (j + 0.5) * g.h
    return np.broadcast_to(x[None, :], (g.ny, g.nx)).copy(), np.broadcast_to(y[:, None], (g.ny, g.nx)).copy()


def gaussian_source(g: GridSpec, cx: float = 0.5, cy: float = 0.5, sigma: float = 0.1) -> np.ndarray:
    """f = exp(-|x - c|^2 / sigma^2) at the grid nodes (shape (ny, nx))."""
    x, y = grid_nodes(g)
    return np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / sigma**2)


def lamb_oseen_params(seed, n_vortices: int = 64, rc_lo: float = 0.01, rc_hi: float = 0.05):
    """Vortex centres ~ U[0,1]^2, circulations ~ N(0,1), core radii ~ U[rc_lo, rc_hi].

    ``seed`` is an int or a tuple of ints fed to PCG64.  Draw order is fixed:
    centres (x then y per vortex), circulations, core radii.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(0.0, 1.0, size=(n_vortices, 2))
    gamma = rng.standard_normal(n_vortices)
    rc = rng.uniform(rc_lo, rc_hi, size=n_vortices)
    return centres, gamma, rc


def _vortex_g(s: np.ndarray, a: float):
    """g(s) = (1 - exp(-s/a))/s and g'(s) for the Lamb-Oseen profile, a = rc^2.

    For s/a < 1e-3 a four-term series is used to avoid cancellation.
    """
    x = s / a
    small = x < 1e-3
    xs = np.where(small, 1.0, x)
    ss = np.where(small, a, s)
    e = np.exp(-xs)
    g = -np.expm1(-xs) / ss
    gp = (ss * e / a - (-np.expm1(-xs))) / ss**2
    # series: (1-e^-x)/x = 1 - x/2 + x^2/6 - x^3/24 ; derivative in s
    g_ser = (1.0 - x / 2.0 + x * x / 6.0 - x**3 / 24.0) / a
    gp_ser = (-0.5 + x / 3.0 - x * x / 8.0 + x**3 / 30.0) / (a * a)
    return np.where(small, g_ser, g), np.where(small, gp_ser, gp)


def vortex_velocity_gradients(x: np.ndarray, y: np.ndarray, centres, gamma, rc):
    """Sum of analytic Lamb-Oseen velocity gradients (u_x, u_y, v_x, v_y).

    Each vortex has azimuthal velocity K (1 - exp(-r^2/rc^2)) / r, K = Gamma/2pi,
    i.e. (u, v) = K g(r^2) (-Y, X) with X = x - xc, Y = y - yc.
    """
    ux = np.zeros_like(x)
    uy = np.zeros_like(x)
    vx = np.zeros_like(x)
    vy = np.zeros_like(x)
    for (xc, yc), gm, r in zip(centres, gamma, rc):
        K = gm / (2.0 * math.pi)
        X = x - xc
        Y = y - yc
        s = X * X + Y * Y
        g, gp = _vortex_g(s, r * r)
        ux += -2.0 * K * X * Y * gp
        uy += -K * (g + 2.0 * Y * Y * gp)
        vx += K * (g + 2.0 * X * X * gp)
        vy += 2.0 * K * X * Y * gp
    return ux, uy, vx, vy


def vortex_velocity(x: np.ndarray, y: np.ndarray, centres, gamma, rc):
    """Sum of Lamb-Oseen velocities (u, v) = K g(r^2) (-Y, X), K = Gamma / 2pi."""
    u = np.zeros_like(x)
    v = np.zeros_like(x)
    for (xc, yc), gm, r in zip(centres, gamma, rc):
        K = gm / (2.0 * math.pi)
        X = x - xc
        Y = y - yc
        g, _ = _vortex_g(X * X + Y * Y, r * r)
        u += -K * g * Y
        v += K * g * X
    return u, v


def vortex_velocity_grid(g: GridSpec, seed, n_vortices: int = 64):
    """(u, v) of `lamb_oseen_params(seed, n_vortices)` at the nodes of g, shape (ny, nx) each."""
    centres, gamma, rc = lamb_oseen_params(seed, n_vortices)
    x, y = grid_nodes(g)
    u, v = vortex_velocity(x.ravel(), y.ravel(), centres, gamma, rc)
    return u.reshape(g.ny, g.nx), v.reshape(g.ny, g.nx)


def smoothed_heaviside(d: np.ndarray, eps: float) -> np.ndarray:
    """0 for d <= -eps, 1 for d >= eps, and 1/2 (1 + d/eps + sin(pi d/eps)/pi) in between
    (a cosine-mollified step of half-width eps)."""
    d = np.asarray(d, dtype=np.float64)
    mid = 0.5 * (1.0 + d / eps + np.sin(math.pi * d / eps) / math.pi)
    return np.where(d <= -eps, 0.0, np.where(d >= eps, 1.0, mid))


def ellipse_body(g: GridSpec, cx: float = 0.5, cy: float = 0.5, a: float = 0.2, b: float = 0.05,
                 omega: float = 1.0, vel=(0.0, 0.0)):
    """Characteristic function and body velocity of a rigid ellipse on the grid: chi is the
    smoothed step (half-width 2h) of the scaled inside distance min(a, b) (1 - rho_e), rho_e the
    ellipse radius function; (us, vs) is a rigid motion with translation vel and rotation omega
    about the centre."""
    x, y = grid_nodes(g)
    re = np.sqrt(((x - cx) / a) ** 2 + ((y - cy) / b) ** 2)
    chi = smoothed_heaviside(min(a, b) * (1.0 - re), 2.0 * g.h)
    us = vel[0] - omega * (y - cy)
    vs = vel[1] + omega * (x - cx)
    return chi, us, vs


def vortex_source(g: GridSpec, seed, n_vortices: int = 64, rho: float = 1.0, mask=None,
                  chunk: int = 1 << 18, workers: int | None = None) -> np.ndarray:
    """f = 2 rho (u_x v_y - u_y v_x) of a seeded Lamb-Oseen superposition.

    The gradients are summed over all vortices before f is formed (f is
    quadratic in the velocity).  Shape (ny, nx).  With ``mask`` ((ny, nx)
    booleans) f is evaluated only where the mask is true and is 0 elsewhere.
    The work is split into chunks of nodes evaluated on a thread pool; each
    node's value does not depend on the chunking.
    """
    import concurrent.futures as cf
    import os

    centres, gamma, rc = lamb_oseen_params(seed, n_vortices)
    f = np.zeros(g.ny * g.nx, dtype=np.float64)
    idx = np.arange(g.ny * g.nx) if mask is None else np.flatnonzero(np.asarray(mask).ravel())
    if idx.size == 0:
        return f.reshape(g.ny, g.nx)

    def run(lo):
        sel = idx[lo:lo + chunk]
        i = (sel % g.nx).astype(np.float64)
        j = (sel // g.nx).astype(np.float64)
        x = g.x0 + (i + 0.5) * g.h
        y = g.y0 + (j + 0.5) * g.h
        ux, uy, vx, vy = vortex_velocity_gradients(x, y, centres, gamma, rc)
        f[sel] = 2.0 * rho * (ux * vy - uy * vx)

    workers = workers or min(16, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(run, range(0, idx.size, chunk)))
    return f.reshape(g.ny, g.nx)


def midline(x: np.ndarray, yc: float = 0.5, amp: float = 0.1, phase: float = 0.0,
            x_head: float = 0.2, length_x: float = 0.6) -> np.ndarray:
    """y_m(x) = yc + amp sin(2 pi ((x - x_head)/length_x - phase)): one wavelength over the body."""
    return yc + amp * np.sin(2.0 * math.pi * ((x - x_head) / length_x - phase))


def band_mask(g: GridSpec, half_width: float = 0.05, **mid_kw) -> np.ndarray:
    """True where x_head <= x <= x_head + length_x and |y - y_m(x)| <= half_width."""
    x, y = grid_nodes(g)
    x_head = mid_kw.get("x_head", 0.2)
    length_x = mid_kw.get("length_x", 0.6)
    inside_x = (x >= x_head) & (x <= x_head + length_x)
    return inside_x & (np.abs(y - midline(x, **mid_kw)) <= half_width)


def envelope_weight(g: GridSpec, centres_y=(0.35, 0.65), phases=(0.0, 0.25), width: float = 0.02,
                    amp: float = 0.1, x_head: float = 0.2, length_x: float = 0.6) -> np.ndarray:
    """E(x) = sum_j exp(-d_j^2 / width^2) around two deforming midlines.

    d_j^2 = (y - y_j(x))^2 + (distance of x outside [x_head, x_head+length_x])^2.
    """
    x, y = grid_nodes(g)
    out_x = np.maximum(0.0, np.maximum(x_head - x, x - (x_head + length_x)))
    e = np.zeros_like(x)
    for cy, ph in zip(centres_y, phases):
        dy = y - midline(x, yc=cy, amp=amp, phase=ph, x_head=x_head, length_x=length_x)
        e += np.exp(-(dy * dy + out_x * out_x) / width**2)
    return e


def ellipse_targets(n: int, cx: float = 0.5, cy: float = 0.5, a: float = 0.2, b: float = 0.05):
    """n points at equal parametric angle 2 pi k / n on an axis-aligned ellipse."""
    t = 2.0 * math.pi * np.arange(n, dtype=np.float64) / n
    return cx + a * np.cos(t), cy + b * np.sin(t)


def fish_half_width(s: np.ndarray, L: float) -> np.ndarray:
    """Half-width w(s) of the zebrafish-like profile, eq. fishWidth (Sec. 3.2).

    w_h = s_b = 0.04 L, s_t = 0.95 L, w_t = 0.01 L; s is arclength from the head.
    """
    wh = sb = 0.04 * L
    st = 0.95 * L
    wt = 0.01 * L
    s = np.asarray(s, dtype=np.float64)
    head = np.sqrt(np.maximum(2.0 * wh * s - s * s, 0.0))
    mid = wh - (wh - wt) * (s - sb) / (st - sb)
    tail = wt * (L - s) / (L - st)
    return np.where(s < sb, head, np.where(s < st, mid, tail))


def fish_surface_targets(n_per_side: int, h: float, yc: float = 0.5, amp: float = 0.1, phase: float = 0.0,
                         x_head: float = 0.2, length_x: float = 0.6, lift: float = 2.0):
    """Body-surface points and lifted-surface points of a fish-like body.

    The midline is the graph y_m(x) over [x_head, x_head + length_x]; the body
    length L is its arclength, and s runs from the head.  Each side gets
    ``n_per_side`` points at s_k = (k + 1/2) L / n_per_side; a surface point is
    midline(s) +- w(s) n(s) with n the unit normal of the midline, and its
    lifted copy is moved a further ``lift * h`` along the same normal.

    Returns (sx, sy, lx, ly): surface and lifted coordinates, each of length
    2 * n_per_side (upper side first, then lower side).
    """
    xs = np.linspace(x_head, x_head + length_x, 200001)
    ys = midline(xs, yc=yc, amp=amp, phase=phase, x_head=x_head, length_x=length_x)
    seg = np.hypot(np.diff(xs), np.diff(ys))
    arc = np.concatenate([[0.0], np.cumsum(seg)])
    L = arc[-1]
    s = (np.arange(n_per_side, dtype=np.float64) + 0.5) * L / n_per_side
    x = np.interp(s, arc, xs)
    y = midline(x, yc=yc, amp=amp, phase=phase, x_head=x_head, length_x=length_x)
    dydx = amp * 2.0 * math.pi / length_x * np.cos(2.0 * math.pi * ((x - x_head) / length_x - phase))
    norm = np.sqrt(1.0 + dydx * dydx)
    nx_, ny_ = -dydx / norm, 1.0 / norm
    w = fish_half_width(s, L)
    sx = np.concatenate([x + w * nx_, x - w * nx_])
    sy = np.concatenate([y + w * ny_, y - w * ny_])
    d = lift * h
    lx = np.concatenate([x + (w + d) * nx_, x - (w + d) * nx_])
    ly = np.concatenate([y + (w + d) * ny_, y - (w + d) * ny_])
    return sx, sy, lx, ly


def polygon_panels(vx, vy):
    """Surface panels of a closed polygon with counter-clockwise vertices (vx, vy):
    panel k runs from vertex k to vertex k+1 (cyclically); returns its midpoint
    (mx, my), its outward unit normal (nx, ny) and its length ds."""
    vx = np.asarray(vx, dtype=np.float64)
    vy = np.asarray(vy, dtype=np.float64)
    ex = np.roll(vx, -1) - vx
    ey = np.roll(vy, -1) - vy
    ds = np.hypot(ex, ey)
    return 0.5 * (vx + np.roll(vx, -1)), 0.5 * (vy + np.roll(vy, -1)), ey / ds, -ex / ds, ds


def ellipse_panels(n: int, cx: float = 0.5, cy: float = 0.5, a: float = 0.2, b: float = 0.05):
    """Panels of the polygon through n points at equal parametric angle on an ellipse."""
    vx, vy = ellipse_targets(n, cx, cy, a, b)
    return polygon_panels(vx, vy)


def fish_panels(n_per_side: int, h: float, **fish_kw):
    """Panels of the closed polygon through the fish-surface points of
    ``fish_surface_targets`` (lower side from head to tail, then the upper side
    back to the head: counter-clockwise)."""
    sx, sy, _, _ = fish_surface_targets(n_per_side, h, **fish_kw)
    upper_x, upper_y = sx[:n_per_side], sy[:n_per_side]
    lower_x, lower_y = sx[n_per_side:], sy[n_per_side:]
    vx = np.concatenate([lower_x, upper_x[::-1]])
    vy = np.concatenate([lower_y, upper_y[::-1]])
    return polygon_panels(vx, vy)


def stretched_axis(n: int, beta: float = 2.0, centre: float = 0.5):
    """Cell centres and widths of a 1-D grid on [0, 1] refined towards `centre`:
    edges proportional to sinh(beta (u - centre)) for uniform u, shifted and
    scaled so that the first edge is 0 and the last is 1."""
    u = np.linspace(0.0, 1.0, n + 1)
    e = np.sinh(beta * (u - centre))
    e = (e - e[0]) / (e[-1] - e[0])
    return 0.5 * (e[1:] + e[:-1]), np.diff(e)


def stretched_sources(n: int, seed, n_vortices: int = 64, beta: float = 2.0, rho: float = 1.0):
    """Scattered sources with their own cell areas: the cell centres of an n x n
    tensor-product grid stretched towards (0.5, 0.5), with f the Lamb-Oseen
    source 2 rho (u_x v_y - u_y v_x) at each centre and w = f dx_i dy_j."""
    cx, dx = stretched_axis(n, beta)
    xx, yy = np.meshgrid(cx, cx)
    ax, ay = np.meshgrid(dx, dx)
    centres, gamma, rc = lamb_oseen_params(seed, n_vortices)
    ux, uy, vx, vy = vortex_velocity_gradients(xx.ravel(), yy.ravel(), centres, gamma, rc)
    f = 2.0 * rho * (ux * vy - uy * vx)
    return xx.ravel(), yy.ravel(), f * (ax * ay).ravel()


def _flat_nodes(g: GridSpec):
    x, y = grid_nodes(g)
    return x.ravel(), y.ravel()


def workload(name: str):
    """Build a named workload.  Returns a dict with keys

    grid (GridSpec), f ((ny, nx) FP64), tx, ty (FP64 targets), p, theta,
    precision ('fp64' or 'mixed'), n_grid_targets (how many leading targets
    are grid nodes), seed, and a short description.
    """
    if name not in WORKLOADS:
        raise KeyError(f"unknown workload {name!r}; have {sorted(WORKLOADS)}")
    return WORKLOADS[name]()


def _gaussian64():
    g = GridSpec(64, 64, 1.0 / 64)
    f = gaussian_source(g)
    tx, ty = _flat_nodes(g)
    return dict(name="gaussian64", grid=g, f=f, tx=tx, ty=ty, p=8, theta=0.5, precision="fp64",
                n_grid_targets=tx.size, seed=None,
                desc="64x64 Gaussian (sigma 0.1) on [0,1]^2, targets = the 4096 nodes, p=8, theta=0.5")


def _vortex_grid(n: int, seed, n_ellipse: int, p: int, theta: float, precision: str, name: str):
    g = GridSpec(n, n, 1.0 / n)
    f = vortex_source(g, seed)
    gx, gy = _flat_nodes(g)
    ex, ey = ellipse_targets(n_ellipse)
    return dict(name=name, grid=g, f=f, tx=np.concatenate([gx, ex]), ty=np.concatenate([gy, ey]),
                p=p, theta=theta, precision=precision, n_grid_targets=gx.size, seed=seed,
                desc=f"{n}x{n} Lamb-Oseen vortex source (64 vortices, seed {seed}), targets = {n*n} nodes"
                     f" + {n_ellipse} ellipse points, p={p}, theta={theta}")


def _vortex512():
    return _vortex_grid(512, 2, 2048, 12, 0.5, "mixed", "vortex512")


def _band2048():
    n = 2048
    g = GridSpec(n, n, 1.0 / n)
    f = vortex_source(g, 3, mask=band_mask(g))
    sx, sy, lx, ly = fish_surface_targets(4096, g.h)
    return dict(name="band2048", grid=g, f=f, tx=np.concatenate([sx, lx]), ty=np.concatenate([sy, ly]),
                p=16, theta=0.4, precision="mixed", n_grid_targets=0, seed=3,
                desc="2048x2048 vortex source masked to a band |y-y_m|<=0.05 around a sinusoidal midline;"
                     " 8192 fish-surface + 8192 lifted (2h) targets; p=16, theta=0.4")


def _envelope4096():
    n = 4096
    g = GridSpec(n, n, 1.0 / n)
    e = envelope_weight(g)
    keep = e >= 1e-16
    f = vortex_source(g, 5, mask=keep) * e
    f[~keep] = 0.0
    txs, tys = [], []
    lxs, lys = [], []
    for cy, ph in ((0.35, 0.0), (0.65, 0.25)):
        sx, sy, lx, ly = fish_surface_targets(4096, g.h, yc=cy, phase=ph)
        txs.append(sx); tys.append(sy); lxs.append(lx); lys.append(ly)
    tx = np.concatenate(txs + lxs)
    ty = np.concatenate(tys + lys)
    return dict(name="envelope4096", grid=g, f=f, tx=tx, ty=ty, p=12, theta=0.5, precision="mixed",
                n_grid_targets=0, seed=5,
                desc="4096x4096 vortex source times a two-band Gaussian envelope (width 0.02), sources with"
                     " envelope < 1e-16 set to zero; 16384 surface + 16384 lifted targets; p=12, theta=0.5")


def points_workload(n: int = 256, n_ellipse: int = 2048, seed=6):
    """Scattered-source case: the stretched-grid sources of `stretched_sources`
    (n x n), targets = every 7th source position (exact coincidences) plus an
    ellipse of n_ellipse points; p = 12, theta = 0.5."""
    sx, sy, w = stretched_sources(n, seed)
    ex, ey = ellipse_targets(n_ellipse)
    return dict(name=f"stretched{n}", sx=sx, sy=sy, w=w, tx=np.concatenate([sx[::7], ex]),
                ty=np.concatenate([sy[::7], ey]), p=12, theta=0.5, seed=seed)


WORKLOADS = {
    "gaussian64": _gaussian64,
    "vortex512": _vortex512,
    "band2048": _band2048,
    "envelope4096": _envelope4096,
}


def vortex_source_device(g: GridSpec, seed, n_vortices: int = 64, rho: float = 1.0, device="cuda"):
    """``vortex_source`` evaluated with torch in FP64 on a device (same parameters and formulas).

    Used where many fields are needed quickly (the serving stream); values agree
    with the NumPy version to rounding.  Returns a (ny, nx) float64 tensor.
    """
    import torch

    centres, gamma, rc = lamb_oseen_params(seed, n_vortices)
    i = torch.arange(g.nx, dtype=torch.float64, device=device)
    j = torch.arange(g.ny, dtype=torch.float64, device=device)
    x = (g.x0 + (i + 0.5) * g.h)[None, :].expand(g.ny, g.nx)
    y = (g.y0 + (j + 0.5) * g.h)[:, None].expand(g.ny, g.nx)
    ux = torch.zeros((g.ny, g.nx), dtype=torch.float64, device=device)
    uy = torch.zeros_like(ux)
    vx = torch.zeros_like(ux)
    vy = torch.zeros_like(ux)
    for (xc, yc), gm, r in zip(centres, gamma, rc):
        K = float(gm) / (2.0 * math.pi)
        a = float(r) * float(r)
        X = x - float(xc)
        Y = y - float(yc)
        s = X * X + Y * Y
        xs = s / a
        small = xs < 1e-3
        xsafe = torch.where(small, torch.ones_like(xs), xs)
        ssafe = torch.where(small, torch.full_like(s, a), s)
        om = -torch.expm1(-xsafe)
        gg = om / ssafe
        gp = (ssafe * torch.exp(-xsafe) / a - om) / (ssafe * ssafe)
        g_ser = (1.0 - xs / 2.0 + xs * xs / 6.0 - xs ** 3 / 24.0) / a
        gp_ser = (-0.5 + xs / 3.0 - xs * xs / 8.0 + xs ** 3 / 30.0) / (a * a)
        gg = torch.where(small, g_ser, gg)
        gp = torch.where(small, gp_ser, gp)
        ux += -2.0 * K * X * Y * gp
        uy += -K * (gg + 2.0 * Y * Y * gp)
        vx += K * (gg + 2.0 * X * X * gp)
        vy += 2.0 * K * X * Y * gp
    return 2.0 * rho * (ux * vy - uy * vx)


def serving_requests(n_requests: int = 256, seed: int = 4, device="cuda"):
    """The serving stream: independent solves of uneven size.

    Request k draws, from PCG64((seed, k)): grid n uniform in {128, 256, 512, 1024}
    (h = 1/n on the unit square), a fresh Lamb-Oseen field with U{16..128}
    vortices (field seed (seed, k, 1)), U{1024..8192} targets that are either
    an ellipse (semi-axes 0.2, 0.05) or a fish surface plus its 2h-lifted copy
    (random phase), each with probability 1/2.  Parameters p = 12, theta = 0.5,
    mixed precision.  Returns a list of dicts with device tensors f, tx, ty.
    """
    import torch

    out = []
    for k in range(n_requests):
        rng = np.random.Generator(np.random.PCG64((seed, k)))
        n = int(rng.choice([128, 256, 512, 1024]))
        nv = int(rng.integers(16, 129))
        m = int(rng.integers(1024, 8193))
        fish = bool(rng.uniform() < 0.5)
        phase = float(rng.uniform())
        g = GridSpec(n, n, 1.0 / n)
        f = vortex_source_device(g, (seed, k, 1), nv, device=device)
        if fish:
            nps = max(1, m // 4)
            sx, sy, lx, ly = fish_surface_targets(nps, g.h, phase=phase)
            tx, ty = np.concatenate([sx, lx]), np.concatenate([sy, ly])
        else:
            tx, ty = ellipse_targets(m)
        out.append(dict(k=k, grid=g, f=f, tx=torch.as_tensor(tx, device=device),
                        ty=torch.as_tensor(ty, device=device), p=12, theta=0.5, precision="mixed",
                        shape="fish" if fish else "ellipse", vortices=nv))
    return out
