"""Plain reference of the steps around the Poisson solve that work on the
gridded velocity: the pressure source and the viscous surface forces.

TEST INFRASTRUCTURE ONLY (it shares no code with the GPU library).

Source (eq. PoissonFinal): f = -rho (grad u^T : grad u) + rho lambda div(chi (u_s - u)),
with grad u^T : grad u = u_{j,i} u_{i,j} = u_x^2 + 2 u_y v_x + v_y^2 in 2-D.
Viscous forces (Sec. 2.3.2): dF = 2 mu D . n dS (eq. Fvisc), D = (grad u + grad u^T) / 2,
with grad u taken on the lifted surface by nearest-neighbour interpolation, i.e. the
finite-difference gradient of the grid node nearest to the lifted point; the net force,
drag and coefficient follow eq. FviscNet and eq. CdNu.

Readings (the paper names neither a difference scheme nor the interpolation details):
* derivatives of node fields are second-order central differences at interior nodes and
  second-order one-sided three-point differences on the first and last row/column
  (a single node along an axis has derivative 0 along it; two nodes use the two-point
  difference);
* the nearest node of a point (x, y) is (floor((x - x0)/h), floor((y - y0)/h)) clamped to
  the grid (node (i, j) sits at the centre of that cell).
Every expression is written with explicit operation order; numpy does not fuse.
"""

from __future__ import annotations

import math

import numpy as np


def derivative(a: np.ndarray, h: float, axis: int) -> np.ndarray:
    """d a / d x (axis = 1, columns) or d a / d y (axis = 0, rows) of a node field a[j, i]."""
    a = np.asarray(a, dtype=np.float64)
    a = np.moveaxis(a, axis, 0)
    n = a.shape[0]
    out = np.zeros_like(a)
    two_h = 2.0 * h
    if n >= 3:
        out[1:-1] = (a[2:] - a[:-2]) / two_h
        out[0] = ((-3.0 * a[0] + 4.0 * a[1]) - a[2]) / two_h
        out[-1] = ((3.0 * a[-1] - 4.0 * a[-2]) + a[-3]) / two_h
    elif n == 2:
        out[0] = (a[1] - a[0]) / h
        out[1] = (a[1] - a[0]) / h
    return np.moveaxis(out, 0, axis)


def velocity_gradients(u, v, h):
    """(u_x, u_y, v_x, v_y) at every node."""
    return derivative(u, h, 1), derivative(u, h, 0), derivative(v, h, 1), derivative(v, h, 0)


def pressure_source(u, v, h, rho: float = 1.0, lam: float = 0.0, chi=None, us=None, vs=None):
    """f of eq. PoissonFinal at every node (shape of u)."""
    ux, uy, vx, vy = velocity_gradients(u, v, h)
    f = -rho * ((ux * ux + 2.0 * (uy * vx)) + vy * vy)
    if chi is not None and lam != 0.0:
        px = np.asarray(chi) * (np.asarray(us) - np.asarray(u))
        py = np.asarray(chi) * (np.asarray(vs) - np.asarray(v))
        f = f + (rho * lam) * (derivative(px, h, 1) + derivative(py, h, 0))
    return f


def nearest_node(x, y, x0: float, y0: float, h: float, nx: int, ny: int):
    i = np.clip(np.floor((np.asarray(x, dtype=np.float64) - x0) / h), 0, nx - 1).astype(np.int64)
    j = np.clip(np.floor((np.asarray(y, dtype=np.float64) - y0) / h), 0, ny - 1).astype(np.int64)
    return i, j


def viscous_forces(u, v, h, x0, y0, lx, ly, nx, ny, ds, seg_start, mu, ux_inf, uy_inf, rho, area):
    """Per-panel traction force (dfx, dfy) = 2 mu D(nearest node of the lifted point) n dS and, per
    segment, the net force, drag and coefficient (exactly rounded sums)."""
    u = np.asarray(u, dtype=np.float64)
    gy_, gx_ = u.shape
    ux, uy, vx, vy = velocity_gradients(u, v, h)
    i, j = nearest_node(lx, ly, x0, y0, h, gx_, gy_)
    dux, duy, dvx, dvy = ux[j, i], uy[j, i], vx[j, i], vy[j, i]
    nx = np.asarray(nx, dtype=np.float64)
    ny = np.asarray(ny, dtype=np.float64)
    ds = np.asarray(ds, dtype=np.float64)
    off = 0.5 * (duy + dvx)
    two_mu = 2.0 * mu
    dfx = (two_mu * (dux * nx + off * ny)) * ds
    dfy = (two_mu * (off * nx + dvy * ny)) * ds
    speed = math.hypot(ux_inf, uy_inf)
    out = []
    for s in range(len(seg_start) - 1):
        a, b = int(seg_start[s]), int(seg_start[s + 1])
        fx = math.fsum(dfx[a:b].tolist())
        fy = math.fsum(dfy[a:b].tolist())
        drag = (fx * ux_inf + fy * uy_inf) / speed
        out.append(dict(fx=fx, fy=fy, drag=drag, cd=2.0 * drag / (rho * speed * speed * area)))
    return dfx, dfy, out
