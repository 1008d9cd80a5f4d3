"""Plain reference of the pressure forces on body surfaces.

TEST INFRASTRUCTURE ONLY (it shares no code with the GPU library).

Sec. 2.3.1 of the paper: the pressure at the exact surface points gives the
pointwise force d F_P = -P n dS (eq. Fpress); its closed surface integral is the
net pressure force F_P (eq. FpressNet), whose projection on the free stream is
the pressure drag, with the drag coefficient 2 Drag / (rho |U|^2 A) (eq. CdP).
On a discretised surface (panels j with normal n_j and length dS_j, P_j the
pressure at the panel point) the integral is the sum over the panels; here it
is summed exactly rounded (math.fsum), one closed surface per segment.
"""

from __future__ import annotations

import math

import numpy as np


def surface_forces(p, nx, ny, ds, seg_start, ux: float, uy: float, rho: float, area: float):
    """Per-panel forces (dfx, dfy) and, per segment [seg_start[s], seg_start[s+1]), the net force,
    the drag along U and the drag coefficient.  Returns (dfx, dfy, [dict(fx, fy, drag, cd), ...])."""
    p = np.asarray(p, dtype=np.float64)
    nx = np.asarray(nx, dtype=np.float64)
    ny = np.asarray(ny, dtype=np.float64)
    ds = np.asarray(ds, dtype=np.float64)
    dfx = -p * nx * ds
    dfy = -p * ny * ds
    speed = math.hypot(ux, uy)
    out = []
    for s in range(len(seg_start) - 1):
        a, b = int(seg_start[s]), int(seg_start[s + 1])
        fx = math.fsum(dfx[a:b].tolist())
        fy = math.fsum(dfy[a:b].tolist())
        drag = (fx * ux + fy * uy) / speed
        cd = 2.0 * drag / (rho * speed * speed * area)
        out.append(dict(fx=fx, fy=fy, drag=drag, cd=cd))
    return dfx, dfy, out
