"""Pins of the reference surface-force sums (eq. Fpress, eq. FpressNet, eq. CdP).

For panels of a closed polygon (normal and length of each edge, pressure at the
edge midpoint): a constant pressure gives no net force; a linear pressure
a x + b y + c gives exactly -(a, b) times the enclosed area (divergence theorem;
the midpoint rule is exact for a linear integrand on each edge); the potential
flow around a cylinder gives zero drag and the known lateral distribution; and
a hand-computed square checks the drag projection and the coefficient.
"""

import math

import numpy as np

from oracle import forces
from workloads import generators as G


def _area(mx, my, nx, ny, ds):
    return 0.5 * math.fsum((mx * nx * ds + my * ny * ds).tolist())


def test_constant_pressure_has_no_net_force():
    mx, my, nx, ny, ds = G.fish_panels(512, 1.0 / 1024)
    _, _, out = forces.surface_forces(np.full(mx.size, 3.7), nx, ny, ds, [0, mx.size], 1.0, 0.0, 1.0, 1.0)
    scale = 3.7 * ds.sum()
    assert abs(out[0]["fx"]) < 1e-15 * scale and abs(out[0]["fy"]) < 1e-15 * scale


def test_linear_pressure_gives_gradient_times_area():
    for mx, my, nx, ny, ds in (G.ellipse_panels(777), G.fish_panels(300, 1.0 / 512)):
        a, b, c = 1.3, -0.7, 2.0
        p = a * mx + b * my + c
        _, _, out = forces.surface_forces(p, nx, ny, ds, [0, mx.size], 1.0, 0.0, 1.0, 1.0)
        A = _area(mx, my, nx, ny, ds)
        assert abs(out[0]["fx"] + a * A) < 1e-14 and abs(out[0]["fy"] + b * A) < 1e-14


def test_potential_flow_cylinder_has_no_drag():
    """P = P_inf + rho U^2 / 2 (1 - 4 sin^2 theta) on a cylinder: d'Alembert, no net force."""
    n = 4096
    R, U, rho = 0.1, 2.0, 1.2
    mx, my, nx, ny, ds = G.ellipse_panels(n, 0.0, 0.0, R, R)
    th = np.arctan2(my, mx)
    p = 5.0 + 0.5 * rho * U * U * (1.0 - 4.0 * np.sin(th) ** 2)
    _, _, out = forces.surface_forces(p, nx, ny, ds, [0, n], U, 0.0, rho, 2 * R)
    assert abs(out[0]["drag"]) < 1e-12 and abs(out[0]["fy"]) < 1e-12 and abs(out[0]["cd"]) < 1e-10


def test_hand_computed_square_and_segments():
    # unit square, CCW, pressure 2 on the left edge and 0 elsewhere: F = (+2, 0) (pushes to +x)
    mx, my, nx, ny, ds = G.polygon_panels([0.0, 1.0, 1.0, 0.0], [0.0, 0.0, 1.0, 1.0])
    p = np.where(mx < 0.25, 2.0, 0.0)
    # two segments: the square alone, then the square again with pressure doubled
    P = np.concatenate([p, 2 * p])
    N = lambda a: np.concatenate([a, a])  # noqa: E731
    dfx, dfy, out = forces.surface_forces(P, N(nx), N(ny), N(ds), [0, 4, 8], 3.0, 4.0, 0.5, 2.0)
    assert out[0]["fx"] == 2.0 and out[0]["fy"] == 0.0
    assert out[1]["fx"] == 4.0
    # drag along U = (3, 4)/5: 2 * 3/5 = 1.2; Cd = 2 * 1.2 / (0.5 * 25 * 2) = 0.096
    assert abs(out[0]["drag"] - 1.2) < 1e-15 and abs(out[0]["cd"] - 0.096) < 1e-15
    assert np.array_equal(dfx[:4], -p * nx * ds)
