"""Pins of the reference source assembly (eq. PoissonFinal) and viscous forces
(eq. Fvisc, FviscNet, CdNu).

The difference formulas are exact for quadratic fields (inside and on the
boundary), so a quadratic velocity gives the analytic source at every node; a
Lamb-Oseen field converges to its analytic source at second order; the
penalisation divergence of a linear field is its trace; and a Poiseuille flow
around a grid-aligned square whose panel midpoints are nodes gives the net
viscous force 2 mu (area, 0) exactly (divergence theorem).
"""

import math

import numpy as np

from oracle import assembly
from workloads import generators as G


def _quadratic(g):
    x, y = G.grid_nodes(g)
    u = 0.3 * x * x - 1.1 * x * y + 0.7 * y * y + 0.2 * x - 0.5 * y + 1.0
    v = -0.4 * x * x + 0.9 * x * y - 0.6 * y * y - 0.3 * x + 0.8 * y - 2.0
    ux = 0.6 * x - 1.1 * y + 0.2
    uy = -1.1 * x + 1.4 * y - 0.5
    vx = -0.8 * x + 0.9 * y - 0.3
    vy = 0.9 * x - 1.2 * y + 0.8
    return u, v, ux, uy, vx, vy


def test_gradients_exact_for_quadratics():
    g = G.GridSpec(17, 11, 0.0625, 0.3, -0.2)
    u, v, ux, uy, vx, vy = _quadratic(g)
    got = assembly.velocity_gradients(u, v, g.h)
    for a, b in zip(got, (ux, uy, vx, vy)):
        assert np.max(np.abs(a - b)) < 1e-12


def test_source_of_quadratic_field_is_analytic():
    g = G.GridSpec(20, 20, 0.05)
    u, v, ux, uy, vx, vy = _quadratic(g)
    rho = 1.3
    f = assembly.pressure_source(u, v, g.h, rho)
    expect = -rho * (ux * ux + 2 * uy * vx + vy * vy)
    assert np.max(np.abs(f - expect)) < 1e-11


def test_lamb_oseen_source_converges_second_order():
    """The FD source of the sampled Lamb-Oseen velocity tends to the analytic 2 rho (u_x v_y - u_y v_x)."""
    errs = []
    for n in (64, 128, 256):
        g = G.GridSpec(n, n, 1.0 / n)
        u, v = G.vortex_velocity_grid(g, 3, 4)
        f = assembly.pressure_source(u, v, g.h)
        exact = G.vortex_source(g, 3, 4)
        inner = (slice(2, -2), slice(2, -2))
        errs.append(np.max(np.abs(f[inner] - exact[inner])) / np.max(np.abs(exact)))
    assert errs[1] < errs[0] / 3.5 and errs[2] < errs[1] / 3.5


def test_penalisation_term_of_a_linear_field():
    g = G.GridSpec(12, 9, 0.1)
    x, y = G.grid_nodes(g)
    u = np.zeros_like(x)
    v = np.zeros_like(x)
    us = 0.4 * x - 0.3 * y + 1.0
    vs = 0.2 * x + 0.7 * y
    f = assembly.pressure_source(u, v, g.h, rho=2.0, lam=5.0, chi=np.ones_like(x), us=us, vs=vs)
    assert np.max(np.abs(f - 2.0 * 5.0 * (0.4 + 0.7))) < 1e-12


def test_viscous_force_of_poiseuille_flow_on_a_square():
    h = 0.01
    n = 60
    g = G.GridSpec(n, n, h)
    x, y = G.grid_nodes(g)
    u, v = y * y, np.zeros_like(y)
    # square with vertices on nodes (i, j) = (10, 10), (30, 10), (30, 30), (10, 30), split into panels of
    # two cells so that every panel midpoint is a node
    corners = [(10, 10), (30, 10), (30, 30), (10, 30)]
    vx, vy = [], []
    for k in range(4):
        (i0, j0), (i1, j1) = corners[k], corners[(k + 1) % 4]
        steps = max(abs(i1 - i0), abs(j1 - j0)) // 2
        for s in range(steps):
            vx.append((i0 + (i1 - i0) * s / steps + 0.5) * h)
            vy.append((j0 + (j1 - j0) * s / steps + 0.5) * h)
    mx, my, nx, ny, ds = G.polygon_panels(np.array(vx), np.array(vy))
    mu = 0.7
    _, _, out = assembly.viscous_forces(u, v, h, 0.0, 0.0, mx, my, nx, ny, ds, [0, mx.size], mu, 1.0, 0.0, 1.0, 1.0)
    area = (20 * h) ** 2
    assert abs(out[0]["fx"] - 2 * mu * area) < 1e-14 and abs(out[0]["fy"]) < 1e-14
    assert abs(out[0]["drag"] - 2 * mu * area) < 1e-14
