"""GPU tests of the pressure surface forces (pp_surface_forces, eq. Fpress,
FpressNet, CdP) against the oracle's exactly rounded sums, alone and after a
pressure solve at the panel points of two fish bodies."""

import numpy as np
import pytest

from oracle import direct, forces
from workloads import generators as G

from gpu_common import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_04398_amd as pp
    s = pp.Solver(0)
    yield s
    s.close()


def _two_bodies(n=700):
    a = G.fish_panels(n, 1.0 / 512, yc=0.35)
    b = G.ellipse_panels(n + 123, 0.5, 0.7, 0.15, 0.04)
    return [np.concatenate([x, y]) for x, y in zip(a, b)], [0, a[0].size, a[0].size + b[0].size]


def test_forces_match_oracle(solver):
    (mx, my, nx, ny, ds), seg = _two_bodies()
    rng = np.random.Generator(np.random.PCG64(2))
    p = rng.standard_normal(mx.size) + 3.0 * mx
    dfx_r, dfy_r, ref = forces.surface_forces(p, nx, ny, ds, seg, 0.3, -0.1, 1.2, 0.08)
    got, dfx, dfy = solver.surface_forces(p, nx, ny, ds, seg, u=(0.3, -0.1), rho=1.2, area=0.08, pointwise=True)
    assert np.array_equal(dfx, dfx_r) and np.array_equal(dfy, dfy_r)
    for g, r, a, b in zip(got, ref, seg[:-1], seg[1:]):
        scale = float(np.sum(np.abs(dfx_r[a:b])) + np.sum(np.abs(dfy_r[a:b])))
        for k in ("fx", "fy", "drag"):
            assert abs(g[k] - r[k]) <= 1e-15 * scale, (k, g[k], r[k])
        assert abs(g["cd"] - r["cd"]) <= 1e-13 * abs(r["cd"]) + 1e-15 * scale


def test_forces_after_solve_device(solver):
    """Two fish bodies: pressure from the tree-code at the panel points, then the forces, all on the
    device; against the oracle's direct pressure and sums."""
    n = 256
    g = G.GridSpec(n, n, 1.0 / n)
    f = G.vortex_source(g, 7, 24)
    (mx, my, nx, ny, ds), seg = _two_bodies(600)
    P_ref = direct.direct_grid(f, g.h, mx, my)
    _, _, ref = forces.surface_forces(P_ref, nx, ny, ds, seg, 1.0, 0.0, 1.0, 0.6)
    fd, txd, tyd, nxd, nyd, dsd = to_dev(f, mx, my, nx, ny, ds)
    Pd = solver.solve_grid(fd, g.h, txd, tyd, p=12, theta=0.5, precision="mixed")
    got = solver.surface_forces(Pd, nxd, nyd, dsd, seg, u=(1.0, 0.0), rho=1.0, area=0.6)
    P = to_host(Pd)
    for gg, r, a, b in zip(got, ref, seg[:-1], seg[1:]):
        scale = float(np.sum(np.abs(P_ref[a:b] * ds[a:b])))
        assert abs(gg["fx"] - r["fx"]) < 1e-5 * scale and abs(gg["fy"] - r["fy"]) < 1e-5 * scale
    # and the GPU forces of the GPU pressure equal the oracle's sums of the same pressure
    _, _, same = forces.surface_forces(P, nx, ny, ds, seg, 1.0, 0.0, 1.0, 0.6)
    for gg, r in zip(got, same):
        assert abs(gg["fx"] - r["fx"]) < 1e-13 and abs(gg["fy"] - r["fy"]) < 1e-13


def test_forces_errors(solver):
    import paper_1610_04398_amd as pp
    (mx, my, nx, ny, ds), seg = _two_bodies(50)
    p = np.ones(mx.size)
    for bad in ([0, 10], [1, mx.size], [0, 80, 60, mx.size]):
        with pytest.raises(pp.PPError) as e:
            solver.surface_forces(p, nx, ny, ds, bad)
        assert e.value.status == -1
    with pytest.raises(pp.PPError):
        solver.surface_forces(p, nx, ny, ds, seg, u=(0.0, 0.0))
    with pytest.raises(pp.PPError):
        solver.surface_forces(p, nx, ny, ds, seg, rho=-1.0)
