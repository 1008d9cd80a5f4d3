"""GPU parity tests of the scattered-source entry points (pp_solve_points,
pp_direct_points) against the FP64 oracle direct sum over the same points."""

import numpy as np
import pytest

from oracle import direct
from workloads import generators as G

from gpu_common import rel_l2, rel_max, to_dev, to_host

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


def _clustered(seed, n=3000, m=1500):
    """Gaussian clusters of sources with signed weights (some exactly zero), targets
    partly on sources (exact coincidence), partly random."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = 5
    c = rng.uniform(0.2, 0.8, (k, 2))
    lab = rng.integers(0, k, n)
    sx = c[lab, 0] + 0.03 * rng.standard_normal(n)
    sy = c[lab, 1] + 0.03 * rng.standard_normal(n)
    w = rng.standard_normal(n) * rng.uniform(0.5, 2.0, n) * 1e-4
    w[rng.uniform(size=n) < 0.1] = 0.0
    tx = np.concatenate([sx[: m // 3], rng.uniform(0.0, 1.0, m - m // 3)])
    ty = np.concatenate([sy[: m // 3], rng.uniform(0.0, 1.0, m - m // 3)])
    return sx, sy, w, tx, ty


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_direct_points(solver, precision, tol):
    sx, sy, w, tx, ty = _clustered(1)
    ref = direct.direct_points(sx, sy, w, tx, ty)
    got = solver.direct_points(sx, sy, w, tx, ty, leaf_max=32, precision=precision)
    assert rel_l2(got, ref) < tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("mixed", 1e-4)])
@pytest.mark.parametrize("seed,leaf_max", [(2, 16), (3, 64)])
def test_tree_points(solver, precision, tol, seed, leaf_max):
    sx, sy, w, tx, ty = _clustered(seed)
    ref = direct.direct_points(sx, sy, w, tx, ty)
    got = solver.solve_points(sx, sy, w, tx, ty, p=12, theta=0.5, leaf_max=leaf_max, precision=precision)
    assert rel_l2(got, ref) < tol
    assert rel_max(got, ref) < 10 * tol
    st = solver.stats()
    assert st["nsources"] == int(np.count_nonzero(w))
    assert st["n_m2l"] > 0


def test_points_match_grid_nodes(solver):
    """Grid nodes given as scattered points with w = f h^2: same sum as the grid entry point."""
    w0 = G.workload("gaussian64")
    g = w0["grid"]
    x, y = G.grid_nodes(g)
    rng = np.random.Generator(np.random.PCG64(9))
    tx = rng.uniform(0.0, 1.0, 800)
    ty = rng.uniform(0.0, 1.0, 800)
    ref = direct.direct_grid(w0["f"], g.h, tx, ty)
    a = solver.solve_grid(w0["f"], g.h, tx, ty, p=12, theta=0.5, precision="fp64")
    b = solver.solve_points(x.ravel(), y.ravel(), (w0["f"] * g.h * g.h).ravel(), tx, ty, p=12, theta=0.5,
                            precision="fp64")
    assert rel_l2(a, ref) < 1e-7 and rel_l2(b, ref) < 1e-7


def test_stretched_sources_device(solver):
    """Stretched-grid sources with per-cell areas, device pointers, every 7th source a target."""
    wl = G.points_workload(256)
    sx, sy, w, tx, ty = to_dev(wl["sx"], wl["sy"], wl["w"], wl["tx"], wl["ty"])
    got = to_host(solver.solve_points(sx, sy, w, tx, ty, p=wl["p"], theta=wl["theta"], precision="mixed"))
    rng = np.random.Generator(np.random.PCG64(5))
    sel = rng.choice(wl["tx"].size, 700, replace=False)
    ref = direct.direct_points(wl["sx"], wl["sy"], wl["w"], wl["tx"][sel], wl["ty"][sel])
    assert rel_l2(got[sel], ref) < 1e-4
    again = to_host(solver.solve_points(sx, sy, w, tx, ty, p=wl["p"], theta=wl["theta"], precision="mixed"))
    assert np.array_equal(got, again)


def test_points_degenerate(solver):
    import paper_1610_04398_amd as pp
    rng = np.random.Generator(np.random.PCG64(4))
    tx, ty = rng.uniform(size=50), rng.uniform(size=50)
    # no sources, and sources with zero weight only
    assert np.all(solver.solve_points(np.zeros(0), np.zeros(0), np.zeros(0), tx, ty) == 0.0)
    z = np.zeros(10)
    assert np.all(solver.solve_points(rng.uniform(size=10), rng.uniform(size=10), z, tx, ty) == 0.0)
    # one source, one coincident target (skipped) and one other target
    sx, sy, w = np.array([0.3]), np.array([0.4]), np.array([2.0])
    got = solver.solve_points(sx, sy, w, np.array([0.3, 0.7]), np.array([0.4, 0.4]), precision="fp64")
    assert got[0] == 0.0
    assert abs(got[1] - 2.0 * np.log(0.4) / (2 * np.pi)) < 1e-14
    # all points coincide
    got = solver.solve_points(np.full(5, 0.5), np.full(5, 0.5), np.ones(5), np.array([0.5]), np.array([0.5]))
    assert got[0] == 0.0
    # the cell-average self rule has no cell here
    with pytest.raises(pp.PPError) as e:
        solver._run_points(pp.pp_solve_points, sx, sy, w, tx, ty, pp.make_params(self_mode="cellavg"), None, None)
    assert e.value.status == -1
    bad = sx.copy()
    bad[0] = np.nan
    with pytest.raises(pp.PPError) as e:
        solver.solve_points(bad, sy, w, tx, ty)
    assert e.value.status == -1


def test_points_multi_tile_sort(solver):
    """Point sources over many sort tiles (32-bit keys, four passes, ragged tail): the tree solve stays
    within the mixed tolerance of the direct sum and counts every nonzero source."""
    sx, sy, w, tx, ty = _clustered(9, n=2 * 4096 + 77, m=2000)
    ref = direct.direct_points(sx, sy, w, tx, ty)
    got = solver.solve_points(sx, sy, w, tx, ty, p=12, theta=0.5, leaf_max=32, precision="mixed")
    assert rel_l2(got, ref) < 1e-4
    assert solver.stats()["nsources"] == int(np.count_nonzero(w))


@pytest.mark.parametrize("method", ["fmm", "treecode"])
def test_points_timed_schedule_matches(monkeypatch, method):
    """The timed schedule (near field between HIP events; the per-leaf packing rides on the list launch)
    gives the same bits as the untimed one, for scattered sources."""
    import paper_1610_04398_amd as pp
    sx, sy, w, tx, ty = _clustered(13, n=5000, m=2500)
    kw = dict(p=12, theta=0.5, leaf_max=32, precision="mixed", method=method)
    monkeypatch.setenv("PP_DIRECT_ISSUE", "0")  # untimed calls replay the second segment from a graph
    s = pp.Solver(0)
    try:
        base = s.solve_points(sx, sy, w, tx, ty, **kw)
        s.set_profiling(2)
        timed = s.solve_points(sx, sy, w, tx, ty, **kw)
        again = s.solve_points(sx, sy, w, tx, ty, **kw)
        assert s.stats()["ms_phase"]["p2p"] > 0.0
    finally:
        s.close()
    assert np.array_equal(base, timed) and np.array_equal(base, again)
    assert rel_l2(base, direct.direct_points(sx, sy, w, tx, ty)) < 1e-4
