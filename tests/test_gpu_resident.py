"""Resident solves (pp_solve_grid_resident through the C ABI): the tree, lists and target sort of the last
grid solve are kept, and a new source on the same grid (with no new nonzero node) is solved without
rebuilding them.  With the same nonzero nodes the result is bitwise that of a fresh pp_solve_grid; with
fewer, it matches the oracle to the accuracy contract; a node that becomes nonzero, or a target that leaves
its finest cell, is refused with the output untouched."""

import numpy as np
import pytest

from oracle import direct
from workloads import generators as G

from gpu_common import rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_04398_amd as pp
    return pp


def _case(seed=3, n=128, masked=True):
    g = G.GridSpec(n, n, 1.0 / n)
    f = G.vortex_source(g, seed, 24)
    if masked:
        f[:, : n // 5] = 0.0  # a region with no sources: the tree is adaptive there
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y = G.grid_nodes(g)
    tx = np.concatenate([x.ravel()[::5], *G.ellipse_targets(700)[:1]])
    ty = np.concatenate([y.ravel()[::5], *G.ellipse_targets(700)[1:]])
    return g, f, tx, ty, rng


def _moved_within_cells(tx, ty, h, rng):
    """Every target moved to another point of the same finest cell (its floor((t - x0) / h) unchanged)."""
    cx, cy = np.floor(tx / h), np.floor(ty / h)
    nx_ = (cx + rng.uniform(0.05, 0.95, tx.size)) * h
    ny_ = (cy + rng.uniform(0.05, 0.95, ty.size)) * h
    keep = (np.floor(nx_ / h) == cx) & (np.floor(ny_ / h) == cy)
    return np.where(keep, nx_, tx), np.where(keep, ny_, ty)


@pytest.mark.parametrize("method", ["fmm", "treecode"])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("lists", ["onepass", "exact"])
def test_resident_equals_fresh_solve(pp, monkeypatch, method, precision, lists):
    """Same nonzero nodes, new values, targets moved inside their cells: bitwise the fresh solve, on two
    resident calls in a row (device inputs; the near field on the side stream, and all on one stream)."""
    if lists == "exact":
        monkeypatch.setenv("PP_EXACT_LISTS", "1")
    s = pp.Solver(0)
    ref = pp.Solver(0)
    monkeypatch.delenv("PP_EXACT_LISTS", raising=False)
    try:
        g, f, tx, ty, rng = _case()
        kw = dict(p=12, theta=0.5, leaf_max=32, precision=precision, method=method)
        fd, txd, tyd = to_dev(f, tx, ty)
        s.solve_grid(fd, g.h, txd, tyd, **kw)
        for it in range(2):
            f2 = f * (1.5 + it) + np.where(f != 0.0, 0.25 * rng.standard_normal(f.shape), 0.0)
            tx2, ty2 = _moved_within_cells(tx, ty, g.h, rng)
            f2d, tx2d, ty2d = to_dev(f2, tx2, ty2)
            got = to_host(s.solve_grid_resident(f2d, tx2d, ty2d))
            want = to_host(ref.solve_grid(f2d, g.h, tx2d, ty2d, **kw))
            assert np.array_equal(got, want), (it, np.max(np.abs(got - want)))
            assert s.stats()["ncells"] == ref.stats()["ncells"]
            assert s.stats()["n_p2p_pairs"] == ref.stats()["n_p2p_pairs"]
    finally:
        s.close()
        ref.close()


def test_resident_with_fewer_sources_matches_oracle(pp):
    """Nodes that became zero keep their place in the tree with weight 0: the result still matches the
    FP64 direct sum of the new f (host inputs here)."""
    s = pp.Solver(0)
    try:
        g, f, tx, ty, rng = _case(seed=4)
        s.solve_grid(f, g.h, tx, ty, precision="mixed")
        f3 = f.copy()
        f3[rng.uniform(size=f.shape) < 0.3] = 0.0
        got = s.solve_grid_resident(f3, tx, ty)
        e = rel_l2(got, direct.direct_grid(f3, g.h, tx, ty))
        assert e < 1e-6, e
    finally:
        s.close()


def test_resident_refuses_a_tree_that_does_not_fit(pp):
    import torch
    s = pp.Solver(0)
    try:
        g, f, tx, ty, rng = _case(seed=5)
        with pytest.raises(pp.PPError) as e:  # nothing retained yet
            s.solve_grid_resident(f, tx, ty)
        assert e.value.status == -1
        base = s.solve_grid(f, g.h, tx, ty, precision="mixed")
        out = torch.full((tx.size,), 7.0, dtype=torch.float64, device="cuda")
        fd, txd, tyd = to_dev(f, tx, ty)
        # a node outside the retained sources becomes nonzero
        f4 = f.copy()
        f4[10, 3] = 1.0
        assert f[10, 3] == 0.0
        with pytest.raises(pp.PPError) as e:
            s.solve_grid_resident(to_dev(f4)[0], txd, tyd, out=out)
        assert e.value.status == -1 and bool(torch.all(out == 7.0))
        # a target leaves its finest cell
        tx5 = tx.copy()
        tx5[17] += g.h
        with pytest.raises(pp.PPError) as e:
            s.solve_grid_resident(fd, to_dev(tx5)[0], tyd, out=out)
        assert e.value.status == -1 and bool(torch.all(out == 7.0))
        # a non-finite value
        f6 = f.copy()
        f6[0, 0] = np.inf
        with pytest.raises(pp.PPError) as e:
            s.solve_grid_resident(to_dev(f6)[0], txd, tyd, out=out)
        assert e.value.status == -1 and bool(torch.all(out == 7.0))
        # the retained tree is still there
        again = to_host(s.solve_grid_resident(fd, txd, tyd, out=out))
        assert np.array_equal(again, base)
        # a scattered-source solve keeps no grid tree
        s.solve_points(np.array([0.3, 0.6]), np.array([0.4, 0.5]), np.array([1.0, -2.0]), tx[:10], ty[:10])
        with pytest.raises(pp.PPError) as e:
            s.solve_grid_resident(f, tx, ty)
        assert e.value.status == -1
    finally:
        s.close()


def test_resident_multi_group_grid(pp):
    """A 1100^2 grid (2,048 Morton tiles, counted in groups of two): with the same nonzero nodes the resident
    solve is bitwise the fresh one; with nodes zeroed it agrees with the fresh solve to the accuracy contract;
    a node that becomes nonzero in a late tile (inside a zero patch) is refused."""
    n = 1100
    h = 1.0 / n
    rng = np.random.Generator(np.random.PCG64(2024))
    f = rng.standard_normal((n, n))
    f[rng.uniform(size=f.shape) < 0.5] = 0.0
    f[900:1000, 900:1000] = 0.0
    tx, ty = rng.uniform(0, 1, 2000), rng.uniform(0, 1, 2000)
    s, ref = pp.Solver(0), pp.Solver(0)
    try:
        kw = dict(p=10, theta=0.5, precision="mixed")
        txd, tyd = to_dev(tx, ty)
        s.solve_grid(to_dev(f)[0], h, txd, tyd, **kw)
        f2d = to_dev(1.7 * f)[0]
        got = to_host(s.solve_grid_resident(f2d, txd, tyd))
        assert np.array_equal(got, to_host(ref.solve_grid(f2d, h, txd, tyd, **kw)))
        f3 = 1.7 * f
        f3[rng.uniform(size=f.shape) < 0.2] = 0.0
        f3d = to_dev(f3)[0]
        got = to_host(s.solve_grid_resident(f3d, txd, tyd))
        assert rel_l2(got, to_host(ref.solve_grid(f3d, h, txd, tyd, **kw))) < 1e-6
        f4 = f.copy()
        f4[950, 950] = 1.0
        with pytest.raises(pp.PPError) as e:
            s.solve_grid_resident(to_dev(f4)[0], txd, tyd)
        assert e.value.status == -1
    finally:
        s.close()
        ref.close()


@pytest.mark.parametrize("method", ["fmm", "treecode"])
def test_resident_graph_replay(pp, monkeypatch, method):
    """With PP_RESIDENT_GRAPH=1, repeated resident solves on the same device buffers (f, targets, output
    changed in place) run as one captured graph from the third call with those buffers on (first launches
    and the whole second segment, no host round trip inside); two sets of buffers used in turn keep a graph
    each.  Each of eight calls, with eager device work between them, equals a fresh solve bit for bit; a
    refused call (a node outside the tree turned nonzero) leaves the output alone and the next one replays
    again."""
    import torch
    monkeypatch.setenv("PP_RESIDENT_GRAPH", "1")
    s = pp.Solver(0)
    monkeypatch.delenv("PP_RESIDENT_GRAPH")
    ref = pp.Solver(0)
    try:
        g, f, tx, ty, rng = _case(seed=6)
        kw = dict(p=12, theta=0.5, leaf_max=32, precision="mixed", method=method)
        sets = [to_dev(f, tx, ty) + [torch.empty(tx.size, dtype=torch.float64, device="cuda")] for _ in range(2)]
        s.solve_grid(sets[0][0], g.h, sets[0][1], sets[0][2], **kw)
        nz = torch.as_tensor(f != 0.0, device="cuda")
        zero = int(np.argwhere(f.ravel() == 0.0)[0, 0])
        for it in range(8):
            fd, txd, tyd, out = sets[it % 2]
            fd.copy_(torch.as_tensor(f * (1.0 + 0.3 * it), device="cuda"))
            fd.add_(0.1 * torch.randn_like(fd) * nz)
            mx, my = _moved_within_cells(tx, ty, g.h, rng)
            txd.copy_(torch.as_tensor(mx, device="cuda"))
            tyd.copy_(torch.as_tensor(my, device="cuda"))
            torch.randn(1 << 16, device="cuda").sum()  # eager work between replays
            if it == 6:
                fd.view(-1)[zero] = 1.0
                out.fill_(7.0)
                with pytest.raises(pp.PPError):
                    s.solve_grid_resident(fd, txd, tyd, out=out)
                assert bool(torch.all(out == 7.0))
                fd.view(-1)[zero] = 0.0
            s.solve_grid_resident(fd, txd, tyd, out=out)
            want = to_host(ref.solve_grid(fd, g.h, txd, tyd, **kw))
            assert np.array_equal(to_host(out), want), it
    finally:
        s.close()
        ref.close()
