"""Batched solves (pp_solve_grid_batch through the C ABI): several requests of one grid geometry solved as one
forest in one set of launches.  Each request's output is bitwise that of its lone pp_solve_grid: the forest
keeps every request's tree, lists and arithmetic.  Checked for 2 to 5 requests (one and two forest levels), mixed
and FP64 precision, both self rules (grid-node targets), a request without targets, and the refusals."""

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


def _requests(n, count, seed):
    """count requests on an n x n grid (h = 1/n): their own vortex fields (some with a zero band), and targets
    that are an ellipse, a fish surface with its lifted copy, or a subset of the grid nodes."""
    g = G.GridSpec(n, n, 1.0 / n)
    x, y = G.grid_nodes(g)
    reqs = []
    for r in range(count):
        rng = np.random.Generator(np.random.PCG64((seed, r)))
        f = G.vortex_source(g, (seed, r), int(rng.integers(8, 32)))
        if r % 2:
            f[:, : n // 4] = 0.0
        kind = r % 3
        if kind == 0:
            tx, ty = G.ellipse_targets(int(rng.integers(200, 3000)))
        elif kind == 1:
            sx, sy, lx, ly = G.fish_surface_targets(int(rng.integers(100, 800)), g.h, phase=float(rng.uniform()))
            tx, ty = np.concatenate([sx, lx]), np.concatenate([sy, ly])
        else:
            pick = rng.choice(x.size, int(rng.integers(500, 4000)), replace=False)
            tx, ty = x.ravel()[pick], y.ravel()[pick]
        reqs.append((f, tx, ty))
    return g, reqs


@pytest.mark.parametrize("n,count", [(128, 2), (128, 4), (256, 3), (64, 5)])
@pytest.mark.parametrize("precision,self_mode", [("mixed", "skip"), ("fp64", "cellavg")])
def test_batch_equals_lone_solves(pp, n, count, precision, self_mode):
    g, reqs = _requests(n, count, seed=n + count)
    kw = dict(p=12, theta=0.5, leaf_max=64, precision=precision, self_mode=self_mode)
    dev = [to_dev(f, tx, ty) for f, tx, ty in reqs]
    s, lone = pp.Solver(0), pp.Solver(0)
    try:
        outs = s.solve_grid_batch([d[0] for d in dev], g.h, [d[1] for d in dev], [d[2] for d in dev], **kw)
        for r, (fd, txd, tyd) in enumerate(dev):
            want = to_host(lone.solve_grid(fd, g.h, txd, tyd, **kw))
            assert np.array_equal(to_host(outs[r]), want), (r, np.max(np.abs(to_host(outs[r]) - want)))
        # and against the oracle for one request
        f, tx, ty = reqs[-1]
        ref = direct.direct_grid(f, g.h, tx, ty, self_mode=1 if self_mode == "cellavg" else 0)
        assert rel_l2(to_host(outs[-1]), ref) < (1e-6 if precision == "mixed" else 1e-8)
    finally:
        s.close()
        lone.close()


def test_batch_request_without_targets_and_repeat(pp):
    """A request with no targets takes part (its sources only); the same context then solves a lone grid and a
    second batch, each bitwise as alone."""
    import torch
    g, reqs = _requests(128, 3, seed=9)
    dev = [to_dev(f, tx, ty) for f, tx, ty in reqs]
    empty = torch.empty(0, dtype=torch.float64, device="cuda")
    s, lone = pp.Solver(0), pp.Solver(0)
    try:
        fs = [d[0] for d in dev]
        txs = [dev[0][1], empty, dev[2][1]]
        tys = [dev[0][2], empty, dev[2][2]]
        outs = s.solve_grid_batch(fs, g.h, txs, tys)
        assert outs[1].numel() == 0
        for r in (0, 2):
            assert np.array_equal(to_host(outs[r]), to_host(lone.solve_grid(fs[r], g.h, txs[r], tys[r])))
        one = to_host(s.solve_grid(fs[1], g.h, dev[1][1], dev[1][2]))
        assert np.array_equal(one, to_host(lone.solve_grid(fs[1], g.h, dev[1][1], dev[1][2])))
        outs = s.solve_grid_batch(fs[:2], g.h, [dev[0][1], dev[1][1]], [dev[0][2], dev[1][2]])
        for r in range(2):
            assert np.array_equal(to_host(outs[r]), to_host(lone.solve_grid(fs[r], g.h, dev[r][1], dev[r][2])))
    finally:
        s.close()
        lone.close()


def test_batch_refusals(pp):
    import torch
    g, reqs = _requests(128, 2, seed=3)
    dev = [to_dev(f, tx, ty) for f, tx, ty in reqs]
    fs, txs, tys = [d[0] for d in dev], [d[1] for d in dev], [d[2] for d in dev]
    s = pp.Solver(0)
    try:
        with pytest.raises(pp.PPError) as e:  # a target outside its request's square
            bad = txs[1].clone()
            bad[3] = 1.5
            s.solve_grid_batch(fs, g.h, [txs[0], bad], tys)
        assert e.value.status == -2
        small = [torch.zeros((16, 16), dtype=torch.float64, device="cuda")] * 2
        with pytest.raises(pp.PPError) as e:  # grids below 33 nodes a side
            s.solve_grid_batch(small, 1.0 / 16, txs, tys)
        assert e.value.status == -1
        with pytest.raises(pp.PPError) as e:  # more than 16 requests
            s.solve_grid_batch(fs * 9, g.h, txs * 9, tys * 9)
        assert e.value.status == -1
        out = s.solve_grid_batch(fs, g.h, txs, tys)  # still usable
        assert all(bool(torch.isfinite(o).all()) for o in out)
    finally:
        s.close()
