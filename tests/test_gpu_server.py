"""GPU tests of the serving loop (pp_server_* through the C ABI).

Each served result must equal the same request solved alone, bit for bit;
admission must keep the estimated footprints in flight within the budget; a
failing request must report its own status without disturbing the others.
"""

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


def _requests(n=10, seed=31):
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for k in range(n):
        size = int(rng.choice([64, 128, 256]))
        g = G.GridSpec(size, size, 1.0 / size)
        f = G.vortex_source(g, (seed, k), int(rng.integers(8, 24)))
        m = int(rng.integers(300, 3000))
        if k % 2:
            tx, ty = G.ellipse_targets(m)
        else:
            sx, sy, lx, ly = G.fish_surface_targets(max(1, m // 4), g.h, phase=float(rng.uniform()))
            tx, ty = np.concatenate([sx, lx]), np.concatenate([sy, ly])
        reqs.append(dict(g=g, f=f, tx=tx, ty=ty))
    return reqs


def test_served_equals_alone(pp):
    reqs = _requests()
    solver = pp.Solver(0)
    alone = [solver.solve_grid(r["f"], r["g"].h, r["tx"], r["ty"], p=12, theta=0.5, precision="mixed")
             for r in reqs]
    solver.close()
    srv = pp.Server(0, max_slots=4)
    outs, tickets = [], []
    for i, r in enumerate(reqs):
        if i % 3 == 0:  # device inputs and outputs for some requests
            f, tx, ty = to_dev(r["f"], r["tx"], r["ty"])
            import torch
            out = torch.empty(tx.numel(), dtype=torch.float64, device="cuda")
        else:
            f, tx, ty = r["f"], r["tx"], r["ty"]
            out = np.empty(tx.size)
        outs.append(out)
        tickets.append(srv.submit(f, r["g"].h, tx, ty, out, p=12, theta=0.5, precision="mixed"))
    infos = [srv.wait(t) for t in tickets]
    srv.close()
    slots = {inf["slot"] for inf in infos}
    for a, o in zip(alone, outs):
        got = to_host(o) if not isinstance(o, np.ndarray) else o
        assert np.array_equal(a, got)
    assert len(slots) > 1  # the work was spread over several slots
    # and the answers are right
    r = reqs[1]
    ref = direct.direct_grid(r["f"], r["g"].h, r["tx"], r["ty"])
    assert rel_l2(alone[1], ref) < 1e-4


def test_admission_respects_budget(pp):
    reqs = _requests(n=8, seed=5)
    fps = [pp.pp_footprint_estimate(r["g"].nx, r["g"].ny, r["tx"].size, 12, 64) for r in reqs]
    budget = max(fps) + min(fps) // 2  # at most ~one request in flight at a time
    srv = pp.Server(0, max_slots=4, hbm_budget_bytes=budget)
    outs = [np.empty(r["tx"].size) for r in reqs]
    tickets = [srv.submit(r["f"], r["g"].h, r["tx"], r["ty"], o) for r, o in zip(reqs, outs)]
    infos = [srv.wait(t) for t in tickets]
    srv.close()
    # at every start, the footprints of the requests then running fit the budget
    for i, a in enumerate(infos):
        running = [j for j, b in enumerate(infos) if b["start_us"] <= a["start_us"] < b["end_us"]]
        assert sum(fps[j] for j in running) <= budget or len(running) == 1, (i, running)


def test_resident_memory_stays_under_budget(pp):
    """Idle slots keep their buffers between requests; the admission counts them, and a slot whose
    buffers leave the total above the budget after a large request releases them, so that once every
    request has finished the slots hold at most the budget (and results stay bitwise those of a lone
    solve)."""
    reqs = _requests(n=8, seed=14)
    fps = sorted(pp.pp_footprint_estimate(r["g"].nx, r["g"].ny, r["tx"].size, 12, 64) for r in reqs)
    budget = fps[-1] + fps[0]
    srv = pp.Server(0, max_slots=3, hbm_budget_bytes=budget)
    outs = [np.empty(r["tx"].size) for r in reqs]
    tickets = [srv.submit(r["f"], r["g"].h, r["tx"], r["ty"], o) for r, o in zip(reqs, outs)]
    for t in tickets:
        srv.wait(t)
    held = srv.device_bytes()
    srv.close()
    assert held <= budget, (held, budget)
    s = pp.Solver(0)
    try:
        for r, o in zip(reqs[:3], outs[:3]):
            assert np.array_equal(s.solve_grid(r["f"], r["g"].h, r["tx"], r["ty"], p=12, theta=0.5,
                                               precision="mixed"), o)
    finally:
        s.close()


def test_failing_request_reports_its_own_status(pp):
    reqs = _requests(n=4, seed=7)
    srv = pp.Server(0, max_slots=2)
    outs = [np.empty(r["tx"].size) for r in reqs]
    bad_tx = reqs[2]["tx"].copy()
    bad_tx[0] = 5.0  # outside the root square
    tickets = []
    for i, (r, o) in enumerate(zip(reqs, outs)):
        tx = bad_tx if i == 2 else r["tx"]
        tickets.append(srv.submit(r["f"], r["g"].h, tx, r["ty"], o))
    for i, t in enumerate(tickets):
        if i == 2:
            with pytest.raises(pp.PPError) as e:
                srv.wait(t)
            assert e.value.status == -2
        else:
            srv.wait(t)
    srv.close()


def test_work_budget_admission(pp):
    """With a work bound, the requests running together never exceed it (a lone request always runs)."""
    reqs = _requests(n=10, seed=12)
    works = [r["g"].nx * r["g"].ny + r["tx"].size for r in reqs]
    budget = max(works)
    srv = pp.Server(0, max_slots=4, work_budget_points=budget)
    outs = [np.empty(r["tx"].size) for r in reqs]
    tickets = [srv.submit(r["f"], r["g"].h, r["tx"], r["ty"], o) for r, o in zip(reqs, outs)]
    infos = [srv.wait(t) for t in tickets]
    srv.close()
    for i, a in enumerate(infos):
        running = [j for j, b in enumerate(infos) if b["start_us"] <= a["start_us"] < b["end_us"]]
        assert sum(works[j] for j in running) <= budget or len(running) == 1, (i, running)


def test_cancel_queued_request(pp):
    """A request still in the queue can be withdrawn; its output stays untouched."""
    reqs = _requests(n=6, seed=13)
    srv = pp.Server(0, max_slots=1)
    outs = [np.full(r["tx"].size, 7.0) for r in reqs]
    tickets = [srv.submit(r["f"], r["g"].h, r["tx"], r["ty"], o) for r, o in zip(reqs, outs)]
    assert srv.cancel(tickets[-1]) is True  # one slot: the last cannot have started yet
    for t in tickets[:-1]:
        srv.wait(t)
    with pytest.raises(pp.PPError) as e:
        srv.wait(tickets[-1])
    assert e.value.status == -7
    assert np.all(outs[-1] == 7.0)
    with pytest.raises(pp.PPError):  # released by its wait: an unknown ticket now
        srv.cancel(tickets[-1])
    srv.close()


def test_fused_batches_equal_alone(pp):
    """With max_batch = 4 and one slot, queued requests of one shape (device inputs and outputs) are solved
    together in one set of launches: several tickets share their start and end; every result is bitwise the
    request's lone solve; a request whose target lies outside its square fails alone (the batch is then
    solved one request at a time) and the others still succeed; host-input requests are served unbatched."""
    import torch
    rng = np.random.Generator(np.random.PCG64(12))
    reqs = []
    for k in range(11):
        size = (128, 256)[k % 2] if k < 9 else 128
        g = G.GridSpec(size, size, 1.0 / size)
        f = G.vortex_source(g, (12, k), int(rng.integers(8, 24)))
        tx, ty = G.ellipse_targets(int(rng.integers(300, 2000)))
        if k == 4:
            tx = tx.copy()
            tx[7] = 1.25  # outside the unit square
        reqs.append(dict(g=g, f=f, tx=tx, ty=ty, host=k == 10))
    solver = pp.Solver(0)
    alone = []
    for r in reqs:
        try:
            alone.append(solver.solve_grid(r["f"], r["g"].h, r["tx"], r["ty"]))
        except pp.PPError as e:
            alone.append(e.status)
    solver.close()
    srv = pp.Server(0, max_slots=1, max_batch=4)
    outs, tickets = [], []
    for r in reqs:
        if r["host"]:
            f, tx, ty, out = r["f"], r["tx"], r["ty"], np.empty(r["tx"].size)
        else:
            f, tx, ty = to_dev(r["f"], r["tx"], r["ty"])
            out = torch.empty(tx.numel(), dtype=torch.float64, device="cuda")
        outs.append(out)
        tickets.append(srv.submit(f, r["g"].h, tx, ty, out))
    infos = []
    for k, t in enumerate(tickets):
        if isinstance(alone[k], int):
            with pytest.raises(pp.PPError) as e:
                srv.wait(t)
            assert e.value.status == alone[k]
            infos.append(None)
        else:
            infos.append(srv.wait(t))
    srv.close()
    for k, (a, o) in enumerate(zip(alone, outs)):
        if isinstance(a, int):
            continue
        got = o if isinstance(o, np.ndarray) else to_host(o)
        assert np.array_equal(a, got), k
    spans = [(i["start_us"], i["end_us"]) for i in infos if i is not None]
    assert len(set(spans)) < len(spans)  # some requests ran as one batch
