#!/usr/bin/env python3
"""Benchmark of the pressure-Poisson tree-code on one MI355X.

Workload (default ``envelope4096``, the largest single-GPU configuration): a
4096 x 4096 grid (h = 1/4096) of sources f = 2(u_x v_y - u_y v_x) from 64
seeded Lamb-Oseen vortices, times a two-band Gaussian envelope (width 0.02)
around two deforming fish midlines; nodes where the envelope is below 1e-16
are zero and culled, leaving 6.16M sources.  Targets: 16,384 points on the two
fish surfaces plus 16,384 lifted 2h along the normals.  p = 12, theta = 0.5,
mixed precision (FP32 + Kahan near field and local evaluation, FP64
expansions).

One step = one complete cold solve (ingest, target sort, tree, interaction
lists, P2M, M2M, M2L, L2L, L2P, P2P, finalize) with the inputs already resident
in device memory.  Also measured: the resident solve (the tree, lists and
target sort of the first solve kept, a new source with the same nonzero nodes
and new targets in the same cells: weights, expansions, near field and
finalize only), the per-phase breakdown with each phase's roofline fraction,
the 512^2 vortex workload (all grid nodes plus an ellipse as targets), and the
serving stream of uneven requests against the one-at-a-time path.

Prints one JSON line: solves/s, effective interactions/s against the GPU
all-pairs direct sum, accuracy against the FP64 CPU oracle on sampled targets,
the roofline of the dominant kernel (HIP events around its launch in the timed
solves) and of every phase, and the CPU oracle timed on a bounded sample on the
host cores.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks: HBM3E 8 TB/s; FP64 vector 78.6 TFLOP/s; FP32 lanes without packed instructions
# 256 CU x 64 lanes x 2.4 GHz = 39.3 T lane-ops/s (the near field's bound: one VALU issue per lane-op)
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Algorithmic FP32 lane operations of one near-field pair: dx, dy, dx^2, +dy^2 (fma), log2, and
# the weighted accumulation w*log2 (fma).  Compensation and loop overhead are not counted.
OPS_PER_PAIR = 6


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash(name: str) -> str:
    with open(os.path.join(ROOT, "paper_1610_04398_amd", "csrc", name), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_from_profile(workload: str, phase: str, **match):
    """HBM bytes per launch of a phase's kernel from the committed rocprofv3 counter summary
    (profiles/<phase>_<workload>_traffic.json), if it was taken on the current kernel source and
    the same settings; else None."""
    path = os.path.join(ROOT, "profiles", f"{phase}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_sha256_16") != kernel_source_hash(rec.get("kernel_source", "p2p.hip")):
        return None
    for k, v in match.items():
        if rec.get(k) != v:
            return None
    return rec.get("bytes_per_launch")


def phase_work(st: dict, w: dict, parts: int) -> dict:
    """Algorithmic work of each phase of one solve: (bound, amount, unit).  Bytes are what the phase
    must move at least (its inputs read once, its outputs written once); flops count an FMA as 2 and
    a complex multiply-add as 8; the near field counts 6 FP32 lane-ops per pair."""
    N, M = int(st["nsources"]), int(st["ntargets"])
    C, Ls = int(st["ncells"]), int(st["nsrc_leaves"])
    X, Y, Q = int(st["n_m2l"]), int(st["n_p2p_lists"]), int(st["n_p2p_pairs"])
    G = w["grid"].nx * w["grid"].ny
    p = int(w["p"])
    D = max(1, math.ceil(math.log2(max(w["grid"].nx, w["grid"].ny))))
    passes = math.ceil(2 * D / 8)
    cp = 16 * (p + 1)  # bytes of one expansion
    return {
        # read f once, write the node index and weight of every kept source (its key is the Morton index
        # of the node, formed where needed)
        "ingest": ("hbm", 8 * G + 12 * N, "B"),
        # target keys from the coordinates, then (key, index) read and written per radix pass
        "sort": ("hbm", 24 * M + passes * 16 * M, "B"),
        # sorted keys read once, cell arrays and list records written once
        "tree": ("hbm", 4 * (N + M) + 72 * C, "B"),
        # list entries written once, cell records read once
        "lists": ("hbm", 4 * (X + Y) + 32 * C, "B"),
        # source records (index, weight in; x, y, w FP32 out), target offsets and self data
        "pack": ("hbm", 24 * N + 64 * M, "B"),
        "p2m": ("fp64", (8 * p + 5) * N, "flop"),
        "m2m": ("fp64", 8 * (p + 1) ** 2 * max(C - 1, 0), "flop"),
        "m2l": ("fp64", 8 * (p + 1) ** 2 * X, "flop"),
        "l2l": ("fp64", 4 * (p + 1) * (p + 2) * C, "flop"),
        "l2p": ("alu", 8 * (p + 1) * M, "op"),
        "p2p": ("alu", OPS_PER_PAIR * Q, "op"),
        "finalize": ("hbm", (8 * parts + 44) * M + cp * min(C, M), "B"),
    }


def roofline_of(work, ms):
    bound, amount, unit = work
    t = ms * 1e-3
    if bound == "hbm":
        ideal = amount / (HBM_PEAK_GBS * 1e9)
        achieved, peak, u = amount / t / 1e9 if t > 0 else None, HBM_PEAK_GBS, "GB/s"
    elif bound == "fp64":
        ideal = amount / (FP64_PEAK_TFLOPS * 1e12)
        achieved, peak, u = amount / t / 1e12 if t > 0 else None, FP64_PEAK_TFLOPS, "TFLOP/s"
    else:
        ideal = amount / (VALU_PEAK_TOPS * 1e12)
        achieved, peak, u = amount / t / 1e12 if t > 0 else None, VALU_PEAK_TOPS, "T lane-op/s"
    return {"bound": bound, "work": amount, "work_unit": unit, "ms": ms, "achieved": achieved, "peak": peak,
            "unit": u, "frac": (achieved / peak) if achieved else None, "ideal_ms": ideal * 1e3}


def host_cpu_info() -> dict:
    """CPU model, sockets and logical CPUs of the host (from /proc/cpuinfo), and the CPUs this process may use."""
    model, sockets, logical = None, set(), 0
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                k, _, v = line.partition(":")
                k = k.strip()
                if k == "processor":
                    logical += 1
                elif k == "model name" and model is None:
                    model = v.strip()
                elif k == "physical id":
                    sockets.add(v.strip())
    except OSError:
        pass
    return {"model": model, "sockets": len(sockets) or None, "logical_cpus": logical or None,
            "usable_cpus": len(os.sched_getaffinity(0))}


def _percentile(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q))


def serving_run(pp, G, args, log):
    """Serving stream: the same Poisson arrival trace fed to a one-slot server (the plain
    one-solve-at-a-time path) and to a multi-slot server (continuous batching)."""
    import threading

    import numpy as np
    import torch

    log(f"[bench] serving: generating {args.serve_requests} requests")
    reqs = G.serving_requests(args.serve_requests, seed=4, device="cuda")
    torch.cuda.synchronize()
    # sequential throughput and the reference (alone) results
    s = pp.Solver(0)
    alone = []
    for r in reqs[:4]:
        s.solve_grid(r["f"], r["grid"].h, r["tx"], r["ty"], p=r["p"], theta=r["theta"], precision=r["precision"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs:
        alone.append(s.solve_grid(r["f"], r["grid"].h, r["tx"], r["ty"], p=r["p"], theta=r["theta"],
                                  precision=r["precision"]))
    torch.cuda.synchronize()
    seq_rate = len(reqs) / (time.perf_counter() - t0)
    s.close()
    lam = args.serve_load * seq_rate
    rng = np.random.Generator(np.random.PCG64(4))
    arrivals = np.cumsum(rng.exponential(1.0 / lam, len(reqs)))
    arrivals -= arrivals[0]

    def run(srv, slots, batch=0):
        outs = [torch.empty(r["tx"].numel(), dtype=torch.float64, device="cuda") for r in reqs]
        tickets = [None] * len(reqs)
        start = time.perf_counter()

        def submitter():
            for i, r in enumerate(reqs):
                delay = arrivals[i] - (time.perf_counter() - start)
                if delay > 0:
                    time.sleep(delay)
                tickets[i] = srv.submit(r["f"], r["grid"].h, r["tx"], r["ty"], outs[i], p=r["p"], theta=r["theta"],
                                        precision=r["precision"])

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        infos = [srv.wait(t) for t in tickets]
        makespan = max(i["end_us"] for i in infos) - min(i["start_us"] - i["queue_us"] for i in infos)
        lat = [i["total_us"] / 1e3 for i in infos]
        same = all(bool(torch.equal(o, a)) for o, a in zip(outs, alone))
        batched = len({(i["start_us"], i["end_us"]) for i in infos})
        return {"p50_ms": _percentile(lat, 50), "p99_ms": _percentile(lat, 99), "mean_ms": float(np.mean(lat)),
                "solves_per_s": len(reqs) / (makespan * 1e-6), "slots": slots, "max_batch": batch,
                "launch_sets": batched, "work_budget_points": args.serve_work_budget if slots > 1 else 0,
                "identical_to_alone": same}

    def median_run(slots, batch=0):
        # One server, in its steady state: the trace once to warm it up (each slot's buffers grow to the
        # largest request or batch it has run, and stay resident), then replayed args.serve_reps times;
        # the run with the median p99 is reported.
        srv = pp.Server(0, max_slots=slots, work_budget_points=args.serve_work_budget if slots > 1 else 0,
                        max_batch=batch)
        run(srv, slots, batch)
        runs = sorted((run(srv, slots, batch) for _ in range(args.serve_reps)), key=lambda r: r["p99_ms"])
        srv.close()
        out = dict(runs[len(runs) // 2])
        out["p99_ms_runs"] = [r["p99_ms"] for r in runs]
        out["identical_to_alone"] = all(r["identical_to_alone"] for r in runs)
        return out

    log("[bench] serving: one-slot (sequential) path")
    seq = median_run(1)
    log(f"[bench] serving: {args.serve_slots}-slot path, requests of one shape fused up to {args.serve_batch}")
    srv = median_run(args.serve_slots, args.serve_batch)
    log(f"[bench] serving: {args.serve_slots}-slot path without fused launches")
    unfused = median_run(args.serve_slots, 0)
    sizes = [r["grid"].nx for r in reqs]
    return {"requests": len(reqs), "arrival": f"Poisson, rate {lam:.1f}/s = {args.serve_load} x sequential "
                                               f"throughput ({seq_rate:.1f} solves/s)",
            "grid_sizes": {str(n): sizes.count(n) for n in sorted(set(sizes))},
            "sequential": seq, "served": srv, "served_without_fused_launches": unfused,
            "p99_speedup": seq["p99_ms"] / srv["p99_ms"] if srv["p99_ms"] > 0 else None,
            "note": "each path is one server in its steady state (the trace run once untimed, then replayed); "
                    "served: max_slots slots, queued requests of one shape solved together (pp_solve_grid_batch, "
                    "one set of launches); launch_sets counts the distinct (start, end) spans, fewer than the "
                    "requests when batches formed"}


def accuracy(P, w, n_samples, seed, oracle_direct):
    """rel-L2 and largest error (relative to max |P|) on seeded sampled grid and surface targets."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))
    M = P.size
    ng = int(w["n_grid_targets"])
    ns = M - ng
    k_grid = min(n_samples * 3 // 4, ng) if ns > 0 else min(n_samples, ng)
    k_surf = min(n_samples - k_grid, ns)
    sel_g = rng.choice(ng, k_grid, replace=False) if k_grid else np.zeros(0, int)
    sel_s = ng + rng.choice(ns, k_surf, replace=False) if k_surf else np.zeros(0, int)
    acc = {}
    for name, sel in (("grid", sel_g), ("surface", sel_s)):
        if sel.size == 0:
            continue
        ref = oracle_direct.direct_grid(w["f"], w["grid"].h, w["tx"][sel], w["ty"][sel])
        acc[name] = {"rel_l2": float(np.linalg.norm(P[sel] - ref) / np.linalg.norm(ref)),
                     "rel_max": float(np.max(np.abs(P[sel] - ref)) / np.max(np.abs(ref))),
                     "targets": int(sel.size)}
    return acc


def timed_solves(s, f, g, tx, ty, out, kw, steps, phase):
    """steps solves with HIP events around `phase`'s launches (on its stream); (solves/s, mean ms of
    the phase).  The solves run in the schedule of an untimed call."""
    import torch
    s.set_profiling(phase=phase)
    ph_sum = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.solve_grid(f, g.h, tx, ty, out=out, **kw)
        ph_sum += s.stats()["ms_phase"][phase]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s.set_profiling(0)
    return steps / el, el / steps * 1e3, ph_sum / steps


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="envelope4096")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--method", default="fmm", choices=["fmm", "treecode"],
                    help="fmm: M2L/L2L/L2P with the dual-tree acceptance; treecode: the paper's own variant (M2P)")
    ap.add_argument("--roofline-phase", default=None,
                    help="phase whose launches are bracketed by HIP events in the timed solves (default: the "
                         "phase with the largest time in the per-phase breakdown)")
    ap.add_argument("--direct-steps", type=int, default=2)
    ap.add_argument("--samples", type=int, default=2000, help="targets checked against the oracle")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--also", default="vortex512", help="second workload timed beside the main one ('' skips)")
    ap.add_argument("--serve-requests", type=int, default=256, help="requests in the serving stream (0: skip)")
    ap.add_argument("--serve-slots", type=int, default=2)
    ap.add_argument("--serve-batch", type=int, default=8, help="requests of one shape fused per launch set")
    ap.add_argument("--serve-reps", type=int, default=3, help="replays of the arrival trace per path (median p99)")
    ap.add_argument("--serve-work-budget", type=int, default=1300000,
                    help="server admission bound on in-flight grid nodes + targets (0: none)")
    ap.add_argument("--serve-load", type=float, default=0.8, help="arrival rate / sequential solves per second")
    ap.add_argument("--forces-panels", type=int, default=4096,
                    help="panels per side of each of two fish bodies for the force steps; 0 skips the source "
                         "assembly and force timings")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (the known-size kernel that scales "
                         "the HBM byte counters of a profile) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1 (sharding the solve over "
                                   "several GPUs is described, not implemented)"}))
        return 2

    import numpy as np
    import torch

    import paper_1610_04398_amd as pp
    from workloads import generators as G

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 1

    if args.copy_calibration > 0:
        n = args.copy_calibration << 17  # doubles
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read": n * 8, "bytes_written": n * 8, "launches": 3}}))
        return 0

    log(f"[bench] generating workload {args.workload}")
    w = G.workload(args.workload)
    g = w["grid"]
    dev = torch.device("cuda:0")
    f = torch.as_tensor(w["f"], device=dev)
    tx = torch.as_tensor(w["tx"], device=dev)
    ty = torch.as_tensor(w["ty"], device=dev)
    out = torch.empty(tx.numel(), dtype=torch.float64, device=dev)
    kw = dict(p=w["p"], theta=w["theta"], leaf_max=64, precision=args.precision, method=args.method)

    s = pp.Solver(0)
    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        s.solve_grid(f, g.h, tx, ty, out=out, **kw)
    torch.cuda.synchronize()

    # phase breakdown: every phase alone on one stream, events between the phases (eager launches)
    s.set_profiling(1)
    nph = max(5, args.steps // 4)
    log(f"[bench] phase breakdown over {nph} solves")
    s.solve_grid(f, g.h, tx, ty, out=out, **kw)
    phase_sum = None
    for _ in range(nph):
        s.solve_grid(f, g.h, tx, ty, out=out, **kw)
        ph = np.array([s.stats()["ms_phase"][k] for k in pp._binding.PHASES])
        phase_sum = ph if phase_sum is None else phase_sum + ph
    torch.cuda.synchronize()
    phases = dict(zip(pp._binding.PHASES, (phase_sum / nph).tolist()))
    s.set_profiling(0)
    rphase = args.roofline_phase or max(phases, key=phases.get)

    # timed region: the default schedule (first segment replayed from its graph unless the bracketed
    # phase is in it, second segment issued directly, near field on the side stream), HIP events
    # around the launches of the dominant phase
    log(f"[bench] timing {args.steps} solves (events around {rphase})")
    value, ms_per_step, rphase_ms = timed_solves(s, f, g, tx, ty, out, kw, args.steps, rphase)
    st = s.stats()
    N, M = int(st["nsources"]), int(st["ntargets"])
    P = out.cpu().numpy()
    p2p_parts = int(s.debug_array("NEAR").size // max(M, 1))

    # the same solves with no timing events at all
    for _ in range(3):
        s.solve_grid(f, g.h, tx, ty, out=out, **kw)
    torch.cuda.synchronize()
    tu0 = time.perf_counter()
    for _ in range(args.steps):
        s.solve_grid(f, g.h, tx, ty, out=out, **kw)
    torch.cuda.synchronize()
    untimed_value = args.steps / (time.perf_counter() - tu0)

    # resident solves: the tree of the last solve kept; the source alternates between two fields with
    # the same nonzero nodes (f and 1.5 f + a seeded perturbation on them), the targets between their
    # positions and positions moved inside their finest cells
    log(f"[bench] resident solves x{args.steps}")
    rng = np.random.Generator(np.random.PCG64(77))
    f_alt = torch.as_tensor(np.where(w["f"] != 0.0, 1.5 * w["f"] + 0.1 * np.abs(w["f"]).max()
                                     * rng.standard_normal(w["f"].shape), 0.0), device=dev)
    cx, cy = np.floor(w["tx"] / g.h), np.floor(w["ty"] / g.h)
    mx = np.clip((cx + rng.uniform(0.1, 0.9, cx.size)) * g.h, cx * g.h, (cx + 1) * g.h)
    my = np.clip((cy + rng.uniform(0.1, 0.9, cy.size)) * g.h, cy * g.h, (cy + 1) * g.h)
    keep = (np.floor(mx / g.h) == cx) & (np.floor(my / g.h) == cy)
    tx_alt = torch.as_tensor(np.where(keep, mx, w["tx"]), device=dev)
    ty_alt = torch.as_tensor(np.where(keep, my, w["ty"]), device=dev)
    inputs = [(f, tx, ty), (f_alt, tx_alt, ty_alt)]
    s.solve_grid(f, g.h, tx, ty, out=out, **kw)
    for i in range(3):
        s.solve_grid_resident(*inputs[i % 2], out=out)
    torch.cuda.synchronize()
    tr0 = time.perf_counter()
    for i in range(args.steps):
        s.solve_grid_resident(*inputs[i % 2], out=out)
    torch.cuda.synchronize()
    resident_value = args.steps / (time.perf_counter() - tr0)
    s.solve_grid_resident(f_alt, tx_alt, ty_alt, out=out)
    P_res = out.cpu().numpy()
    fresh = s.solve_grid(f_alt, g.h, tx_alt, ty_alt, **kw).cpu().numpy()
    resident_same = bool(np.array_equal(P_res, fresh))

    # the same resident solves, each replayed as one captured graph (a context with PP_RESIDENT_GRAPH=1)
    os.environ["PP_RESIDENT_GRAPH"] = "1"
    sg = pp.Solver(0)
    del os.environ["PP_RESIDENT_GRAPH"]
    out_g = torch.empty_like(out)
    sg.solve_grid(f, g.h, tx, ty, out=out_g, **kw)
    for i in range(4):
        sg.solve_grid_resident(*inputs[i % 2], out=out_g)
    torch.cuda.synchronize()
    tg0 = time.perf_counter()
    for i in range(args.steps):
        sg.solve_grid_resident(*inputs[i % 2], out=out_g)
    torch.cuda.synchronize()
    resident_graph_value = args.steps / (time.perf_counter() - tg0)
    sg.solve_grid_resident(f_alt, tx_alt, ty_alt, out=out_g)
    resident_graph_same = bool(np.array_equal(out_g.cpu().numpy(), fresh))
    sg.close()

    direct_s = None
    if args.direct_steps > 0:
        log(f"[bench] GPU all-pairs direct sum x{args.direct_steps}")
        s.direct_grid(f, g.h, tx, ty, out=torch.empty_like(out), precision=args.precision)
        torch.cuda.synchronize()
        td0 = time.perf_counter()
        for _ in range(args.direct_steps):
            s.direct_grid(f, g.h, tx, ty, out=torch.empty_like(out), precision=args.precision)
        torch.cuda.synchronize()
        direct_s = (time.perf_counter() - td0) / args.direct_steps

    from oracle import direct as oracle_direct
    log(f"[bench] oracle on {args.samples} sampled targets")
    acc = accuracy(P, w, args.samples, 2024, oracle_direct)

    # per-phase roofline: each phase's algorithmic work over its time alone (mode 1 above), and the
    # whole solve's fraction sum_phases max(bytes/BW, work/peak) / measured time
    works = phase_work(st, w, p2p_parts)
    per_phase = {k: roofline_of(works[k], phases[k]) for k in pp._binding.PHASES}
    ideal_ms = sum(v["ideal_ms"] for v in per_phase.values())
    overall = {"ideal_ms": ideal_ms, "measured_ms": ms_per_step, "frac": ideal_ms / ms_per_step,
               "note": "sum over phases of max(algorithmic bytes / 8 TB/s, algorithmic work / peak), over the "
                       "timed solve's time"}

    # the headline kernel: HIP events around its launches in the timed solves
    rw = roofline_of(works[rphase], rphase_ms)
    traffic = None
    if rphase == "p2p":
        traffic = traffic_from_profile(args.workload, "p2p", kernel_source="p2p.hip", p2p_parts=p2p_parts,
                                       precision=args.precision, method=args.method)
    elif rphase in ("p2m",):
        traffic = traffic_from_profile(args.workload, rphase, kernel_source="expand.hip",
                                       precision=args.precision, method=args.method)
    elif rphase in ("ingest",):
        traffic = traffic_from_profile(args.workload, rphase, kernel_source="ingest.hip")
    # FP64 work on this path runs on the vector ALUs (no matrix cores): bound "alu" against the FP64 peak
    roofline = {"bound": "hbm" if rw["bound"] == "hbm" else "alu",
                "kernel": rphase, "achieved": rw["achieved"], "peak": rw["peak"],
                "unit": {"hbm": "GB/s", "fp64": "TFLOP/s", "alu": "TFLOP/s"}[rw["bound"]],
                "frac": rw["frac"], "traffic": traffic, "work_per_launch": rw["work"],
                "work_unit": rw["work_unit"], "avg_launch_ms": rphase_ms, "p2p_list_parts": p2p_parts,
                "note": {"hbm": "algorithmic bytes per solve of the phase over its HIP-event time in the timed solves; "
                                "peak = MI355X HBM3E 8 TB/s",
                         "fp64": "FP64 flops (FMA = 2) per solve of the phase over its HIP-event time; peak = "
                                 "MI355X FP64 vector 78.6 TFLOP/s",
                         "alu": "FP32 lane-ops per solve of the phase over its HIP-event time; peak = 256 CU x 64 "
                                "lanes x 2.4 GHz without packed FP32"}[rw["bound"]]}

    # CPU oracle baseline on a bounded sample of the same workload (all host threads), and one thread
    cpu = None
    if not args.no_cpu_baseline:
        info = host_cpu_info()
        probe = 32
        tp0 = time.perf_counter()
        oracle_direct.direct_grid(w["f"], g.h, w["tx"][:probe], w["ty"][:probe])
        t_probe = time.perf_counter() - tp0
        n_sample = int(max(probe, min(M, args.cpu_seconds / max(t_probe / probe, 1e-9))))
        idx = rng.choice(M, n_sample, replace=False)
        log(f"[bench] CPU oracle on {n_sample} targets")
        tc0 = time.perf_counter()
        oracle_direct.direct_grid(w["f"], g.h, w["tx"][idx], w["ty"][idx])
        t_cpu = time.perf_counter() - tc0
        threads = oracle_direct.get_threads()
        oracle_direct.set_threads(1)
        n1 = max(8, int(n_sample * 3.0 / max(t_cpu * threads, 1e-9)))
        n1 = min(n1, 4096)
        log(f"[bench] CPU oracle, one thread, on {n1} targets")
        t10 = time.perf_counter()
        oracle_direct.direct_grid(w["f"], g.h, w["tx"][idx[:n1]], w["ty"][idx[:n1]])
        t1 = time.perf_counter() - t10
        oracle_direct.set_threads(0)
        cpu = {"value": (n_sample / M) / t_cpu, "unit": "solves/s", "cores": threads, "kind": "oracle",
               "sample": f"FP64 direct sum over all {N} nonzero sources at {n_sample} of the {M} targets "
                         f"(seeded), {t_cpu:.2f} s on {threads} threads; rate scaled to whole solves",
               "single_thread": {"value": (n1 / M) / t1, "unit": "solves/s", "targets": n1, "seconds": t1},
               "host": info}

    # the second workload (vortex512: all 262,144 grid nodes and an ellipse as targets)
    also = None
    if args.also:
        log(f"[bench] second workload {args.also}")
        w2 = G.workload(args.also)
        g2 = w2["grid"]
        f2, tx2, ty2 = (torch.as_tensor(w2[k], device=dev) for k in ("f", "tx", "ty"))
        out2 = torch.empty(tx2.numel(), dtype=torch.float64, device=dev)
        kw2 = dict(p=w2["p"], theta=w2["theta"], leaf_max=64, precision=args.precision, method=args.method)
        for _ in range(args.warmup):
            s.solve_grid(f2, g2.h, tx2, ty2, out=out2, **kw2)
        v2, ms2, p2p2 = timed_solves(s, f2, g2, tx2, ty2, out2, kw2, args.steps, "p2p")
        st2 = s.stats()
        P2 = out2.cpu().numpy()
        acc2 = accuracy(P2, w2, args.samples, 2024, oracle_direct)
        s.solve_grid(f2, g2.h, tx2, ty2, out=out2, **kw2)
        for _ in range(3):
            s.solve_grid_resident(f2, tx2, ty2, out=out2)
        torch.cuda.synchronize()
        tr0 = time.perf_counter()
        for _ in range(args.steps):
            s.solve_grid_resident(f2, tx2, ty2, out=out2)
        torch.cuda.synchronize()
        res2 = args.steps / (time.perf_counter() - tr0)
        pr2 = roofline_of(("alu", OPS_PER_PAIR * int(st2["n_p2p_pairs"]), "op"), p2p2)
        also = {"workload": args.also, "solves_per_s": v2, "ms_per_solve": ms2, "resident_solves_per_s": res2,
                "sources_nonzero": int(st2["nsources"]), "targets": int(st2["ntargets"]),
                "interactions_per_s": int(st2["nsources"]) * int(st2["ntargets"]) / (ms2 * 1e-3),
                "accuracy_vs_oracle": acc2,
                "p2p_roofline": {"achieved": pr2["achieved"], "peak": pr2["peak"], "unit": "T lane-op/s",
                                 "frac": pr2["frac"], "avg_launch_ms": p2p2},
                "tree": {k: st2[k] for k in ("depth", "ncells", "nsrc_leaves", "ntgt_leaves", "n_m2l",
                                              "n_p2p_lists", "n_p2p_pairs")}}

    # the steps around the solve, timed alone on the workload's grid: the source from a gridded
    # Lamb-Oseen velocity (eq. PoissonFinal), and the pressure and viscous forces on two fish bodies
    # (eq. Fpress / FpressNet / CdP; eq. Fvisc / FviscNet / CdNu, lifted points 2h out)
    around = None
    if args.forces_panels > 0:
        reps = 20

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            t0_ = time.perf_counter()
            for _ in range(reps):
                r_ = fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0_) / reps * 1e3, r_

        vel = G.vortex_velocity_grid(g, w["seed"] if w["seed"] is not None else 0, 64)
        ud, vd = (torch.as_tensor(a, device=dev) for a in vel)
        del vel
        fa = torch.empty_like(ud)
        src_ms, _ = timed(lambda: s.pressure_source(ud, vd, g.h, out=fa))
        bodies = [G.fish_panels(args.forces_panels, g.h, yc=0.35), G.fish_panels(args.forces_panels, g.h, yc=0.65,
                                                                                 phase=0.25)]
        mx_, my_, fnx, fny, fds = [np.concatenate([b[i] for b in bodies]) for i in range(5)]
        seg = [0, bodies[0][0].size, mx_.size]
        tpx, tpy, dnx, dny, dds = (torch.as_tensor(a, device=dev) for a in (mx_, my_, fnx, fny, fds))
        lxd, lyd = tpx + 2 * g.h * dnx, tpy + 2 * g.h * dny
        Pp = s.solve_grid(f, g.h, tpx, tpy, **kw)
        fp_ms, fr = timed(lambda: s.surface_forces(Pp, dnx, dny, dds, seg, u=(1.0, 0.0), rho=1.0, area=0.6))
        fv_ms, fv = timed(lambda: s.viscous_forces(ud, vd, g.h, lxd, lyd, dnx, dny, dds, seg, mu=1e-3,
                                                   uinf=(1.0, 0.0), rho=1.0, area=0.6))
        nodes = g.nx * g.ny
        around = {
            "source_assembly": {"ms_per_call": src_ms, "grid": [g.nx, g.ny],
                                "algorithmic_bytes": 24 * nodes,
                                "GB_per_s": 24 * nodes / (src_ms * 1e-3) / 1e9,
                                "note": "read u, v and write f (8 B each per node); host wall time per call"},
            "pressure_forces": {"ms_per_call": fp_ms, "panels": int(mx_.size), "bodies": 2, "result": fr},
            "viscous_forces": {"ms_per_call": fv_ms, "panels": int(mx_.size), "mu": 1e-3, "result": fv},
            "note": "U = (1, 0), rho = 1, A = 0.6; host wall time per call including the copy of the results",
        }
        del ud, vd, fa

    served = None
    if args.serve_requests > 0:
        served = serving_run(pp, G, args, log)

    rec = {
        "metric": "pressure solves/s & interactions/s vs direct at rel-L2 1e-4; served p50/p99 ms",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": [g.nx, g.ny], "sources_nonzero": N, "targets": M,
                   "p": w["p"], "theta": w["theta"], "leaf_max": 64, "precision": args.precision,
                   "method": args.method, "seed": w["seed"], "parallelism": "single GPU",
                   "step": "one cold solve (tree rebuilt), inputs resident in HBM"},
        "interactions_per_s": N * M / (ms_per_step * 1e-3),
        "direct": None if direct_s is None else {
            "ms_per_solve": direct_s * 1e3, "interactions_per_s": N * M / direct_s,
            "speedup_tree_vs_direct": direct_s / (ms_per_step * 1e-3)},
        "accuracy_vs_oracle": acc,
        "untimed_solves_per_s": untimed_value,
        "untimed_note": "the same cold solves without any timing events",
        "resident": {"solves_per_s": resident_value, "ms_per_solve": 1e3 / resident_value,
                     "bitwise_equal_to_cold_solve": resident_same,
                     "one_graph": {"solves_per_s": resident_graph_value, "bitwise_equal_to_cold_solve":
                                   resident_graph_same,
                                   "note": "each resident solve replayed as one captured graph (PP_RESIDENT_GRAPH=1; "
                                           "one graph per set of buffers, no host synchronisation inside)"},
                     "note": "pp_solve_grid_resident: tree, lists and target sort kept; each call a new source "
                             "with the same nonzero nodes and targets moved inside their finest cells"},
        "phases_ms": phases,
        "phases_note": f"per-phase HIP-event times from {nph} solves with every phase alone on one stream "
                       "(eager launches); the timed solves overlap the near field with the expansions",
        "phase_roofline": per_phase,
        "overall_roofline": overall,
        "tree": {k: st[k] for k in ("depth", "ncells", "nsrc_leaves", "ntgt_leaves", "n_m2l", "n_p2p_lists",
                                     "n_p2p_pairs")},
        "also": also,
        "served": served,
        "around_the_solve": around,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    s.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
