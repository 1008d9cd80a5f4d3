#!/usr/bin/env python3
"""Benchmark of the pressure-Poisson tree-code on one MI355X.

Workload (default ``vortex512``): a 512 x 512 grid of sources f = 2(u_x v_y -
u_y v_x) from 64 seeded Lamb-Oseen vortices, targets = the 262,144 grid nodes
plus 2,048 points on an ellipse, expansion order p = 12, acceptance theta =
0.5, mixed precision (FP32 + Kahan near field and local evaluation, FP64
expansions).  One step = one complete solve (ingest, target sort, tree,
interaction lists, P2M, M2M, M2L, L2L, L2P, P2P, finalize) with the inputs
already resident in device memory.  Repeated solves replay their launches from
captured HIP graphs (the library does this when shape and pointers repeat),
and the near field runs on a second stream beside the upward and downward
passes.  HIP events around every near-field launch in the timed region (on
that stream) give the kernel's duration for the roofline; a further pass with
events between all phases, each phase alone on one stream, gives the phase
breakdown, and a last pass without any events gives the untimed rate.

Prints one JSON line: solves/s, effective interactions/s against the GPU
all-pairs direct sum, accuracy against the FP64 CPU oracle on sampled targets,
the roofline of the dominant kernel (the near field) and the CPU oracle timed
on a bounded sample on the host cores.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs, 64 FP32 lanes per CU per clock without packed instructions, 2.4 GHz
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Algorithmic FP32 lane operations of one near-field pair: dx, dy, dx^2, +dy^2 (fma), log2, and
# the weighted accumulation w*log2 (fma).  Compensation and loop overhead are not counted, so they
# lower the fraction.
OPS_PER_PAIR = 6


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    with open(os.path.join(ROOT, "paper_1610_04398_amd", "csrc", "p2p.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_from_profile(workload: str, parts: int, precision: str, method: str):
    """HBM bytes per near-field launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source with the same number of list parts per target
    leaf (each part writes its own partial sums), precision and method; else None."""
    path = os.path.join(ROOT, "profiles", f"p2p_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_sha256_16") != kernel_source_hash() or rec.get("p2p_parts") != parts:
        return None
    if rec.get("precision") != precision or rec.get("method") != method:
        return None
    return rec.get("bytes_per_launch")


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

    def run(slots):
        srv = pp.Server(0, max_slots=slots, work_budget_points=args.serve_work_budget if slots > 1 else 0)
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
        srv.close()
        lat = [i["total_us"] / 1e3 for i in infos]
        same = all(bool(torch.equal(o, a)) for o, a in zip(outs, alone))
        return {"p50_ms": _percentile(lat, 50), "p99_ms": _percentile(lat, 99), "mean_ms": float(np.mean(lat)),
                "solves_per_s": len(reqs) / (makespan * 1e-6), "slots": slots,
                "work_budget_points": args.serve_work_budget if slots > 1 else 0, "identical_to_alone": same}

    def median_run(slots):
        # the same trace replayed args.serve_reps times; the run with the median p99 is reported
        runs = sorted((run(slots) for _ in range(args.serve_reps)), key=lambda r: r["p99_ms"])
        out = dict(runs[len(runs) // 2])
        out["p99_ms_runs"] = [r["p99_ms"] for r in runs]
        out["identical_to_alone"] = all(r["identical_to_alone"] for r in runs)
        return out

    log("[bench] serving: one-slot (sequential) path")
    seq = median_run(1)
    log(f"[bench] serving: {args.serve_slots}-slot path")
    srv = median_run(args.serve_slots)
    sizes = [r["grid"].nx for r in reqs]
    return {"requests": len(reqs), "arrival": f"Poisson, rate {lam:.1f}/s = {args.serve_load} x sequential "
                                               f"throughput ({seq_rate:.1f} solves/s)",
            "grid_sizes": {str(n): sizes.count(n) for n in sorted(set(sizes))},
            "sequential": seq, "served": srv,
            "p99_speedup": seq["p99_ms"] / srv["p99_ms"] if srv["p99_ms"] > 0 else None}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="vortex512")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--method", default="fmm", choices=["fmm", "treecode"],
                    help="fmm: M2L/L2L/L2P with the dual-tree acceptance; treecode: the paper's own variant (M2P)")
    ap.add_argument("--direct-steps", type=int, default=3)
    ap.add_argument("--samples", type=int, default=2000, help="targets checked against the oracle")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=256, help="requests in the serving stream (0: skip)")
    ap.add_argument("--serve-slots", type=int, default=2)
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
    # timed region: launches replayed from captured graphs, HIP events around every near-field
    # launch (on the stream it runs on) for the roofline
    s.set_profiling(2)
    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        s.solve_grid(f, g.h, tx, ty, out=out, **kw)
    torch.cuda.synchronize()
    p2p_sum = 0.0
    log(f"[bench] timing {args.steps} solves")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.solve_grid(f, g.h, tx, ty, out=out, **kw)
        p2p_sum += s.stats()["ms_phase"]["p2p"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = args.steps / elapsed
    p2p_ms_timed = p2p_sum / args.steps
    st = s.stats()
    N = int(st["nsources"])
    M = int(st["ntargets"])
    pairs = int(st["n_p2p_pairs"])
    P = out.cpu().numpy()
    # list parts of the near field in this run: its partial sums are [parts][targets]
    p2p_parts = int(s.debug_array("NEAR").size // max(M, 1))

    # phase breakdown: the same solve with events between all phases (launched eagerly)
    s.set_profiling(1)
    nph = max(5, args.steps // 2)
    log(f"[bench] phase breakdown over {nph} solves")
    s.solve_grid(f, g.h, tx, ty, out=out, **kw)
    phase_sum = None
    tp0 = time.perf_counter()
    for _ in range(nph):
        s.solve_grid(f, g.h, tx, ty, out=out, **kw)
        stp = s.stats()
        ph = np.array([stp["ms_phase"][k] for k in pp._binding.PHASES])
        phase_sum = ph if phase_sum is None else phase_sum + ph
    torch.cuda.synchronize()
    ms_eager = 1e3 * (time.perf_counter() - tp0) / nph
    phases = dict(zip(pp._binding.PHASES, (phase_sum / nph).tolist()))
    s.set_profiling(0)

    # the same solves with no timing events at all
    for _ in range(3):
        s.solve_grid(f, g.h, tx, ty, out=out, **kw)
    torch.cuda.synchronize()
    tu0 = time.perf_counter()
    for _ in range(args.steps):
        s.solve_grid(f, g.h, tx, ty, out=out, **kw)
    torch.cuda.synchronize()
    untimed_value = args.steps / (time.perf_counter() - tu0)

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

    # accuracy on sampled targets against the FP64 oracle
    from oracle import direct as oracle_direct
    rng = np.random.Generator(np.random.PCG64(2024))
    ng = int(w["n_grid_targets"])
    ns = M - ng
    k_grid = min(args.samples * 3 // 4, ng) if ns > 0 else min(args.samples, ng)
    k_surf = min(args.samples - k_grid, ns)
    sel_g = rng.choice(ng, k_grid, replace=False) if k_grid else np.zeros(0, int)
    sel_s = ng + rng.choice(ns, k_surf, replace=False) if k_surf else np.zeros(0, int)
    log(f"[bench] oracle on {k_grid + k_surf} sampled targets")
    acc = {}
    for name, sel in (("grid", sel_g), ("surface", sel_s)):
        if sel.size == 0:
            continue
        ref = oracle_direct.direct_grid(w["f"], g.h, w["tx"][sel], w["ty"][sel])
        acc[name] = {"rel_l2": float(np.linalg.norm(P[sel] - ref) / np.linalg.norm(ref)),
                     "rel_max": float(np.max(np.abs(P[sel] - ref)) / np.max(np.abs(ref))),
                     "targets": int(sel.size)}

    # CPU oracle baseline on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        probe = 64
        tp0 = time.perf_counter()
        oracle_direct.direct_grid(w["f"], g.h, w["tx"][:probe], w["ty"][:probe])
        t_probe = time.perf_counter() - tp0
        n_sample = int(max(probe, min(M, args.cpu_seconds / max(t_probe / probe, 1e-9))))
        idx = rng.choice(M, n_sample, replace=False)
        log(f"[bench] CPU oracle on {n_sample} targets")
        tc0 = time.perf_counter()
        oracle_direct.direct_grid(w["f"], g.h, w["tx"][idx], w["ty"][idx])
        t_cpu = time.perf_counter() - tc0
        cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
        cpu = {"value": (n_sample / M) / t_cpu, "unit": "solves/s", "cores": cores, "kind": "oracle",
               "sample": f"FP64 direct sum over all {N} nonzero sources at {n_sample} of the {M} targets "
                         f"(seeded), {t_cpu:.2f} s; rate scaled to whole solves"}

    # the steps around the solve, timed alone on the workload's grid: the source from a gridded
    # Lamb-Oseen velocity (eq. PoissonFinal), and the pressure and viscous forces on two fish bodies
    # (eq. Fpress / FpressNet / CdP; eq. Fvisc / FviscNet / CdNu, lifted points 2h out)
    around = None
    if args.forces_panels > 0:
        reps = 50

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
        fa = torch.empty_like(ud)
        src_ms, _ = timed(lambda: s.pressure_source(ud, vd, g.h, out=fa))
        bodies = [G.fish_panels(args.forces_panels, g.h, yc=0.35), G.fish_panels(args.forces_panels, g.h, yc=0.65,
                                                                                 phase=0.25)]
        mx, my, fnx, fny, fds = [np.concatenate([b[i] for b in bodies]) for i in range(5)]
        seg = [0, bodies[0][0].size, mx.size]
        tpx, tpy, dnx, dny, dds = (torch.as_tensor(a, device=dev) for a in (mx, my, fnx, fny, fds))
        lxd, lyd = tpx + 2 * g.h * dnx, tpy + 2 * g.h * dny
        Pp = s.solve_grid(fa, g.h, tpx, tpy, **kw)
        fp_ms, fr = timed(lambda: s.surface_forces(Pp, dnx, dny, dds, seg, u=(1.0, 0.0), rho=1.0, area=0.6))
        fv_ms, fv = timed(lambda: s.viscous_forces(ud, vd, g.h, lxd, lyd, dnx, dny, dds, seg, mu=1e-3,
                                                   uinf=(1.0, 0.0), rho=1.0, area=0.6))
        nodes = g.nx * g.ny
        around = {
            "source_assembly": {"ms_per_call": src_ms, "grid": [g.nx, g.ny],
                                "algorithmic_bytes": 24 * nodes,
                                "GB_per_s": 24 * nodes / (src_ms * 1e-3) / 1e9,
                                "note": "read u, v and write f (8 B each per node); host wall time per call"},
            "pressure_forces": {"ms_per_call": fp_ms, "panels": int(mx.size), "bodies": 2, "result": fr},
            "viscous_forces": {"ms_per_call": fv_ms, "panels": int(mx.size), "mu": 1e-3, "result": fv},
            "note": "U = (1, 0), rho = 1, A = 0.6; host wall time per call including the copy of the results",
        }

    served = None
    if args.serve_requests > 0:
        served = serving_run(pp, G, args, log)

    p2p_ms = p2p_ms_timed
    achieved = OPS_PER_PAIR * pairs / (p2p_ms * 1e-3) / 1e12 if p2p_ms > 0 else None
    roofline = {"bound": "alu", "kernel": "k_p2p32 (near field)", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                "unit": "TFLOP/s", "frac": (achieved / VALU_PEAK_TOPS) if achieved else None,
                "traffic": traffic_from_profile(args.workload, p2p_parts, args.precision, args.method),
                "ops_per_pair": OPS_PER_PAIR,
                "pairs_per_launch": pairs, "avg_launch_ms": p2p_ms, "p2p_list_parts": p2p_parts,
                "note": "6 algorithmic FP32 VALU lane-ops per near-field pair (sub, sub, mul, fma, log2, fma); "
                        "peak = 256 CU x 64 lanes x 2.4 GHz without packed FP32"}
    if args.precision == "fp64":
        roofline["kernel"] = "k_p2p64 (near field)"

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
                   "method": args.method,
                   "seed": w["seed"], "parallelism": "single GPU"},
        "interactions_per_s": N * M / (ms_per_step * 1e-3),
        "direct": None if direct_s is None else {
            "ms_per_solve": direct_s * 1e3, "interactions_per_s": N * M / direct_s,
            "speedup_tree_vs_direct": direct_s / (ms_per_step * 1e-3)},
        "accuracy_vs_oracle": acc,
        "phases_ms": phases,
        "phases_note": f"per-phase HIP-event times from {nph} further solves launched without graph replay, "
                       f"every phase on one stream ({ms_eager:.3f} ms per solve); the timed solves replay the "
                       "first segment from a graph and run the near field on a second stream beside the expansions",
        "untimed_solves_per_s": untimed_value,
        "untimed_note": "the same solves without the near-field timing events: the first segment one replayed "
                        "graph, the second issued directly in the same order as the timed solves",
        "tree": {k: st[k] for k in ("depth", "ncells", "nsrc_leaves", "ntgt_leaves", "n_m2l", "n_p2p_lists",
                                     "n_p2p_pairs")},
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
