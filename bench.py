#!/usr/bin/env python3
"""Benchmark of the SIP hot path on one MI355X.

Workload: one 256^3 block of first-order upwind convection-diffusion
(D = 1, divergence-free seeded face fluxes with max |F| = 2), b uniform[-1,1]
from seed 1234, alpha = 0.92.  One step = the whole hot path on that block:
reorder into the tile-sheared layout, Stone factorisation (computed in FP64,
stored FP32), and the mixed-precision solve (FP32 sweeps, FP64 residual and
update) to a relative residual of 1e-8.

value = cells * iterations / wall time of the timed steps (cell-iterations/s),
inputs resident in HBM before the timed region.  The line also reports the
same solve in plain FP64, the achieved bandwidth of the persistent solve
kernel (one launch runs every sweep of a solve; timed with HIP events on the
launch stream) against the HBM peak, the two sweeps launched one at a time
for comparison, and the CPU oracle on a bounded sample of the same workload.

With the default 256^3 workload the line also carries, under "configs", the
other configurations at their full sizes, each with its throughput, the
error of the mixed result against the FP64 result, a roofline and the oracle
on a bounded sample: the 64 uneven blocks through one solve server, the
512 x 512 x 256 stretched-grid Poisson block, and the serving stream of 250
systems x 8 right-hand sides at 200 arrivals per second (--no-configs skips
them).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# algorithmic HBM bytes per cell of one sweep launch (each array streamed once)
FWD_BYTES = {"mixed": 56 + 8 + 8 + 16 + 4, "fp64": 56 + 8 + 8 + 32 + 8,   # A, b, x, L (Lb,Lw,Ls,1/Lp), y out
             "fp32": 28 + 4 + 4 + 16 + 4}
A_SYM_SAVING = 56 - 32     # symmetric storage reads A_P, A_E, A_N, A_T only
BWD_BYTES = {"mixed": 12 + 4 + 8 + 8, "fp64": 24 + 8 + 8 + 8,              # U, y, x in, x out
             "fp32": 12 + 4 + 4 + 4}
FP32_RTOL = 1e-5           # the all-FP32 relaxation stalls near 1e-7
# a pair of right-hand sides per sweep: A and the factors once, b, x, y per right-hand side
PAIR_FWD_BYTES = 56 + 16 + 2 * (8 + 8 + 4)     # per cell, both right-hand sides
PAIR_BWD_BYTES = 12 + 2 * (4 + 8 + 8)
RTOL = 1e-8
# Single systems of at least this many cells load the forward sweep's
# coefficient, factor and b streams non-temporally (the library's own
# threshold): the last template argument of the persistent kernel's name.
STREAM_HINT_CELLS = 1 << 22
# Device bytes a mixed system keeps resident per cell (A 56, FP32 factors 28,
# b, x and y 20); a workload whose whole working set fits the 256 MiB
# last-level cache would be a cache measurement, not an HBM one.
RESIDENT_BYTES_MIXED = 104
MALL_BYTES = 256 << 20


def working_set(cells):
    ws = cells * RESIDENT_BYTES_MIXED
    return {"working_set_mib": round(ws / 2 ** 20, 1), "cache_resident": ws <= MALL_BYTES}
SOLVE_BYTES_MIXED = FWD_BYTES["mixed"] + BWD_BYTES["mixed"]   # one mixed iteration, both sweeps
# HBM bytes per launch of the persistent solve kernel (one launch = one whole
# mixed solve) on the 256^3 and the 512x512x256 workloads, and of the two
# launches of the pair workload's two-right-hand-side solve, from the rocprofv3
# FETCH_SIZE / WRITE_SIZE passes summarised in profiles/solve_256cube_cd.md,
# profiles/solve_512x512x256_stretched.md and profiles/solve_pair_256cube_cd.md
# (calibrated against a plain copy), with the iterations of that solve and the
# SHA-256 of the kernel source they were taken with.  Once the source differs the counters no
# longer describe the kernel and traffic is null.
MEASURED = {"kernels_sha256": "5c3497df3e244a4b2c3bcf66754d076ef980a87eaa475b0e66aa594286e91fb6",
            "single": {"iterations": 4069, "persist_bytes": 9723600658445},
            "large": {"iterations": 15239, "persist_bytes": 147052406773563},
            "pair": {"iterations": [4069, 6023], "persist_bytes": 17950146754459}}


def log(msg):
    """Progress of the phases on stderr (the JSON line goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def copy_gbps():
    """Read + write bandwidth of a plain 1 GiB stream on this GPU (the better
    of a device-to-device copy and an elementwise scale), timed with events on
    the current stream: the bandwidth a simple streaming kernel reaches."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    best = 0.0
    for op in (lambda: dst.copy_(src), lambda: torch.mul(src, 2.0, out=dst)):
        for _ in range(3):
            op()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            op()
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / 10
        best = max(best, 2 * src.numel() * 8 / (ms * 1e-3) / 1e9)
    return best


def host_cpu():
    """CPU model of the host that timed the oracle."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def kernels_sha256():
    import hashlib
    with open(os.path.join(ROOT, "paper_1303_4538_amd", "csrc", "sip_kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256, help="block edge (cells)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--no-fp32", action="store_true", help="skip the all-FP32 relaxation comparison")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the two-right-hand-side and multi-block solves of the same block")
    ap.add_argument("--profile-iters", type=int, default=40)
    # oracle samples sized to about 10-30 s of host CPU work each
    ap.add_argument("--cpu-iters", type=int, default=100, help="oracle iterations of the 256^3 block")
    ap.add_argument("--cpu-iters-batched", type=int, default=20,
                    help="oracle iterations per block (batched; 16 processes)")
    ap.add_argument("--cpu-iters-large", type=int, default=20, help="oracle iterations of the 512x512x256 block")
    ap.add_argument("--cpu-iters-serving", type=int, default=100,
                    help="oracle iterations per sampled system (serving; 16 processes)")
    ap.add_argument("--no-configs", action="store_true",
                    help="default line without the batched, large and serving configurations")
    ap.add_argument("--storage", default="full", choices=["full", "symmetric"],
                    help="coefficient storage of the sweeps (symmetric: Poisson workloads only)")
    ap.add_argument("--workload", default="single",
                    choices=["single", "batched", "large", "serving", "pair", "blocks", "tune", "steps"],
                    help="single: 256^3 block (default); batched: 64 uneven blocks through the solve "
                         "server; large: 512x512x256 stretched Poisson; serving: Poisson-arrival "
                         "request stream (8 right-hand sides per system); pair: the 256^3 block with "
                         "two right-hand sides swept together; blocks: the 256^3 domain cut into "
                         "--blocks-per-axis^3 blocks coupled through boundary values; tune: every sweep plan "
                         "(loader phases x poll distance) timed on blocks of 32^3 to 512x512x256, with "
                         "sip_tune's choice; steps: the sweeps' time per tile step on shapes that separate "
                         "the step time from the hop lag")
    ap.add_argument("--blocks-per-axis", type=int, default=2, help="blocks along each axis (workload blocks)")
    ap.add_argument("--serve-systems", type=int, default=40, help="systems in the serving stream (8 rhs each)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="mean arrivals per second")
    ap.add_argument("--serve-budget-gb", type=float, default=16.0, help="server HBM budget")
    ap.add_argument("--epoch-iters", type=int, default=8, help="server iterations per epoch (batched, serving)")
    ap.add_argument("--prof", action="store_true",
                    help="short run for rocprofv3: factor, a few sweeps and one persistent mixed solve of the "
                         "default workload (sweeps: mixed, a pair of right-hand sides, all-FP32; with --workload "
                         "large: the 512x512x256 block, mixed and FP64; with --workload pair: the two-right-hand-"
                         "side solve of the pair workload) and a 512 MiB device copy used to calibrate the HBM "
                         "byte counters")
    return ap.parse_args()


def prof_run(args):
    """Minimal GPU work for counter collection (one process, no CPU oracle)."""
    import numpy as np
    import torch

    from paper_1303_4538_amd import problems, sip

    sip.lib()
    src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")       # 512 MiB
    dst = torch.empty_like(src)
    dst.copy_(src)                                                         # calibration copy
    torch.cuda.synchronize()
    del src, dst
    if args.workload == "large":
        # 512 x 512 x 256 stretched Poisson: the mixed and the FP64 sweeps
        c = problems.config4()
        A = torch.from_numpy(c["A"]).cuda()
        b = torch.from_numpy(c["b"]).cuda()
        for precision in ("mixed", "fp64"):
            S = sip.sip_factor(A, c["alpha"], precision)
            f, bk = sip.sip_profile_sweeps(S, b, torch.zeros_like(b), 5)
            print(f"prof: large {precision} forward {f:.4f} ms, backward {bk:.4f} ms per sweep", flush=True)
            if precision == "mixed":
                _, it, _, sec = sip.sip_solve(S, b, torch.zeros_like(b), RTOL, 200000)
                print(f"prof: large mixed solve, {it} iterations in one persistent launch, {sec:.3f} s", flush=True)
            S.close()
        torch.cuda.synchronize()
        return
    c = problems.config2(args.n)
    A = torch.from_numpy(c["A"]).cuda()
    b = torch.from_numpy(c["b"]).cuda()
    if args.workload == "pair":
        # the two-right-hand-side solve of the pair workload: one pair launch
        # and the continuation of the right-hand side that runs longer
        n = args.n
        b2 = torch.from_numpy(problems.rhs_uniform(
            n, n, n, np.random.default_rng(np.random.SeedSequence(problems.MASTER_SEED).spawn(3)[2]))).cuda()
        S = sip.sip_factor(A, c["alpha"], "mixed")
        _, info = sip.sip_solve_multi(S, [b, b2], [torch.zeros_like(b), torch.zeros_like(b)], RTOL, 200000)
        print(f"prof: pair solve, iterations {[i[0] for i in info]}, "
              f"{sip.sip_system_solve_ms(S):.1f} ms in its persistent launches", flush=True)
        S.close()
        torch.cuda.synchronize()
        return
    S = sip.sip_factor(A, c["alpha"], "mixed")
    x = torch.zeros_like(b)
    fwd_ms, bwd_ms = sip.sip_profile_sweeps(S, b, x, 5)
    print(f"prof: mixed forward {fwd_ms:.4f} ms, backward {bwd_ms:.4f} ms per sweep", flush=True)
    _, it, _, sec = sip.sip_solve(S, b, torch.zeros_like(b), RTOL, 200000)
    print(f"prof: mixed solve, {it} iterations in one persistent launch, {sec:.3f} s", flush=True)
    # the same block with two right-hand sides swept together
    bs = [b, torch.flip(b, dims=(0,)).contiguous()]
    f2, b2 = sip.sip_profile_sweeps_multi(S, bs, [torch.zeros_like(b), torch.zeros_like(b)], 5)
    print(f"prof: pair forward {f2:.4f} ms, backward {b2:.4f} ms per sweep", flush=True)
    S.close()
    S = sip.sip_factor(A, c["alpha"], "fp32")   # the all-FP32 relaxation
    f3, b3 = sip.sip_profile_sweeps(S, b, torch.zeros_like(b), 5)
    print(f"prof: fp32 forward {f3:.4f} ms, backward {b3:.4f} ms per sweep", flush=True)
    S.close()
    torch.cuda.synchronize()


def batched_run(args):
    """64 independent blocks (dims uniform 32..160 per axis, half Poisson, half
    convection-diffusion) submitted at once to the solve server, mixed
    precision to 1e-8; value = total cell-iterations / wall time."""
    import torch

    from paper_1303_4538_amd import problems, sip

    sip.lib()
    meta = problems.config3_meta()
    blocks = []
    for dims, kind, ss in meta:
        A, b = problems.make_block(dims, kind, ss)
        blocks.append((dims, torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda()))
    torch.cuda.synchronize()

    def step(tag, precision="mixed"):
        srv = sip.Server(max_slots=256, epoch_iters=args.epoch_iters)
        xs = [torch.zeros_like(b) for _, _, b in blocks]
        t0 = time.perf_counter()
        tickets = [srv.submit(tag * 1000 + q, A, b, xs[q], precision=precision, rtol=RTOL, max_iter=200000)
                   for q, (_, A, b) in enumerate(blocks)]
        res = [srv.poll(t) for t in tickets]
        t1 = time.perf_counter()
        st = srv.stats()
        srv.close()
        ci = sum(dims[0] * dims[1] * dims[2] * r["iters"] for (dims, _, _), r in zip(blocks, res))
        return t1 - t0, ci, res, st

    for w in range(args.warmup):
        step(w + 1)
    tot_t, tot_ci, last = 0.0, 0, None
    for k in range(args.steps):
        dt, ci, res, st = step(100 + k)
        tot_t += dt
        tot_ci += ci
        last = (res, st)
    res, st = last
    cells = sum(d[0] * d[1] * d[2] for d, _, _ in blocks)
    value = tot_ci / tot_t
    extra, cpu = {}, None
    if not args.no_extras:
        # the same 64 blocks solved one after the other (factor + mixed solve each)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ci1 = 0
        for dims, A, b in blocks:
            S = sip.sip_factor(A, problems.ALPHA, "mixed")
            x = torch.zeros_like(b)
            _, it, _, _ = sip.sip_solve(S, b, x, RTOL, 200000)
            S.close()
            ci1 += dims[0] * dims[1] * dims[2] * it
        torch.cuda.synchronize()
        extra["one_at_a_time_cell_iters_per_s"] = ci1 / (time.perf_counter() - t0)
        # plain FP64 through the same server
        dt64, ci64, res64, _ = step(500, "fp64")
        extra["fp64_batched_cell_iters_per_s"] = ci64 / dt64
        extra["fp64_all_ok"] = all(r["status"] == 0 for r in res64)
        extra["mixed_speedup_vs_fp64"] = value / (ci64 / dt64)
    if not args.no_cpu:
        cpu = batched_cpu_baseline(meta, args.cpu_iters_batched)
    line = {
        "metric": "cell-iterations/s (batched mixed SIP to 1e-8 rel. residual)",
        "value": value, "unit": "cell-iterations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": tot_t / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "64 blocks, dims uniform 32..160 per axis, half Poisson / half upwind "
                               "convection-diffusion, one solve server, factor + mixed solve to 1e-8",
                   "cells": cells, "max_iters": max(r["iters"] for r in res),
                   "all_ok": all(r["status"] == 0 for r in res), "epochs": st["epochs"],
                   "graph_epochs": st["graph_epochs"], "launches": st["launches"],
                   "hbm_gbps_algorithmic": value * (FWD_BYTES["mixed"] + BWD_BYTES["mixed"]) / 1e9, **extra},
        "roofline": solve_roofline(value), "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def _oracle_block_sample(job):
    """One block of the batched workload on one host core: factorisation
    (untimed), then n mixed-form oracle iterations (timed)."""
    dims, kind, ss, n = job
    import numpy as np

    import oracle
    from paper_1303_4538_amd import problems
    A, b = problems.make_block(dims, kind, ss)
    LU = oracle.factor(A, problems.ALPHA)
    t = time.perf_counter()
    oracle.iterate(A, LU, b, np.zeros_like(b), n, mixed=True)
    return dims[0] * dims[1] * dims[2] * n, time.perf_counter() - t


def batched_cpu_baseline(meta, n):
    """The oracle on the batched workload, every block in its own process over
    all host cores (at most 16): n mixed-form iterations per block; the rate is
    the total cell-iterations over the summed iteration time spread across the
    cores."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import oracle
    oracle.build(force=False)
    procs = max(1, min(16, os.cpu_count() or 1))
    # fresh interpreters (no inherited GPU state); a worker that cannot start
    # fails the pool instead of being restarted
    with ProcessPoolExecutor(procs, mp_context=mp.get_context("spawn")) as pool:
        out = list(pool.map(_oracle_block_sample, [(d, k, s, n) for d, k, s in meta]))
    ci = sum(c for c, _ in out)
    busy = sum(t for _, t in out)
    return {"value": ci / (busy / procs), "unit": "cell-iterations/s", "cores": procs, "kind": "oracle",
            "sample": f"all {len(meta)} blocks, {n} mixed-form SIP iterations each (FP64 residual, FP32 sweeps), "
                      f"one process per block on {procs} cores, factorisation untimed",
            "host_cpu": host_cpu(), "host_cpus": os.cpu_count()}


def serve_stream(sip, n_systems, rate, budget_gb, epoch_iters, keep=False):
    """One Poisson-arrival stream against a fresh continuous-batching server:
    each system (lognormal dims 24..192 per axis, half Poisson / half
    convection-diffusion) receives 8 right-hand sides; requests are shuffled
    and submitted at their arrival times; factors stay resident across a
    system's requests.  Returns the latency and throughput figures (and, with
    keep, the systems, requests, coefficients, right-hand sides and results)."""
    import numpy as np
    import torch

    from paper_1303_4538_amd import problems

    systems, reqs = problems.serving_stream(n_systems=n_systems, rhs_per_system=8, rate_hz=rate)
    As = [torch.from_numpy(problems.system_coefficients(dims, kind, ss)).cuda() for dims, kind, ss in systems]
    bs = [torch.from_numpy(problems.request_rhs(systems[s][0], rs)).cuda() for _, s, _, rs in reqs]
    xs = [torch.zeros_like(b) for b in bs]
    torch.cuda.synchronize()
    srv = sip.Server(hbm_budget_bytes=int(budget_gb * (1 << 30)), max_slots=512, epoch_iters=epoch_iters)
    t0 = time.perf_counter()
    tickets = []
    for q, (ta, s, m, _) in enumerate(reqs):
        wait = t0 + ta - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        tickets.append(srv.submit(s, As[s], bs[q], xs[q], precision="mixed", rtol=RTOL, max_iter=200000,
                                  retain=True))
    res = [srv.poll(t) for t in tickets]
    t1 = time.perf_counter()
    st = srv.stats()
    srv.close()
    lat = np.array([r["t_done"] - r["t_submit"] for r in res])
    run = np.array([r["t_done"] - r["t_admit"] for r in res])
    cells = np.array([np.prod(systems[s][0]) for _, s, _, _ in reqs])
    iters = np.array([r["iters"] for r in res])
    span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
    out = dict(n=len(reqs), ci=float((cells * iters).sum()), span=span, wall=t1 - t0,
               solves_per_s=len(res) / span,
               latency_p50_ms=float(np.percentile(lat, 50) * 1e3),
               latency_p99_ms=float(np.percentile(lat, 99) * 1e3),
               run_p50_ms=float(np.percentile(run, 50) * 1e3), run_p99_ms=float(np.percentile(run, 99) * 1e3),
               all_ok=all(r["status"] == 0 for r in res), st=st,
               mean_cells=float(cells.mean()), mean_iters=float(iters.mean()))
    if keep:
        out.update(systems=systems, reqs=reqs, As=As, bs=bs, xs=xs, res=res)
    return out


def serving_run(args):
    """The serving stream (--serve-systems systems x 8 right-hand sides at
    --serve-rate arrivals per second) against one server: latency
    percentiles beside throughput, the offered load (arrival rate over the
    served rate), and as context the same stream at lower arrival rates."""
    from paper_1303_4538_amd import sip

    sip.lib()
    m = serve_stream(sip, args.serve_systems, args.serve_rate, args.serve_budget_gb, args.epoch_iters)
    st = m["st"]
    sweep = []
    if not args.no_extras:
        for rate in (args.serve_rate / 8, args.serve_rate / 4, args.serve_rate / 2):
            r = serve_stream(sip, args.serve_systems, rate, args.serve_budget_gb, args.epoch_iters)
            sweep.append({"offered_per_s": rate, "solves_per_s": r["solves_per_s"],
                          "latency_p50_ms": r["latency_p50_ms"], "latency_p99_ms": r["latency_p99_ms"],
                          "cell_iters_per_s": r["ci"] / r["span"], "all_ok": r["all_ok"]})
    value = m["ci"] / m["span"]
    line = {
        "metric": "served solves: cell-iterations/s and latency (mixed SIP to 1e-8)",
        "value": value, "unit": "cell-iterations/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": m["wall"] * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{m['n']} requests ({args.serve_systems} systems x 8 rhs), Poisson arrivals "
                               f"{args.serve_rate:g}/s, lognormal dims 24..192, half Poisson / half CD, "
                               f"HBM budget {args.serve_budget_gb:g} GB",
                   **_serving_fields(m, args.serve_rate), "rate_sweep": sweep},
        "roofline": solve_roofline(value), "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def _serving_fields(m, rate):
    st = m["st"]
    return {"solves_per_s": m["solves_per_s"], "offered_per_s": rate, "offered_load": rate / m["solves_per_s"],
            "latency_p50_ms": m["latency_p50_ms"], "latency_p99_ms": m["latency_p99_ms"],
            "run_p50_ms": m["run_p50_ms"], "run_p99_ms": m["run_p99_ms"], "all_ok": m["all_ok"],
            "factorisations": st["factorisations"], "evictions": st["evictions"], "epochs": st["epochs"],
            "graph_epochs": st["graph_epochs"], "peak_bytes": st["peak_bytes"],
            "mean_cells": m["mean_cells"], "mean_iters": m["mean_iters"]}


def persist_roofline(cells, iters, solve_ms, storage="full", workload=None):
    """Roofline of the persistent solve kernel k_persist, which runs every
    sweep of one mixed solve in one launch: iters + 1 fused residual + forward
    sweeps (the last one finds the residual below the tolerance) and iters
    backward sweeps, each streaming its arrays once.  solve_ms is the
    launch's device time from HIP events recorded just before and after it on
    its stream (sip_system_solve_ms)."""
    fwd_b = FWD_BYTES["mixed"] - (A_SYM_SAVING if storage == "symmetric" else 0)
    alg = ((iters + 1) * fwd_b + iters * BWD_BYTES["mixed"]) * cells
    achieved = alg / (solve_ms * 1e-3) / 1e9
    traffic = None
    m = MEASURED.get(workload) if workload else None
    if m and storage == "full" and kernels_sha256() == MEASURED["kernels_sha256"] and m["iterations"] == iters:
        traffic = round(m["persist_bytes"] / (solve_ms * 1e-3) / 1e9, 1)
    st = "true" if cells >= STREAM_HINT_CELLS else "false"
    return {"bound": "hbm",
            "kernel": f"k_persist<float, double, 3, 1, false, {st}> (whole mixed solve in one launch: FP64 residual "
                      "+ FP32 forward sweep, FP32 backward sweep + FP64 update, every iteration)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
            "launch_ms": round(solve_ms, 3),
            "basis": f"({iters} + 1) x {fwd_b} + {iters} x {BWD_BYTES['mixed']} algorithmic B per cell per launch"}


def pair_roofline(cells, its, launch_ms):
    """Roofline of a two-right-hand-side solve's persistent launches: the pair
    launch k_persist<float, double, 3, 2, false, ...> sweeps both until the first
    stops at iteration n0 (n0 + 1 pair forward sweeps, n0 pair backward
    sweeps), then the other continues from x_n0 in a one-RHS launch
    (n1 - n0 + 1 forward and n1 - n0 backward sweeps; none when both stop
    together).  launch_ms: the launches' summed device time from HIP events
    around each (sip_system_solve_ms)."""
    n0, n1 = min(its), max(its)
    pair = (n0 + 1) * PAIR_FWD_BYTES + n0 * PAIR_BWD_BYTES
    m = n1 - n0
    cont = (m + 1) * FWD_BYTES["mixed"] + m * BWD_BYTES["mixed"] if m > 0 else 0
    achieved = (pair + cont) * cells / (launch_ms * 1e-3) / 1e9
    st = "true" if cells >= STREAM_HINT_CELLS else "false"
    return {"bound": "hbm",
            "kernel": f"k_persist<float, double, 3, 2, false, {st}> (both right-hand sides in one launch until the "
                      f"first stops) + k_persist<float, double, 3, 1, false, {st}> (the other's continuation)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None, "launch_ms": round(launch_ms, 3),
            "basis": f"({n0} + 1) x {PAIR_FWD_BYTES} + {n0} x {PAIR_BWD_BYTES}"
                     + (f" + ({m} + 1) x {FWD_BYTES['mixed']} + {m} x {BWD_BYTES['mixed']}" if m > 0 else "")
                     + " algorithmic B per cell"}


def sweep_detail(fwd_ms, bwd_ms, cells, storage="full"):
    """The two sweep kernels launched one at a time (HIP events around each
    launch): the per-sweep view of the same work."""
    fwd_b = FWD_BYTES["mixed"] - (A_SYM_SAVING if storage == "symmetric" else 0)
    return {"fwd_ms": round(fwd_ms, 4), "bwd_ms": round(bwd_ms, 4),
            "fwd_gbps": round(fwd_b * cells / (fwd_ms * 1e-3) / 1e9, 1),
            "bwd_gbps": round(BWD_BYTES["mixed"] * cells / (bwd_ms * 1e-3) / 1e9, 1)}


def solve_roofline(rate):
    """Whole-solve bandwidth of a batched or served run: cell-iterations/s times
    the algorithmic bytes of one mixed iteration (forward + backward sweep), as
    a fraction of the HBM peak.  It averages over every launch of the run
    (factorisations, layout copies and idle gaps included), so it bounds the
    sweeps' own fraction from below."""
    achieved = rate * SOLVE_BYTES_MIXED / 1e9
    return {"bound": "hbm", "kernel": "whole solve: every sweep launch (persistent or per-epoch) over all active "
                                      "blocks (mixed)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
            "basis": f"cell-iterations/s x {SOLVE_BYTES_MIXED} algorithmic B per mixed cell-iteration"}


def rel_err(xm, x64):
    """max |x_mixed - x_fp64| / max |x_fp64| (on the device)."""
    s = float(x64.abs().max())
    return float((xm - x64).abs().max()) / s if s > 0 else 0.0


def run_batch(sip, blocks, precision, epoch_iters, tag):
    """All blocks submitted at once to a fresh solve server (factor + solve
    to RTOL); returns wall time, cell-iterations, results, stats, solutions."""
    import torch
    srv = sip.Server(max_slots=256, epoch_iters=epoch_iters)
    xs = [torch.zeros_like(b) for _, _, b in blocks]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = [srv.submit(tag * 1000 + q, A, b, xs[q], precision=precision, rtol=RTOL, max_iter=200000)
               for q, (_, A, b) in enumerate(blocks)]
    res = [srv.poll(t) for t in tickets]
    t1 = time.perf_counter()
    st = srv.stats()
    srv.close()
    ci = sum(dims[0] * dims[1] * dims[2] * r["iters"] for (dims, _, _), r in zip(blocks, res))
    return t1 - t0, ci, res, st, xs


def config3_summary(args, sip):
    """64 uneven blocks (dims uniform 32..160 per axis, half Poisson, half
    convection-diffusion) through one solve server: one mixed and one FP64
    run, the mixed result's error against the FP64 result per block, the
    whole-solve roofline and the oracle on all host cores."""
    import torch

    from paper_1303_4538_amd import problems
    meta = problems.config3_meta()
    blocks = []
    for dims, kind, ss in meta:
        A, b = problems.make_block(dims, kind, ss)
        blocks.append((dims, torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda()))
    log("64 uneven blocks through the solve server: mixed, FP64")
    run_batch(sip, blocks, "mixed", args.epoch_iters, 1)   # warm-up
    dt, ci, res, st, xs = run_batch(sip, blocks, "mixed", args.epoch_iters, 2)
    dt64, ci64, res64, _, xs64 = run_batch(sip, blocks, "fp64", args.epoch_iters, 3)
    errs = [rel_err(x, y) for x, y in zip(xs, xs64)]
    value = ci / dt
    log("64 uneven blocks: the same solved one after the other")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ci1 = 0
    for dims, A, b in blocks:
        S = sip.sip_factor(A, problems.ALPHA, "mixed")
        _, it, _, _ = sip.sip_solve(S, b, torch.zeros_like(b), RTOL, 200000)
        S.close()
        ci1 += dims[0] * dims[1] * dims[2] * it
    torch.cuda.synchronize()
    one_at_a_time = ci1 / (time.perf_counter() - t0)
    out = {"workload": "64 blocks, dims uniform 32..160 per axis, half Poisson / half upwind convection-diffusion, "
                       "one solve server, factor + mixed solve to 1e-8",
           "cells": sum(d[0] * d[1] * d[2] for d, _, _ in blocks),
           **working_set(sum(d[0] * d[1] * d[2] for d, _, _ in blocks)), "value": value, "unit": "cell-iterations/s",
           "seconds": dt, "max_iters": max(r["iters"] for r in res), "max_rel_res": max(r["rel_res"] for r in res),
           "all_ok": all(r["status"] == 0 for r in res) and all(r["status"] == 0 for r in res64),
           "epochs": st["epochs"], "fp64_cell_iters_per_s": ci64 / dt64, "mixed_speedup_vs_fp64": value / (ci64 / dt64),
           "one_at_a_time_cell_iters_per_s": one_at_a_time, "speedup_vs_one_at_a_time": value / one_at_a_time,
           "err_vs_fp64_max": max(errs), "err_vs_fp64_median": sorted(errs)[len(errs) // 2],
           "roofline": solve_roofline(value)}
    if not args.no_cpu:
        log("64 uneven blocks: oracle sample on the host cores")
        out["cpu_baseline"] = batched_cpu_baseline(meta, args.cpu_iters_batched)
    del blocks, xs, xs64
    torch.cuda.empty_cache()
    return out


def config4_summary(args, sip):
    """512 x 512 x 256 stretched-grid Poisson (67 M cells): factor + mixed solve
    to 1e-8 and the same in FP64, the mixed result's error against the FP64
    result, the persistent solve kernel's roofline (HIP events on the launch
    stream) and the oracle on one host core (first iterations)."""
    import numpy as np
    import torch

    from paper_1303_4538_amd import problems
    c = problems.config4()
    cells = 512 * 512 * 256
    A = torch.from_numpy(c["A"]).cuda()
    b = torch.from_numpy(c["b"]).cuda()
    xs, its, secs = {}, {}, {}
    for precision in ("mixed", "fp64"):
        log(f"512x512x256: {precision} solve")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S = sip.sip_factor(A, c["alpha"], precision)
        x = torch.zeros_like(b)
        _, it, rr, _ = sip.sip_solve(S, b, x, RTOL, 200000)
        torch.cuda.synchronize()
        secs[precision] = time.perf_counter() - t0
        if precision == "mixed":
            if os.environ.get("SIP_SOLVE_PERSISTENT", "1") != "0":
                solve_ms = sip.sip_system_solve_ms(S)   # HIP events around the launch, on its stream
            fwd_ms, bwd_ms = sip.sip_profile_sweeps(S, b, torch.zeros_like(b), args.profile_iters)
            rr_mixed = rr
        S.close()
        xs[precision], its[precision] = x, it
    value = cells * its["mixed"] / secs["mixed"]
    if os.environ.get("SIP_SOLVE_PERSISTENT", "1") != "0":
        roofline = persist_roofline(cells, its["mixed"], solve_ms, workload="large")
        roofline["sweeps_one_launch_each"] = sweep_detail(fwd_ms, bwd_ms, cells)
    else:
        achieved = FWD_BYTES["mixed"] * cells / (fwd_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": "k_forward<float, double, 3, 1, 2, true> (FP64 residual + FP32 forward sweep)",
                    "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
                    **sweep_detail(fwd_ms, bwd_ms, cells)}
    out = {"workload": "512x512x256 stretched-grid Poisson (z ratio 1.05), alpha 0.92, factor + mixed solve to 1e-8",
           "cells": cells, **working_set(cells), "value": value, "unit": "cell-iterations/s", "seconds": secs["mixed"],
           "iterations": its["mixed"], "final_rel_res": rr_mixed, "fp64_iterations": its["fp64"],
           "fp64_cell_iters_per_s": cells * its["fp64"] / secs["fp64"],
           "mixed_speedup_vs_fp64": secs["fp64"] / secs["mixed"] * its["mixed"] / its["fp64"],
           "err_vs_fp64": rel_err(xs["mixed"], xs["fp64"]),
           "roofline": roofline}
    del A, b, xs
    torch.cuda.empty_cache()
    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        log("512x512x256: oracle sample")
        LU = oracle.factor(c["A"], c["alpha"])
        t = time.perf_counter()
        oracle.iterate(c["A"], LU, c["b"], np.zeros_like(c["b"]), args.cpu_iters_large, mixed=True)
        dt = time.perf_counter() - t
        out["cpu_baseline"] = {"value": cells * args.cpu_iters_large / dt, "unit": "cell-iterations/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"first {args.cpu_iters_large} mixed-form SIP iterations of the 512x512x256 "
                                         "block, single-threaded C oracle, factorisation untimed"}
        del LU
    return out


def _oracle_stream_sample(job):
    """One served system on one host core: factorisation (untimed), then n
    mixed-form oracle iterations (timed) on one of its right-hand sides."""
    dims, kind, ss, rs, n = job
    import numpy as np

    import oracle
    from paper_1303_4538_amd import problems
    A = problems.system_coefficients(dims, kind, ss)
    b = problems.request_rhs(dims, rs)
    LU = oracle.factor(A, problems.ALPHA)
    t = time.perf_counter()
    oracle.iterate(A, LU, b, np.zeros_like(b), n, mixed=True)
    return dims[0] * dims[1] * dims[2] * n, time.perf_counter() - t


def config5_summary(args, sip):
    """The serving stream at its full size (250 systems x 8 right-hand sides,
    Poisson arrivals at 200/s): latency percentiles and throughput, the
    whole-solve roofline, the mixed results' error against FP64 solves of a 5 %
    sample of the requests, and the oracle on a 5 % sample of the systems over
    all host cores."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import torch
    log("serving stream 250 x 8 at %g/s" % args.serve_rate)
    m = serve_stream(sip, 250, args.serve_rate, args.serve_budget_gb, args.epoch_iters, keep=True)
    log("serving: FP64 solves of a 5 % sample")
    value = m["ci"] / m["span"]
    errs = []
    for q in range(0, m["n"], 20):
        _, s, _, _ = m["reqs"][q]
        S = sip.sip_factor(m["As"][s], 0.92, "fp64")
        x64 = torch.zeros_like(m["bs"][q])
        sip.sip_solve(S, m["bs"][q], x64, RTOL, 200000)
        S.close()
        errs.append(rel_err(m["xs"][q], x64))
    out = {"workload": f"{m['n']} requests (250 systems x 8 rhs), Poisson arrivals {args.serve_rate:g}/s, lognormal "
                       f"dims 24..192, half Poisson / half CD, HBM budget {args.serve_budget_gb:g} GB",
           "value": value, "unit": "cell-iterations/s", "seconds": m["wall"], **_serving_fields(m, args.serve_rate),
           "max_rel_res": max(r["rel_res"] for r in m["res"]),
           "err_vs_fp64_max": max(errs), "err_vs_fp64_median": sorted(errs)[len(errs) // 2],
           "err_vs_fp64_sample": f"every 20th request ({len(errs)} of {m['n']}), FP64 factor + solve to 1e-8",
           "roofline": solve_roofline(value)}
    sample = [m["systems"][s] for s in range(0, len(m["systems"]), 20)]
    first_rhs = {}
    for _, s, _, rs in m["reqs"]:
        first_rhs.setdefault(s, rs)
    del m
    torch.cuda.empty_cache()
    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        log("serving: oracle sample on the host cores")
        procs = max(1, min(16, os.cpu_count() or 1))
        systems = [(d, k, ss, first_rhs[20 * i], args.cpu_iters_serving) for i, (d, k, ss) in enumerate(sample)]
        with ProcessPoolExecutor(procs, mp_context=mp.get_context("spawn")) as pool:
            res = list(pool.map(_oracle_stream_sample, systems))
        ci = sum(c for c, _ in res)
        busy = sum(t for _, t in res)
        out["cpu_baseline"] = {"value": ci / (busy / procs), "unit": "cell-iterations/s", "cores": procs,
                               "kind": "oracle",
                               "sample": f"every 20th system ({len(systems)} of 250), {args.cpu_iters_serving} "
                                         f"mixed-form SIP iterations each on its first right-hand side, one "
                                         f"process per system on {procs} cores, factorisation untimed"}
    return out


def fp32_comparison(sip, A, b, alpha, cells):
    """The paper's all-FP32 relaxation against the mixed form on the same
    block: solve time and iterations to FP32_RTOL (factorisation untimed), the
    sweep kernels' times and the residual level where FP32 stalls."""
    import torch

    def solve(precision):
        S = sip.sip_factor(A, alpha, precision)
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, it, rr, _ = sip.sip_solve(S, b, x, FP32_RTOL, 200000)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        fwd, bwd = sip.sip_profile_sweeps(S, b, torch.zeros_like(b), 20)
        S.close()
        return it, rr, dt, fwd, bwd

    it32, rr32, dt32, f32, b32 = solve("fp32")
    itm, rrm, dtm, fm, bm = solve("mixed")
    S = sip.sip_factor(A, alpha, "fp32")
    hist = sip.sip_iterate(S, b, torch.zeros_like(b), 4 * it32 + 50)
    S.close()
    return {"rtol": FP32_RTOL, "iterations": it32, "mixed_iterations": itm,
            "rel_res": rr32, "mixed_rel_res": rrm,
            "solve_ms": round(dt32 * 1e3, 3), "mixed_solve_ms": round(dtm * 1e3, 3),
            "cell_iters_per_s": cells * it32 / dt32, "mixed_cell_iters_per_s": cells * itm / dtm,
            "fwd_ms": round(f32, 4), "bwd_ms": round(b32, 4), "mixed_fwd_ms": round(fm, 4),
            "mixed_bwd_ms": round(bm, 4),
            "fwd_gbps_algorithmic": round(FWD_BYTES["fp32"] * cells / (f32 * 1e-3) / 1e9, 1),
            "stall_rel_res": float(min(hist))}


def pair_run(args):
    """256^3 convection-diffusion, two right-hand sides (the default one and
    a second seeded one) solved together by sip_solve_multi to 1e-8 (mixed);
    value = right-hand-side cell-iterations / wall time, factorisation in the
    step.  The line also gives the same two solved one after the other."""
    import numpy as np
    import torch

    from paper_1303_4538_amd import problems, sip

    sip.lib()
    dev = torch.device("cuda:0")
    n = args.n
    c = problems.config2(n)
    cells = n ** 3
    b2 = problems.rhs_uniform(n, n, n, np.random.default_rng(np.random.SeedSequence(problems.MASTER_SEED).spawn(3)[2]))
    A = torch.from_numpy(c["A"]).to(dev)
    bs = [torch.from_numpy(c["b"]).to(dev), torch.from_numpy(b2).to(dev)]
    torch.cuda.synchronize()

    persistent = os.environ.get("SIP_SOLVE_PERSISTENT", "1") != "0"
    launch_ms = []   # per timed two-RHS solve: its persistent launches' device time

    def step(together, timed=False):
        S = sip.sip_factor(A, c["alpha"], "mixed")
        xs = [torch.zeros_like(b) for b in bs]
        if together:
            st, info = sip.sip_solve_multi(S, bs, xs, RTOL, 200000)
            its = [i[0] for i in info]
            if timed and persistent:
                launch_ms.append(sip.sip_system_solve_ms(S))
        else:
            its = [sip.sip_solve(S, b, x, RTOL, 200000)[1] for b, x in zip(bs, xs)]
        S.close()
        return its

    for _ in range(args.warmup):
        step(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = [step(True, timed=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = cells * sum(sum(i) for i in its) / elapsed
    t1 = time.perf_counter()
    its1 = step(False)
    torch.cuda.synchronize()
    alone = cells * sum(its1) / (time.perf_counter() - t1)
    S = sip.sip_factor(A, c["alpha"], "mixed")
    fwd_ms, bwd_ms = sip.sip_profile_sweeps_multi(S, bs, [torch.zeros_like(b) for b in bs], args.profile_iters)
    S.close()
    achieved = PAIR_FWD_BYTES * cells / (fwd_ms * 1e-3) / 1e9
    sweeps = {"fwd_ms": round(fwd_ms, 4), "bwd_ms": round(bwd_ms, 4), "fwd_gbps": round(achieved, 1),
              "bwd_gbps": round(PAIR_BWD_BYTES * cells / (bwd_ms * 1e-3) / 1e9, 1)}
    if persistent:
        roof = pair_roofline(cells, its[-1], sum(launch_ms) / len(launch_ms))
        m = MEASURED.get("pair")
        if m and kernels_sha256() == MEASURED["kernels_sha256"] and m["iterations"] == its[-1]:
            roof["traffic"] = round(m["persist_bytes"] / (roof["launch_ms"] * 1e-3) / 1e9, 1)
        roof["sweeps_one_launch_each"] = sweeps
    else:
        roof = {"bound": "hbm", "kernel": "k_forward<float, double, 3, 2, 2, true> (pair forward sweep, one launch)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None, **sweeps}
    line = {
        "metric": "right-hand-side cell-iterations/s (two mixed SIP solves swept together, to 1e-8)",
        "value": value, "unit": "cell-iterations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{n}^3 upwind convection-diffusion (D=1, max|F|=2), two right-hand sides, "
                               f"alpha 0.92, factor + sip_solve_multi to {RTOL:g}",
                   "cells": cells, "iterations": its[-1], "one_after_the_other_cell_iters_per_s": alone,
                   "speedup_vs_one_after_the_other": value / alone},
        "roofline": roof,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def blocks_run(args):
    """The 256^3 convection-diffusion domain cut into q^3 equal blocks, each
    factorised alone and coupled through boundary values once per iteration;
    factor + mixed solve to 1e-8.  value = domain cell-iterations / wall time.
    Block coupling changes the iteration (more iterations than one block)."""
    import torch

    from paper_1303_4538_amd import problems, sip

    sip.lib()
    dev = torch.device("cuda:0")
    n, q = args.n, args.blocks_per_axis
    c = problems.config2(n)
    cells = n ** 3
    cuts = [[n * t // q for t in range(q + 1)]] * 3
    A = torch.from_numpy(c["A"]).to(dev)
    b = torch.from_numpy(c["b"]).to(dev)
    torch.cuda.synchronize()

    def step():
        B = sip.sip_blocks_factor(A, cuts, c["alpha"], "mixed")
        x = torch.zeros_like(b)
        st, it, rr, _ = B.solve(b, x, RTOL, 200000)
        B.close()
        return it, rr

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    its = [it for it, _ in res]
    value = cells * sum(its) / elapsed
    line = {
        "metric": "cell-iterations/s (multi-block mixed SIP to 1e-8 rel. residual)",
        "value": value, "unit": "cell-iterations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{n}^3 upwind convection-diffusion (D=1, max|F|=2) cut into {q}^3 blocks coupled "
                               f"through boundary values, alpha 0.92, factor + mixed solve to {RTOL:g}",
                   "cells": cells, "blocks": q ** 3, "iterations": its[-1],
                   "final_rel_res": max(rr for _, rr in res),
                   "ms_per_iteration": elapsed / sum(its) * 1e3},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def tune_run(args):
    """Every compiled sweep plan (loader phases 1..3 x poll distance 1..3; the
    distances other than 2 with two or three phases) timed per iteration
    (forward + backward launch, HIP events) on mixed solves of blocks from
    32^3 to 512x512x256, and the plan sip_tune picks for each block."""
    import torch

    from paper_1303_4538_amd import problems, sip

    sip.lib()
    shapes = [((32, 32, 32), "cd"), ((64, 64, 64), "cd"), ((160, 160, 160), "cd"), ((256, 256, 256), "cd"),
              ((512, 512, 256), "stretched")]
    plans = [(ph, pd) for ph in (1, 2, 3) for pd in (1, 2, 3) if pd == 2 or ph >= 2]
    table = []
    for dims, kind in shapes:
        ni, nj, nk = dims
        if kind == "stretched":
            c = problems.config4()
            A, b = c["A"], c["b"]
        else:
            A, b = problems.make_block(dims, kind, np_seed(ni))
        At, bt = torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda()
        n_iter = max(4, min(40, int(4e8 // (ni * nj * nk))))
        row = {"dims": list(dims), "kind": kind, "iters_timed": n_iter, "ms_per_iteration": {}}
        for ph, pd in plans:
            os.environ["SIP_SWEEP_PHASES"], os.environ["SIP_POLL_DISTANCE"] = str(ph), str(pd)
            S = sip.sip_factor(At, problems.ALPHA, "mixed")
            assert sip.sip_system_plan(S) == (ph, pd)
            f, bk = sip.sip_profile_sweeps(S, bt, torch.zeros_like(bt), n_iter)
            S.close()
            row["ms_per_iteration"][f"{ph}x{pd}"] = round(f + bk, 5)
        del os.environ["SIP_SWEEP_PHASES"], os.environ["SIP_POLL_DISTANCE"]
        S = sip.sip_factor(At, problems.ALPHA, "mixed")
        sip.sip_tune(S, bt, n_iter)
        row["tuned"] = "%dx%d" % sip.sip_system_plan(S)
        S.close()
        best = min(row["ms_per_iteration"], key=row["ms_per_iteration"].get)
        row["fastest"] = best
        row["default_3x2_vs_fastest"] = round(row["ms_per_iteration"]["3x2"] / row["ms_per_iteration"][best], 4)
        log(f"tune {dims}: fastest {best}, tuned {row['tuned']}, {row['ms_per_iteration']}")
        table.append(row)
        del At, bt
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "sweep plans: ms per mixed iteration (forward + backward launch)",
                      "plans": [f"{ph}x{pd}" for ph, pd in plans], "table": table}), flush=True)


def steps_run(args):
    """Step time and hop lag of the sweeps, separated: sip_profile_sweeps (HIP
    events around each launch) on mixed convection-diffusion blocks whose
    shapes isolate them -- one tile (no exchange, no contention), a row and a
    column of 16 tiles (15 hops in a row), 8 x 8 tiles and the 256^3 block.
    A launch of nk planes takes nk + 14 steps of its last tile (the shear of
    the 8-lane tile edge), so us per step = launch time / (nk + 14)."""
    import torch

    from paper_1303_4538_amd import problems, sip

    sip.lib()
    shapes = [(16, 16, 256), (16, 16, 1024), (256, 16, 256), (16, 256, 256), (128, 128, 256), (256, 256, 256)]
    rows = []
    for dims in shapes:
        ni, nj, nk = dims
        A, b = problems.make_block(dims, "cd", np_seed(ni + 3 * nj + 7 * nk))
        At, bt = torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda()
        S = sip.sip_factor(At, problems.ALPHA, "mixed")
        f, bk = sip.sip_profile_sweeps(S, bt, torch.zeros_like(bt), args.profile_iters)
        plan = "%dx%d" % sip.sip_system_plan(S)
        S.close()
        row = {"dims": list(dims), "tiles": (ni // 16) * (nj // 16), "plan": plan, "fwd_ms": round(f, 4),
               "bwd_ms": round(bk, 4), "fwd_us_per_step": round(f * 1e3 / (nk + 14), 3),
               "bwd_us_per_step": round(bk * 1e3 / (nk + 14), 3)}
        log(f"steps {dims}: {row}")
        rows.append(row)
        del At, bt
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "sweep step time: us per tile step (launch time / (nk + 14))", "table": rows}),
          flush=True)


def np_seed(k):
    import numpy as np
    return np.random.SeedSequence(1234 + k)


def pair_and_blocks(sip, A, b, alpha, n):
    """The same block and b: (1) with a second seeded right-hand side, both
    solved together (sip_solve_multi) against one after the other; (2) cut
    into 2^3 blocks coupled through boundary values.  Mixed, to RTOL, one solve
    each (kernels already warm), factorisation untimed."""
    import numpy as np
    import torch

    from paper_1303_4538_amd import problems

    cells = n ** 3
    b2 = torch.from_numpy(problems.rhs_uniform(
        n, n, n, np.random.default_rng(np.random.SeedSequence(problems.MASTER_SEED).spawn(3)[2]))).to(b.device)
    S = sip.sip_factor(A, alpha, "mixed")
    xs = [torch.zeros_like(b), torch.zeros_like(b)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = sip.sip_solve_multi(S, [b, b2], xs, RTOL, 200000)
    torch.cuda.synchronize()
    t_pair = time.perf_counter() - t0
    its = [i[0] for i in info]
    pair_roof = None
    if os.environ.get("SIP_SOLVE_PERSISTENT", "1") != "0":
        r = pair_roofline(cells, its, sip.sip_system_solve_ms(S))
        pair_roof = {k: r[k] for k in ("achieved", "frac", "launch_ms")}
    t0 = time.perf_counter()
    for rhs in (b, b2):
        sip.sip_solve(S, rhs, torch.zeros_like(b), RTOL, 200000)
    torch.cuda.synchronize()
    t_alone = time.perf_counter() - t0
    S.close()
    cuts = [[0, n // 2, n]] * 3
    B = sip.sip_blocks_factor(A, cuts, alpha, "mixed")
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, itb, rrb, _ = B.solve(b, x, RTOL, 200000)
    torch.cuda.synchronize()
    t_blk = time.perf_counter() - t0
    B.close()
    return {"two_rhs_iterations": its,
            "two_rhs_cell_iters_per_s": cells * sum(its) / t_pair,
            "one_after_the_other_cell_iters_per_s": cells * sum(its) / t_alone,
            "two_rhs_speedup": t_alone / t_pair,
            "two_rhs_persistent_launches": pair_roof,
            "blocks_2x2x2_iterations": itb, "blocks_2x2x2_rel_res": rrb,
            "blocks_2x2x2_cell_iters_per_s": cells * itb / t_blk,
            "blocks_2x2x2_solve_s": round(t_blk, 3)}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only; --gpus must be 1 (the library does not shard a solve "
              "across GPUs)", file=sys.stderr)
        sys.exit(2)
    if args.prof:
        prof_run(args)
        return
    if args.workload == "batched":
        batched_run(args)
        return
    if args.workload == "serving":
        serving_run(args)
        return
    if args.workload == "pair":
        pair_run(args)
        return
    if args.workload == "blocks":
        blocks_run(args)
        return
    if args.workload == "tune":
        tune_run(args)
        return
    if args.workload == "steps":
        steps_run(args)
        return
    import numpy as np
    import torch

    from paper_1303_4538_amd import problems, sip

    sip.lib()                       # raises if the HIP library is not built
    dev = torch.device("cuda:0")
    n = args.n
    if args.workload == "large":
        c = problems.config4()
        cells = 512 * 512 * 256
        label = "512x512x256 stretched-grid Poisson (z ratio 1.05)"
    else:
        c = problems.config2(n)
        cells = n ** 3
        label = f"{n}^3 upwind convection-diffusion (D=1, max|F|=2)"
    A = torch.from_numpy(c["A"]).to(dev)
    b = torch.from_numpy(c["b"]).to(dev)
    torch.cuda.synchronize()

    xkeep = {}
    persistent = os.environ.get("SIP_SOLVE_PERSISTENT", "1") != "0"
    launch_ms, call_ms = [], []   # per timed solve: the persistent launch, the whole sip_solve call

    def step(precision, timed=False):
        S = sip.sip_factor(A, c["alpha"], precision, storage=args.storage)
        x = torch.zeros_like(b)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        st, it, rr, _ = sip.sip_solve(S, b, x, RTOL, 200000)
        e1.record()
        if timed:
            e1.synchronize()
            call_ms.append(e0.elapsed_time(e1))
            if persistent:   # HIP events around the launch, on its stream
                launch_ms.append(sip.sip_system_solve_ms(S))
        S.close()
        xkeep[precision] = x
        return it, rr

    log(f"{label}: {args.warmup} warm-up and {args.steps} timed steps")
    for _ in range(args.warmup):
        step("mixed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step("mixed", timed=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    iters = [it for it, _ in results]
    value = cells * sum(iters) / elapsed
    ms_per_step = elapsed / args.steps * 1e3

    extra = {}
    log("timed steps done; FP64, all-FP32, pair and block comparisons")
    if not args.no_fp64:
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        it64, rr64 = step("fp64")
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        extra["fp64_iterations"] = it64
        extra["fp64_cell_iters_per_s"] = cells * it64 / (t3 - t2)
        extra["fp64_ms_per_solve"] = (t3 - t2) * 1e3
        extra["mixed_speedup_vs_fp64"] = (t3 - t2) / (elapsed / args.steps)
        extra["err_vs_fp64"] = rel_err(xkeep["mixed"], xkeep["fp64"])
    if not args.no_fp32 and args.storage == "full":
        extra["fp32_relaxation"] = fp32_comparison(sip, A, b, c["alpha"], cells)
    if not args.no_extras and args.storage == "full" and args.workload == "single":
        extra["two_rhs_and_blocks"] = pair_and_blocks(sip, A, b, c["alpha"], n)

    # the sweeps launched one at a time (events around each launch)
    S = sip.sip_factor(A, c["alpha"], "mixed", storage=args.storage)
    x = torch.zeros_like(b)
    fwd_ms, bwd_ms = sip.sip_profile_sweeps(S, b, x, args.profile_iters)
    S.close()
    fwd_bytes = FWD_BYTES["mixed"] - (A_SYM_SAVING if args.storage == "symmetric" else 0)
    if persistent:
        # dominant kernel: the persistent solve, one launch per timed solve
        same_iters = len(set(iters)) == 1
        wl = ("large" if args.workload == "large" else "single" if args.n == 256 else None) if same_iters else None
        roofline = persist_roofline(cells, iters[0], sum(launch_ms) / len(launch_ms), args.storage, wl)
        roofline["solve_call_ms"] = round(sum(call_ms) / len(call_ms), 3)
        roofline["sweeps_one_launch_each"] = sweep_detail(fwd_ms, bwd_ms, cells, args.storage)
        achieved = roofline["achieved"]
    else:
        # chunked graph replays: the fused residual + forward sweep dominates
        achieved = fwd_bytes * cells / (fwd_ms * 1e-3) / 1e9
        phases = int(os.environ.get("SIP_SWEEP_PHASES", "3"))   # the single-system default: 3 loader phases
        poll = int(os.environ.get("SIP_POLL_DISTANCE", "2"))    # and polls 2 steps ahead
        st = "true" if cells >= STREAM_HINT_CELLS and phases == 3 and poll == 2 else "false"
        roofline = {"bound": "hbm",
                    "kernel": f"k_forward<float, double, {phases}, 1, {poll}, {st}> (FP64 residual + FP32 forward "
                              "sweep)",
                    "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
                    **sweep_detail(fwd_ms, bwd_ms, cells, args.storage)}
    # what a plain device copy reaches on this GPU, as context for the fraction
    copy = copy_gbps()
    roofline["copy_gbps"] = round(copy, 1)
    roofline["frac_of_copy"] = round(achieved / copy, 4)

    cpu = None
    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        An, bn = c["A"], c["b"]
        LU = oracle.factor(An, c["alpha"])
        t4 = time.perf_counter()
        oracle.iterate(An, LU, bn, np.zeros_like(bn), args.cpu_iters, mixed=True)
        t5 = time.perf_counter()
        cpu = {"value": cells * args.cpu_iters / (t5 - t4), "unit": "cell-iterations/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{label}, first {args.cpu_iters} mixed-form SIP iterations "
                         f"(FP64 residual, FP32 sweeps), single-threaded C oracle, factorisation untimed",
               "host_cpu": host_cpu(), "host_cpus": os.cpu_count()}

    configs = None
    if not args.no_configs and args.workload == "single" and args.storage == "full" and args.n == 256:
        del A, b, xkeep
        torch.cuda.empty_cache()
        configs = {"batched_64_blocks": config3_summary(args, sip),
                   "large_512x512x256": config4_summary(args, sip),
                   "serving_250x8_at_200_per_s": config5_summary(args, sip)}

    mean_it = sum(iters) / len(iters)
    line = {
        "metric": "cell-iterations/s (mixed SIP to 1e-8 rel. residual)",
        "value": value,
        "unit": "cell-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"{label}, alpha 0.92, factor + mixed solve to {RTOL:g}"
                        + (", symmetric coefficient storage" if args.storage == "symmetric" else ""),
            "cells": cells,
            **working_set(cells),
            "iterations": mean_it,
            "final_rel_res": max(rr for _, rr in results),
            "hbm_gbps_algorithmic": value * (fwd_bytes + BWD_BYTES["mixed"]) / 1e9,
            **extra,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if configs is not None:
        line["configs"] = configs
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
