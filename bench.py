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
same solve in plain FP64, the forward-sweep kernel's achieved bandwidth
against the HBM peak (timed with HIP events on the launch stream) and the CPU
oracle on a bounded sample of the same workload.
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
FWD_BYTES = {"mixed": 56 + 8 + 8 + 16 + 4, "fp64": 56 + 8 + 8 + 32 + 8}    # A, b, x, L (Lb,Lw,Ls,1/Lp), y out
BWD_BYTES = {"mixed": 12 + 4 + 8 + 8, "fp64": 24 + 8 + 8 + 8}              # U, y, x in, x out
RTOL = 1e-8


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256, help="block edge (cells)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--profile-iters", type=int, default=40)
    ap.add_argument("--cpu-iters", type=int, default=12)
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1 (multi-GPU sharding is "
              "described in DESIGN.md, not implemented)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1303_4538_amd import problems, sip

    sip.lib()                       # raises if the HIP library is not built
    dev = torch.device("cuda:0")
    n = args.n
    cells = n ** 3
    c = problems.config2(n)
    A = torch.from_numpy(c["A"]).to(dev)
    b = torch.from_numpy(c["b"]).to(dev)
    torch.cuda.synchronize()

    def step(precision):
        S = sip.sip_factor(A, c["alpha"], precision)
        x = torch.zeros_like(b)
        st, it, rr, _ = sip.sip_solve(S, b, x, RTOL, 200000)
        S.close()
        return it, rr

    for _ in range(args.warmup):
        step("mixed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step("mixed") for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    iters = [it for it, _ in results]
    value = cells * sum(iters) / elapsed
    ms_per_step = elapsed / args.steps * 1e3

    extra = {}
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

    # dominant kernel: the fused residual + forward sweep (events on the launch stream)
    S = sip.sip_factor(A, c["alpha"], "mixed")
    x = torch.zeros_like(b)
    fwd_ms, bwd_ms = sip.sip_profile_sweeps(S, b, x, args.profile_iters)
    S.close()
    achieved = FWD_BYTES["mixed"] * cells / (fwd_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": "k_forward<float> (residual + forward sweep)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
                "fwd_ms": round(fwd_ms, 4), "bwd_ms": round(bwd_ms, 4),
                "bwd_gbps": round(BWD_BYTES["mixed"] * cells / (bwd_ms * 1e-3) / 1e9, 1)}

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
               "sample": f"{n}^3 convection-diffusion block, first {args.cpu_iters} mixed-form SIP iterations "
                         f"(FP64 residual, FP32 sweeps), single-threaded C oracle, factorisation untimed"}

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
            "workload": f"{n}^3 upwind convection-diffusion (D=1, max|F|=2), alpha 0.92, factor + mixed "
                        f"solve to {RTOL:g}",
            "cells": cells,
            "iterations": mean_it,
            "final_rel_res": max(rr for _, rr in results),
            "hbm_gbps_algorithmic": value * (FWD_BYTES["mixed"] + BWD_BYTES["mixed"]) / 1e9,
            **extra,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
