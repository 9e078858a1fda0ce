#!/usr/bin/env python3
"""Benchmark of the exact symbolic hot path on one MI355X.

Workload (one step): the projection step of a curve analysis,
R = res_y(f, f_y) and gcd(R, R') in Z[x], for f dense of total degree 24
with uniform signed 16-bit coefficients (seeded).  The inputs are planned and
uploaded once (resident in HBM); a timed step runs the whole device path --
reduction mod 35 primes, evaluation and elimination at 553 points per prime,
interpolation, CRT to exact integers, then the modular gcd of R and R' with
its certificate -- and returns both results to the host.

Prints one JSON line.  Also reported: per-stage device times (HIP events on
the launch stream), the roofline of the dominant kernel, the oracle timed on
the host cores, and batched vs plain resultants/s on 512 random pairs.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # int32 VALU lane-ops/s of the MI355X (39.32 T)


def eval_elim_lane_ops(m: int, n: int, T: int) -> int:
    """Essential VALU lane-ops of one (prime, point) instance of the fused
    evaluate+eliminate kernel: 3 per Horner step (64-bit multiply-add, low
    multiply, multiply-add), 4 per two-product update lc(Y) X_i - lc(X) Y_i and
    3 per scale-only update lc(Y) X_i, over the normal remainder sequence."""
    ops = 3 * T
    if m < n:
        m, n = n, m
    if n == 0:
        return ops
    a, b, s = m, n, m - n + 1
    while b >= 1:
        dX = a
        for _ in range(s):
            ops += 4 * b + 3 * (dX - b)
            dX -= 1
        a, b, s = b, b - 1, 2
    return ops


def cpu_baseline(f, g, cores: int):
    """The oracle (exact Bareiss at every point + Newton interpolation) on the
    host cores, for res_y of the same workload."""
    from oracle import resultant as R
    t0 = time.perf_counter()
    r = R.resultant_y_by_points(f, g, processes=cores)
    dt = time.perf_counter() - t0
    return r, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on a single GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if world != 1:
        print("bench.py: single-GPU benchmark; launch without torch.distributed.run", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1103_4697_amd as snc
    import synth

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    ctx = snc.Context(0)
    f, g = synth.config1()
    plan = snc.resultant_plan(f, g)
    D, k = plan.deg_bound, plan.nprimes

    batch = snc.ResultantBatch([(f, g)], ctx)   # planned and uploaded once: inputs resident

    def step():
        batch.run()
        d = batch.out[0].deg
        Rl = batch.bufs[0][: d + 1]
        G = snc.gcd_z_limbs(Rl, snc.derivative_limbs(Rl), ctx)
        return d, G

    progress("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        d, G = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    value = args.steps / dt

    progress(f"timed {args.steps} steps: {dt / args.steps * 1e3:.3f} ms/step")
    # correctness of the last step against the stored oracle values
    ref = json.load(open(os.path.join(ROOT, "tests", "golden", "config1.json")))
    Rints = snc.limbs_to_ints(batch.bufs[0][: d + 1])
    q61 = (1 << 61) - 1
    parity = ([c % q61 for c in Rints] == ref["mod_2_61_minus_1"]
              and snc.limbs_to_ints(G) == [int(c) for c in ref["gcd_r_rprime"]])

    # per-stage device times of the same resultant on the plain path (events on its stream)
    ctx.set_timing(True)
    stages = {}
    nrep = 10
    for _ in range(nrep):
        snc.resultant_y(f, g, ctx)
        for name, ms, _n in ctx.timing():
            stages[name] = stages.get(name, 0.0) + ms / nrep
    gstages = {}
    Rl = batch.bufs[0][: d + 1]
    Rpl = snc.derivative_limbs(Rl)
    for _ in range(nrep):
        snc.gcd_z_limbs(Rl, Rpl, ctx)
        for name, ms, _n in ctx.timing():
            gstages[name] = gstages.get(name, 0.0) + ms / nrep
    ctx.set_timing(False)
    ee_ms = stages.get("eval_elim", float("nan"))
    m, n = f.shape[0] - 1, g.shape[0] - 1
    T = sum(int(np.max(np.nonzero(row)[0]) + 1) if np.any(row) else 0 for row in f) + \
        sum(int(np.max(np.nonzero(row)[0]) + 1) if np.any(row) else 0 for row in g)
    ops_launch = eval_elim_lane_ops(m, n, T) * k * (D + 1)
    achieved = ops_launch / (ee_ms * 1e-3) / 1e12

    out = {
        "metric": "exact resultants/sec (res_y(f, f_y) + gcd(R, R'), bit-exact)",
        "value": round(value, 3),
        "unit": "resultants/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "curve-analysis projection: f dense total degree 24, uniform signed "
                               "16-bit coefficients, g = df/dy; res_y then gcd(R, R')",
                   "deg_bound": D, "primes": k, "points": D + 1, "parallelism": "single GPU"},
        "parity_ok": bool(parity),
        "mod_p_evals_per_s": round(k * (D + 1) / (ms_per_step * 1e-3), 1),
        "stage_ms": {kk: round(v, 4) for kk, v in stages.items()},
        "gcd_stage_ms": {kk: round(v, 4) for kk, v in gstages.items()},
        "roofline": {"kernel": "eval_elim", "bound": "alu", "achieved": round(achieved, 4),
                     "peak": round(PEAK_VALU_TOPS, 3), "unit": "TOP/s (int32 VALU lane-ops)",
                     "frac": round(achieved / PEAK_VALU_TOPS, 5), "traffic": None,
                     "ops_per_launch": ops_launch, "avg_launch_ms": round(ee_ms, 5)},
    }

    progress(f"stages {stages}")
    progress(f"gcd stages {gstages}")
    if not args.no_batch:
        progress("batched workload")
        pairs, _common = synth.config2()
        b512 = snc.ResultantBatch(pairs, ctx)
        b512.run()
        torch.cuda.synchronize()
        nb = 5
        t0 = time.perf_counter()
        for _ in range(nb):
            b512.run()
        torch.cuda.synchronize()
        bt = (time.perf_counter() - t0) / nb
        nplain = 64
        t0 = time.perf_counter()
        for i in range(nplain):
            snc.resultant_y(*pairs[i], ctx)
        torch.cuda.synchronize()
        pt = (time.perf_counter() - t0) / nplain
        out["batched"] = {"workload": "512 random dense pairs, total degrees 8..40, 8..32-bit, 10% with a "
                                      "common factor",
                          "batched_resultants_per_s": round(len(pairs) / bt, 2),
                          "plain_resultants_per_s": round(1.0 / pt, 2),
                          "speedup": round((len(pairs) / bt) * pt, 3),
                          "batched_ms": round(bt * 1e3, 3)}

    if not args.no_cpu_baseline:
        progress("cpu baseline")
        cores = min(16, os.cpu_count() or 1)
        r, cdt = cpu_baseline(f, g, cores)
        out["cpu_baseline"] = {"value": round(1.0 / cdt, 5), "unit": "resultants/s", "cores": cores,
                               "kind": "oracle",
                               "sample": "res_y(f, f_y) of the same workload, exact Bareiss at all 553 points "
                                         "+ Newton interpolation, one full run (gcd excluded)",
                               "agrees": r == Rints}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
