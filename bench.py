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
    evaluate+eliminate kernel: Horner's rule in x^4 costs 6 per 4
    coefficients (four 64-bit multiply-adds, low multiply, multiply-add);
    every normal remainder (the first one when deg A = deg B + 1, and all
    later ones) is one fused update of three products and one REDC, 5 per
    coefficient of the new remainder; a first remainder with a larger degree
    gap takes elementary steps, 4 per two-product update lc(Y) X_i -
    lc(X) Y_i and 3 per scale-only update lc(Y) X_i."""
    ops = (3 * T) // 2
    if m < n:
        m, n = n, m
    if n == 0:
        return ops
    if m == n + 1:
        ops += 5 * n
    else:
        dX = m
        for _ in range(m - n + 1):
            ops += 4 * n + 3 * (dX - n)
            dX -= 1
    b = n - 1
    while b >= 1:
        ops += 5 * b
        b -= 1
    return ops


def gcd_euclid_lane_ops(da: int, db: int) -> int:
    """Essential VALU lane-ops of one prime of the modular Euclid kernel on a
    normal remainder sequence (each remainder one degree below its divisor,
    the generic case): a remainder of d coefficients costs 3 products and one
    REDC (2 ops) per coefficient; the first reduction of a by b takes
    (da - db + 1) elementary steps of 4 ops per coefficient of b."""
    if da < db:
        da, db = db, da
    ops = 4 * db * (da - db + 1) if da > db + 1 else 0
    d = db - 1 if da > db + 1 else db
    while d >= 1:
        ops += 5 * d
        d -= 1
    return ops


def profiled_traffic(kernel: str, source: str):
    """HBM bytes per launch of a kernel from the committed counter summary
    (profiles/<kernel>_*.md, FETCH_SIZE + WRITE_SIZE scaled by a copy of known
    size), or None when there is none or the kernel source changed since."""
    import glob
    import hashlib
    sha = hashlib.sha256(open(os.path.join(ROOT, source), "rb").read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"{kernel}_*.md"))):
        fields = {}
        for line in open(path):
            if ":" in line and line.strip().startswith("- "):
                key, val = line.strip()[2:].split(":", 1)
                tok = val.split()
                fields[key.strip()] = tok[0].strip("`") if tok else ""
        if fields.get("kernel_source_sha256") == sha and "traffic_bytes_per_launch" in fields:
            return int(float(fields["traffic_bytes_per_launch"]))
    return None


def cpu_baseline(f, g, cores: int):
    """The oracle (exact Bareiss at every point + Newton interpolation) on the
    host cores, for res_y of the same workload."""
    from oracle import resultant as R
    t0 = time.perf_counter()
    r = R.resultant_y_by_points(f, g, processes=cores)
    dt = time.perf_counter() - t0
    return r, dt


def serving(snc, synth, ctx, nreq, progress):
    """Request stream of resultants and gcds (4:1) through the serving loop:
    saturation throughput with everything queued, then Poisson arrivals at
    0.5x and 0.8x of it; latency = finish - submit on the server's clock."""
    import numpy as np

    reqs = synth.config4(nreq)
    srv = snc.Server(pool_bytes=8 << 30, max_slots=256, nstreams=4, ctx=ctx)

    def submit(kind, x, y):
        return srv.submit_resultant(x, y) if kind == "res" else srv.submit_gcd(x, y)

    done = 0
    res = {"workload": "4:1 mix of res_y requests (total degrees 10..50, 8..64-bit) and gcd requests "
                       "(degree 100..2000 with a shared factor of degree 5..50)", "requests": nreq}
    # saturation
    t0 = time.perf_counter()
    tickets = [submit(k, x, y) for k, x, y in reqs]
    ok = srv.wait(done + nreq, 600.0)
    t1 = time.perf_counter()
    done += nreq
    sat = nreq / (t1 - t0)
    lat = np.array([srv.times(t)[1] - srv.times(t)[0] for t in tickets])
    results = [srv.poll(t) for t in tickets]
    # each result equals the same request computed alone (sampled)
    sample = list(range(0, nreq, max(1, nreq // 24)))
    same = all(results[i] == (snc.resultant_y(reqs[i][1], reqs[i][2], ctx) if reqs[i][0] == "res"
                              else snc.gcd_z(reqs[i][1], reqs[i][2], ctx)) for i in sample)
    res.update({"saturation_req_per_s": round(sat, 2), "all_finished": bool(ok),
                "saturation_p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "saturation_p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                "alone_vs_mix_identical_sample": bool(same), "sample_size": len(sample)})
    progress(f"serving saturation {sat:.1f} req/s")
    rng = np.random.default_rng(4321)
    for frac in (0.5, 0.8):
        rate = frac * sat
        arr = synth.poisson_arrivals(rng, rate, nreq)
        tickets = []
        start = time.perf_counter()
        for (k, x, y), at in zip(reqs, arr):
            while time.perf_counter() - start < at:
                pass
            tickets.append(submit(k, x, y))
        ok = srv.wait(done + nreq, 600.0)
        t_end = time.perf_counter()
        done += nreq
        lat = np.array([srv.times(t)[1] - srv.times(t)[0] for t in tickets])
        for t in tickets:
            srv.poll(t)
        res[f"rate_{frac}"] = {"offered_req_per_s": round(rate, 2),
                               "completed_req_per_s": round(nreq / (t_end - start), 2),
                               "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                               "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                               "all_finished": bool(ok)}
        progress(f"serving at {frac} x saturation: p50 {res[f'rate_{frac}']['p50_ms']} ms")
    srv.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-sqfree", action="store_true")
    ap.add_argument("--no-curve-sets", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run one device copy of this many MiB (reference for HBM byte counters)")
    ap.add_argument("--profile-curve-set", default="",
                    help="D:B -- only run the five-curve set of degree D and B-bit coefficients five times "
                         "(for a profiler) and exit")
    ap.add_argument("--profile-batch", type=int, default=0,
                    help="only replay the 512-pair batched workload this many times (for profilers) and exit")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many resultant+gcd steps (for profilers) and exit")
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
    if args.calibrate_copy_mib:
        nbytes = args.calibrate_copy_mib << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        progress(f"copy calibration: {nbytes} bytes read and written")
        del src, dst
    ctx = snc.Context(0)
    f, g = synth.config1()
    plan = snc.resultant_plan(f, g)
    D, k = plan.deg_bound, plan.nprimes

    batch = snc.ResultantBatch([(f, g)], ctx)   # planned and uploaded once: inputs resident

    def step():
        # R and gcd(R, R') in one pass: the Euclid runs on R mod p beside the CRT
        batch.run_sqfree()
        d = batch.out[0].deg
        G = batch.gbufs[0][: batch.gout[0].deg + 1]
        return d, G

    if args.profile_curve_set:
        d, bits = (int(v) for v in args.profile_curve_set.split(":"))
        bs = snc.ResultantBatch(synth.random_curve_set(np.random.default_rng(100 * d + bits), d, bits), ctx)
        for _ in range(5):
            bs.run()
        torch.cuda.synchronize()
        progress(f"profile run: curve set degree {d}, {bits} bits, 5 runs done")
        return
    if args.profile_batch:
        pairs, _common = synth.config2()
        bb = snc.ResultantBatch(pairs, ctx)
        for _ in range(args.profile_batch):
            bb.run()
        torch.cuda.synchronize()
        progress(f"profile run: 512-pair batch, {args.profile_batch} runs done")
        return
    if args.profile_steps:
        for _ in range(args.profile_steps):
            step()
        torch.cuda.synchronize()
        progress(f"profile run: {args.profile_steps} steps done")
        return
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
    gcd_primes = 0
    Rl = batch.bufs[0][: d + 1]
    for _ in range(nrep):
        snc.gcd_z_deriv_limbs(Rl, ctx)
        for name, ms, nl in ctx.timing():
            gstages[name] = gstages.get(name, 0.0) + ms / nrep
            if name == "gcd_euclid":
                gcd_primes = nl
    # the step's own Euclid (on the resultant's primes, beside the CRT)
    fu_ms, fu_primes = 0.0, 0
    for _ in range(nrep):
        batch.run_sqfree()
        for name, ms, nl in ctx.timing():
            if name == "sqfree_euclid":
                fu_ms += ms / nrep
                fu_primes = nl
    ctx.set_timing(False)
    ee_ms = stages.get("eval_elim", float("nan"))
    m, n = f.shape[0] - 1, g.shape[0] - 1
    T = sum(int(np.max(np.nonzero(row)[0]) + 1) if np.any(row) else 0 for row in f) + \
        sum(int(np.max(np.nonzero(row)[0]) + 1) if np.any(row) else 0 for row in g)
    ee_ops = eval_elim_lane_ops(m, n, T) * k * (D + 1)
    ee_achieved = ee_ops / (ee_ms * 1e-3) / 1e12
    eu_ms = fu_ms
    eu_ops = gcd_euclid_lane_ops(d, d - 1) * fu_primes
    eu_achieved = eu_ops / (eu_ms * 1e-3) / 1e12

    def roof(kernel, ops, ms, achieved, traffic):
        return {"kernel": kernel, "bound": "alu", "achieved": round(achieved, 4),
                "peak": round(PEAK_VALU_TOPS, 3), "unit": "TOP/s (int32 VALU lane-ops)",
                "frac": round(achieved / PEAK_VALU_TOPS, 5), "traffic": traffic,
                "ops_per_launch": ops, "avg_launch_ms": round(ms, 5)}
    roof_eu = roof("gcd_euclid", eu_ops, eu_ms, eu_achieved,
                   profiled_traffic("gcd_euclid", "paper_1103_4697_amd/csrc/kernels_gcd.hip"))
    roof_ee = roof("eval_elim", ee_ops, ee_ms, ee_achieved,
                   profiled_traffic("eval_elim", "paper_1103_4697_amd/csrc/kernels_res.hip"))
    roof_eu["primes_per_launch"] = fu_primes
    dominant, secondary = (roof_eu, roof_ee) if eu_ms >= ee_ms else (roof_ee, roof_eu)

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
        "roofline": dominant,
        "roofline_other": secondary,
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

    if not args.no_curve_sets:
        progress("random curve sets")
        sets = {}
        for d in (6, 9, 12, 15):
            for bits in (10, 128, 512, 2048):
                pairs = synth.random_curve_set(np.random.default_rng(100 * d + bits), d, bits)
                bs = snc.ResultantBatch(pairs, ctx)
                bs.run()
                torch.cuda.synchronize()
                nrep = 3
                t0 = time.perf_counter()
                for _ in range(nrep):
                    bs.run()
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) / nrep * 1e3
                kmax = max(snc.resultant_plan(*pr).nprimes for pr in pairs)
                sets[f"d{d}_b{bits}"] = {"ms": round(ms, 3), "max_primes": kmax}
                progress(f"curve set degree {d}, {bits} bits: {ms:.3f} ms ({kmax} primes)")
        out["random_curve_sets"] = {"workload": "five random dense curves of total degree d with signed b-bit "
                                                "coefficients: res_y(f, f_y) of each and res_y(f, h) of every "
                                                "pair (15 resultants) in one batch",
                                    "sets": sets}

    if not args.no_curve_sets:
        progress("content in y")
        hx = [-1, 3, 1]  # x^2 + 3x - 1: the vertical lines at its two real roots
        fh = [synth.univariate_product(hx, [int(c) for c in row]) for row in f]
        got = snc.content_y(fh, ctx)  # warm-up (workspace)
        torch.cuda.synchronize()
        nrep = 5
        t0 = time.perf_counter()
        for _ in range(nrep):
            got = snc.content_y(fh, ctx)
        torch.cuda.synchronize()
        ct = (time.perf_counter() - t0) / nrep
        out["content_y"] = {"workload": "content in y of (x^2 + 3x - 1) f for the step's curve f (25 rows of "
                                        "degree up to 26): row gcds in a tree of batched modular gcds",
                            "ms": round(ct * 1e3, 3), "parity_ok": got == hx}

    if not args.no_curve_sets:
        progress("FastLift Q")
        q = snc.fastlift_q(f, ctx)  # warm-up
        torch.cuda.synchronize()
        nrep = 5
        t0 = time.perf_counter()
        for _ in range(nrep):
            q = snc.fastlift_q(f, ctx)
        torch.cuda.synchronize()
        qt = (time.perf_counter() - t0) / nrep
        out["fastlift_q"] = {"workload": "Q = res_y(f_x / h, f_y / h), h = gcd(f_x, f_y), for the step's curve f: "
                                         "h certified constant in y and in x mod p on the host, then one resultant",
                             "ms": round(qt * 1e3, 3), "deg_Q": len(q) - 1}

    if not args.no_sqfree:
        progress("square-free factorisation")
        a, want = synth.sqfree_request(np.random.default_rng(2024))
        got = snc.sqfree_factor(a, ctx)  # warm-up (plans, workspace)
        torch.cuda.synchronize()
        nrep = 5
        t0 = time.perf_counter()
        for _ in range(nrep):
            got = snc.sqfree_factor(a, ctx)
        torch.cuda.synchronize()
        st_ = (time.perf_counter() - t0) / nrep
        out["sqfree_factor"] = {"workload": "a = -6 f1 f2^2 f3^3, monic f_i of degrees 120, 60, 30 with signed "
                                            "8-bit coefficients (degree 330); Yun's algorithm, one modular gcd "
                                            "per step",
                                "factorisations_per_s": round(1.0 / st_, 2),
                                "ms": round(st_ * 1e3, 3),
                                "parity_ok": got == (-6, want)}

    if not args.no_serving:
        progress("serving workload")
        out["serving"] = serving(snc, synth, ctx, args.serving_requests, progress)

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
