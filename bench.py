#!/usr/bin/env python3
"""Benchmark of the exact symbolic hot path on one MI355X.

Headline (one step): the batched workload -- 512 random dense pairs
f, g in Z[x, y] with total degrees uniform in 8..40 and signed coefficients
of 8..32 bits, 10% of them built with a common factor (res_y = 0) -- planned
and uploaded once (inputs resident in HBM); a step replays the captured
pipeline over every pair's (prime, point) instances -- reduction mod the
primes, evaluation and elimination, interpolation, Chinese remaindering --
and returns all 512 resultants to the host.  value = resultants/s of the
batched form; the plain form (one library call per pair, synchronised, no
graph) runs the same pairs beside it.

Also reported: per-stage device times of the batch (HIP events on the launch
stream), the roofline of its dominant kernel against the int32 VALU peak and
a measured Montgomery-product ceiling, algorithmic HBM GB/s of the
evaluation, interpolation and CRT stages, the large single instance (degrees
64/48, int64), the curve-analysis projection step (res_y(f, f_y) and
gcd(R, R')), the paper's random curve sets, content, FastLift's Q, Yun,
serving, and the oracle timed on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # int32 VALU lane-ops/s of the MI355X (39.32 T)
PEAK_HBM_GBPS = 8000.0


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# Essential work per kernel (algorithmic counts, not instructions issued)
# ---------------------------------------------------------------------------

def eval_elim_lane_ops(m: int, n: int, T: int) -> int:
    """Essential VALU lane-ops of one (prime, point) instance of the fused
    evaluate+eliminate kernel: Horner's rule in x^4 costs 6 per 4
    coefficients (four 64-bit multiply-adds, low multiply, multiply-add);
    every normal remainder (the first one when deg A = deg B + 1, and all
    later ones) is one fused update of three products and one REDC, 5 per
    coefficient of the new remainder; a first remainder with another degree
    gap takes s = m - n + 1 elementary steps, each an update of two products
    and one REDC (4) on the n coefficients that meet B, plus 6 for the
    entries above them, which are only scaled by lc(B): one coefficient
    enters the updated part per step, scaled by the running power of lc(B)
    (3), and that power takes one more product (3)."""
    ops = (3 * T) // 2
    if m < n:
        m, n = n, m
    if n == 0:
        return ops
    if m == n + 1:
        ops += 5 * n
    else:
        ops += (m - n + 1) * (4 * n + 6)
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


def interp_lane_ops(D: int) -> int:
    """Essential lane-ops of the interpolation of one prime from D+1 values:
    the Newton coefficients are a convolution of (D+1)^2/2 products and the
    Newton-to-monomial expansion another (D+1)^2/2; each product is one
    64-bit multiply-add, and every eight share a 3-op reduction."""
    return (11 * (D + 1) * (D + 1)) // 8


def crt_lane_ops(k: int, L: int) -> int:
    """Essential lane-ops of the Chinese remaindering of one coefficient from
    k residues: Garner's digits take k(k-1)/2 modular products (one 64-bit
    multiply-add each, a 3-op reduction per sixteen), the binary value
    sum_j y_j P_j about k L / 2 limb multiply-adds with their carries
    (2 ops each)."""
    return (k * (k - 1) // 2) * 19 // 16 + k * L


def pair_shape(f, g):
    """(m, n, T) of a pair: y-degrees over Z[x] and stored coefficients."""
    def rows(F):
        out = []
        for row in F:
            nz = [i for i, c in enumerate(row) if int(c) != 0]
            out.append(nz[-1] + 1 if nz else 0)
        while out and out[-1] == 0:
            out.pop()
        return out
    rf, rg = rows(f), rows(g)
    return len(rf) - 1, len(rg) - 1, sum(rf) + sum(rg)


def source_sha(source) -> str:
    """sha256 of a kernel's source file, or of the concatenation of several."""
    import hashlib
    h = hashlib.sha256()
    for src in ((source,) if isinstance(source, str) else source):
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return h.hexdigest()


def profiled_traffic(kernel: str, source, workload: str):
    """HBM bytes per launch of a kernel on a workload from the committed
    counter summary (profiles/<kernel>_<workload>_counters.md: FETCH_SIZE +
    WRITE_SIZE scaled by a copy of known size), or None when there is none
    or the kernel source (one file or several) changed since."""
    sha = source_sha(source)
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            key, val = line.strip()[2:].split(":", 1)
            tok = val.split()
            fields[key.strip()] = tok[0].strip("`") if tok else ""
    if fields.get("kernel_source_sha256") == sha and "traffic_bytes_per_launch" in fields:
        return int(float(fields["traffic_bytes_per_launch"]))
    return None


def roof(kernel, ops, ms, traffic, ceilings, algo_bytes=None):
    achieved = ops / (ms * 1e-3) / 1e12
    r = {"kernel": kernel, "bound": "alu", "achieved": round(achieved, 4), "peak": round(PEAK_VALU_TOPS, 3),
         "unit": "TOP/s (int32 VALU lane-ops)", "frac": round(achieved / PEAK_VALU_TOPS, 5), "traffic": traffic,
         "ops_per_launch": int(ops), "avg_launch_ms": round(ms, 5)}
    if algo_bytes is not None:
        r["algorithmic_bytes"] = int(algo_bytes)
        r["hbm_gbps"] = round(algo_bytes / (ms * 1e-3) / 1e9, 2)
    if ceilings.get("mad_u64_per_s"):
        r["frac_of_measured_mad_rate"] = round(ops / (ms * 1e-3) / ceilings["mad_u64_per_s"], 5)
    return r


def stage_times(ctx, run, nrep):
    """Average per-stage device times (ms) over nrep timed runs."""
    ctx.set_timing(True)
    acc = {}
    try:
        for _ in range(nrep):
            run()
            for name, ms, _n in ctx.timing():
                acc[name] = acc.get(name, 0.0) + ms / nrep
    finally:
        ctx.set_timing(False)
    return acc


def cpu_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"os_cpu_count": os.cpu_count(), "cpu_model": model, "python": platform.python_version()}


# ---------------------------------------------------------------------------
# The oracle leg: timed on the host cores, and the checker of the GPU results
# ---------------------------------------------------------------------------

def _oracle_point(args):
    from oracle import resultant as R
    f, g, x0 = args
    t0 = time.perf_counter()
    v = R.resultant_at(f, g, x0)
    return v, time.perf_counter() - t0


def _oracle_modq(args):
    from oracle import resultant as R
    f, g, x0, q = args
    return R.resultant_at_mod(f, g, x0, q)


def cpu_baseline_leg(pairs, common, results, plans, cores, nsample, npoints, nexact):
    """The oracle on the host cores for the batched workload, and the
    oracle's checks of the GPU results.

    Timing (extrapolated, labelled so): nsample pairs drawn from the batch
    (seeded), the exact Sylvester determinant of each at npoints random
    integer points of its balanced range; the oracle's full resultant of a
    pair is D+1 such determinants plus an interpolation, so its cost is
    taken as (D+1) times the mean point time.  Rate on C cores =
    C / (mean cost over the sample), the oracle parallelising over points.

    Checks: the timed values equal the GPU resultants evaluated at the same
    points; every pair's GPU resultant agrees with the oracle's determinant
    modulo a 61-bit prime at a random point; the nexact cheapest pairs
    equal the oracle's full resultant coefficient by coefficient."""
    import multiprocessing as mp
    import random

    from oracle import resultant as R
    from oracle import zx

    rng = random.Random(20260)
    idx = sorted(rng.sample(range(len(pairs)), nsample))
    tasks = []
    for i in idx:
        D = plans[i].deg_bound
        for _ in range(npoints):
            tasks.append((i, rng.randint(-(D // 2), (D + 1) // 2)))
    q = (1 << 61) - 1
    xq = [rng.randrange(q) for _ in pairs]
    ctx_mp = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx_mp.Pool(cores) as pool:
        out = pool.map(_oracle_point, [(pairs[i][0], pairs[i][1], x0) for i, x0 in tasks], chunksize=1)
    wall = time.perf_counter() - t0
    with ctx_mp.Pool(cores) as pool:
        modq = pool.map(_oracle_modq, [(f, g, xq[i], q) for i, (f, g) in enumerate(pairs)], chunksize=4)
    per_pair = {}
    exact_ok = True
    for (i, x0), (v, dt) in zip(tasks, out):
        per_pair.setdefault(i, []).append(dt)
        exact_ok &= zx.evaluate(results[i], x0) == v
    costs = [(plans[i].deg_bound + 1) * (sum(ts) / len(ts)) for i, ts in per_pair.items()]
    mean_cost = sum(costs) / len(costs)
    modq_ok = all(zx.evaluate(results[i], xq[i]) % q == modq[i] for i in range(len(pairs)))
    cheap = sorted(range(len(pairs)), key=lambda i: (plans[i].deg_bound + 1) * len(pairs[i][0]) ** 3)[:nexact]
    elem_ok = all(results[i] == R.resultant_y_by_points(pairs[i][0], pairs[i][1], processes=cores) for i in cheap)
    zeros_ok = all(results[i] == [] for i in common)
    return ({"value": round(cores / mean_cost, 6), "unit": "resultants/s", "cores": cores, "kind": "oracle",
             "single_core_resultants_per_s": round(1.0 / mean_cost, 7),
             "sample": f"{nsample} of the 512 pairs (seeded), exact Sylvester determinant (fraction-free "
                       f"Bareiss over Z) at {npoints} random integer points each; a pair's full oracle "
                       f"resultant (D+1 points + interpolation) extrapolated as (D+1) x its mean point time; "
                       f"rate on {cores} cores = cores / mean pair cost",
             "extrapolated": True, "sample_wall_s": round(wall, 2),
             "sample_core_s": round(sum(dt for _v, dt in out), 2), **cpu_info()},
            {"exact_values_at_sampled_points": bool(exact_ok), "mod_q_all_pairs": bool(modq_ok),
             "elementwise_pairs": cheap, "elementwise_ok": bool(elem_ok), "planted_zero_pairs_ok": bool(zeros_ok)})


# ---------------------------------------------------------------------------
# Sections
# ---------------------------------------------------------------------------

def measure_ceilings(ctx):
    out = {}
    for kind in ("montgomery", "mul_lo", "mad_u64"):
        out[f"{kind}_per_s"] = round(ctx.microbench(kind), 1)
    return out


def batch_stage_roofline(snc, pairs, plans, stages, ceilings, workload_tag):
    """Roofline records of the batch's stages from their device times."""
    ee_ops, ip_ops, crt_ops = 0, 0, 0
    ee_bytes = ip_bytes = crd_bytes = crc_bytes = 0
    for (f, g), p in zip(pairs, plans):
        if p.nprimes == 0:
            continue
        m, n, T = pair_shape(f, g)
        k, D, L = p.nprimes, p.deg_bound, p.out_nlimbs
        nl = snc.bivariate_limbs(f)[3]
        ee_ops += eval_elim_lane_ops(m, n, T) * k * (D + 1)
        ip_ops += interp_lane_ops(D) * k
        crt_ops += crt_lane_ops(k, L) * (D + 1)
        ee_bytes += 4 * nl * T + 4 * k * T + 4 * k * (D + 1)      # limbs in, residues kept, values out
        ip_bytes += 12 * k * (D + 1)                               # values, 1/t! table, coefficients
        crd_bytes += 4 * k * (D + 1) + 2 * k * k                   # coefficients mod p in, constants P_j mod p_i
        crc_bytes += 4 * (D + 1) * L + 4 * k * L                    # output limbs, prefix products P_j
    ee_ms = sum(v for kk, v in stages.items() if kk.startswith("eval_elim"))
    crt_ms = sum(v for kk, v in stages.items() if kk.startswith("crt"))
    src_res = "paper_1103_4697_amd/csrc/kernels_res.hip"
    recs = {
        "eval_elim": roof("eval_elim (all register classes)", ee_ops, ee_ms,
                          profiled_traffic("eval_elim", "paper_1103_4697_amd/csrc/eval_elim.hpp", workload_tag),
                          ceilings, ee_bytes),
        "interp": roof("interp", ip_ops, stages.get("interp", float("nan")),
                       profiled_traffic("interp", src_res, workload_tag), ceilings, ip_bytes),
        "crt": roof("crt (all launches: digits and binary value)", crt_ops, crt_ms,
                    profiled_traffic("crt", src_res, workload_tag), ceilings, crd_bytes + crc_bytes),
    }
    hbm = {"eval_elim": recs["eval_elim"]["hbm_gbps"], "interp": recs["interp"]["hbm_gbps"],
           "crt": recs["crt"]["hbm_gbps"], "peak": PEAK_HBM_GBPS}
    return recs, hbm, ee_ms


def large_single(snc, synth, ctx, nrep):
    """f dense of total degree 64, g dense of total degree 48, uniform signed
    64-bit coefficients: D = 3072, several hundred primes, multi-word CRT."""
    import torch
    f, g = synth.config3()
    p = snc.resultant_plan(f, g)
    b = snc.ResultantBatch([(f, g)], ctx)
    b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nrep):
        b.run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / nrep * 1e3
    r = b.results()[0]
    ref = json.load(open(os.path.join(ROOT, "tests", "golden", "config3.json")))
    top = ref["top_degree"]
    parity = (len(r) - 1 == top and r[0] == int(ref["res_at_0"]) and r[top] == int(ref["top_coefficient"]))
    st = stage_times(ctx, b.run, 3)
    m, n, T = pair_shape(f, g)
    ops = eval_elim_lane_ops(m, n, T) * p.nprimes * (p.deg_bound + 1)
    ee_ms = sum(v for kk, v in st.items() if kk.startswith("eval_elim"))
    return {"workload": "f dense total degree 64, g dense total degree 48, uniform signed 64-bit coefficients",
            "deg_bound": p.deg_bound, "primes": p.nprimes, "out_limbs": p.out_nlimbs,
            "ms": round(ms, 3), "resultants_per_s": round(1e3 / ms, 2),
            "mod_p_evals_per_s": round(p.nprimes * (p.deg_bound + 1) / (ms * 1e-3), 1),
            "parity_ok": bool(parity), "parity_check": "exact bottom and top coefficients against stored oracle values",
            "stage_ms": {kk: round(v, 4) for kk, v in st.items()},
            "eval_elim_valu_frac": round(ops / (ee_ms * 1e-3) / 1e12 / PEAK_VALU_TOPS, 5)}


def curve_analysis(snc, synth, ctx, nsteps):
    """The projection step of a curve analysis: R = res_y(f, f_y) for f dense
    of total degree 24 with signed 16-bit coefficients, and gcd(R, R')."""
    import numpy as np
    import torch
    f, g = synth.config1()
    plan = snc.resultant_plan(f, g)
    D, k = plan.deg_bound, plan.nprimes
    batch = snc.ResultantBatch([(f, g)], ctx)
    for _ in range(3):
        batch.run_sqfree()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nsteps):
        batch.run_sqfree()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / nsteps * 1e3
    d = batch.out[0].deg
    G = batch.gbufs[0][: batch.gout[0].deg + 1]
    ref = json.load(open(os.path.join(ROOT, "tests", "golden", "config1.json")))
    q61 = (1 << 61) - 1
    Rints = snc.limbs_to_ints(batch.bufs[0][: d + 1])
    parity = ([c % q61 for c in Rints] == ref["mod_2_61_minus_1"]
              and snc.limbs_to_ints(G) == [int(c) for c in ref["gcd_r_rprime"]])
    ctx.set_timing(True)
    eu_ms, eu_primes = 0.0, 0
    nrep = 10
    for _ in range(nrep):
        batch.run_sqfree()
        for name, t, nl in ctx.timing():
            if name == "sqfree_euclid":
                eu_ms += t / nrep
                eu_primes = nl
    ctx.set_timing(False)
    st = stage_times(ctx, lambda: snc.resultant_y(f, g, ctx), nrep)
    m, n = f.shape[0] - 1, g.shape[0] - 1
    T = sum(int(np.max(np.nonzero(row)[0]) + 1) if np.any(row) else 0 for row in f) + \
        sum(int(np.max(np.nonzero(row)[0]) + 1) if np.any(row) else 0 for row in g)
    ee_ms = sum(v for kk, v in st.items() if kk.startswith("eval_elim"))
    eu_ops = gcd_euclid_lane_ops(d, d - 1) * eu_primes
    ee_ops = eval_elim_lane_ops(m, n, T) * k * (D + 1)
    src_gcd = ("paper_1103_4697_amd/csrc/kernels_gcd.hip", "paper_1103_4697_amd/csrc/gcd_reg.hpp")
    return {"workload": "curve-analysis projection: f dense total degree 24, uniform signed 16-bit "
                        "coefficients, g = df/dy; res_y then gcd(R, R') in one pass",
            "deg_bound": D, "primes": k, "ms_per_step": round(ms, 4), "steps_per_s": round(1e3 / ms, 2),
            "parity_ok": bool(parity),
            "stage_ms": {kk: round(v, 4) for kk, v in st.items()},
            "euclid": roof("gcd_euclid", eu_ops, eu_ms, profiled_traffic("gcd_euclid", src_gcd, "curve_d552"), {}),
            "eval_elim": roof("eval_elim", ee_ops, ee_ms,
                              profiled_traffic("eval_elim", "paper_1103_4697_amd/csrc/eval_elim.hpp",
                                               "curve_d552"), {})}


def curve_sets(snc, synth, ctx):
    import numpy as np
    import torch
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
            bs.close()
    return {"workload": "five random dense curves of total degree d with signed b-bit coefficients: "
                        "res_y(f, f_y) of each and res_y(f, h) of every pair (15 resultants) in one batch",
            "sets": sets}


def arrangements(snc, synth, ctx):
    """The projection phase of an arrangement of a curve set: contents of all
    curves in one tree of batched gcds (at preparation), then res_y(p, p_y)
    of every primitive part and res_y(p_i, p_j) of every pair as one batch."""
    import numpy as np
    import torch
    out = {"workload": "sets of planar curves cycling through circles, ellipses, random dense curves of degree 3..8 "
                       "(10-bit), graphs of rational functions and curves with a factor in x alone; n contents, "
                       "then n + n(n-1)/2 resultants per run"}
    for n in (20, 50):
        curves = synth.arrangement_set(np.random.default_rng(3000 + n), n)
        t0 = time.perf_counter()
        A = snc.Arrangement(curves, ctx)
        prep = time.perf_counter() - t0
        A.run()
        torch.cuda.synchronize()
        nrep = 5
        t0 = time.perf_counter()
        for _ in range(nrep):
            A.run()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / nrep * 1e3
        npairs = n + n * (n - 1) // 2
        out[f"n{n}"] = {"resultants": npairs, "contents_and_primitive_parts_ms": round(prep * 1e3, 2),
                        "run_ms": round(ms, 3), "resultants_per_s": round(npairs / (ms * 1e-3), 1)}
        progress(f"arrangement of {n} curves: {npairs} resultants in {ms:.2f} ms")
        A.close()
    return out


def timed(fn, nrep):
    import torch
    out = fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nrep):
        out = fn()
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t0) / nrep


def serving(snc, synth, ctx, nreq):
    """Request stream of resultants and gcds (4:1) through the serving loop:
    saturation throughput with everything queued, then Poisson arrivals at
    0.5x and 0.8x of it; latency = finish - submit on the server's clock.
    Every result is compared with the same request computed alone."""
    import numpy as np

    reqs = synth.config4(nreq)
    srv = snc.Server(pool_bytes=8 << 30, max_slots=256, nstreams=4, ctx=ctx)

    def submit(kind, x, y):
        return srv.submit_resultant(x, y) if kind == "res" else srv.submit_gcd(x, y)

    done = 0
    res = {"workload": "4:1 mix of res_y requests (total degrees 10..50, 8..64-bit) and gcd requests "
                       "(degree 100..2000 with a shared factor of degree 5..50)", "requests": nreq}
    t0 = time.perf_counter()
    tickets = [submit(k, x, y) for k, x, y in reqs]
    ok = srv.wait(done + nreq, 600.0)
    t1 = time.perf_counter()
    done += nreq
    sat = nreq / (t1 - t0)
    lat = np.array([srv.times(t)[1] - srv.times(t)[0] for t in tickets])
    results = [srv.poll(t) for t in tickets]
    # the same requests alone: resultants as plain calls, gcds one at a time
    alone = []
    for kind, x, y in reqs:
        alone.append(snc.resultant_y(x, y, ctx) if kind == "res" else snc.gcd_z(x, y, ctx))
    same = results == alone
    res.update({"saturation_req_per_s": round(sat, 2), "all_finished": bool(ok),
                "saturation_p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "saturation_p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                "alone_vs_mix_identical": bool(same), "compared": nreq})
    progress(f"serving saturation {sat:.1f} req/s, identical to alone: {same}")
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
        got = [srv.poll(t) for t in tickets]
        res[f"rate_{frac}"] = {"offered_req_per_s": round(rate, 2),
                               "completed_req_per_s": round(nreq / (t_end - start), 2),
                               "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                               "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                               "all_finished": bool(ok), "identical_to_alone": got == alone}
        progress(f"serving at {frac} x saturation: p50 {res[f'rate_{frac}']['p50_ms']} ms")
    srv.close()
    res["parity_ok"] = bool(same and all(res[f"rate_{fr}"]["identical_to_alone"] for fr in (0.5, 0.8)))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the headline batch, its parity and roofline")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--cpu-sample-pairs", type=int, default=64)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run one device copy of this many MiB (reference for HBM byte counters)")
    ap.add_argument("--ceilings", action="store_true",
                    help="only measure the integer-operation ceilings (Montgomery product, mul_lo, mad_u64)")
    ap.add_argument("--profile-curve-set", default="",
                    help="D:B -- only run the five-curve set of degree D and B-bit coefficients five times")
    ap.add_argument("--profile-batch", type=int, default=0,
                    help="only replay the 512-pair batched workload this many times (for profilers)")
    ap.add_argument("--profile-large", type=int, default=0,
                    help="only run the degree-64/48 int64 instance this many times (for profilers)")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many curve-analysis projection steps (for profilers)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on a single GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: single-GPU benchmark; launch without torch.distributed.run", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1103_4697_amd as snc
    import synth

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

    if args.ceilings:
        print(json.dumps({"ceilings": measure_ceilings(ctx), "peak_int32_valu_tops": round(PEAK_VALU_TOPS, 3)}))
        return
    if args.profile_curve_set:
        d, bits = (int(v) for v in args.profile_curve_set.split(":"))
        bs = snc.ResultantBatch(synth.random_curve_set(np.random.default_rng(100 * d + bits), d, bits), ctx)
        for _ in range(5):
            bs.run()
        torch.cuda.synchronize()
        progress(f"profile run: curve set degree {d}, {bits} bits, 5 runs done")
        return
    if args.profile_large:
        bl = snc.ResultantBatch([synth.config3()], ctx)
        for _ in range(args.profile_large):
            bl.run()
        torch.cuda.synchronize()
        progress(f"profile run: degree-64/48 int64 instance, {args.profile_large} runs done")
        return
    if args.profile_steps:
        f1, g1 = synth.config1()
        b1 = snc.ResultantBatch([(f1, g1)], ctx)
        for _ in range(args.profile_steps):
            b1.run_sqfree()
        torch.cuda.synchronize()
        progress(f"profile run: {args.profile_steps} projection steps done")
        return

    progress("planning and uploading the 512-pair batch")
    pairs, common = synth.config2()
    t_prep = time.perf_counter()
    batch = snc.ResultantBatch(pairs, ctx)
    prep_s = time.perf_counter() - t_prep
    tune_rep, tune_ms = ctx.tuning()
    if args.profile_batch:
        for _ in range(args.profile_batch):
            batch.run()
        torch.cuda.synchronize()
        progress(f"profile run: 512-pair batch, {args.profile_batch} runs done")
        return
    plans = list(batch.each)
    ninst = sum(p.nprimes * (p.deg_bound + 1) for p in plans if p.nprimes > 0)

    progress("warmup")
    for _ in range(args.warmup):
        batch.run()
        batch.collect(batch.submit())
    torch.cuda.synchronize()
    # one run at a time: plan-free replay, download and widening of each
    # step before the next starts (the latency of one batch)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.run()
    torch.cuda.synchronize()
    ms_single = (time.perf_counter() - t0) / args.steps * 1e3
    serial_results = batch.results()
    # the timed steps: each step's results download and are widened while
    # the next step's kernels run (two steps in flight)
    t0 = time.perf_counter()
    inflight = []
    for _ in range(args.steps):
        inflight.append(batch.submit())
        if len(inflight) == 2:
            batch.collect(inflight.pop(0))
    while inflight:
        batch.collect(inflight.pop(0))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    value = len(pairs) * args.steps / dt
    progress(f"timed {args.steps} batched steps: {ms_per_step:.3f} ms/step, {value:.1f} resultants/s "
             f"(one at a time: {ms_single:.3f} ms/step)")
    results = batch.results()
    pipelined_same = results == serial_results

    # the plain form on the same pairs
    plain = snc.PlainResultants(pairs, ctx)
    plain.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain.run()
    torch.cuda.synchronize()
    pt = time.perf_counter() - t0
    plain_rate = len(pairs) / pt
    plain_res = plain.results()
    progress(f"plain: {pt * 1e3:.1f} ms for {len(pairs)} pairs, {plain_rate:.1f} resultants/s")

    same_as_plain = plain_res == results and pipelined_same
    zeros_ok = all(results[i] == [] for i in common)
    nonzero_ok = all(results[i] != [] for i in range(len(pairs)) if i not in common)

    stages = stage_times(ctx, batch.run, 5)
    ceilings = measure_ceilings(ctx)
    recs, hbm, _ee_ms = batch_stage_roofline(snc, pairs, plans, stages, ceilings, "batch512")
    order = sorted(recs, key=lambda kk: -recs[kk]["avg_launch_ms"])
    dominant, secondary = recs[order[0]], recs[order[1]]

    out = {
        "metric": "exact resultants/sec, batched vs plain, bit-exact",
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
        "config": {"workload": "batched: 512 random dense pairs f, g in Z[x,y], total degrees uniform 8..40, "
                               "uniform signed coefficients of 8..32 bits, 51 pairs (10%) built as f = h a, "
                               "g = h b with a common factor h of y-degree 1..3 (res_y = 0); every pair's "
                               "(prime, point) instances in one graph replay; consecutive steps pipelined "
                               "(a step's result download and widening beside the next step's kernels)",
                   "pairs": len(pairs), "instances": ninst,
                   "max_deg_bound": max(p.deg_bound for p in plans),
                   "max_primes": max(p.nprimes for p in plans), "parallelism": "single GPU"},
        "parity_ok": bool(same_as_plain and zeros_ok and nonzero_ok),
        "ms_per_step_one_at_a_time": round(ms_single, 4),
        "resultants_per_s_one_at_a_time": round(len(pairs) / (ms_single * 1e-3), 2),
        "parity": {"batched_equals_plain_all_pairs": bool(same_as_plain),
                   "pipelined_equals_one_at_a_time": bool(pipelined_same),
                   "planted_zero_pairs_exact": bool(zeros_ok),
                   "other_pairs_nonzero": bool(nonzero_ok)},
        "plain_resultants_per_s": round(plain_rate, 2),
        "batched_vs_plain": round(value / plain_rate, 3),
        "mod_p_evals_per_s": round(ninst / (ms_per_step * 1e-3), 1),
        "stage_ms": {kk: round(v, 4) for kk, v in stages.items()},
        "roofline": dominant,
        "roofline_other": secondary,
        "roofline_stages": recs,
        "hbm_gbps_algorithmic": hbm,
        "ceilings": ceilings,
        "autotune": {"classes": tune_rep, "tuning_ms": round(tune_ms, 1),
                     "prepare_s_including_tuning": round(prep_s, 3),
                     "note": "one-time: variants chosen at preparation (measured, or read from the cache file)"},
    }

    if not args.no_extras:
        progress("large single instance (degrees 64/48, int64)")
        out["large_single"] = large_single(snc, synth, ctx, 3)
        progress("curve-analysis projection step")
        out["curve_analysis"] = curve_analysis(snc, synth, ctx, 20)
        progress("random curve sets")
        out["random_curve_sets"] = curve_sets(snc, synth, ctx)
        f, _g = synth.config1()
        progress("content in y")
        hx = [-1, 3, 1]  # x^2 + 3x - 1: the vertical lines at its two real roots
        fh = [synth.univariate_product(hx, [int(c) for c in row]) for row in f]
        got, ct = timed(lambda: snc.content_y(fh, ctx), 5)
        out["content_y"] = {"workload": "content in y of (x^2 + 3x - 1) f for the curve-analysis f (25 rows of "
                                        "degree up to 26): row gcds in a tree of batched modular gcds",
                            "ms": round(ct * 1e3, 3), "parity_ok": got == hx}
        progress("FastLift Q")
        q, qt = timed(lambda: snc.fastlift_q(f, ctx), 5)
        out["fastlift_q"] = {"workload": "Q = res_y(f_x / h, f_y / h), h = gcd(f_x, f_y), for the curve-analysis f",
                             "ms": round(qt * 1e3, 3), "deg_Q": len(q) - 1}
        # a curve with a squared component: h = gcd(f_x, f_y) depends on y (bivariate modular gcd)
        gsq = [[int(c) for c in row] for row in synth.dense_bivariate(np.random.default_rng(77), 4, bits=8)]
        ksq = [[int(c) for c in row] for row in synth.dense_bivariate(np.random.default_rng(78), 6, bits=8)]
        fsq = synth.bivariate_product(synth.bivariate_product(gsq, gsq), ksq)
        q2, qt2 = timed(lambda: snc.fastlift_q(fsq, ctx), 3)
        out["fastlift_q_y_factor"] = {"workload": "f = g^2 k with g, k random dense of total degrees 4 and 6 "
                                                  "(8-bit): h = gcd(f_x, f_y) has y-degree 4 (bivariate modular gcd)",
                                      "ms": round(qt2 * 1e3, 3), "deg_Q": len(q2) - 1}
        progress("arrangements")
        out["arrangements"] = arrangements(snc, synth, ctx)
        progress("square-free factorisation")
        a, want = synth.sqfree_request(np.random.default_rng(2024))
        got, st_ = timed(lambda: snc.sqfree_factor(a, ctx), 5)
        out["sqfree_factor"] = {"workload": "a = -6 f1 f2^2 f3^3, monic f_i of degrees 120, 60, 30 with signed "
                                            "8-bit coefficients (degree 330); Yun's algorithm",
                                "factorisations_per_s": round(1.0 / st_, 2), "ms": round(st_ * 1e3, 3),
                                "parity_ok": got == (-6, want)}
        if not args.no_serving:
            progress("serving workload")
            out["serving"] = serving(snc, synth, ctx, args.serving_requests)

    if not args.no_cpu_baseline:
        progress("cpu baseline (the oracle on the host cores) and the oracle's checks")
        cores = min(16, os.cpu_count() or 1)
        base, checks = cpu_baseline_leg(pairs, common, results, plans, cores, args.cpu_sample_pairs, 2, 3)
        out["cpu_baseline"] = base
        out["parity"]["oracle"] = checks
        out["parity_ok"] = bool(out["parity_ok"] and all(v for kk, v in checks.items() if kk.endswith("_ok")
                                                         or kk in ("exact_values_at_sampled_points",
                                                                   "mod_q_all_pairs")))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
