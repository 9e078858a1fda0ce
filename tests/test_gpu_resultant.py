"""GPU parity of res_y(f, g) through the C ABI against the CPU oracle.

Exact integers: every comparison is bit-identical (tolerance 0).
* small and medium random pairs (several point tiles, ragged tails, all
  register classes, multi-limb coefficients) against the oracle;
* edge cases: zero operands, constants in y, swapped degrees, leading
  coefficients vanishing at a point or modulo a table prime, a root shared
  at x = 0, a common factor, y-degree above the register classes;
* the curve-analysis workload against stored oracle values;
* the large workload on sampled outputs (exact bottom and top coefficients,
  values modulo 61-bit primes at random points).
"""
import hashlib
import json
import os
import random

import numpy as np
import pytest

import synth
from oracle import resultant as R
from oracle import zx

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
Q61 = (1 << 61) - 1


@pytest.fixture(scope="module")
def snc():
    import paper_1103_4697_amd as m
    return m


def rand_pair(rng, m, n, dxf, dxg, bits):
    lim = 1 << (bits - 1)

    def draw(dy, dx):
        rows = [[int(v) for v in rng.integers(-lim, lim, size=dx + 1, dtype=np.int64)] if bits <= 63
                else [random.Random(int(rng.integers(1 << 30))).randrange(-lim, lim) for _ in range(dx + 1)]
                for _ in range(dy + 1)]
        if all(v == 0 for v in rows[-1]):
            rows[-1][0] = 1
        return rows
    return draw(m, dxf), draw(n, dxg)


def check(snc, f, g, ref=None):
    got = snc.resultant_y(f, g)
    if ref is None:
        ref = R.resultant_y_by_points(f, g, processes=1)
    assert got == ref
    return got


def test_config0_exact(snc):
    f, g = synth.config0()
    assert snc.resultant_y(f, g) == R.resultant_y(f, g)


@pytest.mark.parametrize("seed", range(14))
def test_random_parity(snc, seed):
    rng = np.random.default_rng(5000 + seed)
    m = int(rng.integers(0, 13))
    n = int(rng.integers(0, 13))
    dxf = int(rng.integers(0, 9))
    dxg = int(rng.integers(0, 9))
    bits = [8, 20, 32, 63, 100][seed % 5]
    f, g = rand_pair(rng, m, n, dxf, dxg, bits)
    if seed % 4 == 1 and m > 0:
        f[m - 1] = [0] * (dxf + 1)           # a zero row inside
    check(snc, f, g)


def test_register_classes_and_ragged_tiles(snc):
    # y-degrees hitting each register class (<=8, <=16, <=32, <=48, <=64)
    rng = np.random.default_rng(77)
    for m, n, dx in [(8, 5, 3), (16, 9, 2), (20, 20, 1), (40, 33, 1), (60, 2, 1)]:
        f, g = rand_pair(rng, m, n, dx, dx, 16)
        check(snc, f, g)


# (deg_y f, deg_y g) through every form of the first remainder and every
# phase width: the normal step (m = n + 1) at and below a class's top
# width, m = n (one elementary step) with the whole width meeting g at the
# top, large gaps with g of degree 1 or 2 (a narrow window, most of f only
# scaled), and windows of each width in steps of 8
FIRST_REMAINDER_SHAPES = [(48, 47), (47, 46), (48, 48), (47, 47), (48, 1), (48, 2), (40, 8), (41, 15),
                          (45, 31), (33, 32), (32, 32), (32, 1), (30, 16), (17, 16), (16, 16), (16, 7),
                          (9, 9), (8, 8), (8, 7), (8, 2), (7, 1), (64, 64), (64, 63), (64, 5), (4, 4),
                          (3, 2), (2, 1), (40, 40), (40, 39), (40, 1), (39, 38), (36, 20)]


def test_first_remainder_shapes(snc, assert_same):
    rng = np.random.default_rng(4242)
    pairs = [rand_pair(rng, m, n, 1, 2, 12) for m, n in FIRST_REMAINDER_SHAPES]
    pairs += [(g, f) for f, g in pairs[:4]]   # the smaller degree first
    batch = snc.resultant_y_batch(pairs)
    rs = random.Random(17)
    for (f, g), r in zip(pairs, batch):
        m, n = len(f) - 1, len(g) - 1
        assert len(r) - 1 <= snc.resultant_plan(f, g).deg_bound, (m, n)
        for x0 in (0, 1, rs.randrange(Q61)):
            assert zx.evaluate(r, x0) % Q61 == R.resultant_at_mod(f, g, x0, Q61), (m, n, x0)
    for i in (0, 2, 4, 21, 27):
        assert_same(snc.resultant_y(*pairs[i]), batch[i])


def test_edge_cases(snc):
    one = [[1]]
    f = [[3, 1], [0, 2], [1]]
    assert snc.resultant_y([[0]], f) == []                         # f = 0
    assert snc.resultant_y(f, [[0], [0]]) == []                    # g = 0
    assert snc.resultant_y([[2, 3]], [[7, 0, 1]]) == [1]            # m = n = 0
    assert snc.resultant_y([[1, 1]], f) == R.resultant_y([[1, 1]], f)  # m = 0
    assert snc.resultant_y(f, [[5, 0, 2]]) == R.resultant_y(f, [[5, 0, 2]])  # n = 0
    assert snc.resultant_y(one, one) == [1]
    # swapped degrees with m*n odd (sign)
    rng = np.random.default_rng(3)
    a, b = rand_pair(rng, 1, 3, 2, 2, 10)
    check(snc, a, b)
    check(snc, b, a)
    # leading y-coefficient vanishing at x = 0 (formal degree kept there)
    f2 = [[1, 2], [3, 0, 1], [0, 1]]
    g2 = [[2, 1], [1, 1], [0, 0, 3]]
    check(snc, f2, g2)
    # f(0, y) and g(0, y) share the root y = 1: abnormal remainder at x = 0
    f3 = [[-1, 2], [0, 1], [1, 3]]
    g3 = [[-3, 1], [1, 1], [2, 0, 1]]
    assert R.resultant_at(f3, g3, 0) == 0
    check(snc, f3, g3)
    # common factor: every instance degenerates, result 0
    h = [[1, 1], [2], [1]]
    ua = [[3], [1, 1]]
    vb = [[-1, 2], [0, 0, 1], [1]]
    fa = synth.bivariate_product(h, ua)
    gb = synth.bivariate_product(h, vb)
    assert snc.resultant_y(fa, gb) == []
    # leading coefficient divisible by the first table prime
    p0 = snc.prime(0)
    f4 = [[1, 5, 7], [2, 1], [p0, 0, p0]]
    g4 = [[3, 1, 1], [1, 0, 4], [1, 2], [5]]
    check(snc, f4, g4)


def sparse_abnormal_pair(rng, dx1, dx2, bits):
    """f = y^4 + c1(x), g = y^2 + c2(x): at every point the first remainder
    f rem g = c1 + c2^2 is a constant where a linear one is expected, so
    every (prime, point) instance takes the general elimination.  With g's
    roots +-sqrt(-c2), res_y(f, g) = (c1 + c2^2)^2."""
    lim = 1 << (bits - 1)
    c1 = [int(v) for v in rng.integers(-lim, lim, size=dx1 + 1)]
    c2 = [int(v) for v in rng.integers(-lim, lim, size=dx2 + 1)]
    f = [c1, [0], [0], [0], [1]]
    g = [c2, [0], [1]]
    s = zx.add(c1, zx.mul(c2, c2))
    return f, g, zx.mul(s, s)


def test_abnormal_instances_list_and_scan(snc):
    """Abnormal instances within the list's capacity (list mode) and beyond
    it (scan of the values for the marker), alone and beside normal pairs
    and a common-factor pair."""
    rng = np.random.default_rng(41)
    small = sparse_abnormal_pair(rng, 20, 10, 8)       # few instances: list
    large = sparse_abnormal_pair(rng, 200, 100, 32)    # k (D+1) > 4096: scan
    assert snc.resultant_plan(*large[:2]).nprimes * (snc.resultant_plan(*large[:2]).deg_bound + 1) > 4096
    for f, g, want in (small, large):
        assert snc.resultant_y(f, g) == want == R.resultant_y(f, g)
    h = [[1, 1], [2], [1]]
    fa = synth.bivariate_product(h, [[3], [1, 1]])
    gb = synth.bivariate_product(h, [[-1, 2], [0, 0, 1], [1]])
    a, b = rand_pair(rng, 6, 5, 4, 4, 16)
    pairs = [(a, b), large[:2], (fa, gb), small[:2], (b, a)]
    got = snc.resultant_y_batch(pairs)
    assert got[1] == large[2] and got[3] == small[2] and got[2] == []
    assert got[0] == R.resultant_y(a, b) and got[4] == R.resultant_y(b, a)


def test_general_path_above_register_classes(snc):
    rng = np.random.default_rng(11)
    f, g = rand_pair(rng, 70, 3, 1, 2, 12)
    check(snc, f, g)


def test_multilimb_and_mixed_widths(snc):
    rng = random.Random(9)
    f = [[rng.randrange(-(1 << 127), 1 << 127) for _ in range(3)] for _ in range(4)]
    g = [[rng.randrange(-99, 99) for _ in range(4)] for _ in range(3)]
    check(snc, f, g)
    f64 = synth.dense_bivariate(np.random.default_rng(1), 5, bits=64)
    check(snc, f64, g)


def test_config1_against_golden(snc):
    ref = json.load(open(os.path.join(GOLDEN, "config1.json")))
    f, g = synth.config1()
    r = snc.resultant_y(f, g)
    assert len(r) - 1 == ref["degree"]
    assert [c % Q61 for c in r] == ref["mod_2_61_minus_1"]
    assert hashlib.sha256(",".join(str(c) for c in r).encode()).hexdigest() == ref["sha256"]
    assert r[0] == R.resultant_at(f, g, 0)


def test_config3_sampled(snc):
    ref = json.load(open(os.path.join(GOLDEN, "config3.json")))
    f, g = synth.config3()
    r = snc.resultant_y(f, g)
    assert len(r) - 1 <= ref["degree_bound"]
    assert r[0] == int(ref["res_at_0"])
    top = r[ref["top_degree"]] if len(r) > ref["top_degree"] else 0
    assert top == int(ref["top_coefficient"])
    assert len(r) - 1 == ref["top_degree"]
    rng = random.Random(2024)
    for q in (Q61, (1 << 61) - 31):
        for _ in range(3):
            x0 = rng.randrange(q)
            assert zx.evaluate(r, x0) % q == R.resultant_at_mod(f, g, x0, q)


def test_largest_degree_bound(snc):
    """Total degrees 100 and 100: the degree bound 10000 is the largest the
    library accepts (interpolation buffers fill the LDS of a CU), y-degree
    100 takes the general elimination.  Checked on sampled values."""
    rng = np.random.default_rng(77)
    f = synth.dense_bivariate(rng, 100, bits=3)
    g = synth.dense_bivariate(rng, 100, bits=3)
    assert snc.resultant_plan(f, g).deg_bound == 10000
    r = snc.resultant_y(f, g)
    assert len(r) - 1 <= 10000
    rs = random.Random(5)
    for q in (Q61, (1 << 61) - 31):
        for x0 in (0, 1, 9999, rs.randrange(q)):
            assert zx.evaluate(r, x0) % q == R.resultant_at_mod(f, g, x0, q)


def test_batch_matches_plain_and_oracle(snc, assert_same):
    pairs, common = synth.config2(npairs=48, frac_common=0.1)
    batch = snc.resultant_y_batch(pairs)
    for i, (f, g) in enumerate(pairs):
        if i in common:
            assert batch[i] == []
    # plain path on a subset, oracle mod q on all pairs at one random point
    for i in range(0, len(pairs), 6):
        assert batch[i] == snc.resultant_y(*pairs[i])
    rng = random.Random(7)
    for i, (f, g) in enumerate(pairs):
        x0 = rng.randrange(Q61)
        assert zx.evaluate(batch[i], x0) % Q61 == R.resultant_at_mod(f, g, x0, Q61)
    # replaying the captured graph gives the same results
    b = snc.ResultantBatch(pairs)
    b.run()
    first = b.results()
    b.run()
    assert_same(first, batch)
    assert_same(b.results(), first)


def test_config2_full_draw(snc, assert_same):
    """The batched workload exactly as it is timed: all 512 pairs of the
    seeded draw in one prepared batch.  The 51 planted common-factor pairs
    are exactly 0 and no other pair is; every pair equals its plain run;
    every pair agrees with the oracle's determinant modulo a 61-bit prime at
    a random point; the three cheapest pairs equal the oracle's resultant
    coefficient by coefficient; the stage-by-stage run (timing on) gives the
    same results as the graph, and so do three more graph replays after it."""
    pairs, common = synth.config2()
    assert len(pairs) == 512 and len(common) == 51
    b = snc.ResultantBatch(pairs)
    b.run()
    got = b.results()
    for i in range(len(pairs)):
        assert (got[i] == []) == (i in common), i
    plain = snc.PlainResultants(pairs)
    plain.run()
    assert_same(plain.results(), got)
    rng = random.Random(512)
    for i, (f, g) in enumerate(pairs):
        x0 = rng.randrange(Q61)
        assert zx.evaluate(got[i], x0) % Q61 == R.resultant_at_mod(f, g, x0, Q61), i
    cost = sorted(range(len(pairs)), key=lambda i: (b.each[i].deg_bound + 1) * len(pairs[i][0]) ** 3)
    for i in cost[:3]:
        assert got[i] == R.resultant_y_by_points(*pairs[i], processes=1), i
    b.run()
    assert_same(b.results(), got)   # a second replay of the captured graph
    # with stage timing on, the same launches go to the stream one by one
    # between events instead of the captured graph: the same results
    b.ctx.set_timing(True)
    try:
        b.run()
        assert_same(b.results(), got)
    finally:
        b.ctx.set_timing(False)
    # the captured graph (its CRT classes on two branches) replayed again
    # after that eager work: the same results on every replay
    for _ in range(3):
        b.run()
        assert_same(b.results(), got)


@pytest.mark.parametrize("da,db", [(63, 20), (64, 32), (1000, 500), (1023, 300), (1024, 512)])
def test_interpolation_block_boundaries(snc, da, db):
    """res_y(y^2 - a, y - b) = b^2 - a exactly (f at the root y = b of the
    monic g).  The degree bounds 63/64 (one and two blocks of 64), 1000 and
    1023 (sixteen blocks, the last row of the falling-factorial table) take
    the block-parallel interpolation; 1024 takes the one-workgroup kernel.
    Plain calls and a batch replay agree with the exact value."""
    rng = random.Random(da)
    a = [rng.randrange(-(1 << 40), 1 << 40) for _ in range(da + 1)]
    a[-1] = a[-1] or 1
    b = [rng.randrange(-(1 << 20), 1 << 20) for _ in range(db + 1)]
    b[-1] = b[-1] or 1
    want = zx.sub(zx.mul(b, b), a)
    n = max(da, db) + 1
    f = [[-c for c in a] + [0] * (n - len(a)), [0] * n, [1] + [0] * (n - 1)]
    g = [[-c for c in b] + [0] * (n - len(b)), [1] + [0] * (n - 1)]
    assert snc.resultant_y(f, g) == want
    batch = snc.ResultantBatch([(f, g), (g, f)])
    for _ in range(2):
        batch.run()
        r_fg, r_gf = batch.results()
        assert r_fg == want and r_gf == want  # (-1)^(2*1) = 1


@pytest.mark.parametrize("d,bits,pair", [(10, 128, False), (10, 512, False), (6, 1024, False), (4, 2048, False),
                                         (9, 2048, False), (15, 2048, False), (15, 2048, True)])
def test_multilimb_curves(snc, d, bits, pair):
    """The paper's 128..2048-bit random curves: R = res_y(f, f_y) (or
    res_y(f, h) of two such curves) for dense f of total degree d with
    bits-bit coefficients, checked on sampled values mod two 61-bit primes
    against the oracle's determinant at the point, plus the degree bound and
    a batch replay.  Degree 15 at 2048 bits needs about 2000 primes."""
    rng = np.random.default_rng(bits + d)
    f, g = synth.bigcoef_curve(rng, d, bits)
    if pair:
        g, _ = synth.bigcoef_curve(rng, d, bits)
    plan = snc.resultant_plan(f, g)
    r = snc.resultant_y(f, g)
    assert len(r) - 1 <= plan.deg_bound
    rs = random.Random(bits)
    for q in (Q61, (1 << 61) - 31):
        for x0 in (0, 1, plan.deg_bound, rs.randrange(q)):
            assert zx.evaluate(r, x0) % q == R.resultant_at_mod(f, g, x0, q)
    batch = snc.ResultantBatch([(f, g)])
    for _ in range(2):
        batch.run()
        assert batch.results()[0] == r


def test_random_curve_set_batch(snc):
    """Projection phase of five random degree-9, 512-bit curves in one batch:
    each curve with its y-derivative and every pair; every result matches the
    single call and the oracle's determinant at sampled points."""
    pairs = synth.random_curve_set(np.random.default_rng(7), 9, 512)
    batch = snc.ResultantBatch(pairs)
    batch.run()
    got = batch.results()
    rs = random.Random(9)
    for (f, g), r in zip(pairs, got):
        assert r == snc.resultant_y(f, g)
        x0 = rs.randrange(Q61)
        assert zx.evaluate(r, x0) % Q61 == R.resultant_at_mod(f, g, x0, Q61)


def _class_spanning_pairs(seed):
    """Pairs whose larger y-degree falls in every register class from 16 to
    64, with ragged point tiles, small and multi-word coefficients and one
    planted common factor (resultant 0)."""
    rng = np.random.default_rng(seed)
    shapes = [(12, 10, 16, 20), (20, 17, 24, 12), (30, 26, 8, 32), (40, 36, 16, 16), (44, 46, 10, 12),
              (60, 58, 8, 8)]
    pairs = [synth.random_pair(rng, *sh) for sh in shapes]
    pairs.append(synth.common_factor_pair(rng, 38, 35, 12, 12))
    return pairs


def test_eval_variants_identical(snc, assert_same):
    """Every launch variant of the evaluation kernel the autotuner can pick
    (register budget for 1..4 wavefronts per SIMD; one workgroup per block
    or a persistent grid taking 1 or 4 blocks at a time) gives the same
    resultants; those equal the plain calls, and a pair checked against the
    oracle mod a 61-bit prime at a random point."""
    pairs = _class_spanning_pairs(8801)
    ctx = snc.Context(0)
    ctx.set_tuning(0)
    ref = snc.resultant_y_batch(pairs, ctx)
    assert ref[-1] == []
    assert all(r != [] for r in ref[:-1])
    for (f, g), r in zip(pairs[:3], ref):
        assert snc.resultant_y(f, g, ctx) == r
    rng = random.Random(8802)
    f, g = pairs[3]
    x0 = rng.randrange(Q61)
    assert zx.evaluate(ref[3], x0) % Q61 == R.resultant_at_mod(f, g, x0, Q61)
    for wpe in (1, 2, 3, 4):
        for chunk in (0, 1, 4):
            for cap in (16, 32, 40, 48, 64):
                ctx.set_eval_variant(cap, wpe, chunk)
            got = snc.resultant_y_batch(pairs, ctx)
            rep, _ = ctx.tuning()
            assert {e["source"] for e in rep} == {"forced"}
            assert all(e["wpe"] == wpe and e["chunk"] == chunk for e in rep)
            assert_same(got, ref, f"variant {(wpe, chunk)}")
    for cap in (16, 32, 40, 48, 64):
        ctx.set_eval_variant(cap, 0, 0)
    # the prepared graph of a persistent variant replayed several times
    for cap in (16, 32, 40, 48, 64):
        ctx.set_eval_variant(cap, 2, 1)
    b = snc.ResultantBatch(pairs, ctx)
    for _ in range(3):
        b.run()
        assert_same(b.results(), ref)
    b.close()
    for cap in (16, 32, 40, 48, 64):
        ctx.set_eval_variant(cap, 0, 0)


def test_autotuner_measures_and_caches(snc, assert_same):
    """The autotuner times every candidate of each class the batch uses,
    keeps one no slower than the default, and a later preparation of the
    same shape reuses it from its table; results are unchanged."""
    pairs = _class_spanning_pairs(8803)
    ctx = snc.Context(0)
    ctx.set_tuning(0)
    ref = snc.resultant_y_batch(pairs, ctx)
    ctx.set_tuning(2)
    b = snc.ResultantBatch(pairs, ctx)
    rep, tune_ms = ctx.tuning()
    assert tune_ms > 0.0
    assert {e["class"] for e in rep} == {16, 32, 40, 48, 64}
    for e in rep:
        assert e["source"] == "measured"
        assert e["candidates"] >= 4
        assert 0.0 < e["best_ms"] <= e["default_ms"] + 1e-6
        assert 1 <= e["wpe"] <= 4 and e["chunk"] in (0, 1, 4)
    b.run()
    assert_same(b.results(), ref)
    b.close()
    ctx.set_tuning(1)
    b2 = snc.ResultantBatch(pairs, ctx)
    rep2, _ = ctx.tuning()
    assert {e["source"] for e in rep2} == {"cached"}
    assert [(e["wpe"], e["chunk"]) for e in rep2] == [(e["wpe"], e["chunk"]) for e in rep]
    b2.run()
    assert_same(b2.results(), ref)
    b2.close()


def test_one_wavefront_interpolation_batch(snc, assert_same):
    """A batch with more than 4096 (pair, prime) instances and degree bounds
    below 4096 takes the one-wavefront interpolation (in place from the top
    block down); every result equals the single-pair call, which
    interpolates with the workgroup kernels.  Degree bounds 63 and 64 sit on
    the 64-point block boundary, 1600 is the largest."""
    rng = np.random.default_rng(8811)
    shapes = [(7, 9, 12, 12), (8, 8, 16, 16), (9, 7, 20, 8), (16, 8, 30, 30), (8, 16, 30, 30), (31, 33, 24, 24),
              (40, 40, 32, 32), (20, 25, 32, 32)]
    pairs = [synth.random_pair(rng, *sh) for sh in shapes]
    while sum(snc.resultant_plan(f, g).nprimes for f, g in pairs) < 4300:
        df, dg = int(rng.integers(8, 41)), int(rng.integers(8, 41))
        pairs.append(synth.random_pair(rng, df, dg, int(rng.integers(8, 33)), int(rng.integers(8, 33))))
    got = snc.resultant_y_batch(pairs)
    assert_same(got, [snc.resultant_y(f, g) for f, g in pairs])
    qr = random.Random(8812)
    f, g = pairs[6]
    x0 = qr.randrange(Q61)
    assert zx.evaluate(got[6], x0) % Q61 == R.resultant_at_mod(f, g, x0, Q61)


def test_pipelined_submit_collect(snc, assert_same):
    """snc_prepared_submit / _collect: every collected run equals a plain
    run of the prepared batch, with two runs outstanding, a third submit
    refused until one is collected, a prepared run between them, an unknown
    ticket refused, and a handle destroyed with a run outstanding."""
    pairs, common = synth.config2(npairs=48, frac_common=0.1)
    b = snc.ResultantBatch(pairs)
    b.run()
    ref = b.results()
    t0 = b.submit()
    t1 = b.submit()
    with pytest.raises(snc.SncError) as ei:
        b.submit()
    assert ei.value.status == snc.SNC_EAGAIN
    b.collect(t0)
    assert_same(b.results(), ref)
    t2 = b.submit()
    b.run()                      # the plain run between pipelined ones
    assert_same(b.results(), ref)
    b.collect(t1)
    assert_same(b.results(), ref)
    b.collect(t2)
    assert_same(b.results(), ref)
    with pytest.raises(snc.SncError) as ei:
        b.collect(t2)
    assert ei.value.status == snc.SNC_EINVAL
    assert [t0, t1, t2] == [0, 1, 2]
    for i in common:
        assert ref[i] == []
    # a staging buffer below snc_prepared_stage_bytes is refused before any work
    import ctypes
    need = snc.lib().snc_prepared_stage_bytes(b.h)
    assert need >= 2 * 4 * sum(len(r) for r in ref)
    t = ctypes.c_int64(-1)
    st = snc.lib().snc_prepared_submit(b.h, ctypes.c_void_p(b.stage.data_ptr()), ctypes.c_size_t(need - 1),
                                       b.ctx.stream_handle(None), ctypes.byref(t))
    assert st == snc.SNC_ENOMEM and t.value == -1
    t3 = b.submit()
    assert t3 == 3
    b.close()                    # waits for the outstanding download
