"""GPU parity of gcd(a, b) in Z[x] through the C ABI against the CPU oracle
(Euclid over Q where it is fast enough, the oracle's certificate at larger
sizes).  Results are exact integers compared bit for bit."""
import json
import os
import random
from math import gcd as igcd

import numpy as np
import pytest

import synth
from oracle import gcd as G
from oracle import resultant as R
from oracle import zx

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
Q61 = (1 << 61) - 1


@pytest.fixture(scope="module")
def snc():
    import paper_1103_4697_amd as m
    return m


def rpoly(rng, deg, bits):
    lim = 1 << (bits - 1)
    c = [rng.randrange(-lim, lim) for _ in range(deg + 1)]
    if c[-1] == 0:
        c[-1] = 1
    return c


def test_golden(snc):
    data = json.load(open(os.path.join(GOLDEN, "worked_examples.json")))
    for ex in data["gcds"]:
        assert snc.gcd_z(ex["a"], ex["b"]) == ex["gcd"], ex["name"]


@pytest.mark.parametrize("seed", range(10))
def test_by_construction_vs_euclid(snc, seed):
    rng = random.Random(100 + seed)
    h = rpoly(rng, rng.randint(0, 8), rng.choice([4, 16, 40]))
    u = rpoly(rng, rng.randint(0, 30), rng.choice([8, 32, 70]))
    v = rpoly(rng, rng.randint(0, 30), rng.choice([8, 32, 70]))
    if seed % 3 == 0:
        u = zx.scale(u, 6)
        v = zx.scale(v, 10)
    a, b = synth.univariate_product(h, u), synth.univariate_product(h, v)
    got = snc.gcd_z(a, b)
    assert got == G.gcd_zx(a, b)


def test_special_cases(snc):
    assert snc.gcd_z([], []) == []
    assert snc.gcd_z([0, -2, -4], []) == [0, 2, 4]
    assert snc.gcd_z([], [-7]) == [7]
    assert snc.gcd_z([12], [0, 18, 6]) == [6]
    assert snc.gcd_z([4, 0, 2], [-6]) == [2]
    assert snc.gcd_z([1, 1], [1, 1]) == [1, 1]
    assert snc.gcd_z([-3, -3], [6, 6]) == [3, 3]


def test_unlucky_prime_and_lc_divisible(snc):
    p0 = snc.prime(0)
    rng = random.Random(5)
    u = rpoly(rng, 12, 20)
    v = rpoly(rng, 9, 20)
    lin = [1, 1]
    # b = v (x+1) + p0 x^3: coprime to a = u (x+1) over Q, common factor mod p0
    a = synth.univariate_product(u, lin)
    b = zx.add(synth.univariate_product(v, lin), [0, 0, 0, p0])
    assert snc.gcd_z(a, b) == G.gcd_zx(a, b)
    # same with a shared factor h: the gcd is h, prime p0 sees h (x+1)
    h = rpoly(rng, 4, 16)
    a2 = synth.univariate_product(h, a)
    b2 = synth.univariate_product(h, b)
    assert snc.gcd_z(a2, b2) == G.gcd_zx(a2, b2)
    # leading coefficients divisible by p0 (p0 divides beta: that prime is skipped)
    a3 = synth.univariate_product(h, u[:-1] + [p0 * 3])
    b3 = synth.univariate_product(h, v[:-1] + [p0 * 5])
    assert snc.gcd_z(a3, b3) == G.gcd_zx(a3, b3)


def test_resultant_squarefree_config0(snc):
    f, g = synth.config0()
    r = snc.resultant_y(f, g)
    rp = zx.deriv(r)
    assert snc.gcd_z(r, rp) == G.gcd_zx(r, rp)


def test_config1_squarefree_against_golden(snc):
    ref = json.load(open(os.path.join(GOLDEN, "config1.json")))
    f, g = synth.config1()
    r = snc.resultant_y(f, g)
    gg = snc.gcd_z(r, zx.deriv(r))
    assert gg == [int(c) for c in ref["gcd_r_rprime"]]


@pytest.mark.parametrize("target,dh", [(300, 12), (1200, 40)])
def test_serving_shape_certified(snc, target, dh):
    rng = np.random.default_rng(target)
    a, b, h = synth.gcd_request(rng, target, target, dh, dh, 8, 32)
    got = snc.gcd_z(a, b)
    assert zx.deg(got) >= dh
    assert G.certify_gcd(a, b, got)


def test_gcd_with_derivative_against_oracle(snc):
    """gcd(a, a') with a' formed in the library: polynomials with repeated
    factors (a = h^2 u, a = h^3), square-free ones, contents, negative leading
    coefficients; equal to the oracle and to gcd(a, a') through snc_gcd_z."""
    rng = random.Random(31)
    cases = []
    for _ in range(6):
        h = rpoly(rng, rng.randint(1, 6), 8)
        u = rpoly(rng, rng.randint(0, 30), 12)
        cases.append(zx.mul(zx.mul(h, h), u))
        cases.append(zx.mul(zx.mul(h, h), h))
        cases.append([c * 6 for c in rpoly(rng, rng.randint(1, 40), 20)])
        cases.append([-c for c in rpoly(rng, rng.randint(1, 25), 70)])
    for a in cases:
        ref = G.gcd_zx(a, zx.deriv(a))
        assert snc.gcd_z_deriv(a) == ref
        assert snc.gcd_z(a, zx.deriv(a)) == ref


def test_gcd_with_derivative_edge_cases(snc):
    assert snc.gcd_z_deriv([]) == []
    assert snc.gcd_z_deriv([-7]) == [7]          # gcd(-7, 0)
    assert snc.gcd_z_deriv([4, 6]) == [2]        # gcd(6x + 4, 6)
    assert snc.gcd_z_deriv([1, 2, 1]) == [1, 1]  # (x + 1)^2
    assert snc.gcd_z_deriv([0, 0, 0, 5]) == [0, 0, 5]  # gcd(5x^3, 15x^2) = 5x^2


def test_gcd_with_derivative_of_curve_resultant(snc):
    """The projection step: gcd(R, R') of R = res_y(f, f_y) on the curve-analysis
    workload, from limbs, against the stored oracle value."""
    ref = json.load(open(os.path.join(GOLDEN, "config1.json")))
    f, g = synth.config1()
    r = snc.resultant_y(f, g)
    limbs = snc.ints_to_limbs(r, max(1, max(c.bit_length() for c in r) // 32 + 2))
    got = snc.limbs_to_ints(snc.gcd_z_deriv_limbs(limbs))
    assert got == [int(c) for c in ref["gcd_r_rprime"]]


def test_batch_equals_single_and_oracle(snc):
    """snc_gcd_z_batch on a mix: shared factors of several degrees (register
    classes 2..9 and degrees above 64 E), square-free pairs, contents,
    derivative pairs, trivial entries and a repeated problem; every result
    equals the single call and the oracle (Euclid over Q where fast, else
    the divisibility certificate)."""
    rng = random.Random(77)
    pairs = []
    for deg_h, deg_u in ((3, 20), (12, 60), (30, 200), (8, 500), (2, 2), (40, 40)):
        h = rpoly(rng, deg_h, 10)
        pairs.append((zx.mul(h, rpoly(rng, deg_u, 12)), zx.mul(h, rpoly(rng, deg_u + 3, 12))))
    pairs.append(([c * 4 for c in rpoly(rng, 30, 20)], [c * 6 for c in rpoly(rng, 25, 20)]))
    a = zx.mul(zx.mul([1, 1], [1, 1]), rpoly(rng, 15, 8))
    pairs.append((a, zx.deriv(a)))
    pairs += [([], []), ([5], []), ([0, 3], [6]), pairs[0]]
    got = snc.gcd_z_batch(pairs)
    assert len(got) == len(pairs)
    for (a, b), g in zip(pairs, got):
        assert g == snc.gcd_z(a, b)
        if max(len(a), len(b)) <= 80:
            assert g == G.gcd_zx(a, b)
        assert G.certify_gcd(a, b, g)   # divides both, content, coprime cofactors
    assert got[-1] == got[0]
    assert snc.gcd_z_batch([]) == []


def test_batch_output_too_small(snc):
    """SNC_ERANGE: the entries that are too small receive the sizes they need."""
    import ctypes as C
    keep = []
    pairs = [([1, 2, 1], [1, 1]), ([3, 0, 0, 1], [2, 5])]
    n = len(pairs)
    A = (snc.Upoly * n)()
    B = (snc.Upoly * n)()
    for i, (a, b) in enumerate(pairs):
        A[i] = snc._as_upoly(a, keep)
        B[i] = snc._as_upoly(b, keep)
    each = (snc.Plan * n)()
    total = snc.Plan()
    assert snc.lib().snc_gcd_z_batch_plan(n, A, B, each, C.byref(total)) == 0
    out = (snc.Upoly * n)()
    bufs = []
    for i in range(n):
        u, buf = snc._out_upoly(each[i].deg_bound, each[i].out_nlimbs, keep)
        out[i] = u
        bufs.append(buf)
    out[0].deg = -1  # too small on purpose (host-side check, no device work started)
    ctx = snc.default_context()
    ws = ctx.workspace(total.workspace_bytes)
    st = snc.lib().snc_gcd_z_batch(ctx.h, n, A, B, C.c_void_p(ws.data_ptr()), C.c_size_t(ws.numel()),
                                   ctx.stream_handle(), out)
    assert st == snc.SNC_ERANGE
    assert out[0].deg == each[0].deg_bound and out[0].nlimbs >= 1


def _sq_pair(a, b):
    """f = y - a(x), g = y - b(x): res_y(f, g) = a(x) - b(x) (formal degrees 1, 1)."""
    n = max(len(a), len(b))
    return ([[-c for c in a] + [0] * (n - len(a)), [1] + [0] * (n - 1)],
            [[-c for c in b] + [0] * (n - len(b)), [1] + [0] * (n - 1)])


def test_resultant_with_sqfree_gcd(snc):
    """One pass for R = res_y(f, g) and gcd(R, R'): the fused check on the
    resultant's primes (square-free R), the full gcd when R has a repeated
    root, zero and constant resultants, and random pairs; R equal to the plain
    run and G to the oracle."""
    rng = random.Random(5)
    pairs = []
    for _ in range(4):
        f = synth.dense_bivariate(np.random.default_rng(rng.randrange(1 << 30)), rng.randint(2, 6), bits=10)
        g = synth.dense_bivariate(np.random.default_rng(rng.randrange(1 << 30)), rng.randint(2, 6), bits=10)
        pairs.append((f, g))
    d = zx.mul(zx.mul([-1, 1], [-1, 1]), [2, 1])            # (x - 1)^2 (x + 2): a repeated root
    pairs.append(_sq_pair(zx.add([3, 0, 5], [c * 7 for c in d]), [3, 0, 5]))
    h = [[1, 2], [3], [1]]                                     # common factor in y: R = 0
    pairs.append((synth.bivariate_product(h, [[1, 1], [1]]), synth.bivariate_product(h, [[2], [1]])))
    pairs.append(([[5]], [[7]]))                               # constants in y: R = 1
    pairs.append(_sq_pair([4, 0, 0, 1], [4]))                  # R = -x^3 (a triple root at 0)
    # contents: R scaled by 3^3 (one-word running gcd reduced from the limbs),
    # and by 6^6 10^6 > 2^32 (a two-word content)
    rg = np.random.default_rng(11)
    pairs.append((3 * synth.dense_bivariate(rg, 4, bits=10), synth.dense_bivariate(rg, 3, bits=10)))
    pairs.append((6 * synth.dense_bivariate(rg, 6, bits=8), 10 * synth.dense_bivariate(rg, 6, bits=8)))
    batch = snc.ResultantBatch(pairs)
    for _ in range(2):                                         # graph capture, then replay
        batch.run_sqfree()
        R_all = batch.results()
        G_all = batch.sqfree_results()
        for (f, g), r, gg in zip(pairs, R_all, G_all):
            assert r == snc.resultant_y(f, g)
            assert gg == G.gcd_zx(r, zx.deriv(r))
    assert R_all[5] == [] and G_all[5] == []


def test_resultant_with_sqfree_gcd_curve_workload(snc):
    ref = json.load(open(os.path.join(GOLDEN, "config1.json")))
    f, g = synth.config1()
    batch = snc.ResultantBatch([(f, g)])
    batch.run_sqfree()
    r = batch.results()[0]
    assert len(r) - 1 == ref["degree"]
    assert [c % Q61 for c in r] == ref["mod_2_61_minus_1"]
    assert batch.sqfree_results()[0] == [int(c) for c in ref["gcd_r_rprime"]]


def _gcd_mod_p(a, b, p):
    """Monic gcd of two integer polynomials (coefficient lists, constant
    first) reduced mod p, by the plain Euclidean algorithm."""
    def trim(v):
        v = [c % p for c in v]
        while v and v[-1] == 0:
            v.pop()
        return v
    a, b = trim(a), trim(b)
    while b:
        inv = pow(b[-1], p - 2, p)
        while len(a) >= len(b):
            q = a[-1] * inv % p
            s = len(a) - len(b)
            for i, c in enumerate(b):
                a[s + i] = (a[s + i] - q * c) % p
            a = trim(a)
        a, b = b, a
    inv = pow(a[-1], p - 2, p)
    return [c * inv % p for c in a]


def test_sqfree_check_large_degree(snc):
    """The fused check at degree 420 and above: R = w (square-free,
    primitive), 6 w (content 6), u^2 w (repeated factor u) for a random w of
    degree 420: gcd(R, R') is 1, 6 and u by construction once w is square-free
    and coprime to u, which is checked mod a prime.  The fast path must settle
    the two square-free cases (no full gcd), and the gcds must equal the plain
    modular gcd of R and R'."""
    rng = random.Random(23)
    p = 1000003
    u = [-7, 3, 1]
    while True:
        w = [rng.randint(-60, 60) for _ in range(420)] + [1]
        if _gcd_mod_p(w, zx.deriv(w), p) == [1] and _gcd_mod_p(w, u, p) == [1]:
            break
    cases = [(w, [1]), ([6 * c for c in w], [6]), (zx.mul(zx.mul(u, u), w), u)]
    pairs = [_sq_pair(r, [0]) for r, _ in cases]
    batch = snc.ResultantBatch(pairs)
    ctx = batch.ctx
    ctx.set_timing(True)
    try:
        batch.run_sqfree()
        stages = {name: launches for name, _, launches in ctx.timing()}
    finally:
        ctx.set_timing(False)
    R_all, G_all = batch.results(), batch.sqfree_results()
    for (r, g), (f2, g2), rr, gg in zip(cases, pairs, R_all, G_all):
        # res_y(y - r, y - 0) = r exactly (closed form; the oracle agrees at a point)
        assert R.resultant_at(f2, g2, 3) == zx.evaluate(r, 3)
        assert rr == r
        assert gg == g
        assert gg == snc.gcd_z_deriv(rr)
    assert stages["sqfree_full_gcd"] == 1          # only u^2 w needs the full gcd
    assert stages["sqfree_euclid"] > 0              # (pair, prime) items of the fused check
    batch.run_sqfree()                             # replay of the captured pipeline
    assert batch.sqfree_results() == G_all   # short lists of small polynomials


def test_sqfree_factor_against_oracle(snc):
    """snc_sqfree (Yun's algorithm on the modular gcd with lifted cofactors)
    against the oracle's repeated-gcd factorisation: random products of
    powers with contents and signs, special cases, and the projection
    resultant of the small curve workload."""
    rng = random.Random(41)
    cases = [[], [7], [-12], [0, 1], [-2, 2], [0, 0, 0, 5], zx.power([1, 1], 5),
             zx.mul([0, -3], zx.power([1, 0, 1], 2))]
    for _ in range(10):
        a = [rng.choice([1, -1, 6, -10])]
        for _ in range(rng.randint(1, 4)):
            a = zx.mul(a, zx.power(rpoly(rng, rng.randint(1, 6), 12), rng.randint(1, 4)))
        cases.append(a)
    for a in cases:
        assert snc.sqfree_factor(a) == G.sqfree_zx(a), a[:4]
    # the small curve workload's resultant against the oracle; its square and
    # (x + 3)^3 r by construction from that (the oracle's gcds over Q are slow there)
    f, g = synth.config0()
    r = snc.resultant_y(f, g)
    c, fr = G.sqfree_zx(r)
    assert snc.sqfree_factor(r) == (c, fr)
    assert snc.sqfree_factor(zx.mul(r, r)) == (c * c, [(h, 2 * m) for h, m in fr])
    if all(zx.evaluate(h, -3) != 0 for h, _ in fr) and all(m != 3 for _, m in fr):
        want = sorted(fr + [([3, 1], 3)], key=lambda t: t[1])
        assert snc.sqfree_factor(zx.mul(zx.power([3, 1], 3), r)) == (c, want)


def test_sqfree_factor_large_by_construction(snc):
    """a = -6 f1 f2^2 f3^3 with f1, f2, f3 of degrees 120, 60, 30 (total degree
    330): the factorisation is known once the f_i are square-free and
    pairwise coprime, which is checked mod a prime."""
    rng = random.Random(57)
    p = 1000003
    fs = []
    for d in (120, 60, 30):
        while True:
            f = [rng.randint(-40, 40) for _ in range(d)] + [1]
            if igcd(*f) != 1:
                continue
            if _gcd_mod_p(f, zx.deriv(f), p) != [1] or any(_gcd_mod_p(f, h, p) != [1] for h in fs):
                continue
            fs.append(f)
            break
    a = [-6]
    for i, f in enumerate(fs):
        a = zx.mul(a, zx.power(f, i + 1))
    c, got = snc.sqfree_factor(a)
    assert c == -6
    assert got == [(fs[0], 1), (fs[1], 2), (fs[2], 3)]


def _content_cases():
    rng = np.random.default_rng(31)
    pr = random.Random(31)
    cases = []
    # random dense curves: content 1
    for d, bits in [(9, 10), (12, 128), (6, 512)]:
        f, _ = synth.bigcoef_curve(rng, d, bits)
        cases.append((f"random_d{d}_b{bits}", f))
    # a non-trivial content h times a curve, with an odd number of rows
    h = [pr.randrange(-50, 50) for _ in range(4)] + [3]
    g, _ = synth.bigcoef_curve(rng, 6, 16)
    cases.append(("h_times_curve", [zx.mul(h, [int(c) for c in row]) for row in g]))
    # integer content only; a zero row in between; rows of mixed degree
    cases.append(("integer", [[6, 12, 18], [0], [30, -6], [12]]))
    # one non-zero row (negative leading coefficient)
    cases.append(("one_row", [[0], [5, -3, 0, -7]]))
    # the content of a product curve (x^2 + 1)^2 (y^2 - x) at 300 bits
    big = (1 << 300) + 12345
    h2 = zx.scale(zx.mul([1, 0, 1], [1, 0, 1]), big)
    cases.append(("big_content", [zx.scale(h2, -1), [0], [int(c) for c in h2]]))
    return cases


@pytest.mark.parametrize("name,f", _content_cases(), ids=[c[0] for c in _content_cases()])
def test_content_y(snc, name, f):
    """Content in y on the device (a tree of batched row gcds) against the
    oracle's fold of exact gcds; the content divides every row."""
    got = snc.content_y(f)
    want = G.content_y(f)
    assert got == want
    for row in f:
        if any(int(c) for c in row):
            assert zx.divides(got, [int(c) for c in row])


def test_content_y_zero(snc):
    assert snc.content_y([[0, 0], [0]]) == []


def _fastlift_cases():
    rng = np.random.default_rng(41)
    cases = []
    for d, bits in [(4, 8), (6, 16), (7, 6), (5, 128)]:  # the oracle's gcd (pseudo-remainders) limits the degree
        f, _ = synth.bigcoef_curve(rng, d, bits)
        cases.append((f"random_d{d}_b{bits}", [[int(c) for c in row] for row in f]))
    # f = 5 + x^2 C(x, y): f_x and f_y share x
    C, _ = synth.bigcoef_curve(rng, 4, 6)
    rows = [zx.mul([0, 0, 1], [int(c) for c in r]) for r in C]
    rows[0] = zx.add(rows[0], [5])
    cases.append(("shared_x", rows))
    # every coefficient of f_x and f_y even: h = 2
    f, _ = synth.bigcoef_curve(rng, 5, 8)
    cases.append(("even", [[2 * int(c) for c in row] for row in f]))
    return cases


@pytest.mark.parametrize("name,f", _fastlift_cases(), ids=[c[0] for c in _fastlift_cases()])
def test_fastlift_q(snc, name, f):
    """Q = res_y(f_x / h, f_y / h) on the device against the oracle (its own
    bivariate gcd by pseudo-remainders and Bareiss over Z[x])."""
    from oracle import fastlift as FL
    want, h = FL.fastlift_q(f)
    assert len(h) == 1  # these inputs have h constant in y
    assert snc.fastlift_q(f) == want


def _fastlift_y_cases():
    """Curves whose f_x and f_y share a factor that depends on y."""
    rng = np.random.default_rng(43)
    cases = [("square_y_minus_x", [[0, 0, 1], [0, -2, 1], [1, -2], [1]])]  # (y - x)^2 (y + 1)

    def bi(rows):
        return [[int(c) for c in r] for r in rows]

    g = [[1, -2], [3]]                       # 3y - 2x + 1
    k = bi(synth.dense_bivariate(rng, 2, bits=5))
    cases.append(("square_times_random", bi(synth.bivariate_product(synth.bivariate_product(g, g), k))))
    g3 = [[0, 1], [2], [1]]                  # y^2 + 2y + x
    cases.append(("cube", bi(synth.bivariate_product(synth.bivariate_product(g3, g3), g3))))
    # x^2 (y - x^2)^2 (y^2 + 5): the shared factor carries a content in x
    a = [[0, 0, -1], [1]]
    f = synth.bivariate_product(synth.bivariate_product(a, a), [[5], [0], [1]])
    cases.append(("content_and_square", bi([zx.mul([0, 0, 1], [int(c) for c in r]) for r in f])))
    # a 40-bit square factor times a random cubic
    g4 = [[int(c) for c in synth.uniform_signed(rng, (3,), 40)], [int(c) for c in synth.uniform_signed(rng, (2,), 40)],
          [1]]
    k4 = bi(synth.dense_bivariate(rng, 3, bits=8))
    cases.append(("square_40bit", bi(synth.bivariate_product(synth.bivariate_product(g4, g4), k4))))
    return cases


@pytest.mark.parametrize("name,f", _fastlift_y_cases(), ids=[c[0] for c in _fastlift_y_cases()])
def test_fastlift_q_y_factor(snc, name, f):
    """h = gcd(f_x, f_y) depending on y: the library's bivariate modular gcd
    (images per (prime, point) on the device, interpolation and Chinese
    remaindering, exact division) gives the oracle's Q."""
    from oracle import fastlift as FL
    want, h = FL.fastlift_q(f)
    assert len(h) > 1  # h depends on y
    assert snc.fastlift_q(f) == want


def test_blocked_euclid_matches_one_wavefront(snc, assert_same):
    """The square-free check's Euclid as a workgroup per (pair, prime) (blocks
    of up to 31 normal steps decided from the top 64 coefficients, each
    block's 2x2 polynomial matrix applied to the full remainders) against one
    wavefront per (pair, prime): identical d = deg R mod p and e = deg gcd(R,
    R') mod p for every prime, in the four register classes it serves
    (resultant degrees 300, 552, 700, 1000), for square-free resultants,
    repeated factors of degree 20 and 100 (the zero remainder arrives inside a
    block), a leading coefficient divisible by the first prime, and x^552 + 5
    (the first remainder is a constant); e and d equal the oracle's on sampled
    primes, and the gcds agree."""
    rng = random.Random(31)

    def rand_poly(n, bits=24):
        return [rng.randint(-(1 << bits), 1 << bits) for _ in range(n)] + [rng.choice((-1, 1)) * rng.randint(1, 99)]

    cases = [rand_poly(d) for d in (300, 552, 700, 1000)]
    u20, u100 = rand_poly(20, 8), rand_poly(100, 8)
    cases.append(zx.mul(zx.mul(u20, u20), rand_poly(512, 8)))
    cases.append(zx.mul(zx.mul(u100, u100), rand_poly(350, 8)))
    lead_div = rand_poly(552)
    lead_div[-1] = snc.prime(0) * 3
    cases.append(lead_div)
    cases.append([5] + [0] * 551 + [1])
    pairs = [_sq_pair(r, [0]) for r in cases]
    batch = snc.ResultantBatch(pairs)
    ctx = batch.ctx
    got = {}
    try:
        for v in (1, 2):
            ctx.set_gcd_variant(v)
            batch.run_sqfree()
            got[v] = ([batch.sqfree_degrees(i) for i in range(len(pairs))], batch.sqfree_results())
    finally:
        ctx.set_gcd_variant(0)
    assert_same(got[2][0], got[1][0], "per-prime (d, e)")
    assert_same(got[2][1], got[1][1], "gcds")
    for i, r in enumerate(cases):
        d, e = got[2][0][i]
        assert len(d) == len(e) > 0
        for q in sorted(set(rng.sample(range(len(e)), min(3, len(e))) + [0])):
            p = snc.prime(q)
            rp = zx.trim([c % p for c in r])
            assert d[q] == len(rp) - 1, (i, q)
            assert e[q] == G._gcd_mod_degree(r, zx.deriv(r), p), (i, q)
    assert max(got[2][0][4][1]) == 20 and max(got[2][0][5][1]) == 100
    assert got[2][0][6][0][0] == 551      # the leading coefficient vanishes mod the first prime
