"""CPU tests of the C ABI: the library loads and exports every function that
include/snc.h declares, and its host-only planning (prime table, degree and
coefficient bounds, workspace sizing, argument checks) agrees with the
oracle's bounds.  No device work is started here."""
import os
import re
import subprocess
from math import gcd

import numpy as np
import pytest

import synth
from oracle import resultant as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "snc.h")


@pytest.fixture(scope="module")
def snc():
    import paper_1103_4697_amd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_1103_4697_amd.build import build
        build()
    return m


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(snc_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(snc):
    names = declared_functions()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", snc.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (snc_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, f"declared but not exported: {missing}"
    lib = snc.lib()
    for n in names:
        assert getattr(lib, n) is not None


def test_status_strings_and_version(snc):
    lib = snc.lib()
    assert lib.snc_version() >= 100
    for st in range(-6, 1):
        assert lib.snc_status_str(st)


def is_prime(n):
    if n < 2:
        return False
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def test_prime_table(snc):
    ps = [snc.prime(i) for i in range(3072)]
    assert ps == sorted(ps, reverse=True) and len(set(ps)) == 3072
    assert all(2 ** 29 < p < 2 ** 30 for p in ps)
    assert all(is_prime(p) for p in ps[:64] + ps[-64:])
    # no prime of the range above the last one is skipped
    assert all(not is_prime(n) for n in range(ps[0] + 2, 2 ** 30, 2))
    assert snc.prime(-1) == 0 and snc.prime(3072) == 0


@pytest.mark.parametrize("which", ["c0", "c1", "c3", "small", "swapped", "big512", "big2048", "big2048d15"])
def test_resultant_plan_bounds(snc, which):
    rng = np.random.default_rng(1)
    if which.startswith("big"):  # norms far beyond the range of a double
        d = 15 if which.endswith("d15") else 6
        f, g = synth.bigcoef_curve(rng, d, int(which[3:7]))
    elif which == "c0":
        f, g = synth.config0()
    elif which == "c1":
        f, g = synth.config1()
    elif which == "c3":
        f, g = synth.config3()
    elif which == "small":
        f = synth.dense_bivariate(rng, 3, bits=40)
        g = synth.dense_bivariate(rng, 7, bits=10)
    else:
        f = synth.dense_bivariate(rng, 2, bits=12)
        g = synth.dense_bivariate(rng, 9, bits=12)
    p = snc.resultant_plan(f, g)
    assert p.deg_bound == R.degree_bound(f, g)
    B2 = R.coeff_bound_sq(f, g)
    M = 1
    for i in range(p.nprimes):
        M *= snc.prime(i)
    assert M * M > 4 * B2                       # prod p > 2B: balanced CRT recovers every coefficient
    M_prev = M // snc.prime(p.nprimes - 1)
    assert not (M_prev * M_prev * 10000 > 4 * B2 * 10001) or p.nprimes <= 2   # no prime is wasted
    assert (1 << (32 * p.out_nlimbs - 1)) ** 2 > B2  # two's complement limbs hold +-B
    assert p.workspace_bytes > 0


def test_trivial_and_invalid_plans(snc):
    p = snc.resultant_plan([[0]], [[1], [2]])
    assert p.nprimes == 0 and p.workspace_bytes == 0
    p = snc.resultant_plan([[3, 1]], [[2]])
    assert p.nprimes == 0
    import ctypes as C
    lib = snc.lib()
    assert lib.snc_resultant_y_plan(None, None, None) == snc.SNC_EINVAL
    bad = snc.Bipoly()
    bad.limbs, bad.dy, bad.dx, bad.nlimbs = None, 2, 2, 1
    ok = snc.Bipoly()
    ok.limbs, ok.dy, ok.dx, ok.nlimbs = None, -1, 0, 1
    pl = snc.Plan()
    assert lib.snc_resultant_y_plan(C.byref(bad), C.byref(ok), C.byref(pl)) == snc.SNC_EINVAL
    # degree bound above the supported maximum (total degrees 101 and 100)
    rng = np.random.default_rng(77)
    with pytest.raises(snc.SncError):
        snc.resultant_plan(synth.dense_bivariate(rng, 101, bits=3), synth.dense_bivariate(rng, 100, bits=3))
    # y-degree above the supported maximum
    big = np.zeros((300, 1), dtype=np.int64)
    big[299, 0] = 1
    with pytest.raises(snc.SncError):
        snc.resultant_plan(big, [[1], [1]])


def test_batch_plan_totals(snc):
    pairs, _ = synth.config2(npairs=16)
    import ctypes as C
    keep = []
    n = len(pairs)
    F = (snc.Bipoly * n)()
    G = (snc.Bipoly * n)()
    for i, (f, g) in enumerate(pairs):
        F[i] = snc._as_bipoly(f, keep)
        G[i] = snc._as_bipoly(g, keep)
    each = (snc.Plan * n)()
    total = snc.Plan()
    assert snc.lib().snc_resultant_y_batch_plan(n, F, G, each, C.byref(total)) == 0
    for i, (f, g) in enumerate(pairs):
        assert each[i].deg_bound == R.degree_bound(f, g)
    assert total.deg_bound == max(e.deg_bound for e in each)
    assert total.workspace_bytes >= max(snc.resultant_plan(f, g).workspace_bytes for f, g in pairs)


def test_gcd_plan(snc):
    import ctypes as C
    keep = []

    def plan(a, b):
        ua, ub = snc._as_upoly(a, keep), snc._as_upoly(b, keep)
        p = snc.Plan()
        st = snc.lib().snc_gcd_z_plan(C.byref(ua), C.byref(ub), C.byref(p))
        assert st == 0
        return p
    assert plan([], []).workspace_bytes == 0
    assert plan([3, 4], []).deg_bound == 1
    p = plan([1, 2, 3, 4], [5, 6, 7])
    assert p.deg_bound == 2 and p.nprimes > 0 and p.workspace_bytes > 0
    # Mignotte: the output limbs hold 2^deg * ||a||_2
    a = [(-1) ** i * (1 << 40) for i in range(30)]
    b = [7] * 25
    p = plan(a, b)
    norm = min(sum(c * c for c in a), sum(c * c for c in b)) ** 0.5
    assert 32 * p.out_nlimbs - 1 >= 24 + np.log2(norm)


def test_gcd_batch_plan(snc):
    """The batch plan covers every problem: per-problem plans equal the single
    plans, and the total workspace holds all of them (trivial ones need none)."""
    import ctypes as C
    keep = []
    rng = np.random.default_rng(3)
    pairs = [([1, 2, 3, 4], [5, 6, 7]), ([], [3]), ([0, 0, 5], [0, 2]),
             ([int(v) for v in rng.integers(-99, 99, 300)] + [1], [int(v) for v in rng.integers(-99, 99, 40)] + [7])]
    n = len(pairs)
    A = (snc.Upoly * n)()
    B = (snc.Upoly * n)()
    for i, (a, b) in enumerate(pairs):
        A[i] = snc._as_upoly(a, keep)
        B[i] = snc._as_upoly(b, keep)
    each = (snc.Plan * n)()
    total = snc.Plan()
    assert snc.lib().snc_gcd_z_batch_plan(n, A, B, each, C.byref(total)) == 0
    ws_sum = 0
    for i in range(n):
        one = snc.Plan()
        assert snc.lib().snc_gcd_z_plan(C.byref(A[i]), C.byref(B[i]), C.byref(one)) == 0
        assert (each[i].deg_bound, each[i].out_nlimbs, each[i].nprimes) == (one.deg_bound, one.out_nlimbs, one.nprimes)
        ws_sum += one.workspace_bytes
    assert each[1].workspace_bytes == 0
    assert max(e.workspace_bytes for e in each) <= total.workspace_bytes <= ws_sum
    assert snc.lib().snc_gcd_z_batch_plan(0, None, None, None, C.byref(total)) == 0
    assert total.workspace_bytes == 0
    assert snc.lib().snc_gcd_z_batch_plan(-1, None, None, None, C.byref(total)) == snc.SNC_EINVAL


def test_gcd_degree_limit(snc):
    """Degrees above the supported maximum (13000) are refused at planning."""
    import ctypes as C
    keep = []
    ua = snc._as_upoly([1] * 13002, keep)       # degree 13001
    ub = snc._as_upoly([1, 1], keep)
    p = snc.Plan()
    assert snc.lib().snc_gcd_z_plan(C.byref(ua), C.byref(ub), C.byref(p)) == snc.SNC_EINVAL
    ua = snc._as_upoly([1] * 13001, keep)       # degree 13000
    assert snc.lib().snc_gcd_z_plan(C.byref(ua), C.byref(ub), C.byref(p)) == 0


def test_content_plan(snc):
    """Planning the content in y needs no device: the degree bound is the
    least row degree, and the zero polynomial needs nothing."""
    import ctypes as C
    keep = []
    p = snc.Plan()
    f = [[1, 2, 3], [0], [5, 0, 0, 0, 7], [2, 1]]
    assert snc.lib().snc_content_y_plan(C.byref(snc._as_bipoly(f, keep)), C.byref(p)) == snc.SNC_OK
    assert p.deg_bound == 1 and p.out_nlimbs >= 1 and p.workspace_bytes > 0
    assert snc.lib().snc_content_y_plan(C.byref(snc._as_bipoly([[0]], keep)), C.byref(p)) == snc.SNC_OK
    assert p.deg_bound == 0 and p.workspace_bytes == 0
    assert snc.lib().snc_content_y_plan(None, C.byref(p)) == snc.SNC_EINVAL
