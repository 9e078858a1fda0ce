"""Pins for the oracle's sampled checker R(x0) mod q = det S(x0) mod q.

``resultant_at_mod`` and ``det_mod`` decide every large-size parity test
(the degree-64/48 pair, the 2048-bit curves, the batches, the largest degree
bound), so they are pinned here against values that do not come from the
oracle's own Sylvester construction:

* ``det_mod`` against the Leibniz expansion on integer matrices whose pivots
  vanish (the row-swap branch and its sign), and on singular matrices;
* ``resultant_at_mod`` against closed forms evaluated at the point: for
  f = c(x) y - a(x), res_y(f, g) = sum_j g_j(x) a(x)^j c(x)^(n-j); for
  f = c prod (y - a_i), g = e prod (y - b_j), res = c^n e^m prod (a_i - b_j);
  at points where a leading y-coefficient vanishes (formal degree kept, so
  elimination must swap rows) and where it does not;
* agreement with the exact determinant (``resultant_at``) and with the
  Z[x] Bareiss result evaluated at the point, for random pairs and a small
  prime where pivots vanish modulo q;
* planted mistakes in the oracle's code (the row-swap sign dropped, the
  operands' row blocks exchanged, coefficients in ascending order inside a
  row, the wrong evaluation point) each fail these pins.
"""
import inspect
import itertools
import textwrap

import numpy as np
import pytest

from oracle import resultant as R
from oracle import zx

Q61 = (1 << 61) - 1
QSMALL = 101  # pivots vanish modulo a small prime often


def leibniz_int(M) -> int:
    n = len(M)
    tot = 0
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        t = 1
        for i in range(n):
            t *= int(M[i][perm[i]])
            if t == 0:
                break
        tot += -t if inv % 2 else t
    return tot


def rand_zx(rng, deg, lo=-6, hi=6):
    c = [int(v) for v in rng.integers(lo, hi + 1, size=deg + 1)]
    if c[-1] == 0:
        c[-1] = 1
    return zx.trim(c)


def with_root(rng, x0, deg):
    """A polynomial of degree deg >= 1 that vanishes at x0: (x - x0) * r(x)."""
    return zx.mul([-x0, 1], rand_zx(rng, deg - 1))


def from_roots(c, roots):
    """c(x) prod (y - r(x)) as rows over Z[x]."""
    rows = [c]
    for r in roots:
        new = [[] for _ in range(len(rows) + 1)]
        for i, ri in enumerate(rows):
            new[i + 1] = zx.add(new[i + 1], ri)
            new[i] = zx.sub(new[i], zx.mul(r, ri))
        rows = new
    return rows


# ---------------------------------------------------------------------------
# Pin cases: (f, g, x0, q, expected) with expected from closed forms only
# ---------------------------------------------------------------------------

def closed_form_cases():
    rng = np.random.default_rng(31337)
    cases = []
    for t in range(12):
        x0 = int(rng.integers(-5, 6))
        q = Q61 if t % 3 else QSMALL
        n = int(rng.integers(1, 5))
        a = rand_zx(rng, int(rng.integers(0, 3)))
        # c vanishes at x0 in half the cases: the formal degree 1 is kept there
        c = with_root(rng, x0, 1 + t % 2) if t % 2 == 0 else rand_zx(rng, int(rng.integers(0, 2)))
        g = [rand_zx(rng, int(rng.integers(0, 3))) for _ in range(n + 1)]
        if t % 4 == 0:
            g[-1] = with_root(rng, x0, 1)  # g's leading coefficient vanishes there too
        f = [zx.neg(a), c]
        res = []
        for j, gj in enumerate(g):
            res = zx.add(res, zx.mul(gj, zx.mul(zx.power(a, j), zx.power(c, n - j))))
        cases.append((f, g, x0, q, zx.evaluate(res, x0) % q))
        # and with the operands exchanged: res(g, f) = (-1)^(1 n) res(f, g)
        cases.append((g, f, x0, q, (-1) ** n * zx.evaluate(res, x0) % q))
    for t in range(10):
        x0 = int(rng.integers(-4, 5))
        q = Q61 if t % 3 else QSMALL
        m, n = int(rng.integers(1, 4)), int(rng.integers(1, 4))
        c = with_root(rng, x0, 1) if t % 2 == 0 else rand_zx(rng, 1)
        e = with_root(rng, x0, 1) if t % 3 == 0 else rand_zx(rng, 1)
        A = [rand_zx(rng, int(rng.integers(0, 2)), -4, 4) for _ in range(m)]
        B = [rand_zx(rng, int(rng.integers(0, 2)), -4, 4) for _ in range(n)]
        res = zx.mul(zx.power(c, n), zx.power(e, m))
        for ai in A:
            for bj in B:
                res = zx.mul(res, zx.sub(ai, bj))
        cases.append((from_roots(c, A), from_roots(e, B), x0, q, zx.evaluate(res, x0) % q))
    return cases


CASES = closed_form_cases()


def det_cases():
    """Integer matrices with vanishing pivots, and their Leibniz determinants."""
    rng = np.random.default_rng(4242)
    out = []
    for t in range(30):
        n = int(rng.integers(2, 7))
        M = [[int(v) for v in rng.integers(-9, 10, size=n)] for _ in range(n)]
        # zero the leading column entries of the first rows: swaps at several steps
        z = int(rng.integers(1, n))
        for i in range(z):
            M[i][0] = 0
        if t % 3 == 0 and n >= 3:
            M[1][1] = 0
            M[0][1] = 0
        if t % 5 == 0:
            M[-1] = [2 * v for v in M[0]]  # singular
        q = Q61 if t % 2 else QSMALL
        out.append((M, q, leibniz_int(M) % q))
    # a permutation matrix with an odd permutation (one swap of rows 0 and 1)
    P = [[0, 1, 0], [1, 0, 0], [0, 0, 1]]
    out.append((P, Q61, Q61 - 1))
    return out


DETS = det_cases()


def all_pass(cases=CASES, dets=DETS) -> bool:
    ok = all(R.det_mod(M, q) == want for M, q, want in dets)
    return ok and all(R.resultant_at_mod(f, g, x0, q) == want for f, g, x0, q, want in cases)


# ---------------------------------------------------------------------------

def test_det_mod_against_leibniz_with_zero_pivots():
    assert any(M[0][0] == 0 for M, _, _ in DETS)
    for M, q, want in DETS:
        assert R.det_mod(M, q) == want


@pytest.mark.parametrize("idx", range(len(CASES)))
def test_resultant_at_mod_closed_forms(idx):
    f, g, x0, q, want = CASES[idx]
    assert R.resultant_at_mod(f, g, x0, q) == want


def test_closed_form_cases_need_row_swaps():
    """Some pin points make the leading y-coefficient vanish, so the first
    pivot of S(x0) is zero and the elimination must swap rows."""
    swaps = 0
    for f, g, x0, q, _ in CASES:
        S = R.sylvester_at(R.rows_of(f), R.rows_of(g), x0)
        swaps += S[0][0] % q == 0
    assert swaps >= 5


@pytest.mark.parametrize("seed", range(8))
def test_resultant_at_mod_matches_exact(seed):
    rng = np.random.default_rng(900 + seed)
    m, n = int(rng.integers(1, 6)), int(rng.integers(1, 6))
    f = [rand_zx(rng, int(rng.integers(0, 4)), -50, 50) for _ in range(m + 1)]
    g = [rand_zx(rng, int(rng.integers(0, 4)), -50, 50) for _ in range(n + 1)]
    x0 = int(rng.integers(-6, 7))
    if seed % 2:
        f[-1] = with_root(rng, x0, 2)  # lc_y(f)(x0) = 0
    r = R.resultant_y(f, g)
    for q in (Q61, QSMALL, 7):
        want = zx.evaluate(r, x0) % q
        assert R.resultant_at(f, g, x0) % q == want
        assert R.resultant_at_mod(f, g, x0, q) == want


# ---------------------------------------------------------------------------
# Planted mistakes in the oracle's code fail the pins
# ---------------------------------------------------------------------------

def _mutant(fn, old, new):
    """A copy of an oracle function with one source fragment replaced,
    compiled in the oracle module's namespace."""
    src = textwrap.dedent(inspect.getsource(fn))
    assert old in src, f"fragment {old!r} not in {fn.__name__}"
    ns = dict(vars(R))
    exec(compile(src.replace(old, new, 1), f"<mutant {fn.__name__}>", "exec"), ns)
    return ns[fn.__name__]


def test_dropped_swap_sign_is_caught(monkeypatch):
    monkeypatch.setattr(R, "det_mod", _mutant(R.det_mod, "det = -det", "det = det"))
    assert not all_pass()


def test_exchanged_row_blocks_are_caught(monkeypatch):
    orig = R.sylvester

    def blocks_exchanged(frows, grows):
        S = orig(frows, grows)
        n = R.ydeg(grows)
        return S[n:] + S[:n]
    monkeypatch.setattr(R, "sylvester", blocks_exchanged)
    assert not all_pass()


def test_ascending_row_order_is_caught(monkeypatch):
    monkeypatch.setattr(R, "sylvester", _mutant(R.sylvester, "frows[m - t]", "frows[t]"))
    assert not all_pass()


def test_wrong_point_is_caught(monkeypatch):
    monkeypatch.setattr(R, "resultant_at_mod",
                        _mutant(R.resultant_at_mod, "zx.evaluate(e, x0) % q", "zx.evaluate(e, x0 + 1) % q"))
    assert not all_pass()


def test_unmutated_oracle_passes():
    assert all_pass()
