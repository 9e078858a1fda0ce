"""Pins for the resultant oracle: it is checked against facts fixed by the
mathematics, not against itself.

* hand-derived worked examples (tests/golden/worked_examples.json);
* closed form res_y(y - a(x), g) = g(x, a(x));
* product form: f = c prod (y - a_i), g = e prod (y - b_j) gives
  c^n e^m prod (a_i - b_j);
* Leibniz expansion over all permutations for N <= 7;
* quadratic discriminant: res_y(A y^2 + B y + C, 2Ay + B) = -A (B^2 - 4AC);
* invariants: antisymmetry, multiplicativity, scaling, y-translation,
  common factor -> 0, degree and coefficient bounds;
* top coefficient from the top homogeneous forms;
* sympy's resultant where its sign convention agrees (deg_y f >= deg_y g).
"""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import resultant as R
from oracle import zx

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


def rand_zx(rng, deg, lo=-9, hi=9):
    c = [int(v) for v in rng.integers(lo, hi + 1, size=deg + 1)]
    if c[-1] == 0:
        c[-1] = 1
    return zx.trim(c)


def rand_rows(rng, m, xdeg, lo=-9, hi=9):
    rows = [zx.trim([int(v) for v in rng.integers(lo, hi + 1, size=xdeg + 1)]) for _ in range(m + 1)]
    if not rows[-1]:
        rows[-1] = [1]
    return rows


def poly_y_from_roots(c, roots):
    """c(x) * prod (y - r(x)) as rows over Z[x]."""
    rows = [c]
    for r in roots:
        # multiply by (y - r): new_i = old_{i-1} - r * old_i
        new = [[] for _ in range(len(rows) + 1)]
        for i, ri in enumerate(rows):
            new[i + 1] = zx.add(new[i + 1], ri)
            new[i] = zx.sub(new[i], zx.mul(r, ri))
        rows = new
    return rows


def subst_y(rows, a):
    """g(x, a(x))."""
    acc = []
    for r in reversed(rows):
        acc = zx.add(zx.mul(acc, a), r)
    return acc


def leibniz_det(M):
    n = len(M)
    total = []
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        term = [1]
        for i in range(n):
            term = zx.mul(term, M[i][perm[i]])
            if not term:
                break
        if term:
            total = zx.add(total, zx.neg(term) if inv % 2 else term)
    return total


# ---------------------------------------------------------------------------

def test_golden_worked_examples():
    data = json.load(open(GOLDEN))
    for ex in data["resultants"]:
        got = R.resultant_y(ex["f"], ex["g"])
        assert got == ex["res"], ex["name"]
        assert R.resultant_y_by_points(ex["f"], ex["g"]) == ex["res"], ex["name"]


@pytest.mark.parametrize("seed", range(6))
def test_closed_form_linear_in_y(seed):
    rng = np.random.default_rng(seed)
    a = rand_zx(rng, int(rng.integers(0, 4)))
    n = int(rng.integers(1, 6))
    g = rand_rows(rng, n, int(rng.integers(0, 4)))
    f = [zx.neg(a), [1]]
    expect = subst_y(g, a)
    assert R.resultant_y(f, g) == expect
    assert R.resultant_y_by_points(f, g) == expect
    # with a non-monic linear factor c(x) y - a(x): res = sum g_j a^j c^(n-j)
    c = rand_zx(rng, int(rng.integers(0, 3)))
    f2 = [zx.neg(a), c]
    expect2 = []
    for j, gj in enumerate(g):
        expect2 = zx.add(expect2, zx.mul(gj, zx.mul(zx.power(a, j), zx.power(c, n - j))))
    assert R.resultant_y(f2, g) == expect2


@pytest.mark.parametrize("m,n,use_points", [(1, 1, False), (2, 3, False), (3, 2, False),
                                            (4, 4, False), (5, 3, False), (8, 7, True)])
def test_product_form(m, n, use_points):
    rng = np.random.default_rng(100 + 10 * m + n)
    c = rand_zx(rng, 1)
    e = rand_zx(rng, 1)
    A = [rand_zx(rng, int(rng.integers(0, 3)), -5, 5) for _ in range(m)]
    B = [rand_zx(rng, int(rng.integers(0, 3)), -5, 5) for _ in range(n)]
    f = poly_y_from_roots(c, A)
    g = poly_y_from_roots(e, B)
    expect = zx.mul(zx.power(c, n), zx.power(e, m))
    for ai in A:
        for bj in B:
            expect = zx.mul(expect, zx.sub(ai, bj))
    got = R.resultant_y_by_points(f, g) if use_points else R.resultant_y(f, g)
    assert got == expect


@pytest.mark.parametrize("seed", range(8))
def test_leibniz_brute_force(seed):
    rng = np.random.default_rng(200 + seed)
    m = int(rng.integers(0, 5))
    n = int(rng.integers(0, 5))
    if m + n > 7 or m + n == 0:
        m, n = 3, 2
    f = rand_rows(rng, m, 2)
    g = rand_rows(rng, n, 2)
    # force zero pivots: clear some entries so Bareiss must swap rows
    if seed % 2 and m >= 1:
        f[m - 1] = []
        f[0] = []
    S = R.sylvester(R.rows_of(f), R.rows_of(g))
    assert R.resultant_y(f, g) == leibniz_det(S)


@pytest.mark.parametrize("seed", range(5))
def test_quadratic_discriminant(seed):
    rng = np.random.default_rng(300 + seed)
    A, B, C = (rand_zx(rng, 2) for _ in range(3))
    f = [C, B, A]
    fy = [B, zx.scale(A, 2)]
    expect = zx.neg(zx.mul(A, zx.sub(zx.mul(B, B), zx.scale(zx.mul(A, C), 4))))
    assert R.resultant_y(f, fy) == expect


@pytest.mark.parametrize("seed", range(4))
def test_invariants(seed):
    rng = np.random.default_rng(400 + seed)
    m, n = int(rng.integers(1, 5)), int(rng.integers(1, 5))
    f = rand_rows(rng, m, 2)
    g = rand_rows(rng, n, 2)
    r = R.resultant_y(f, g)
    # antisymmetry
    rg = R.resultant_y(g, f)
    assert rg == (zx.neg(r) if (m * n) % 2 else r)
    # scaling by a constant
    assert R.resultant_y([zx.scale(row, 3) for row in f], g) == zx.scale(r, 3 ** n)
    # multiplicativity in the first argument
    f2 = rand_rows(rng, 1, 1)
    prod = [[] for _ in range(m + 2)]
    for i, a in enumerate(f):
        for j, b in enumerate(f2):
            prod[i + j] = zx.add(prod[i + j], zx.mul(a, b))
    assert R.resultant_y(prod, g) == zx.mul(r, R.resultant_y(f2, g))
    # translation y -> y + t(x)
    t = rand_zx(rng, 1, -3, 3)

    def shift(rows):
        acc = []
        for row in reversed(rows):
            # acc = acc * (y + t) + row
            nxt = [[] for _ in range(len(acc) + 1)]
            for i, ai in enumerate(acc):
                nxt[i + 1] = zx.add(nxt[i + 1], ai)
                nxt[i] = zx.add(nxt[i], zx.mul(ai, t))
            nxt[0] = zx.add(nxt[0], row)
            acc = nxt
        return acc
    assert R.resultant_y(shift(f), shift(g)) == r


def test_common_factor_gives_zero():
    rng = np.random.default_rng(7)
    h = rand_rows(rng, 2, 1)
    a = rand_rows(rng, 2, 1)
    b = rand_rows(rng, 3, 1)

    def mulrows(P, Q):
        out = [[] for _ in range(len(P) + len(Q) - 1)]
        for i, x in enumerate(P):
            for j, y in enumerate(Q):
                out[i + j] = zx.add(out[i + j], zx.mul(x, y))
        return out
    assert R.resultant_y(mulrows(h, a), mulrows(h, b)) == []
    assert R.resultant_y_by_points(mulrows(h, a), mulrows(h, b)) == []


@pytest.mark.parametrize("seed", range(6))
def test_two_oracle_forms_agree_and_bounds(seed):
    rng = np.random.default_rng(500 + seed)
    m, n = int(rng.integers(0, 6)), int(rng.integers(0, 6))
    f = rand_rows(rng, m, int(rng.integers(0, 5)), -99, 99)
    g = rand_rows(rng, n, int(rng.integers(0, 5)), -99, 99)
    if seed % 3 == 0:
        f[0] = []            # zero constant row
    r1 = R.resultant_y(f, g)
    r2 = R.resultant_y_by_points(f, g)
    assert r1 == r2
    assert zx.deg(r1) <= R.degree_bound(f, g)
    if r1:
        assert max(c * c for c in r1) <= R.coeff_bound_sq(f, g)


def test_dense_degree_bound_is_attained_and_top_coefficient():
    import synth
    f, g = synth.config0()
    r = R.resultant_y(f, g)
    D = R.degree_bound(f, g)
    assert D == 36 and zx.deg(r) == D
    # top coefficient = res_t(f_top(1, t), g_top(1, t)) from the top forms
    ftop = [[int(f[i][6 - i])] for i in range(7)]
    gtop = [[int(g[i][6 - i])] for i in range(7)]
    assert r[-1] == R.resultant_y(ftop, gtop)[0]
    # bottom coefficient = det S(0)
    assert r[0] == R.resultant_at(f, g, 0)


def test_sympy_agrees_when_deg_f_ge_deg_g():
    sympy = pytest.importorskip("sympy")
    x, y = sympy.symbols("x y")
    rng = np.random.default_rng(600)
    for _ in range(4):
        m = int(rng.integers(1, 5))
        n = int(rng.integers(1, m + 1))
        f = rand_rows(rng, m, 2)
        g = rand_rows(rng, n, 2)
        fs = sum(c * x ** k * y ** i for i, row in enumerate(f) for k, c in enumerate(row))
        gs = sum(c * x ** k * y ** i for i, row in enumerate(g) for k, c in enumerate(row))
        rs = sympy.Poly(sympy.resultant(fs, gs, y), x)
        expect = [int(c) for c in reversed(rs.all_coeffs())] if not rs.is_zero else []
        assert R.resultant_y(f, g) == zx.trim(expect)


def test_det_mod_matches_exact():
    rng = np.random.default_rng(9)
    q = 2305843009213693951
    for n in (1, 3, 6):
        M = [[int(v) for v in rng.integers(-50, 50, size=n)] for _ in range(n)]
        assert R.det_mod(M, q) == R.det_bareiss_z(M) % q
        assert R.det_mod(M, q) == int(round(np.linalg.det(np.array(M, dtype=float)))) % q


@pytest.mark.parametrize("seed", range(6))
def test_bareiss_zx_pivoting_matches_leibniz(seed):
    """General polynomial matrices with zeroed leading entries force row
    swaps inside the Z[x] elimination."""
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(2, 6))
    M = [[rand_zx(rng, int(rng.integers(0, 3)), -4, 4) for _ in range(n)] for _ in range(n)]
    M[0][0] = []
    if n > 2 and seed % 2:
        M[1][1] = []
        M[1][0] = []
    assert R.det_bareiss_zx(M) == leibniz_det(M)
    # scalar elimination on the same matrix at a point
    Mx = [[zx.evaluate(e, 2) for e in row] for row in M]
    assert R.det_bareiss_z(Mx) == zx.evaluate(leibniz_det(M), 2)
