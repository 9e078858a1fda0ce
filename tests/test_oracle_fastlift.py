"""Pins of the oracle for FastLift's Q = res_y(f_x / h, f_y / h) with
h = gcd(f_x, f_y) (Section 2.1, "Lifting Phase"): the bivariate gcd against sympy and
planted factors, the exact bivariate division, and the identity
res(f_x, f_y) = h^(m + n) Q for h in Z[x] (m, n the y-degrees of f_x / h
and f_y / h) against the independently pinned resultant oracle."""
import random

import pytest

from oracle import fastlift as FL
from oracle import resultant as R
from oracle import zx


def rand_bi(rng, d, bits=4):
    """Dense bivariate of total degree d (rows in y, ascending in x)."""
    f = [[rng.randrange(-(1 << bits), (1 << bits) + 1) for _ in range(d + 1 - i)] for i in range(d + 1)]
    f[d][0] = f[d][0] or 1
    return FL.trim_rows(f)


def mul_bi(a, b):
    out = [[] for _ in range(len(a) + len(b) - 1)]
    for i, r in enumerate(a):
        for j, s in enumerate(b):
            out[i + j] = zx.add(out[i + j], zx.mul(r, s))
    return FL.trim_rows(out)


def test_gcd_against_sympy():
    sympy = pytest.importorskip("sympy")
    x, y = sympy.symbols("x y")
    rng = random.Random(5)

    def sym(f):
        return sum(c * x**k * y**i for i, r in enumerate(f) for k, c in enumerate(r))

    for _ in range(5):
        h, u, v = rand_bi(rng, 1, 3), rand_bi(rng, 2, 3), rand_bi(rng, 2, 3)
        a, b = mul_bi(h, u), mul_bi(h, v)
        g = FL.bivariate_gcd(a, b)
        sg = sympy.Poly(sympy.gcd(sym(a), sym(b)), y, x)
        rows = [[0] * (sg.degree(x) + 1) for _ in range(sg.degree(y) + 1)]
        for (i, k), c in sg.terms():
            rows[i][k] = int(c)
        assert g == FL._normalise(FL.trim_rows(rows))
        assert FL.divexact_bivariate(a, g) and FL.divexact_bivariate(b, g)


def test_planted_gcd_and_division():
    rng = random.Random(6)
    h = [[1, 2], [3], [1]]          # y^2 + 3y + (2x + 1)
    u, v = rand_bi(rng, 2), rand_bi(rng, 3)
    assert FL.divexact_bivariate(mul_bi(h, u), h) == u
    g = FL.bivariate_gcd(mul_bi(h, u), mul_bi(h, v))
    assert len(g) == 3 and FL.divexact_bivariate(g, h)  # h divides the gcd (u, v coprime here)


def test_generic_curve_q_is_res_fx_fy():
    rng = random.Random(7)
    for d in (3, 4, 5):
        f = rand_bi(rng, d)
        q, h = FL.fastlift_q(f)
        assert h == [[1]]
        assert q == R.resultant_y(FL.partial_x(f), FL.partial_y(f))


def test_planted_x_factor():
    """f = c + x^2 C(x, y): f_x and f_y share x, and res(f_x, f_y) = x^(m+n) Q."""
    rng = random.Random(8)
    C = rand_bi(rng, 3)
    f = FL.trim_rows([zx.add([5] if i == 0 else [], zx.mul([0, 0, 1], r)) for i, r in enumerate(C)])
    q, h = FL.fastlift_q(f)
    assert len(h) == 1 and zx.divides([0, 1], h[0])
    fx, fy = FL.partial_x(f), FL.partial_y(f)
    m = len(FL.divexact_bivariate(fx, h)) - 1
    n = len(FL.divexact_bivariate(fy, h)) - 1
    hp = [1]
    for _ in range(m + n):
        hp = zx.mul(hp, h[0])
    assert zx.mul(hp, q) == R.resultant_y(fx, fy)


def test_planted_mistake_fails():
    """Forgetting to divide by h breaks the identity on the planted curve."""
    rng = random.Random(8)
    C = rand_bi(rng, 3)
    f = FL.trim_rows([zx.add([5] if i == 0 else [], zx.mul([0, 0, 1], r)) for i, r in enumerate(C)])
    q, h = FL.fastlift_q(f)
    assert q != R.resultant_y(FL.partial_x(f), FL.partial_y(f))
