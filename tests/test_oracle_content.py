"""Pins of the oracle's content in y (the gcd of a curve's rows in Z[x],
removed before the curve analysis, Section 2.1): construction with a known
content, sympy's multivariate gcd over ZZ, special cases, and planted wrong
answers."""
import random

import pytest

from oracle import gcd as G
from oracle import zx


def rand_poly(rng, deg, bits=8):
    p = [rng.randrange(-(1 << bits), 1 << bits) for _ in range(deg + 1)]
    p[-1] = p[-1] or 1
    return p


@pytest.mark.parametrize("seed", range(4))
def test_by_construction(seed):
    """f = c h g with a row of g equal to 1: the content is |c| h (sign of lc)."""
    rng = random.Random(seed)
    h = rand_poly(rng, rng.randrange(1, 5))
    c = rng.choice([1, -1, 6, -35])
    rows = [rand_poly(rng, rng.randrange(0, 6)) for _ in range(rng.randrange(2, 7))]
    rows[rng.randrange(len(rows))] = [1]
    f = [zx.scale(zx.mul(h, r), c) for r in rows]
    want = zx.scale(h, abs(c))
    if want[-1] < 0:
        want = zx.neg(want)
    got = G.content_y(f)
    assert got == want
    for r in f:
        assert zx.divides(got, r)


def test_sympy_agrees():
    sympy = pytest.importorskip("sympy")
    x = sympy.symbols("x")
    rng = random.Random(11)
    for _ in range(6):
        h = rand_poly(rng, rng.randrange(0, 4), bits=4)
        rows = [zx.mul(h, rand_poly(rng, rng.randrange(0, 5), bits=5)) for _ in range(rng.randrange(1, 6))]
        polys = [sympy.Poly(list(reversed(r)), x, domain="ZZ") for r in rows]
        sg = polys[0]
        for q in polys[1:]:
            sg = sympy.gcd(sg, q)
        want = [int(v) for v in reversed(sg.all_coeffs())]
        if want[-1] < 0:
            want = [-v for v in want]
        assert G.content_y(rows) == want


def test_special_cases():
    assert G.content_y([]) == []
    assert G.content_y([[0], [0, 0]]) == []
    assert G.content_y([[0], [-4, 0, -2]]) == [4, 0, 2]         # one non-zero row, sign normalised
    assert G.content_y([[6, 12], [0], [9]]) == [3]              # integer content only
    assert G.content_y([[1, 1], [-1, 0, 1], [0]]) == [1, 1]     # x + 1 divides x^2 - 1


def test_planted_mistakes_fail():
    """Dropping a row, or forgetting the integer content, changes the answer
    on inputs built for it."""
    f = [[2, 2], [0, 2, 2], [4]]  # rows 2(x+1), 2x(x+1), 4: content 2
    assert G.content_y(f) == [2]
    assert G.content_y(f[:2]) == [2, 2]  # without the constant row the content is 2(x+1)
    assert G.content_y([G.primitive_part(r) for r in f]) == [1]
