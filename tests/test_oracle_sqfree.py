"""Pins of the oracle's square-free factorisation (CPU): factorisations known
by construction, sympy's sqf_list, and the defining properties."""
import random

import pytest

from oracle import gcd as G
from oracle import zx


def _rand_poly(rng, deg, lim):
    c = [rng.randint(-lim, lim) for _ in range(deg + 1)]
    c[-1] = c[-1] or 1
    return c


def _normal(f):
    f = G.primitive_part(f)
    return zx.neg(f) if f[-1] < 0 else f


def _coprime_squarefree_factors(rng, degs, lim):
    fs = []
    while len(fs) < len(degs):
        f = _normal(_rand_poly(rng, degs[len(fs)], lim))
        if len(f) - 1 != degs[len(fs)] or G.gcd_zx(f, zx.deriv(f)) != [1]:
            continue
        if any(G.gcd_zx(f, h) != [1] for h in fs):
            continue
        fs.append(f)
    return fs


@pytest.mark.parametrize("seed", range(6))
def test_by_construction(seed):
    rng = random.Random(900 + seed)
    mults = sorted(rng.sample(range(1, 6), rng.randint(1, 3)))
    fs = _coprime_squarefree_factors(rng, [rng.randint(1, 4) for _ in mults], 9)
    c = rng.choice([1, -1, 6, -35])
    a = [c]
    for f, m in zip(fs, mults):
        a = zx.mul(a, zx.power(f, m))
    got_c, got = G.sqfree_zx(a)
    assert got_c == c
    assert got == list(zip(fs, mults))


def test_special_cases():
    assert G.sqfree_zx([]) == (0, [])
    assert G.sqfree_zx([-12]) == (-12, [])
    assert G.sqfree_zx([0, 0, 0, 0, 5]) == (5, [([0, 1], 4)])                  # 5 x^4
    assert G.sqfree_zx([-2, 2]) == (2, [([-1, 1], 1)])                          # 2 (x - 1)
    assert G.sqfree_zx(zx.power([1, 1], 5)) == (1, [([1, 1], 5)])
    assert G.sqfree_zx(zx.mul([0, -3], zx.power([1, 0, 1], 2))) == (-3, [([0, 1], 1), ([1, 0, 1], 2)])


def test_sympy_sqf_list_agrees():
    sympy = pytest.importorskip("sympy")
    x = sympy.Symbol("x")
    rng = random.Random(77)
    for _ in range(8):
        a = [1]
        for _ in range(rng.randint(1, 4)):
            a = zx.mul(a, zx.power(_rand_poly(rng, rng.randint(1, 3), 7), rng.randint(1, 3)))
        a = zx.scale(a, rng.choice([1, -2, 15]))
        coeff, facs = sympy.sqf_list(sympy.Poly(list(reversed(a)), x))
        want = [([int(v) for v in reversed(p.all_coeffs())], m) for p, m in facs]
        # sympy leaves the sign and content in coeff and may return factors with negative leading coefficient
        want = [(_normal(f), m) for f, m in want]
        c, got = G.sqfree_zx(a)
        assert got == sorted(want, key=lambda t: t[1])
        prod = [c]
        for f, m in got:
            prod = zx.mul(prod, zx.power(f, m))
        assert prod == zx.trim(a)


def test_planted_mistakes_fail():
    """A wrong multiplicity or a missing factor breaks the product identity."""
    a = zx.mul(zx.power([1, 1], 2), [-3, 0, 1])
    c, got = G.sqfree_zx(a)
    assert got == [([-3, 0, 1], 1), ([1, 1], 2)]
    bad = [([-3, 0, 1], 1), ([1, 1], 3)]
    prod = [c]
    for f, m in bad:
        prod = zx.mul(prod, zx.power(f, m))
    assert prod != a
