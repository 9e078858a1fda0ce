"""Pins for the gcd oracle and its certificate: worked examples, gcds by
construction (a = h*u, b = h*v with u, v coprime, witnessed by a non-zero
resultant), sympy's gcd over ZZ, special cases, and planted wrong answers that
the certificate must reject."""
import json
import os
from math import gcd as igcd

import numpy as np
import pytest

from oracle import gcd as G
from oracle import resultant as R
from oracle import zx

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


def rand_poly(rng, deg, bits=8):
    lim = 1 << (bits - 1)
    c = [int(v) for v in rng.integers(-lim, lim, size=deg + 1)]
    if c[-1] == 0:
        c[-1] = 1
    return c


def normalise(p):
    return zx.neg(p) if p and p[-1] < 0 else p


def test_golden():
    data = json.load(open(GOLDEN))
    for ex in data["gcds"]:
        assert G.gcd_zx(ex["a"], ex["b"]) == ex["gcd"], ex["name"]
        assert G.certify_gcd(ex["a"], ex["b"], ex["gcd"]), ex["name"]


@pytest.mark.parametrize("seed", range(6))
def test_by_construction(seed):
    rng = np.random.default_rng(700 + seed)
    h = rand_poly(rng, int(rng.integers(0, 6)))
    u = rand_poly(rng, int(rng.integers(0, 12)))
    v = rand_poly(rng, int(rng.integers(0, 12)))
    if seed % 2:
        u = zx.scale(u, 6)
        v = zx.scale(v, 4)
    # u, v coprime over Q iff their resultant is non-zero
    if zx.deg(u) > 0 and zx.deg(v) > 0:
        assert R.resultant_y([[c] for c in u], [[c] for c in v]) != []
    a, b = zx.mul(h, u), zx.mul(h, v)
    expect = normalise(zx.scale(h, igcd(zx.content(u), zx.content(v))))
    got = G.gcd_zx(a, b)
    assert got == expect
    assert G.certify_gcd(a, b, got)


def test_sympy_gcd_agrees():
    sympy = pytest.importorskip("sympy")
    x = sympy.symbols("x")
    rng = np.random.default_rng(800)
    for _ in range(5):
        h = rand_poly(rng, 3)
        a = zx.mul(h, rand_poly(rng, 6))
        b = zx.mul(h, rand_poly(rng, 5))
        sa = sum(c * x ** i for i, c in enumerate(a))
        sb = sum(c * x ** i for i, c in enumerate(b))
        sg = sympy.Poly(sympy.gcd(sa, sb), x)
        expect = normalise([int(c) for c in reversed(sg.all_coeffs())])
        assert G.gcd_zx(a, b) == expect


def test_certificate_rejects_wrong_answers():
    rng = np.random.default_rng(900)
    h = rand_poly(rng, 3)
    a = zx.mul(h, rand_poly(rng, 7))
    b = zx.mul(h, rand_poly(rng, 6))
    g = G.gcd_zx(a, b)
    assert G.certify_gcd(a, b, g)
    assert not G.certify_gcd(a, b, zx.scale(g, 2))       # too much content
    assert not G.certify_gcd(a, b, zx.neg(g))            # wrong sign
    assert not G.certify_gcd(a, b, [1])                  # misses the factor
    if zx.deg(g) > 0:
        assert not G.certify_gcd(a, b, G.primitive_part(g[1:]) or [1])
    # a common factor that the claimed gcd misses is detected by coprimality
    lin = [1, 1]
    a2, b2 = zx.mul(a, lin), zx.mul(b, lin)
    assert not G.certify_gcd(a2, b2, g)
    assert G.certify_gcd(a2, b2, G.gcd_zx(a2, b2))


def test_special_cases():
    assert G.gcd_zx([], []) == []
    assert G.gcd_zx([0, -2, -4], []) == [0, 2, 4]
    assert G.gcd_zx([], [3]) == [3]
    assert G.gcd_zx([5], [7, 1]) == [1]
    assert G.certify_gcd([], [], [])
    assert G.certify_gcd([0, -2, -4], [], [0, 2, 4])


def test_projection_resultant_content_invariant():
    """For R = res_y(f, f_y) with constant lc_y f, |lc_y f| divides
    gcd(R, R') (R is lc_y f times a discriminant)."""
    import synth
    f, fy = synth.config0()[0], None
    fy = synth.y_derivative(f)
    r = R.resultant_y(f, fy)
    g = G.gcd_zx(r, zx.deriv(r))
    assert G.certify_gcd(r, zx.deriv(r), g)
    lc = abs(int(f[6][0]))
    assert all(c % lc == 0 for c in g)
