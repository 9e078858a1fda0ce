"""Oracle for the gcd in Z[x] (test infrastructure only).

The paper runs gcds in Z[x] on the projection resultant (Yun's square-free
factorisation of R, Section 2.1 "Projection Phase") and on the y-coefficients
of f (the content removal at the start of Section 2.1).  It does not fix a
normalisation; the one taken here is the gcd in Z[x] including the integer
content, with a positive leading coefficient:

    gcd(a, b) = gcd(cont a, cont b) * pp(G_Q),  lc > 0,

where G_Q is the monic gcd over Q.  gcd(0, 0) = 0 and gcd(a, 0) = +-a with a
positive leading coefficient.
"""
from __future__ import annotations

from fractions import Fraction
from math import gcd as igcd, lcm

from . import zx


def _normalise_sign(a):
    return zx.neg(a) if a and a[-1] < 0 else list(a)


def _rem_q(a, b):
    """Remainder of a by b over Q (Fraction lists, trimmed)."""
    r = list(a)
    db, lb = len(b) - 1, b[-1]
    while r and len(r) - 1 >= db:
        c = r[-1] / lb
        s = len(r) - 1 - db
        for i, y in enumerate(b):
            r[s + i] -= c * y
        while r and r[-1] == 0:
            r.pop()
    return r


def primitive_part(a):
    c = zx.content(a)
    return [x // c for x in a] if c else []


def gcd_zx(a, b):
    """gcd(a, b) in Z[x] by Euclid over Q, normalised as above.
    Practical up to degree ~100 with moderate coefficients."""
    a, b = zx.trim(a), zx.trim(b)
    if not a and not b:
        return []
    if not b:
        return _normalise_sign(a)
    if not a:
        return _normalise_sign(b)
    c = igcd(zx.content(a), zx.content(b))
    A = [Fraction(x) for x in a]
    B = [Fraction(x) for x in b]
    while B:
        A, B = B, _rem_q(A, B)
    den = 1
    for x in A:
        den = lcm(den, x.denominator)
    G = zx.trim([int(x * den) for x in A])
    G = primitive_part(G)
    return _normalise_sign(zx.scale(G, c))


def _gcd_mod_degree(a, b, q: int) -> int:
    """Degree of gcd(a mod q, b mod q) over GF(q) (plain Euclid)."""
    A = zx.trim([x % q for x in a])
    B = zx.trim([x % q for x in b])
    while B:
        inv = pow(B[-1], q - 2, q)
        R = list(A)
        while R and len(R) >= len(B):
            c = R[-1] * inv % q
            s = len(R) - len(B)
            for i, y in enumerate(B):
                R[s + i] = (R[s + i] - c * y) % q
            while R and R[-1] == 0:
                R.pop()
        A, B = B, R
    return len(A) - 1


# Primes just below 2^61 used as coprimality witnesses.
WITNESS_PRIMES = (2305843009213693951, 2305843009213693921, 2305843009213693907,
                  2305843009213693669, 2305843009213693613)


def certify_gcd(a, b, G) -> bool:
    """True iff G is gcd(a, b) in the normalisation above, at any size.

    Checks: G divides a and b exactly in Z[x]; lc(G) > 0; cont(G) equals
    gcd(cont a, cont b); and the cofactors a/G, b/G are coprime over Q,
    witnessed by a prime q not dividing lc(a/G) with gcd(a/G, b/G) = 1 mod q
    (a common factor over Q would survive reduction mod such a q).
    """
    a, b, G = zx.trim(a), zx.trim(b), zx.trim(G)
    if not a and not b:
        return G == []
    if not G or G[-1] <= 0:
        return False
    if not (zx.divides(G, a) and zx.divides(G, b)):
        return False
    if zx.content(G) != igcd(zx.content(a), zx.content(b)):
        return False
    A = zx.divexact(a, G) if a else []
    B = zx.divexact(b, G) if b else []
    if not A:
        return zx.deg(B) == 0          # gcd(0, b) = b up to a unit
    if not B:
        return zx.deg(A) == 0
    if zx.deg(A) == 0 or zx.deg(B) == 0:
        return True
    for q in WITNESS_PRIMES:
        if A[-1] % q == 0:
            continue
        if _gcd_mod_degree(A, B, q) == 0:
            return True
    return False


def squarefree_part_sqfree(R, G):
    """R / G for G = gcd(R, R') (the square-free part up to content)."""
    return zx.divexact(R, G)


def sqfree_zx(a):
    """Square-free factorisation in Z[x]: a = c * prod_k f_k^k with c = cont(a)
    carrying the sign of lc(a), the f_k primitive with positive leading
    coefficients, square-free and pairwise coprime (the decomposition the
    projection step of Section 2.1 takes of R).  Computed from repeated gcds
    with the derivative: D_0 = pp(a), D_k = gcd(D_{k-1}, D_{k-1}'), so
    D_k = prod_{i > k} f_i^{i-k}; E_k = D_{k-1} / D_k = prod_{i >= k} f_i and
    f_k = E_k / E_{k+1}.  Returns (c, [(f_k, k), ...]) for the f_k of positive
    degree, k increasing; (0, []) for a = 0."""
    a = zx.trim(list(a))
    if not a:
        return 0, []
    c = zx.content(a)
    if a[-1] < 0:
        c = -c
    P = [x // c for x in a]
    if len(P) == 1:
        return c, []
    D = [P]
    while len(D[-1]) > 1:
        D.append(gcd_zx(D[-1], zx.deriv(D[-1])))
    E = [zx.divexact(D[k - 1], D[k]) for k in range(1, len(D))] + [[1]]
    out = []
    for k in range(1, len(D)):
        f = zx.divexact(E[k - 1], E[k])
        if len(f) > 1:
            out.append((f, k))
    return c, out


def content_y(f):
    """Content of a bivariate f in y: the gcd in Z[x] of its rows f_i(x)
    (f = sum_i f_i(x) y^i, rows ascending in x), normalised as gcd_zx.
    Section 2.1 opens by dividing this content out of the curve: its real
    roots are vertical lines of the curve.  [] for f = 0."""
    h = []
    for row in f:
        h = gcd_zx(h, [int(c) for c in row])
    return h
