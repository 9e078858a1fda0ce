"""Oracle for FastLift's resultant Q (test infrastructure only).

Section 2.1, "Lifting Phase" (the bound m*_alpha of FastLift): with
h = gcd(f_x, f_y) in Z[x, y], f_x* = f_x / h and f_y* = f_y / h,

    Q(x) = res(f_x*, f_y*, y),

whose multiplicity at a critical x-value bounds the number of distinct
complex roots of f(alpha, y) from above (m*_alpha = deg_y f - mult(R, alpha)
+ mult(Q, alpha)).  The paper does not normalise h; any unit (+-1) changes Q
at most by a sign, and the oracle fixes h to the primitive-in-y gcd times the
gcd of the contents with a positive leading coefficient (the leading
coefficient in y, then in x).

Bivariate polynomials are lists of rows in y (row i = coefficient of y^i, a
Z[x] list ascending in x), trimmed: no zero rows above the y-degree.

The bivariate gcd is Euclid's algorithm in Z[x][y] with pseudo-remainders,
each remainder made primitive in y (its content in Z[x] divided out), and the
gcd of the two contents (oracle.gcd.content_y, gcd_zx) multiplied back.
"""
from __future__ import annotations

from . import gcd as G
from . import resultant as R
from . import zx


def trim_rows(f):
    rows = [zx.trim(r) for r in f]
    while rows and not rows[-1]:
        rows.pop()
    return rows


def partial_x(f):
    return trim_rows([zx.deriv(r) for r in trim_rows(f)])


def partial_y(f):
    rows = trim_rows(f)
    return trim_rows([zx.scale(rows[i], i) for i in range(1, len(rows))])


def _prem(a, b):
    """Pseudo-remainder of a by b in Z[x][y]: lc(b)^(da-db+1) a mod b."""
    r = [list(x) for x in a]
    db, lb = len(b) - 1, b[-1]
    e = len(a) - len(b) + 1
    while r and len(r) - 1 >= db:
        c = r[-1]
        s = len(r) - 1 - db
        r = [zx.mul(x, lb) for x in r]
        for i, y in enumerate(b):
            r[s + i] = zx.sub(r[s + i], zx.mul(c, y))
        r = trim_rows(r)
        e -= 1
    lbe = [1]
    for _ in range(max(e, 0)):
        lbe = zx.mul(lbe, lb)
    return trim_rows([zx.mul(x, lbe) for x in r])


def _pp_y(a):
    """Primitive part in y: the rows divided by their gcd in Z[x] (content_y)."""
    c = G.content_y(a)
    return [zx.divexact(r, c) for r in a], c


def _normalise(h):
    if h and h[-1] and h[-1][-1] < 0:
        return [zx.neg(r) for r in h]
    return h


def bivariate_gcd(a, b):
    """gcd(a, b) in Z[x, y] as described in the module docstring."""
    a, b = trim_rows(a), trim_rows(b)
    if not a:
        return _normalise(b)
    if not b:
        return _normalise(a)
    pa, ca = _pp_y(a)
    pb, cb = _pp_y(b)
    c = G.gcd_zx(ca, cb)
    if len(pa) < len(pb):
        pa, pb = pb, pa
    while pb and len(pb) > 1:
        r = _prem(pa, pb)
        pa = pb
        pb = _pp_y(r)[0] if r else []
    g = pa if not pb else [[1]]  # a remainder constant in y: the primitive parts are coprime
    return _normalise([zx.mul(c, r) for r in g])


def divexact_bivariate(a, h):
    """a / h in Z[x][y] (long division in y with exact divisions in Z[x])."""
    r = [list(x) for x in trim_rows(a)]
    dh = len(h) - 1
    q = [[] for _ in range(max(len(r) - dh, 1))]
    while r and len(r) - 1 >= dh:
        s = len(r) - 1 - dh
        c = zx.divexact(r[-1], h[-1])
        q[s] = c
        for i, y in enumerate(h):
            r[s + i] = zx.sub(r[s + i], zx.mul(c, y))
        r = trim_rows(r)
    assert not r, "inexact bivariate division"
    return trim_rows(q)


def fastlift_q(f):
    """(Q, h): Q = res_y(f_x / h, f_y / h) with h = gcd(f_x, f_y)."""
    fx, fy = partial_x(f), partial_y(f)
    h = bivariate_gcd(fx, fy)
    if not h:
        return [], h
    return R.resultant_y(divexact_bivariate(fx, h), divexact_bivariate(fy, h)), h
