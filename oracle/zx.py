"""Plain arithmetic in Z[x] (oracle support; test infrastructure only).

A polynomial is a list of Python ints in ascending powers of x, always
trimmed: the zero polynomial is ``[]`` and the last entry is non-zero.
"""
from __future__ import annotations

from math import gcd as igcd


def trim(a):
    a = [int(c) for c in a]
    while a and a[-1] == 0:
        a.pop()
    return a


def deg(a) -> int:
    return len(a) - 1  # -1 for the zero polynomial


def add(a, b):
    n = max(len(a), len(b))
    return trim([(a[i] if i < len(a) else 0) + (b[i] if i < len(b) else 0) for i in range(n)])


def neg(a):
    return [-c for c in a]


def sub(a, b):
    return add(a, neg(b))


def scale(a, c: int):
    return trim([c * x for x in a]) if c else []


def mul(a, b):
    if not a or not b:
        return []
    out = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        if x:
            for j, y in enumerate(b):
                out[i + j] += x * y
    return trim(out)


def divmod_exact(a, b):
    """Division with remainder in Z[x] when it exists without fractions:
    returns (q, r) with a = q*b + r, deg r < deg b, or None if some step
    needs a non-integer quotient coefficient."""
    if not b:
        raise ZeroDivisionError("division by the zero polynomial")
    r = list(a)
    db, lb = deg(b), b[-1]
    q = [0] * max(len(a) - db, 0)
    while r and deg(r) >= db:
        c, rem = divmod(r[-1], lb)
        if rem:
            return None
        s = deg(r) - db
        q[s] = c
        for i, y in enumerate(b):
            r[s + i] -= c * y
        r = trim(r)
    return trim(q), r


def divexact(a, b):
    """a / b in Z[x]; raises AssertionError unless b divides a exactly."""
    res = divmod_exact(a, b)
    assert res is not None and not res[1], "inexact division in Z[x]"
    return res[0]


def divides(b, a) -> bool:
    res = divmod_exact(a, b)
    return res is not None and not res[1]


def evaluate(a, x0: int) -> int:
    acc = 0
    for c in reversed(a):
        acc = acc * x0 + c
    return acc


def deriv(a):
    return trim([i * a[i] for i in range(1, len(a))])


def content(a) -> int:
    g = 0
    for c in a:
        g = igcd(g, c)
    return g


def compose(a, b):
    """a(b(x))."""
    acc = []
    for c in reversed(a):
        acc = add(mul(acc, b), [c] if c else [])
    return acc


def power(a, e: int):
    r = [1]
    for _ in range(e):
        r = mul(r, a)
    return r
