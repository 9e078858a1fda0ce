"""Seeded synthetic workloads for the multi-modular resultant and gcd.

The paper's curve-analysis experiments (Section 4.1, family R) run on random
dense curves of moderate total degree with coefficients of a given bit size;
its data sets are not available here, so every input is drawn from a seeded
generator shaped like them.  This module is shared by the oracle side (tests,
CPU baseline) and the device side (binding, bench): it holds input
construction only (random draws, formal derivative of the input, products of
random factors for planted common factors) and none of the arithmetic of the
resultant or gcd computation.

Conventions
-----------
* RNG: ``numpy.random.Generator(PCG64(1000 * config + instance))``.
* A bivariate polynomial ``f = sum_i f_i(x) y^i`` is an integer array
  ``F[i][k]`` = coefficient of ``y^i x^k`` (numpy int64 when it fits, else a
  list of lists of Python ints).
* "Dense of total degree d": every monomial ``x^k y^i`` with ``i + k <= d``;
  entries above the anti-diagonal are zero; the ``y^d`` coefficient is redrawn
  until non-zero so that the y-degree over Z[x] is exactly ``d``.
* "Uniform signed b-bit": uniform on ``[-2^(b-1), 2^(b-1) - 1]``.
* Univariate polynomials in Z[x] are lists of Python ints, ascending powers.
"""
from __future__ import annotations

import numpy as np

INT64_MIN = -(1 << 63)
INT64_MAX = (1 << 63) - 1


def rng_for(config: int, instance: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * config + instance))


def uniform_signed(rng: np.random.Generator, shape, bits: int) -> np.ndarray:
    """Uniform signed ``bits``-bit integers (int64 array); bits <= 64."""
    if not 1 <= bits <= 64:
        raise ValueError("bits must be in 1..64")
    if bits == 64:
        return rng.integers(INT64_MIN, INT64_MAX, size=shape, dtype=np.int64, endpoint=True)
    lo = -(1 << (bits - 1))
    hi = (1 << (bits - 1)) - 1
    return rng.integers(lo, hi, size=shape, dtype=np.int64, endpoint=True)


def uniform_range(rng: np.random.Generator, shape, lo: int, hi: int) -> np.ndarray:
    """Uniform integers on the closed range [lo, hi] (int64)."""
    return rng.integers(lo, hi, size=shape, dtype=np.int64, endpoint=True)


def _mask_total_degree(F: np.ndarray, d: int) -> np.ndarray:
    i = np.arange(F.shape[0])[:, None]
    k = np.arange(F.shape[1])[None, :]
    F = F.copy()
    F[i + k > d] = 0
    return F


def dense_bivariate(rng: np.random.Generator, d: int, bits: int | None = None,
                    lo: int | None = None, hi: int | None = None) -> np.ndarray:
    """Dense bivariate polynomial of total degree ``d`` as an int64 array
    ``[d+1][d+1]``; coefficients are uniform signed ``bits``-bit, or uniform on
    ``[lo, hi]`` when a range is given.  ``F[d][0]`` is non-zero."""
    def draw(shape):
        if bits is not None:
            return uniform_signed(rng, shape, bits)
        return uniform_range(rng, shape, lo, hi)

    F = _mask_total_degree(draw((d + 1, d + 1)), d)
    while F[d, 0] == 0:
        F[d, 0] = draw(())
    return F


def y_derivative(F: np.ndarray) -> np.ndarray:
    """Formal partial derivative in y of an int64 coefficient array
    (``G[j][k] = (j+1) F[j+1][k]``); asserts the result fits int64."""
    dy = F.shape[0] - 1
    if dy == 0:
        return np.zeros((1, F.shape[1]), dtype=np.int64)
    rows = []
    for j in range(dy):
        r = [(j + 1) * int(c) for c in F[j + 1]]
        assert all(INT64_MIN <= c <= INT64_MAX for c in r)
        rows.append(r)
    return np.array(rows, dtype=np.int64)


def bivariate_product(A, B) -> list[list[int]]:
    """Exact product of two bivariate coefficient arrays (Python ints).
    Used only to plant a common factor into generated inputs."""
    A = [[int(c) for c in row] for row in A]
    B = [[int(c) for c in row] for row in B]
    ny = len(A) + len(B) - 1
    nx = max(len(r) for r in A) + max(len(r) for r in B) - 1
    C = [[0] * nx for _ in range(ny)]
    for i, ra in enumerate(A):
        for k, a in enumerate(ra):
            if a == 0:
                continue
            for j, rb in enumerate(B):
                row = C[i + j]
                for l, b in enumerate(rb):
                    if b:
                        row[k + l] += a * b
    return C


def univariate_product(a: list[int], b: list[int]) -> list[int]:
    """Exact product of two univariate integer polynomials (ascending).
    Used only to plant a common factor into generated gcd inputs."""
    if not a or not b:
        return []
    A = np.array([int(x) for x in a], dtype=object)
    B = np.array([int(y) for y in b], dtype=object)
    return [int(v) for v in np.convolve(A, B)]


def as_int64(C) -> np.ndarray:
    arr = np.array([[int(c) for c in row] for row in C], dtype=object)
    assert all(INT64_MIN <= int(c) <= INT64_MAX for c in arr.flat), "coefficient exceeds int64"
    return arr.astype(np.int64)


# ---------------------------------------------------------------------------
# The five workload shapes
# ---------------------------------------------------------------------------

def config0():
    """Smallest instance: f, g dense of total degree 6, coefficients uniform
    on [-127, 127]."""
    rng = rng_for(0)
    f = dense_bivariate(rng, 6, lo=-127, hi=127)
    g = dense_bivariate(rng, 6, lo=-127, hi=127)
    return f, g


def config1():
    """Curve-analysis shape: f dense of total degree 24 with uniform signed
    16-bit coefficients and g = df/dy (the projection resultant's operands)."""
    rng = rng_for(1)
    f = dense_bivariate(rng, 24, bits=16)
    return f, y_derivative(f)


def random_pair(rng, df, dg, bf, bg):
    return dense_bivariate(rng, df, bits=bf), dense_bivariate(rng, dg, bits=bg)


def common_factor_pair(rng, df, dg, bf, bg):
    """f = h*a, g = h*b with h dense of total degree t ~ U{1..3} (y^t
    coefficient non-zero) and a, b dense of total degrees df - t, dg - t; the
    factors carry ceil(b/2)-bit coefficients.  Returns int64 arrays padded to
    [df+1][df+1] and [dg+1][dg+1]."""
    t = int(rng.integers(1, 3, endpoint=True))
    t = min(t, df, dg)
    bh = max(2, (min(bf, bg) + 1) // 2)
    h = dense_bivariate(rng, t, bits=bh)
    a = dense_bivariate(rng, df - t, bits=max(2, (bf + 1) // 2))
    b = dense_bivariate(rng, dg - t, bits=max(2, (bg + 1) // 2))
    f = as_int64(bivariate_product(h, a))
    g = as_int64(bivariate_product(h, b))
    return f, g


def config2(npairs: int = 512, frac_common: float = 0.10):
    """Batched: ``npairs`` pairs, total degrees ~ U{8..40} and bit sizes
    ~ U{8..32} drawn independently for f and g; round(frac_common * npairs)
    pairs (indices from the seed) carry a planted common factor, so their
    resultant is zero.  Returns (pairs, common_index_set)."""
    rng = rng_for(2)
    ncommon = int(round(frac_common * npairs))
    common = set(int(i) for i in rng.choice(npairs, size=ncommon, replace=False))
    pairs = []
    for i in range(npairs):
        df = int(rng.integers(8, 40, endpoint=True))
        dg = int(rng.integers(8, 40, endpoint=True))
        bf = int(rng.integers(8, 32, endpoint=True))
        bg = int(rng.integers(8, 32, endpoint=True))
        if i in common:
            pairs.append(common_factor_pair(rng, df, dg, bf, bg))
        else:
            pairs.append(random_pair(rng, df, dg, bf, bg))
    return pairs, common


def config3():
    """Large single instance: f dense of total degree 64, g dense of total
    degree 48, both with uniform signed 64-bit coefficients."""
    rng = rng_for(3)
    return dense_bivariate(rng, 64, bits=64), dense_bivariate(rng, 48, bits=64)


def random_univariate(rng, deg: int, bits: int) -> list[int]:
    """Dense univariate polynomial of exact degree ``deg`` with uniform
    signed ``bits``-bit coefficients (leading coefficient non-zero)."""
    c = [int(v) for v in uniform_signed(rng, deg + 1, bits)]
    while c[-1] == 0:
        c[-1] = int(uniform_signed(rng, (), bits))
    return c


def gcd_request(rng, target_lo=100, target_hi=2000, h_lo=5, h_hi=50, bits_lo=8, bits_hi=32):
    """Univariate gcd input a = h*u, b = h*v with a shared random factor h
    of degree ~ U{h_lo..h_hi} and cofactors of degree target - deg h."""
    dh = int(rng.integers(h_lo, h_hi, endpoint=True))
    ta = int(rng.integers(target_lo, target_hi, endpoint=True))
    tb = int(rng.integers(target_lo, target_hi, endpoint=True))
    h = random_univariate(rng, dh, int(rng.integers(bits_lo, bits_hi, endpoint=True)))
    u = random_univariate(rng, max(ta - dh, 0), int(rng.integers(bits_lo, bits_hi, endpoint=True)))
    v = random_univariate(rng, max(tb - dh, 0), int(rng.integers(bits_lo, bits_hi, endpoint=True)))
    return univariate_product(h, u), univariate_product(h, v), h


def bigcoef_curve(rng, d: int, bits: int):
    """Dense f of total degree d with uniform signed coefficients of up to
    `bits` bits (any size: Python ints), and g = df/dy.  Lists of rows, row i
    the coefficient of y^i as a polynomial in x (ascending)."""
    def coef():
        words = [int(w) for w in rng.integers(0, 1 << 32, size=(bits + 31) // 32, dtype=np.uint64)]
        v = 0
        for w in words:
            v = (v << 32) | w
        v &= (1 << (bits - 1)) - 1
        return -v if rng.integers(0, 2) else v
    f = [[coef() if i + k <= d else 0 for k in range(d + 1)] for i in range(d + 1)]
    while f[d][0] == 0:
        f[d][0] = coef()
    g = [[(i + 1) * c for c in f[i + 1]] for i in range(d)]
    return f, g


def random_curve_set(rng, d: int, bits: int, ncurves: int = 5):
    """The resultants of the projection phase of an arrangement of `ncurves`
    random dense curves of total degree d with `bits`-bit coefficients:
    res_y(f, f_y) of every curve, then res_y(f, h) of every pair."""
    curves = [bigcoef_curve(rng, d, bits) for _ in range(ncurves)]
    pairs = [(f, fy) for f, fy in curves]
    pairs += [(curves[i][0], curves[j][0]) for i in range(ncurves) for j in range(i + 1, ncurves)]
    return pairs


def circle(a: int, b: int, r2: int):
    """(x - a)^2 + (y - b)^2 - r2 as rows in y (row i = coefficient of y^i)."""
    return [[a * a + b * b - r2, -2 * a, 1], [-2 * b], [1]]


def ellipse(A: int, B: int, a: int, b: int, C: int):
    """A (x - a)^2 + B (y - b)^2 - C as rows in y."""
    return [[A * a * a + B * b * b - C, -2 * A * a, A], [-2 * B * b], [B]]


def arrangement_set(rng, ncurves: int, kinds=("circle", "ellipse", "random", "graph", "content")):
    """A set of `ncurves` planar curves for an arrangement (rows in y of
    Python ints), cycling through the families: circles and ellipses with
    integer centres and radii, random dense curves of total degree 3..8
    with signed 10-bit coefficients, graphs of rational functions
    q(x) y - p(x) (deg p <= 4, deg q <= 3), and random curves of degree
    3..5 times a factor in x alone (x - c or x^2 + c1 x + c0), whose content
    in y is that factor times the integer content."""
    curves = []
    for i in range(ncurves):
        kind = kinds[i % len(kinds)]
        if kind == "circle":
            a, b = (int(v) for v in rng.integers(-20, 21, size=2))
            curves.append(circle(a, b, int(rng.integers(1, 226))))
        elif kind == "ellipse":
            A, B = (int(v) for v in rng.integers(1, 10, size=2))
            a, b = (int(v) for v in rng.integers(-20, 21, size=2))
            curves.append(ellipse(A, B, a, b, int(rng.integers(1, 400))))
        elif kind == "random":
            d = int(rng.integers(3, 9))
            F = dense_bivariate(rng, d, bits=10)
            curves.append([[int(c) for c in row] for row in F])
        elif kind == "graph":
            pp = [int(c) for c in rng.integers(-50, 51, size=int(rng.integers(1, 6)))]
            qq = [int(c) for c in rng.integers(-50, 51, size=int(rng.integers(1, 5)))]
            if not any(qq):
                qq = [1]
            curves.append([[-c for c in pp], qq])
        else:
            d = int(rng.integers(3, 6))
            F = [[int(c) for c in row] for row in dense_bivariate(rng, d, bits=8)]
            c = int(rng.integers(-9, 10))
            h = [-c, 1] if rng.integers(0, 2) else [int(rng.integers(-9, 10)), int(rng.integers(-9, 10)), 1]
            curves.append([univariate_product(h, row) for row in F])
    return curves


def sqfree_request(rng, degs=(120, 60, 30), bits=8, content=-6):
    """Square-free factorisation input a = content * prod_i f_i^i with monic
    random f_i of the given degrees (coefficients uniform signed `bits`-bit),
    and the factor list [(f_1, 1), (f_2, 2), ...].  Random f_i of these
    degrees are square-free and pairwise coprime with overwhelming
    probability; tests that rely on it check it."""
    fs = []
    for d in degs:
        f = [int(c) for c in uniform_signed(rng, (d,), bits)] + [1]
        fs.append(f)
    a = [content]
    for i, f in enumerate(fs):
        for _ in range(i + 1):
            a = univariate_product(a, f)
    return [int(c) for c in a], [(f, i + 1) for i, f in enumerate(fs)]


def config4(nreq: int = 2000):
    """Serving stream: requests mixed 4:1 resultant : gcd.  Resultant
    requests have total degrees ~ U{10..50} and coefficient bits ~ U{8..64};
    gcd requests are products with a shared random factor (see gcd_request).
    Returns a list of ("res", f, g) / ("gcd", a, b) tuples."""
    rng = rng_for(4)
    reqs = []
    for _ in range(nreq):
        if rng.random() < 0.8:
            df = int(rng.integers(10, 50, endpoint=True))
            dg = int(rng.integers(10, 50, endpoint=True))
            bf = int(rng.integers(8, 64, endpoint=True))
            bg = int(rng.integers(8, 64, endpoint=True))
            f, g = random_pair(rng, df, dg, bf, bg)
            reqs.append(("res", f, g))
        else:
            a, b, _h = gcd_request(rng)
            reqs.append(("gcd", a, b))
    return reqs


def poisson_arrivals(rng, rate: float, n: int) -> np.ndarray:
    """Seeded arrival times (seconds) of a Poisson stream with the given rate."""
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
