"""Oracle for ``res_y(f, g)`` in Z[x] (test infrastructure only).

Definition followed.  The paper names the projection resultant
``R(x) = res(f, f_y, y)`` (Section 2.1, "Projection Phase") and the curve-pair
resultant ``R_CD = res(f, g, y)`` (Section 3) without spelling out a matrix,
so the oracle takes the textbook definition: with
``f = sum_{i<=m} f_i(x) y^i`` and ``g = sum_{j<=n} g_j(x) y^j`` (m, n the
y-degrees over Z[x], i.e. the highest non-zero rows), the Sylvester matrix is
the (m+n) x (m+n) matrix whose first n rows hold the coefficients of f in
descending order, each shifted one column to the right of the row above, and
whose last m rows hold those of g the same way; ``res_y(f, g) = det S``.

Conventions where the definition needs one:
* ``f = 0`` or ``g = 0``: the resultant is 0;
* ``m = n = 0`` (both non-zero constants in y): the empty determinant, 1;
* the formal degrees m, n stay fixed when x is specialised, so
  ``R(x0) = det S(x0)`` for every integer x0.

Two evaluations of the same determinant:
* ``resultant_y``: fraction-free Bareiss elimination over the integral domain
  Z[x] (every division is an exact polynomial division, asserted);
* ``resultant_y_by_points``: exact scalar Bareiss over Z at D+1 consecutive
  integer points around 0 and exact Newton interpolation by forward
  differences, D the degree bound below.
"""
from __future__ import annotations

from math import factorial

import numpy as np

from . import zx


# ---------------------------------------------------------------------------
# Input handling
# ---------------------------------------------------------------------------

def rows_of(F):
    """Coefficient array ``F[i][k]`` (y^i x^k) -> trimmed list of Z[x] rows,
    with zero rows above the y-degree removed."""
    rows = [zx.trim([int(c) for c in r]) for r in F]
    while rows and not rows[-1]:
        rows.pop()
    return rows


def ydeg(rows) -> int:
    return len(rows) - 1


def total_degree(rows) -> int:
    return max((i + zx.deg(r) for i, r in enumerate(rows) if r), default=-1)


# ---------------------------------------------------------------------------
# Sylvester matrix and determinants
# ---------------------------------------------------------------------------

def sylvester(frows, grows):
    """Sylvester matrix over Z[x] of f (y-degree m) and g (y-degree n)."""
    m, n = ydeg(frows), ydeg(grows)
    N = m + n
    S = [[[] for _ in range(N)] for _ in range(N)]
    for r in range(n):
        for t in range(m + 1):
            S[r][r + t] = list(frows[m - t])
    for r in range(m):
        for t in range(n + 1):
            S[n + r][r + t] = list(grows[n - t])
    return S


def det_bareiss_zx(M):
    """Determinant over Z[x] by fraction-free (Bareiss) elimination."""
    n = len(M)
    if n == 0:
        return [1]
    A = [[list(e) for e in row] for row in M]
    sign = 1
    prev = [1]
    for k in range(n - 1):
        if not A[k][k]:
            r = next((i for i in range(k + 1, n) if A[i][k]), None)
            if r is None:
                return []
            A[k], A[r] = A[r], A[k]
            sign = -sign
        piv = A[k][k]
        for i in range(k + 1, n):
            aik = A[i][k]
            for j in range(k + 1, n):
                num = zx.sub(zx.mul(piv, A[i][j]), zx.mul(aik, A[k][j]))
                A[i][j] = zx.divexact(num, prev)
        prev = piv
    d = A[n - 1][n - 1]
    return zx.neg(d) if sign < 0 else d


def det_bareiss_z(M) -> int:
    """Determinant of an integer matrix by fraction-free (Bareiss)
    elimination; exact divisions are asserted."""
    n = len(M)
    if n == 0:
        return 1
    A = np.empty((n, n), dtype=object)
    for i in range(n):
        for j in range(n):
            A[i, j] = int(M[i][j])
    sign = 1
    prev = 1
    for k in range(n - 1):
        if A[k, k] == 0:
            nz = [i for i in range(k + 1, n) if A[i, k] != 0]
            if not nz:
                return 0
            r = nz[0]
            A[[k, r]] = A[[r, k]]
            sign = -sign
        piv = A[k, k]
        num = piv * A[k + 1:, k + 1:] - np.outer(A[k + 1:, k], A[k, k + 1:])
        if prev != 1:
            q = num // prev
            assert not (num - q * prev).any(), "inexact Bareiss division"
            num = q
        A[k + 1:, k + 1:] = num
        prev = piv
    return sign * int(A[n - 1, n - 1])


# ---------------------------------------------------------------------------
# Resultant
# ---------------------------------------------------------------------------

def _trivial(frows, grows):
    """Result for the conventions, or None if the general case applies."""
    if not frows or not grows:
        return []
    if ydeg(frows) == 0 and ydeg(grows) == 0:
        return [1]
    return None


def resultant_y(F, G):
    """``res_y(f, g)`` in Z[x] (ascending coefficient list, [] for zero) by
    Bareiss over Z[x].  Cost grows like N^3 polynomial products; use for
    small inputs (total degree up to about 12)."""
    frows, grows = rows_of(F), rows_of(G)
    t = _trivial(frows, grows)
    if t is not None:
        return t
    return det_bareiss_zx(sylvester(frows, grows))


def sylvester_at(frows, grows, x0: int):
    """Integer Sylvester matrix of f(x0, y), g(x0, y) with the formal
    y-degrees of f and g over Z[x]."""
    return [[zx.evaluate(e, x0) for e in row] for row in sylvester(frows, grows)]


def resultant_at(F, G, x0: int) -> int:
    """R(x0) = det S(x0), exact."""
    frows, grows = rows_of(F), rows_of(G)
    t = _trivial(frows, grows)
    if t is not None:
        return zx.evaluate(t, x0)
    return det_bareiss_z(sylvester_at(frows, grows, x0))


def degree_bound(F, G) -> int:
    """Bound D on deg R.  Along any permutation of S the x-degree is at most
    n*d_f + m*d_g - m*n (d_f, d_g total degrees), and at most
    n*max deg f_i + m*max deg g_j (row bound); D is the smaller."""
    frows, grows = rows_of(F), rows_of(G)
    if _trivial(frows, grows) is not None:
        return 0
    m, n = ydeg(frows), ydeg(grows)
    df, dg = total_degree(frows), total_degree(grows)
    row_f = max(zx.deg(r) for r in frows)
    row_g = max(zx.deg(r) for r in grows)
    return max(0, min(n * df + m * dg - m * n, n * row_f + m * row_g))


def coeff_bound_sq(F, G) -> int:
    """B^2 for the Hadamard-type bound B on every |coefficient of R|: for
    |z| = 1 each f-row of S(z) has 2-norm at most sqrt(sum_i ||f_i||_1^2)
    (likewise for g-rows), so |R(z)| <= B := (sum ||f_i||_1^2)^(n/2) *
    (sum ||g_j||_1^2)^(m/2), and a coefficient of R is bounded by the
    maximum of |R| on the unit circle."""
    frows, grows = rows_of(F), rows_of(G)
    if _trivial(frows, grows) is not None:
        return 1
    m, n = ydeg(frows), ydeg(grows)
    sf = sum(sum(abs(c) for c in r) ** 2 for r in frows)
    sg = sum(sum(abs(c) for c in r) ** 2 for r in grows)
    return sf ** n * sg ** m


def interpolate_consecutive(x_start: int, values):
    """The polynomial of degree <= len(values)-1 through (x_start + t, v_t),
    by Newton's forward-difference form; every division by t! is exact for
    integer-coefficient results (asserted)."""
    D = len(values) - 1
    diff = [int(v) for v in values]
    newton = []
    for kappa in range(D + 1):
        q, r = divmod(diff[0], factorial(kappa))
        assert r == 0, "non-integer Newton coefficient"
        newton.append(q)
        diff = [diff[i + 1] - diff[i] for i in range(len(diff) - 1)]
    # Newton form -> monomials: P <- P * (x - x_start - kappa) + a_kappa
    P = []
    for kappa in range(D, -1, -1):
        P = zx.add(zx.mul(P, [-(x_start + kappa), 1]), [newton[kappa]] if newton[kappa] else [])
    return P


def _points_worker(args):
    F, G, xs = args
    return [resultant_at(F, G, x0) for x0 in xs]


def resultant_y_by_points(F, G, processes: int = 1):
    """``res_y(f, g)`` from exact values at D+1 consecutive integer points in
    [-floor(D/2), ceil(D/2)] and exact interpolation.  ``processes > 1``
    spreads the points over a process pool."""
    frows, grows = rows_of(F), rows_of(G)
    t = _trivial(frows, grows)
    if t is not None:
        return t
    D = degree_bound(F, G)
    x0 = -(D // 2)
    xs = list(range(x0, x0 + D + 1))
    Fl = [list(map(int, r)) for r in F]
    Gl = [list(map(int, r)) for r in G]
    if processes > 1 and len(xs) > 1:
        import multiprocessing as mp
        chunks = [xs[i::processes] for i in range(processes)]
        with mp.get_context("fork").Pool(processes) as pool:
            parts = pool.map(_points_worker, [(Fl, Gl, c) for c in chunks])
        vals = {}
        for c, p in zip(chunks, parts):
            vals.update(zip(c, p))
        values = [vals[x] for x in xs]
    else:
        values = _points_worker((Fl, Gl, xs))
    return interpolate_consecutive(x0, values)


# ---------------------------------------------------------------------------
# Modular sampled checks (for sizes where the exact oracle is too slow)
# ---------------------------------------------------------------------------

def det_mod(M, q: int) -> int:
    """Determinant of an integer matrix modulo a prime q by Gaussian
    elimination over GF(q)."""
    n = len(M)
    A = [[int(v) % q for v in row] for row in M]
    det = 1
    for k in range(n):
        r = next((i for i in range(k, n) if A[i][k]), None)
        if r is None:
            return 0
        if r != k:
            A[k], A[r] = A[r], A[k]
            det = -det
        piv = A[k][k]
        det = det * piv % q
        inv = pow(piv, q - 2, q)
        rowk = A[k]
        for i in range(k + 1, n):
            if A[i][k]:
                c = A[i][k] * inv % q
                rowi = A[i]
                for j in range(k, n):
                    rowi[j] = (rowi[j] - c * rowk[j]) % q
    return det % q


def resultant_at_mod(F, G, x0: int, q: int) -> int:
    """R(x0) mod q = det S(x0) mod q (q prime), with the formal degrees."""
    frows, grows = rows_of(F), rows_of(G)
    t = _trivial(frows, grows)
    if t is not None:
        return zx.evaluate(t, x0) % q
    S = [[zx.evaluate(e, x0) % q for e in row] for row in sylvester(frows, grows)]
    return det_mod(S, q)
