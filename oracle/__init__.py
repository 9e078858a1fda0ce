"""CPU oracle for the exact resultant and gcd path -- test infrastructure only.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package; the library path never does.  It shares no code with the
device implementation: it computes the plain definitions with Python integers.

* ``resultant``: ``res_y(f, g)`` as the determinant of the Sylvester matrix of
  ``f, g`` viewed as polynomials in y over Z[x] (the projection resultant
  ``R = res(f, f_y, y)`` of Section 2.1 "Projection Phase" and the curve-pair
  resultant ``R_CD = res(f, g, y)`` of Section 3), by fraction-free Bareiss
  elimination over Z[x], or by exact scalar Bareiss at integer points followed
  by exact Newton interpolation.
* ``gcd``: the gcd in Z[x] (used by the square-free factorisation of R in
  Section 2.1 and for the content of f), by Euclid over Q, plus a certificate
  that checks a claimed gcd at any size.
* ``modp``: plain modular stage definitions (residues, evaluation,
  determinant mod q) used for sampled checks at sizes where the exact oracle
  is too slow.
"""
