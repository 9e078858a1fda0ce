"""Write the stored expected values under tests/golden/ from the oracle.

    python tests/golden/make_golden.py

Calls only ``oracle`` (the CPU oracle) and ``synth`` (the seeded inputs).
Outputs:
* ``config1.json`` -- the projection resultant R = res_y(f, f_y) of the
  curve-analysis workload (f dense of total degree 24, 16-bit coefficients)
  computed by exact evaluation at 553 points and Newton interpolation, its
  SHA-256, R mod 2^61-1, and gcd(R, R') certified by ``certify_gcd``;
* ``config3.json`` -- for the large workload (f, g dense of total degrees 64
  and 48, 64-bit coefficients), whose full oracle run takes core-days: the
  exact bottom coefficient R(0) = det S(0) and the exact top coefficient
  res_t(f_top(1, t), g_top(1, t)) of x^(64*48), from the top homogeneous
  forms of f and g.
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import gcd as G  # noqa: E402
from oracle import resultant as R  # noqa: E402
from oracle import zx  # noqa: E402

Q61 = (1 << 61) - 1


def digest(coeffs) -> str:
    return hashlib.sha256(",".join(str(int(c)) for c in coeffs).encode()).hexdigest()


def main():
    t0 = time.time()
    f, g = synth.config1()
    r = R.resultant_y_by_points(f, g, processes=os.cpu_count() or 1)
    rp = zx.deriv(r)
    cand = [abs(__import__("math").gcd(zx.content(r), zx.content(rp)))]
    assert G.certify_gcd(r, rp, cand), "content gcd is not gcd(R, R')"
    out = {
        "workload": "f dense total degree 24, uniform signed 16-bit coefficients (seed 1000), g = df/dy",
        "source": "oracle.resultant.resultant_y_by_points; gcd certified by oracle.gcd.certify_gcd",
        "degree_bound": R.degree_bound(f, g),
        "degree": zx.deg(r),
        "sha256": digest(r),
        "res_at_0": str(r[0]),
        "leading": str(r[-1]),
        "mod_2_61_minus_1": [c % Q61 for c in r],
        "gcd_r_rprime": [str(c) for c in cand],
        "sqfree_sha256": digest(zx.divexact(r, cand)),
    }
    with open(os.path.join(HERE, "config1.json"), "w") as fh:
        json.dump(out, fh, indent=0)
    print(f"config1.json written in {time.time() - t0:.1f} s (deg {out['degree']})")
    t0 = time.time()
    f, g = synth.config3()
    df, dg = f.shape[0] - 1, g.shape[0] - 1
    ftop = [[int(f[i][df - i])] for i in range(df + 1)]
    gtop = [[int(g[i][dg - i])] for i in range(dg + 1)]
    top = R.resultant_y(ftop, gtop)
    out3 = {
        "workload": "f dense total degree 64, g dense total degree 48, uniform signed 64-bit (seed 3000)",
        "source": "oracle.resultant.resultant_at(f, g, 0); top coefficient = oracle.resultant.resultant_y of the top forms",
        "degree_bound": R.degree_bound(f, g),
        "res_at_0": str(R.resultant_at(f, g, 0)),
        "top_degree": df * dg,
        "top_coefficient": str(top[0] if top else 0),
    }
    with open(os.path.join(HERE, "config3.json"), "w") as fh:
        json.dump(out3, fh, indent=0)
    print(f"config3.json written in {time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
