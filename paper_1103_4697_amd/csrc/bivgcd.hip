// Per-(prime, point) step of the bivariate modular gcd gcd(A, B) in Z[x, y]
// (Section 2.1, "Lifting Phase": FastLift's Q needs h = gcd(f_x, f_y)).
// Brown's dense method: for primitive A, B (in y over Z[x]) and
// gamma = gcd(lc_y A, lc_y B) in Z[x], the images
//   W(x0, y) = gamma(x0) * monic gcd(A(x0, y), B(x0, y)) mod p
// of W = (gamma / lc_y h) h at enough points x0 and primes p are
// interpolated in x and combined by Chinese remaindering; pp_y(W) = h.
// One lane per (prime, point): a wavefront holds 64 consecutive points of
// one prime, so the coefficient residues are uniform across it.  The
// univariate Euclid runs on two arrays in LDS, one column per lane.
#include <hip/hip_runtime.h>

#include "snc_internal.hpp"

namespace snc {

namespace {

// Montgomery residues of a polynomial in y whose row i (coefficient of y^i,
// a polynomial in x of degree <= dx) starts at r + i (dx + 1), evaluated at
// the point X (Montgomery) into the lane's LDS column v (canonical).
__device__ __forceinline__ void eval_rows_y(const uint32_t* r, int m, int dx, uint32_t X, uint32_t* v,
                                            const PrimeC& c) {
  for (int i = 0; i <= m; ++i) {
    const uint32_t* row = r + (int64_t)i * (dx + 1);
    uint32_t acc = 0;
    for (int k = dx; k >= 0; --k) acc = mhorner(acc, X, row[k], c.p, c.pinv);
    v[i * 64] = canon(acc, c.p);
  }
}

__global__ __launch_bounds__(64) void k_ygcd(YGcdArgs a) {
  extern __shared__ uint32_t lds[];  // two columns of (cap + 1) words per lane, lane-interleaved
  const int lane = threadIdx.x;
  const int nbp = (a.npts + 63) / 64;
  const int pi = blockIdx.x / nbp;
  const int j0 = (blockIdx.x % nbp) * 64 + lane;
  if (pi >= a.k) return;
  const bool live = j0 < a.npts;
  const int j = live ? j0 : a.npts - 1;
  const PrimeC c = a.primes[pi];
  const uint32_t X = to_mont((uint32_t)j + a.shift, c);
  const uint32_t* res = a.res + (int64_t)pi * a.T;
  uint32_t* va = lds + lane;
  uint32_t* vb = lds + (a.cap + 1) * 64 + lane;
  eval_rows_y(res + a.offA, a.mA, a.dxA, X, va, c);
  eval_rows_y(res + a.offB, a.mB, a.dxB, X, vb, c);
  uint32_t g = 0;  // gamma(x0)
  for (int k = a.dg; k >= 0; --k) g = mhorner(g, X, res[a.offG + k], c.p, c.pinv);
  g = canon(g, c.p);
  int da = a.mA, db = a.mB;
  int e = -1;
  if (va[da * 64] != 0 && vb[db * 64] != 0 && g != 0) {
    // Euclid with true remainders: A <- A mod B, then swap, until B = 0
    uint32_t* pa = va;
    uint32_t* pb = vb;
    while (db >= 0) {
      const uint32_t inv = minv(pb[db * 64], c);
      while (da >= db) {
        const uint32_t q = mmulc(pa[da * 64], inv, c.p, c.pinv);
        const uint32_t nq = mneg(q, c.p);
        for (int i = 0; i < db; ++i) {
          const int t = (da - db + i) * 64;
          pa[t] = canon2(mmul2(nq, pb[i * 64], c.r1, pa[t], c.p, c.pinv), c.p);
        }
        pa[da * 64] = 0;
        --da;
        while (da >= 0 && pa[da * 64] == 0) --da;
      }
      uint32_t* tp = pa; pa = pb; pb = tp;
      const int td = da; da = db; db = td;
    }
    // gcd = pa (degree da), made monic and scaled by gamma(x0)
    e = da;
    const uint32_t s = mmulc(g, minv(pa[da * 64], c), c.p, c.pinv);
    for (int i = 0; i <= a.emax; ++i) {
      const uint32_t w = i <= da ? mmulc(pa[i * 64], s, c.p, c.pinv) : 0u;
      if (live) a.w[a.w_off + (int64_t)i * a.w_stride + (int64_t)pi * a.npts + j] = w;
    }
  }
  if (live) a.e_out[(int64_t)pi * a.npts + j] = e;
}

}  // namespace

size_t ygcd_lds_bytes(int cap) { return (size_t)2 * (cap + 1) * 64 * sizeof(uint32_t); }

hipError_t configure_ygcd_kernel() {
  static_assert((size_t)2 * (MAXY_GEN + 1) * 64 * sizeof(uint32_t) <= 160 * 1024, "LDS columns of the largest y-degree");
  return hipFuncSetAttribute((const void*)k_ygcd, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)ygcd_lds_bytes(MAXY_GEN));
}

void launch_ygcd(const YGcdArgs& a, hipStream_t s) {
  const int nbp = (a.npts + 63) / 64;
  if (a.k <= 0 || nbp <= 0) return;
  hipLaunchKernelGGL(k_ygcd, dim3((unsigned)(a.k * nbp)), dim3(64), ygcd_lds_bytes(a.cap), s, a);
}

}  // namespace snc
