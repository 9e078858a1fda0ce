// HIP kernels of the modular gcd in Z[x] (Section 2.1: gcds of R and its
// derivative in the square-free factorisation, and the content of f;
// Section 4, "Symbolic Speedups": the gcd follows the same modular scheme).
//
// Per prime p (one workgroup each): the primitive parts a/cont(a) and
// b/cont(b) reduced mod p, their monic gcd G_p by Euclid in LDS, the scaled
// gcd w_p = beta * G_p (beta = gcd of the leading coefficients of the
// primitive parts) and the cofactors u_p = a_p / G_p, v_p = b_p / G_p by
// exact division mod p.  The host keeps the primes of minimal gcd degree,
// lifts w, u, v by Chinese remaindering and certifies beta*a = w*u,
// beta*b = w*v over Z from a norm bound.
#include <hip/hip_runtime.h>

#include "snc_internal.hpp"

namespace snc {

__device__ __forceinline__ uint32_t reduce_coef(const uint32_t* limbs, int nl, const PrimeC& c) {
  const uint32_t mask = (limbs[nl - 1] >> 31) ? 0xffffffffu : 0u;
  uint32_t acc = 0;
  for (int l = nl - 1; l >= 0; --l) {
    uint64_t v = (uint64_t)acc * c.r2 + (uint64_t)(limbs[l] ^ mask) * c.r2;
    acc = redc(v, c.p, c.pinv);
  }
  acc = canon(acc, c.p);
  if (mask) acc = mneg(madd(acc, c.r1, c.p), c.p);
  return acc;
}

__global__ __launch_bounds__(256) void k_gcd_reduce(GcdDesc G, const PrimeC* primes, uint32_t* ws) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int T = G.da + G.db + 2;
  if (t >= T) return;
  const int slot = G.slot0 + blockIdx.y;
  const int pidx = ((const int32_t*)(ws + G.slot_prime_off))[slot];
  const PrimeC c = primes[pidx];
  ws[G.res_off + (int64_t)slot * T + t] = reduce_coef(ws + G.coef_off + (int64_t)t * G.nl, G.nl, c);
}

__global__ __launch_bounds__(GCD_THREADS) void k_gcd_modp(GcdDesc G, const PrimeC* primes, uint32_t* ws) {
  extern __shared__ uint32_t sm[];
  const int tid = threadIdx.x;
  const int slot = G.slot0 + blockIdx.x;
  const int pidx = ((const int32_t*)(ws + G.slot_prime_off))[slot];
  const PrimeC c = primes[pidx];
  const uint32_t* sc = ws + G.slot_scale_off + 3 * (int64_t)slot;
  const uint32_t ia = to_mont(sc[0], c), ib = to_mont(sc[1], c);
  const int maxd = G.da > G.db ? G.da : G.db;
  uint32_t* P0 = sm;
  uint32_t* P1 = sm + (maxd + 1);
  uint32_t* Gm = sm + 2 * (maxd + 1);
  const int T = G.da + G.db + 2;
  const uint32_t* ra = ws + G.res_off + (int64_t)slot * T;
  const uint32_t* rb = ra + G.da + 1;
  for (int i = tid; i <= maxd; i += GCD_THREADS) {
    P0[i] = i <= G.da ? mmulc(ra[i], ia, c.p, c.pinv) : 0u;
    P1[i] = i <= G.db ? mmulc(rb[i], ib, c.p, c.pinv) : 0u;
  }
  __syncthreads();
  uint32_t* A = P0;
  uint32_t* B = P1;
  int dA = G.da;
  while (dA >= 0 && A[dA] == 0) --dA;
  int dB = G.db;
  while (dB >= 0 && B[dB] == 0) --dB;
  // Euclid, division-free: A <- lc(B) A - lc(A) x^(dA-dB) B cancels the top term
  while (true) {
    if (dA < dB) {
      uint32_t* t = A; A = B; B = t;
      int td = dA; dA = dB; dB = td;
    }
    if (dB < 0) break;  // divisor is zero: A is the gcd
    const uint32_t lcA = A[dA], lcB = B[dB];
    const uint32_t nlA = c.p - lcA;
    const int k = dA - dB;
    for (int i = tid; i < dA; i += GCD_THREADS) {
      const uint32_t bv = i >= k ? B[i - k] : 0u;
      A[i] = canon(mmul2(lcB, A[i], nlA, bv, c.p, c.pinv), c.p);
    }
    __syncthreads();
    --dA;
    while (dA >= 0 && A[dA] == 0) --dA;
  }
  const int e = dA;  // gcd degree mod p (>= 0: the inputs are non-zero mod p)
  const uint32_t inv = minv(A[e], c);
  for (int i = tid; i <= e; i += GCD_THREADS) Gm[i] = mmulc(A[i], inv, c.p, c.pinv);
  __syncthreads();
  uint32_t* w = ws + G.w_off + (int64_t)slot * G.wl;
  for (int i = tid; i < G.wl; i += GCD_THREADS) w[i] = i <= e ? from_mont(Gm[i], c) : 0u;
  if (tid == 0) ((int32_t*)(ws + G.e_off))[slot] = e;
  if (e == 0) {
    // constant gcd: the cofactors are the primitive parts themselves
    uint32_t* u = ws + G.u_off + (int64_t)slot * (G.da + 1);
    uint32_t* v = ws + G.v_off + (int64_t)slot * (G.db + 1);
    for (int i = tid; i <= G.da; i += GCD_THREADS) u[i] = from_mont(mmulc(ra[i], ia, c.p, c.pinv), c);
    for (int i = tid; i <= G.db; i += GCD_THREADS) v[i] = from_mont(mmulc(rb[i], ib, c.p, c.pinv), c);
    return;
  }
  // exact division of the primitive parts by the monic gcd, in LDS
  for (int pass = 0; pass < 2; ++pass) {
    const int dn = pass ? G.db : G.da;
    const uint32_t* rs = pass ? rb : ra;
    const uint32_t sc2 = pass ? ib : ia;
    uint32_t* q = ws + (pass ? G.v_off : G.u_off) + (int64_t)slot * (dn + 1);
    uint32_t* Rr = P0;
    __syncthreads();
    for (int i = tid; i <= dn; i += GCD_THREADS) Rr[i] = mmulc(rs[i], sc2, c.p, c.pinv);
    for (int i = tid; i <= dn; i += GCD_THREADS) q[i] = 0u;
    __syncthreads();
    int dr = dn;
    while (dr >= 0 && Rr[dr] == 0) --dr;
    for (int t = dr - e; t >= 0; --t) {
      const uint32_t qt = Rr[t + e];
      if (tid == 0) q[t] = from_mont(qt, c);
      const uint32_t nq = mneg(qt, c.p);
      for (int i = tid; i < e; i += GCD_THREADS)
        Rr[t + i] = canon(mmul2(c.r1, Rr[t + i], nq, Gm[i], c.p, c.pinv), c.p);
      __syncthreads();
    }
  }
}

// copy the rows of the selected primes into compact [k][len] arrays; the
// monic gcd is scaled by beta mod p on the way (w = beta * monic gcd)
__global__ void k_gcd_gather(GcdDesc G, const int32_t* sel, const uint32_t* betas, const PrimeC* sprimes,
                             int ks, int e, uint32_t* ws, int64_t wv, int64_t uv, int64_t vv) {
  const int j = blockIdx.y;
  const int s = sel[j];
  const PrimeC c = sprimes[j];
  const uint32_t bm = to_mont(betas[j], c);
  const int nw = e + 1, nu = G.da - e + 1, nv = G.db - e + 1;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nw + nu + nv; i += gridDim.x * blockDim.x) {
    if (i < nw) ws[wv + (int64_t)j * nw + i] = mmulc(bm, ws[G.w_off + (int64_t)s * G.wl + i], c.p, c.pinv);
    else if (i < nw + nu) ws[uv + (int64_t)j * nu + (i - nw)] = ws[G.u_off + (int64_t)s * (G.da + 1) + (i - nw)];
    else ws[vv + (int64_t)j * nv + (i - nw - nu)] = ws[G.v_off + (int64_t)s * (G.db + 1) + (i - nw - nu)];
  }
  (void)ks;
}

void launch_gcd_round(const GcdDesc& G, int nslots, uint32_t* ws, hipStream_t s) {
  if (nslots <= 0) return;
  const int T = G.da + G.db + 2;
  const PrimeC* primes = global_crt_tables().primes;
  hipLaunchKernelGGL(k_gcd_reduce, dim3((T + 255) / 256, nslots), dim3(256), 0, s, G, primes, ws);
  const int maxd = G.da > G.db ? G.da : G.db;
  const size_t shmem = (size_t)(3 * (maxd + 1)) * sizeof(uint32_t);
  hipLaunchKernelGGL(k_gcd_modp, dim3(nslots), dim3(GCD_THREADS), shmem, s, G, primes, ws);
}

void launch_gcd_gather(const GcdDesc& G, const int32_t* sel_d, const uint32_t* betas_d, const PrimeC* sprimes_d,
                       int ks, int e, uint32_t* ws, int64_t wv, int64_t uv, int64_t vv, hipStream_t s) {
  const int n = G.da + G.db + 3 - e;
  hipLaunchKernelGGL(k_gcd_gather, dim3((n + 255) / 256, ks), dim3(256), 0, s, G, sel_d, betas_d, sprimes_d, ks, e,
                     ws, wv, uv, vv);
}

hipError_t configure_gcd_kernels() {
  return hipFuncSetAttribute((const void*)k_gcd_modp, hipFuncAttributeMaxDynamicSharedMemorySize,
                             160 * 1024);
}

}  // namespace snc
