// HIP kernels of the modular gcd in Z[x] (Section 2.1: gcds of R and its
// derivative in the square-free factorisation, and the content of f;
// Section 4, "Symbolic Speedups": the gcd follows the same modular scheme).
//
// Per (problem, prime p), one wavefront (or one workgroup above degree 2047):
// a and b reduced mod p (b = a' formed from a's residues when asked), their
// monic gcd G_p by Euclid, and a / G_p, b / G_p by exact division mod p.  A
// prime dividing both leading coefficients is marked unusable.  The gather
// kernel scales the selected primes' rows to w_p = beta G_p (beta = gcd of the
// leading coefficients of the primitive parts), u_p = (a / cont a) / G_p and
// v_p = (b / cont b) / G_p.  The host keeps the primes of minimal gcd degree,
// lifts w, u, v by Chinese remaindering and certifies beta abar = w u,
// beta bbar = w v over Z from a norm bound.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gcd_reg.hpp"
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

// Work items are (problem, slot) pairs: items[2w] indexes descs, items[2w+1]
// is the slot (prime) of that problem.
//
// Residues of the stored rows (a's rows, then b's unless b = a'): a block
// stages rpb consecutive rows in LDS with coalesced loads and reduces them for
// up to GCD_RED_ITEMS work items; with b = a', row i also gives b_{i-1} = i a_i.
constexpr int GCD_RED_ITEMS = 1;

__global__ __launch_bounds__(256) void k_gcd_reduce(const GcdDesc* descs, const int32_t* items, int nitems, int rpb,
                                                    const PrimeC* primes, uint32_t* ws) {
  extern __shared__ uint32_t lm[];  // rpb rows of nl limbs
  const int row0 = blockIdx.x * rpb;
  const int w0 = blockIdx.y * GCD_RED_ITEMS;
  const int w1 = min(w0 + GCD_RED_ITEMS, nitems);
  int staged = -1;
  for (int w = w0; w < w1; ++w) {
    const int pb = items[2 * w], slot = items[2 * w + 1];
    const GcdDesc G = descs[pb];
    const int rows = G.deriv ? G.da + 1 : G.da + G.db + 2;
    if (row0 >= rows) continue;  // uniform over the block
    const int nr = min(rpb, rows - row0);
    if (pb != staged) {
      __syncthreads();
      for (int x = threadIdx.x; x < nr * G.nl; x += 256) lm[x] = ws[G.coef_off + (int64_t)row0 * G.nl + x];
      __syncthreads();
      staged = pb;
    }
    if ((int)threadIdx.x < nr) {
      const int i = row0 + threadIdx.x;
      const PrimeC c = primes[((const int32_t*)(ws + G.slot_prime_off))[slot]];
      uint32_t* res = ws + G.res_off + (int64_t)slot * (G.da + G.db + 2);
      const uint32_t r = reduce_coef(lm + threadIdx.x * G.nl, G.nl, c);
      res[i] = r;
      if (G.deriv && i >= 1) res[G.da + i] = mmulc(r, to_mont((uint32_t)i, c), c.p, c.pinv);  // b_{i-1} = i a_i
    }
  }
}

__global__ __launch_bounds__(GCD_THREADS) void k_gcd_modp(const GcdDesc* descs, const int32_t* items,
                                                           const PrimeC* primes, uint32_t* ws) {
  extern __shared__ uint32_t sm[];
  const int tid = threadIdx.x;
  const GcdDesc G = descs[items[2 * blockIdx.x]];
  const int slot = items[2 * blockIdx.x + 1];
  const int pidx = ((const int32_t*)(ws + G.slot_prime_off))[slot];
  const PrimeC c = primes[pidx];

  const int maxd = G.da > G.db ? G.da : G.db;
  uint32_t* P0 = sm;
  uint32_t* P1 = sm + (maxd + 1);
  uint32_t* Gm = sm + 2 * (maxd + 1);
  const int T = G.da + G.db + 2;
  const uint32_t* ra = ws + G.res_off + (int64_t)slot * T;
  const uint32_t* rb = ra + G.da + 1;
  if (G.fused) {  // given residues of a (plain), b = a'
    const uint32_t* va = G.vals + (int64_t)slot * G.vstride;
    for (int i = tid; i <= maxd; i += GCD_THREADS) P0[i] = i <= G.da ? to_mont(va[i], c) : 0u;
    for (int i = tid; i <= maxd; i += GCD_THREADS)
      P1[i] = i <= G.db ? mmulc(to_mont(va[i + 1], c), to_mont((uint32_t)(i + 1), c), c.p, c.pinv) : 0u;
  } else {
    for (int i = tid; i <= maxd; i += GCD_THREADS) {
      P0[i] = i <= G.da ? ra[i] : 0u;
      P1[i] = i <= G.db ? rb[i] : 0u;
    }
  }
  __syncthreads();
  uint32_t* A = P0;
  uint32_t* B = P1;
  int dA = G.da;
  while (dA >= 0 && A[dA] == 0) --dA;
  int dB = G.db;
  while (dB >= 0 && B[dB] == 0) --dB;
  if (G.fused && tid == 0) fused_out(G, ws)[G.d_off + slot] = dA;
  if (!G.fused && dA < G.da && dB < G.db) {
    if (tid == 0) ((int32_t*)(ws + G.e_off))[slot] = GCD_SLOT_UNUSABLE;
    return;
  }
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
  const int e = dA;  // gcd degree mod p (>= 0 unless both operands vanish mod p)
  if (tid == 0) (G.fused ? fused_out(G, ws) : (int32_t*)ws)[G.e_off + slot] = e;
  if (e <= 0 || G.fused) return;  // a usable prime with a constant gcd ends the problem on the host: no rows needed
  const uint32_t inv = minv(A[e], c);
  for (int i = tid; i <= e; i += GCD_THREADS) Gm[i] = mmulc(A[i], inv, c.p, c.pinv);
  __syncthreads();
  uint32_t* w = ws + G.w_off + (int64_t)slot * G.wl;
  for (int i = tid; i < G.wl; i += GCD_THREADS) w[i] = i <= e ? from_mont(Gm[i], c) : 0u;
  // exact division of the primitive parts by the monic gcd, in LDS
  for (int pass = 0; pass < 2; ++pass) {
    const int dn = pass ? G.db : G.da;
    const uint32_t* rs = pass ? rb : ra;
    uint32_t* q = ws + (pass ? G.v_off : G.u_off) + (int64_t)slot * (dn + 1);
    uint32_t* Rr = P0;
    __syncthreads();
    for (int i = tid; i <= dn; i += GCD_THREADS) Rr[i] = rs[i];
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

template <int E>
__device__ __forceinline__ void reg_cofactor(uint32_t (&R)[E], const uint32_t (&G)[E], int e, const uint32_t* row,
                                             int deg, uint32_t* q, uint32_t* sm, int lane, const PrimeC& c) {
  reg_load_staged<E>(R, row, deg, sm, lane);
  for (int i = lane; i <= deg; i += 64) q[i] = 0u;
  const int dR = reg_trim<E>(R, deg, c);
  for (int t = dR - e; t >= 0; --t) {
    const uint32_t qt = lead(R[0], c.p);  // coefficient of x^t of the quotient (G is monic)
    if (lane == 0) q[t] = from_mont(qt, c);
    reg_step<E>(R, G, c.r1, mneg(qt, c.p), c);
  }
}

template <int E>
__global__ __launch_bounds__(64) void k_gcd_modp_reg(const GcdDesc* descs, const int32_t* items,
                                                      const PrimeC* primes, uint32_t* ws) {
  const int lane = threadIdx.x;
  const GcdDesc G = descs[items[2 * blockIdx.x]];
  const int slot = items[2 * blockIdx.x + 1];
  const int pidx = ((const int32_t*)(ws + G.slot_prime_off))[slot];
  const PrimeC c = primes[pidx];

  const int T = G.da + G.db + 2;
  const uint32_t* ra = ws + G.res_off + (int64_t)slot * T;
  const uint32_t* rb = ra + G.da + 1;
  extern __shared__ uint32_t sm[];  // 2 * 64 * E words
  uint32_t X[E], Y[E], Gm[E];
  if (G.fused) {  // given residues of a (plain), b = a': element i of b is (da - i) times element i of a
    reg_load_staged<E>(X, G.vals + (int64_t)slot * G.vstride, G.da, sm, lane);
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int i = lane * E + s;
      X[s] = i <= G.da ? to_mont(X[s], c) : 0u;
      Y[s] = i <= G.db ? mmulc(X[s], to_mont((uint32_t)(G.da - i), c), c.p, c.pinv) : 0u;
    }
  } else {
    reg_load_staged<E>(X, ra, G.da, sm, lane);
    reg_load_staged<E>(Y, rb, G.db, sm, lane);
  }
  const int dX = reg_trim<E>(X, G.da, c);
  const int dY = reg_trim<E>(Y, G.db, c);
  if (G.fused) {
    if (lane == 0) fused_out(G, ws)[G.d_off + slot] = dX;
    const int e = dX < 0 ? -1 : euclid_levels<E>(X, dX, Y, dY, sm, lane, c);
    if (lane == 0) fused_out(G, ws)[G.e_off + slot] = e;
    return;
  }
  if (dX < G.da && dY < G.db) {
    if (lane == 0) ((int32_t*)(ws + G.e_off))[slot] = GCD_SLOT_UNUSABLE;
    return;
  }
  const int e = euclid_levels<E>(X, dX, Y, dY, sm, lane, c);
  if (lane == 0) ((int32_t*)(ws + G.e_off))[slot] = e;
  if (e == 0) return;  // a usable prime with a constant gcd ends the problem on the host: no rows needed
  __syncthreads();
  reg_fetch<E>(Gm, sm, e, lane);
  const uint32_t inv = minv(lead(Gm[0], c.p), c);
#pragma unroll
  for (int s = 0; s < E; ++s) Gm[s] = mmulc(Gm[s], inv, c.p, c.pinv);
  uint32_t* w = ws + G.w_off + (int64_t)slot * G.wl;
  for (int i = lane; i < G.wl; i += 64) w[i] = 0u;
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int i = lane * E + s;
    if (i <= e) w[e - i] = from_mont(Gm[s], c);
  }
  uint32_t* u = ws + G.u_off + (int64_t)slot * (G.da + 1);
  uint32_t* v = ws + G.v_off + (int64_t)slot * (G.db + 1);
  reg_cofactor<E>(X, Gm, e, ra, G.da, u, sm, lane, c);
  reg_cofactor<E>(X, Gm, e, rb, G.db, v, sm, lane, c);
}

static const int kGcdE[] = {2, 4, 6, 9, 12, 16, 24, 32};

// copy the rows of the selected primes into compact [k][len] arrays; the
// monic gcd is scaled by beta mod p on the way (w = beta * monic gcd)
__global__ void k_gcd_gather(GcdDesc G, const int32_t* sel, const uint32_t* scales, const PrimeC* sprimes,
                             int ks, int e, uint32_t* ws, int64_t wv, int64_t uv, int64_t vv) {
  const int j = blockIdx.y;
  const int s = sel[j];
  const PrimeC c = sprimes[j];
  const uint32_t bm = to_mont(scales[3 * j + 0], c);  // beta
  const uint32_t ia = to_mont(scales[3 * j + 1], c);  // 1 / cont(a)
  const uint32_t ib = to_mont(scales[3 * j + 2], c);  // 1 / cont(b)
  const int nw = e + 1, nu = G.da - e + 1, nv = G.db - e + 1;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nw + nu + nv; i += gridDim.x * blockDim.x) {
    if (i < nw) {
      ws[wv + (int64_t)j * nw + i] = mmulc(bm, ws[G.w_off + (int64_t)s * G.wl + i], c.p, c.pinv);
    } else if (i < nw + nu) {
      const uint32_t x = ws[G.u_off + (int64_t)s * (G.da + 1) + (i - nw)];
      ws[uv + (int64_t)j * nu + (i - nw)] = mmulc(ia, x, c.p, c.pinv);
    } else {
      const uint32_t x = ws[G.v_off + (int64_t)s * (G.db + 1) + (i - nw - nu)];
      ws[vv + (int64_t)j * nv + (i - nw - nu)] = mmulc(ib, x, c.p, c.pinv);
    }
  }
  (void)ks;
}

void launch_gcd_reduce(const GcdDesc* descs, const int32_t* items, int nitems, int max_rows, int max_nl,
                       uint32_t* ws, hipStream_t s) {
  if (nitems <= 0 || max_rows <= 0) return;
  const int rpb = std::max(1, std::min(256, 12288 / std::max(max_nl, 1)));
  const dim3 grid((max_rows + rpb - 1) / rpb, (nitems + GCD_RED_ITEMS - 1) / GCD_RED_ITEMS);
  hipLaunchKernelGGL(k_gcd_reduce, grid, dim3(256), (size_t)rpb * max_nl * sizeof(uint32_t), s, descs, items, nitems,
                     rpb, global_crt_tables().primes, ws);
}

int gcd_reg_slots(int maxd) {
  for (int e : kGcdE)
    if (64 * e >= maxd + 1) return e;
  return 0;
}

void launch_gcd_euclid(const GcdDesc* descs, const int32_t* items, int nitems, int slots, int maxd, uint32_t* ws,
                       hipStream_t s) {
  if (nitems <= 0) return;
  const PrimeC* primes = global_crt_tables().primes;
  const dim3 grid(nitems), blk(64);
  switch (slots) {
#define SNC_GCD_REG(E) \
    case E: hipLaunchKernelGGL(k_gcd_modp_reg<E>, grid, blk, 2 * 64 * E * 4, s, descs, items, primes, ws); return;
    SNC_GCD_REG(2) SNC_GCD_REG(4) SNC_GCD_REG(6) SNC_GCD_REG(9)
    SNC_GCD_REG(12) SNC_GCD_REG(16) SNC_GCD_REG(24) SNC_GCD_REG(32)
#undef SNC_GCD_REG
    default: break;
  }
  const size_t shmem = (size_t)(3 * (maxd + 1)) * sizeof(uint32_t);
  hipLaunchKernelGGL(k_gcd_modp, grid, dim3(GCD_THREADS), shmem, s, descs, items, primes, ws);
}

void launch_gcd_gather(const GcdDesc& G, const int32_t* sel_d, const uint32_t* scales_d, const PrimeC* sprimes_d,
                       int ks, int e, uint32_t* ws, int64_t wv, int64_t uv, int64_t vv, hipStream_t s) {
  const int n = G.da + G.db + 3 - e;
  hipLaunchKernelGGL(k_gcd_gather, dim3((n + 255) / 256, ks), dim3(256), 0, s, G, sel_d, scales_d, sprimes_d, ks, e,
                     ws, wv, uv, vv);
}

hipError_t configure_gcd_kernels() {
  return hipFuncSetAttribute((const void*)k_gcd_modp, hipFuncAttributeMaxDynamicSharedMemorySize,
                             160 * 1024);
}

}  // namespace snc
