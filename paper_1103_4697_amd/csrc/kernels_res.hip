// HIP kernels of the multi-modular resultant res_y(f, g) (Section 4,
// "Symbolic Speedups": modular and evaluation homomorphisms, one problem per
// (prime, point) over Z_p, interpolation and Chinese remaindering), written
// for gfx950: 64-wide wavefronts, full-rate 32-bit multiplies, LDS staging.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "eval_elim.hpp"

namespace snc {

// ---------------------------------------------------------------------------
// Constant tables (filled once per device by upload_tables)
// ---------------------------------------------------------------------------
__device__ PrimeC g_primes[KMAX];
__device__ uint32_t g_garner[KMAX];            // Montgomery form of (P_i mod p_i)^-1
__device__ uint32_t g_wtab[KMAX * KMAX];       // [j*KMAX + i] = Montgomery form of P_j mod p_i (j < i)
__device__ uint32_t g_ptab[(KMAX + 1) * LPS];  // row j: P_j = prod_{l<j} p_l, little-endian limbs

__global__ void k_interp(const ResJob* jobs, const int64_t* prefix, int njobs, uint32_t* ws, uint32_t* zero_word);

// per-device kernel attributes (called once per device before any launch)
__global__ void k_crt_combine(CrtTables tb, const ResJob* jobs, const int32_t* job_list, const int64_t* prefix,
                              int njobs, int lx_max, uint32_t* ws);

hipError_t configure_kernels() {
  hipError_t e = hipFuncSetAttribute((const void*)k_interp, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     160 * 1024);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_crt_combine, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(CRT_COMB_PER_BLOCK * 3 * lx_of(KMAX) * sizeof(uint32_t)));
}

void upload_tables(const PrimeC* primes, const uint32_t* garner_c, const uint32_t* wtab,
                   const uint32_t* ptab, hipStream_t s) {
  (void)hipMemcpyToSymbolAsync(HIP_SYMBOL(g_primes), primes, sizeof(PrimeC) * KMAX, 0,
                               hipMemcpyHostToDevice, s);
  (void)hipMemcpyToSymbolAsync(HIP_SYMBOL(g_garner), garner_c, sizeof(uint32_t) * KMAX, 0,
                               hipMemcpyHostToDevice, s);
  (void)hipMemcpyToSymbolAsync(HIP_SYMBOL(g_wtab), wtab, sizeof(uint32_t) * KMAX * KMAX, 0,
                               hipMemcpyHostToDevice, s);
  (void)hipMemcpyToSymbolAsync(HIP_SYMBOL(g_ptab), ptab, sizeof(uint32_t) * (KMAX + 1) * LPS, 0,
                               hipMemcpyHostToDevice, s);
}

__global__ void k_zero_u32(uint32_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

void launch_zero_u32(uint32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
}

// ---------------------------------------------------------------------------
// (1) Modular reduction of the input coefficients (moved on-device; the
//     paper notes the host-side reduction as a bottleneck).
//     residue[prime][t] = Montgomery form of c_t mod p, c_t signed, nl limbs.
// ---------------------------------------------------------------------------
constexpr int RED_THREADS = 256;

__global__ __launch_bounds__(RED_THREADS) void k_reduce(const ResJob* jobs, const int64_t* prefix,
                                                        int njobs, const uint32_t* ws,
                                                        uint32_t* wsw, uint32_t* zero_word) {
  const int64_t b = blockIdx.x;
  if (b == 0 && threadIdx.x == 0 && zero_word) *zero_word = 0u;  // the abnormal-instance counter
  const int jj = find_job(prefix, njobs, b);
  const ResJob J = jobs[jj];
  const int nb = (J.T + RED_THREADS - 1) / RED_THREADS;
  const int64_t lb = b - prefix[jj];
  const int pi = (int)(lb / nb);
  const int t = (int)(lb % nb) * RED_THREADS + threadIdx.x;
  if (t >= J.T) return;
  const PrimeC c = g_primes[pi];
  wsw[J.res_off + (int64_t)pi * J.T + t] = reduce_limbs(ws + J.coef_off + t, J.nl, J.T, c);
}

void launch_reduce(const ResJob* jobs_d, const int64_t* blk_prefix_d, int njobs, int64_t nblocks,
                   const uint32_t* ws, uint32_t* res_base, uint32_t* zero_word, hipStream_t s) {
  if (nblocks <= 0) {
    if (zero_word) launch_zero_u32(zero_word, 1, s);
    return;
  }
  hipLaunchKernelGGL(k_reduce, dim3((unsigned)nblocks), dim3(RED_THREADS), 0, s, jobs_d,
                     blk_prefix_d, njobs, ws, res_base, zero_word);
}

// ---------------------------------------------------------------------------
// General elimination for one instance, any degree pattern: formal-degree
// corrections (res_{m,n} = (-1)^{n(m-m')} g_n^{m-m'} res_{m',n} when f's
// leading coefficients vanish, = f_m^{n-n'} res_{m,n'} when g's do, 0 when
// both do), then Euclid with true remainders.  Arrays are bottom-aligned
// (index = y-degree); runs for the rare abnormal lanes, or for every
// instance when a y-degree exceeds the register classes.
// ---------------------------------------------------------------------------
__device__ uint32_t res_general(uint32_t* F, int m, uint32_t* G, int n, const PrimeC& c) {
  if (m == 0 && n == 0) return c.r1;
  if (n == 0) return mpow(G[0], (uint32_t)m, c);
  if (m == 0) return mpow(F[0], (uint32_t)n, c);
  int mm = m;
  while (mm >= 0 && F[mm] == 0) --mm;
  int nn = n;
  while (nn >= 0 && G[nn] == 0) --nn;
  if (mm < 0 || nn < 0) return 0;
  if (mm < m && nn < n) return 0;
  uint32_t acc = c.r1;
  if (mm < m) {
    acc = mmulc(acc, mpow(G[n], (uint32_t)(m - mm), c), c.p, c.pinv);
    if ((n * (m - mm)) & 1) acc = mneg(acc, c.p);
  }
  if (nn < n) acc = mmulc(acc, mpow(F[m], (uint32_t)(n - nn), c), c.p, c.pinv);
  uint32_t* Ap = F;
  uint32_t* Bp = G;
  int a = mm, b = nn;
  while (true) {
    if (a == 0) return mmulc(acc, mpow(Ap[0], (uint32_t)b, c), c.p, c.pinv);
    if (b == 0) return mmulc(acc, mpow(Bp[0], (uint32_t)a, c), c.p, c.pinv);
    if (a < b) {
      uint32_t* t = Ap; Ap = Bp; Bp = t;
      int ti = a; a = b; b = ti;
      if ((a * b) & 1) acc = mneg(acc, c.p);
      continue;
    }
    const uint32_t inv = minv(Bp[b], c);
    int r = a;
    while (r >= b) {
      const uint32_t q = mmulc(Ap[r], inv, c.p, c.pinv);
      if (q) {
        for (int i = 0; i < b; ++i)
          Ap[r - b + i] = msub(Ap[r - b + i], mmulc(q, Bp[i], c.p, c.pinv), c.p);
      }
      Ap[r] = 0;
      --r;
      while (r >= 0 && Ap[r] == 0) --r;
    }
    if (r < 0) return 0;
    acc = mmulc(acc, mpow(Bp[b], (uint32_t)(a - r), c), c.p, c.pinv);
    if ((a * b) & 1) acc = mneg(acc, c.p);
    uint32_t* t = Ap; Ap = Bp; Bp = t;  // (A, B) <- (B, R)
    a = b; b = r;
  }
}

// MAXY: the largest y-degree of the instances this variant runs (the size
// of the per-lane value arrays)
template <int MAXY>
__device__ void general_instance(const ResJob& J, const RowDesc* rows, uint32_t* ws, int pi, int j) {
  const PrimeC c = g_primes[pi];
  const uint32_t* r = ws + J.res_off + (int64_t)pi * J.T;
  const uint32_t X = to_mont((uint32_t)j, c);
  const RowDesc* ra = rows + J.rows_off;
  const RowDesc* rb = ra + J.rstride;
  uint32_t F[MAXY + 1], G[MAXY + 1];
  for (int t = 0; t <= J.m; ++t) F[J.m - t] = canon(horner_grouped(r, ra[t / ROWGRP], t % ROWGRP, X, c), c.p);
  for (int t = 0; t <= J.n; ++t) G[J.n - t] = canon(horner_grouped(r, rb[t / ROWGRP], t % ROWGRP, X, c), c.p);
  uint32_t res = res_general(F, J.m, G, J.n, c);
  if (J.sign) res = mneg(res, c.p);
  ws[J.pts_off + (int64_t)pi * (J.D + 1) + j] = res;
}

// The abnormal instances of the register-resident elimination (y-degrees up
// to MAXY_FAST): from the list when it held them all, else every instance
// of the batch whose value carries the marker (inst_prefix: instances per
// job, prefix sums over the njobs jobs).
__global__ void k_elim_general(const ResJob* jobs, const RowDesc* rows, uint32_t* ws,
                               const uint32_t* abn_count, const AbnEntry* list, uint32_t cap,
                               const int64_t* inst_prefix, int njobs) {
  const uint32_t cnt = *abn_count;
  if (cnt == 0) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cnt <= cap) {
    for (int64_t idx = t0; idx < cnt; idx += stride) {
      const AbnEntry e = list[idx];
      const ResJob J = jobs[e.job];
      general_instance<MAXY_FAST>(J, rows, ws, e.prime, e.point);
    }
    return;
  }
  const int64_t ninst = inst_prefix[njobs];
  for (int64_t idx = t0; idx < ninst; idx += stride) {
    const int jj = find_job(inst_prefix, njobs, idx);
    const ResJob J = jobs[jj];
    const int64_t li = idx - inst_prefix[jj];
    const int pi = (int)(li / (J.D + 1)), j = (int)(li % (J.D + 1));
    if (J.m > MAXY_FAST) continue;  // computed whole by the general kernel, never marked
    if (ws[J.pts_off + (int64_t)pi * (J.D + 1) + j] == ABN_MARK) general_instance<MAXY_FAST>(J, rows, ws, pi, j);
  }
}

void launch_elim_general(const ResJob* jobs_d, const RowDesc* rows_d, uint32_t* ws,
                         const uint32_t* abn_count, const AbnEntry* abn_list, uint32_t cap,
                         const int64_t* inst_prefix_d, int njobs, hipStream_t s) {
  // enough lanes for a full list, at most 16 wavefronts per CU (grid-stride beyond)
  int64_t blocks = ((int64_t)cap + 63) / 64;
  blocks = blocks < 1 ? 1 : blocks > 256 * 16 ? 256 * 16 : blocks;
  hipLaunchKernelGGL(k_elim_general, dim3((unsigned)blocks), dim3(64), 0, s, jobs_d, rows_d, ws, abn_count, abn_list,
                     cap, inst_prefix_d, njobs);
}

__global__ void k_elim_general_all(const ResJob* jobs, const int32_t* job_list,
                                   const int64_t* prefix, int njobs, int64_t ninst,
                                   const RowDesc* rows, uint32_t* ws) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < ninst;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int jj = find_job(prefix, njobs, idx);
    const ResJob J = jobs[job_list[jj]];
    const int64_t li = idx - prefix[jj];
    general_instance<MAXY_GEN>(J, rows, ws, (int)(li / (J.D + 1)), (int)(li % (J.D + 1)));
  }
}

void launch_elim_general_all(const ResJob* jobs_d, const int32_t* job_list_d,
                             const int64_t* inst_prefix_d, int njobs, int64_t ninst,
                             const RowDesc* rows_d, uint32_t* ws, hipStream_t s) {
  if (ninst <= 0) return;
  int64_t blocks = (ninst + 63) / 64;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_elim_general_all, dim3((unsigned)blocks), dim3(64), 0, s, jobs_d, job_list_d,
                     inst_prefix_d, njobs, ninst, rows_d, ws);
}

// ---------------------------------------------------------------------------
// (4) Interpolation mod p from the values at x = 0..D, one workgroup per
//     (resultant, prime).
//   Newton coefficients of equispaced data, a_k = (Delta^k v_0) / k!, are the
//   convolution a_k = sum_{i<=k} (v_i / i!) ((-1)^{k-i} / (k-i)!).  The Newton
//   form P = sum_k a_k N_k, N_k = x (x-1) ... (x-k+1), is expanded blockwise:
//   with blocks of 64 terms starting at b = 64j,
//     Q_j = sum_{t<64} a_{b+t} prod_{i=b}^{b+t-1} (x - i),   F_j = prod_{i=b}^{b+63} (x - i),
//   and P = Q_0 + F_0 (Q_1 + F_1 (Q_2 + ...)).
//   Both the convolution and the products P F_j are Toeplitz sums; a
//   wavefront owns 64 consecutive outputs (one per lane), takes the uniform
//   operand from a register by readlane and the sliding one from LDS (one
//   coalesced read per product), and reduces every 8 products.  Q_j and F_j
//   are built by the wavefront that computed a_{64j..64j+63}, by 64 steps of
//   a one-lane shift (DPP) and a multiply-add, without barriers.
// ---------------------------------------------------------------------------
constexpr int IB = 64;    // Newton terms per block (one per lane)
constexpr int IPAD = 64;  // zero words below index 0 of the sliding operands
static_assert((4 * ((MAX_D + IB) / IB * IB) + 2 * IPAD) * 4 <= 160 * 1024,
              "interpolation buffers for the largest degree bound exceed the LDS of a CU");

// Montgomery form of 1/t! for every prime of the table and t <= MAX_D
// (filled once per device by k_ifact_init).
__device__ uint32_t g_ifact[(int64_t)KMAX * (MAX_D + 1)];

__global__ void k_ifact_init() {
  const int pi = blockIdx.x * blockDim.x + threadIdx.x;
  if (pi >= KMAX) return;
  const PrimeC c = g_primes[pi];
  uint32_t f = c.r1;
  for (int t = 2; t <= MAX_D; ++t) f = mmulc(f, to_mont((uint32_t)t, c), c.p, c.pinv);
  uint32_t inv = minv(f, c);  // 1/MAX_D!
  uint32_t* row = g_ifact + (int64_t)pi * (MAX_D + 1);
  for (int t = MAX_D; t >= 1; --t) {
    row[t] = inv;
    inv = mmulc(inv, to_mont((uint32_t)t, c), c.p, c.pinv);
  }
  row[0] = inv;
}

void launch_ffact_init(hipStream_t s);

// Montgomery coefficients of x^0 .. x^63 of F_j = (x - 64j)(x - 64j - 1) ... (x - 64j - 63)
// (x^64 implied) for every prime and the blocks j < IW_NBLK of the one-wavefront interpolation
constexpr int IW_NBLK = (IW_MAXD + 1) / 64;
static_assert(64 * IW_NBLK == IW_MAXD + 1, "whole blocks");
__device__ uint32_t g_fblk[(int64_t)KMAX * IW_NBLK * 64];

__device__ __forceinline__ uint32_t lane_shr1(uint32_t v);

// one wavefront per (prime, block): F <- F (x - (64 j + t)) for t = 0..63,
// coefficient of x^lane in lane (the x^64 term leaves lane 63 and is implied)
__global__ __launch_bounds__(64) void k_fblk_init() {
  const int pi = blockIdx.x / IW_NBLK, j = blockIdx.x % IW_NBLK, lane = threadIdx.x;
  const PrimeC c = g_primes[pi];
  uint32_t f = lane == 0 ? c.r1 : 0u;
  for (int t = 0; t < 64; ++t) {
    const uint32_t nk = to_mont(c.p - (uint32_t)(64 * j + t), c);  // -(64 j + t)
    const uint32_t fprev = lane_shr1(f);
    f = canon(redc((uint64_t)nk * f + ((uint64_t)fprev << 32), c.p, c.pinv), c.p);
  }
  g_fblk[((int64_t)pi * IW_NBLK + j) * 64 + lane] = f;
}

void launch_ifact_init(hipStream_t s) {
  hipLaunchKernelGGL(k_ifact_init, dim3(KMAX / 64), dim3(64), 0, s);
  hipLaunchKernelGGL(k_fblk_init, dim3(KMAX * IW_NBLK), dim3(64), 0, s);
  launch_ffact_init(s);
}

// lane L receives lane L-1 of v, lane 0 receives 0
__device__ __forceinline__ uint32_t lane_shr1(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138 /* wave_shr:1 */, 0xf, 0xf, true);
}

__device__ __forceinline__ uint32_t bcast(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// s + a 2^-32 mod p for a sum a of sixteen canonical products: a stays below
// 16 p^2 < 2^64, and a 2^-32 = hi + REDC(lo) mod p splits it without REDC's
// own sum (which could pass 2^64): hi = a >> 32 < 4p is taken below 2p,
// REDC(lo) = mulhi(lo pinv, p) + (lo != 0) <= p (lo plus the low word of m p
// is 0 mod 2^32), so hi + REDC(lo) < 3p and s + it < 4p.
__device__ __forceinline__ uint32_t fold16(uint32_t s, uint64_t a, const PrimeC& c) {
  uint32_t hi = (uint32_t)(a >> 32);
  const uint32_t h2 = hi - 2 * c.p;
  hi = h2 < hi ? h2 : hi;
  const uint32_t lo = (uint32_t)a;
  const uint32_t r = __umulhi(lo * c.pinv, c.p) + (lo != 0u ? 1u : 0u);
  return canon(s + hi + r, c.p);
}

// s + sum_{q<64} u_q S[-q] with u_q = lane q of u (broadcast by readlane) and
// S per lane; s canonical in, out
__device__ __forceinline__ uint32_t toeplitz64_bc(uint32_t s, uint32_t u, const uint32_t* S, const PrimeC& c) {
#pragma unroll
  for (int g = 0; g < IB; g += 8) {
    uint64_t acc = 0;
#pragma unroll
    for (int q = g; q < g + 8; ++q) acc += (uint64_t)bcast(u, q) * S[-q];  // 8 p^2 < 2^63
    s = canon(s + redc(acc, c.p, c.pinv), c.p);
  }
  return s;
}

// The same with U in LDS (16-byte aligned), read four words at a time at one
// address for the whole wavefront (no vector-unit instruction per word), and
// sixteen products per reduction (fold16).
__device__ __forceinline__ uint32_t toeplitz64(uint32_t s, const uint32_t* U, const uint32_t* S, const PrimeC& c) {
#pragma unroll
  for (int g = 0; g < IB; g += 16) {
    const uint4* U4 = reinterpret_cast<const uint4*>(U + g);
    const uint4 ua = U4[0], ub = U4[1], uc = U4[2], ud = U4[3];
    const uint32_t w16[16] = {ua.x, ua.y, ua.z, ua.w, ub.x, ub.y, ub.z, ub.w,
                              uc.x, uc.y, uc.z, uc.w, ud.x, ud.y, ud.z, ud.w};
    uint64_t acc = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += (uint64_t)w16[q] * S[-(g + q)];
    s = fold16(s, acc, c);
  }
  return s;
}

__global__ __launch_bounds__(INTERP_THREADS) void k_interp(const ResJob* jobs, const int64_t* prefix,
                                                           int njobs, uint32_t* ws, uint32_t* zero_word) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *zero_word = 0u;  // abnormal counter, read by now
  extern __shared__ uint4 sm4[];  // sections 16-byte aligned: IPAD and Dp are multiples of 64 words
  uint32_t* sm = reinterpret_cast<uint32_t*>(sm4);
  constexpr int NW = INTERP_THREADS / 64;
  const int64_t b = blockIdx.x;
  const int jj = find_job(prefix, njobs, b);
  const ResJob J = jobs[jj];
  const int pi = (int)(b - prefix[jj]);
  const PrimeC c = g_primes[pi];
  const int n1 = J.D + 1;
  const int nblk = (n1 + IB - 1) / IB;
  const int Dp = nblk * IB;
  const uint32_t* V = ws + J.pts_off + (int64_t)pi * n1;  // values at the points
  uint32_t* C = ws + J.val_off + (int64_t)pi * n1;        // coefficients
  const uint32_t* IF = g_ifact + (int64_t)pi * (MAX_D + 1);
  uint32_t* Wp = sm;             // [IPAD + Dp]: zeros, then w_j = (-1)^j / j!; later a P buffer
  uint32_t* Qb = Wp + IPAD + Dp; // [Dp]: Q_j at 64j
  uint32_t* Fb = Qb + Dp;        // [Dp]: coefficients 0..63 of F_j at 64j (x^64 implied)
  uint32_t* P1 = Fb + Dp;        // [IPAD + Dp]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // w_j = (-1)^j / j! behind IPAD zeros; u_i = v_i / i! staged in P1 (free until the expansion)
  uint32_t* U = P1;
  for (int t = tid; t < IPAD + Dp; t += INTERP_THREADS) {
    const int j = t - IPAD;
    uint32_t w = 0;
    if (j >= 0 && j < n1) {
      const uint32_t f = IF[j];
      w = (j & 1) ? mneg(f, c.p) : f;
    }
    Wp[t] = w;
    if (t < Dp) U[t] = t < n1 ? mmulc(canon(V[t], c.p), IF[t], c.p, c.pinv) : 0u;
  }
  __syncthreads();

  for (int ob = wave; ob < nblk; ob += NW) {
    const int b0 = ob * IB;
    // a_k for k = b0 + lane
    const uint32_t* wk = Wp + IPAD + b0 + lane;
    uint32_t a = 0;
    for (int ib = 0; ib <= ob; ++ib) a = toeplitz64(a, U + ib * IB, wk - ib * IB, c);
    // Q_ob and F_ob, coefficient of x^lane in lane (F_ob from its table when
    // the block has one)
    const int len = min(IB, n1 - b0);
    const uint32_t nk = to_mont(c.p - (uint32_t)(b0 + lane), c);  // -(b0 + lane)
    uint32_t q = lane == 0 ? bcast(a, len - 1) : 0u;
    const bool ftab = ob < IW_NBLK;  // uniform
    uint32_t f = ftab ? g_fblk[((int64_t)pi * IW_NBLK + ob) * 64 + lane] : (lane == 0 ? c.r1 : 0u);
    for (int s = 0; s < IB; ++s) {
      if (!ftab) {
        const uint32_t fprev = lane_shr1(f);  // F <- F (x - (b0 + s))
        f = canon(redc((uint64_t)bcast(nk, s) * f + ((uint64_t)fprev << 32), c.p, c.pinv), c.p);
      }
      const int kq = len - 2 - s;           // Q <- Q (x - (b0 + kq)) + a_{b0 + kq}
      if (kq >= 0) {
        const uint32_t add = bcast(a, kq);
        const uint32_t qprev = lane_shr1(q) + (lane == 0 ? add : 0u);
        q = canon(redc((uint64_t)bcast(nk, kq) * q + ((uint64_t)qprev << 32), c.p, c.pinv), c.p);
      }
    }
    Qb[b0 + lane] = q;
    Fb[b0 + lane] = f;
  }
  __syncthreads();

  // P = Q_{nblk-1}; P <- P F_j + Q_j for j = nblk-2 .. 0.  Entries above the
  // current degree stay zero, so whole 64-blocks are computed and stored.
  uint32_t* Pa = Wp;
  uint32_t* Pb = P1;
  const int lastb = (nblk - 1) * IB;
  const int lastlen = n1 - lastb;
  for (int t = tid; t < IPAD + Dp; t += INTERP_THREADS) {
    const int x = t - IPAD;
    Pa[t] = (x >= 0 && x < lastlen) ? Qb[lastb + x] : 0u;
    Pb[t] = 0u;
  }
  __syncthreads();
  int dP = lastlen - 1;
  for (int j = nblk - 2; j >= 0; --j) {
    const int dN = dP + IB;
    const int nob = dN / IB + 1;
    for (int ob = wave; ob < nob; ob += NW) {
      const int t = ob * IB + lane;
      const uint32_t* pt = Pa + IPAD + t;  // P[t - i] = pt[-i]
      uint32_t s = pt[-IB];                // x^64 term of F_j
      if (t < IB) s = madd(s, Qb[j * IB + t], c.p);
      Pb[IPAD + t] = toeplitz64(s, Fb + j * IB, pt, c);
    }
    __syncthreads();
    uint32_t* tmp = Pa; Pa = Pb; Pb = tmp;
    dP = dN;
  }
  for (int t = tid; t < n1; t += INTERP_THREADS) C[t] = from_mont(Pa[IPAD + t], c);
}

// ---------------------------------------------------------------------------
// One-wavefront interpolation (batches with many (resultant, prime) pairs and
// degree bounds up to IW_MAXD): the same Newton convolution, Newton blocks and
// blockwise expansion as k_interp, by one wavefront per (resultant, prime)
// with no barriers between wavefronts.  LDS holds only the sliding operand:
// w_j = (-1)^j / j! for the convolution, then P, updated in place from its top
// block down (a block's new values depend on its own and the next lower
// block's old ones).  The uniform operand, 64 words, is staged in LDS too and
// read four words at a time at one address for the whole wavefront (a
// broadcast; no vector-unit instruction per word), shared by two output
// blocks; the Newton blocks Q_j (two Horner steps per iteration) go to the
// workspace, the F_j come from their table.
// ---------------------------------------------------------------------------
// s1 += sum_q U[q] S1[-q], and (TWO) s2 += sum_q U[q] S2[-q], U in LDS
// (16-byte aligned), sixteen products per reduction (fold16).
template <bool TWO>
__device__ __forceinline__ void toeplitz64_w(uint32_t& s1, uint32_t& s2, const uint32_t* U, const uint32_t* S1,
                                             const uint32_t* S2, const PrimeC& c) {
#pragma unroll
  for (int g = 0; g < 64; g += 16) {
    const uint4* U4 = reinterpret_cast<const uint4*>(U + g);
    const uint4 ua = U4[0], ub = U4[1], uc = U4[2], ud = U4[3];
    const uint32_t w16[16] = {ua.x, ua.y, ua.z, ua.w, ub.x, ub.y, ub.z, ub.w,
                              uc.x, uc.y, uc.z, uc.w, ud.x, ud.y, ud.z, ud.w};
    uint64_t a1 = 0, a2 = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const uint64_t w = w16[q];
      a1 += w * S1[-(g + q)];
      if constexpr (TWO) a2 += w * S2[-(g + q)];
    }
    s1 = fold16(s1, a1, c);
    if constexpr (TWO) s2 = fold16(s2, a2, c);
  }
}

// Two adjacent outputs per lane: with P at word t (t even) and
// V_j = P[1 - j], so += sum_{q<64} U[q] V_q and se += sum_{q<64} U[q] V_{q+1}:
// the Toeplitz sums of outputs t + 1 and t.  One read of the two words
// P[-2i], P[1-2i] = V_{2i+1}, V_{2i} feeds four products, so the sliding
// operand costs half the LDS bytes of one output per lane; sixteen products
// per reduction (fold16), the same sums as toeplitz64_w.
__device__ __forceinline__ void toeplitz64_pair(uint32_t& se, uint32_t& so, const uint32_t* U, const uint32_t* P,
                                                const PrimeC& c) {
  const uint2* P2 = reinterpret_cast<const uint2*>(P);  // P2[-i] = (V_{2i+1}, V_{2i})
  uint2 cur = P2[0];
#pragma unroll
  for (int g = 0; g < 64; g += 16) {
    uint32_t V[18];  // V[k] = V_{g+k}
    V[0] = cur.y;
    V[1] = cur.x;
#pragma unroll
    for (int i = 1; i <= 8; ++i) {
      const uint2 x = P2[-(g / 2 + i)];
      V[2 * i] = x.y;
      V[2 * i + 1] = x.x;
    }
    cur = make_uint2(V[17], V[16]);
    const uint4* U4 = reinterpret_cast<const uint4*>(U + g);
    const uint4 ua = U4[0], ub = U4[1], uc = U4[2], ud = U4[3];
    const uint32_t w16[16] = {ua.x, ua.y, ua.z, ua.w, ub.x, ub.y, ub.z, ub.w,
                              uc.x, uc.y, uc.z, uc.w, ud.x, ud.y, ud.z, ud.w};
    uint64_t ao = 0, ae = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const uint64_t w = w16[q];
      ao += w * V[q];
      ae += w * V[q + 1];
    }
    so = fold16(so, ao, c);
    se = fold16(se, ae, c);
  }
}

// Newton block -> monomial: Q = sum_{s < len} a_{b0+s} prod_{t < s} (x - (b0 + t)),
// a_{b0+s} in lane s, by Horner's rule from the top with two steps per
// iteration:
//   Q <- (Q (x - c1) + a_k)(x - c2) + a_{k-1}
//      = Q (x^2 + B x + A) + a_k x + (a_{k-1} - c2 a_k),
// c1 = b0 + k, c2 = c1 - 1, A = c1 c2, B = -(c1 + c2): per coefficient two
// products and one reduction, Q[i-1] and Q[i-2] by two lane shifts, instead
// of two products and two reductions.  Lane it first computes iteration it's
// constants (Montgomery forms of A and B, the corrections of coefficients 0
// and 1) into K; a is staged in La.  La: 64 words, K: 4 x 32 words, 16-byte
// aligned; one wavefront (the barriers order its own LDS accesses).  The sum
// below REDC stays under 2p^2 + 2p 2^32 + 2^32 p < 2^64, its result under 4p.
__device__ __forceinline__ uint32_t newton_block2(uint32_t a, int b0, int len, int lane, const PrimeC& c,
                                                  uint32_t* La, uint32_t* K) {
  __syncthreads();
  La[lane] = a;
  __syncthreads();
  const int nit = (len - 1) / 2;
  if (lane < nit) {
    const int k = len - 2 - 2 * lane;                      // the iteration's first Horner index, >= 1
    const uint32_t c1 = (uint32_t)(b0 + k), c2 = c1 - 1;  // below 2^13: c1 c2 < p
    const uint32_t ak = La[k], ak1 = La[k - 1];
    uint4 v;
    v.x = to_mont(c1 * c2, c);
    v.y = to_mont(c.p - c1 - c2, c);
    v.z = msub(ak1, mmulc(to_mont(c2, c), ak, c.p, c.pinv), c.p);
    v.w = ak;
    reinterpret_cast<uint4*>(K)[lane] = v;
  }
  __syncthreads();
  uint32_t q = lane == 0 ? La[len - 1] : 0u;
  for (int it = 0; it < nit; ++it) {
    const uint4 v = reinterpret_cast<const uint4*>(K)[it];
    const uint32_t q1 = lane_shr1(q);
    const uint32_t q2 = lane_shr1(q1) + (lane == 0 ? v.z : lane == 1 ? v.w : 0u);
    q = canon(redc((uint64_t)v.x * q + (uint64_t)v.y * q1 + ((uint64_t)q2 << 32), c.p, c.pinv), c.p);
  }
  if ((len - 1) & 1) {  // the last step alone, k = 0
    const uint32_t nk = to_mont(c.p - (uint32_t)b0, c);
    const uint32_t qprev = lane_shr1(q) + (lane == 0 ? La[0] : 0u);
    q = canon(redc((uint64_t)nk * q + ((uint64_t)qprev << 32), c.p, c.pinv), c.p);
  }
  return q;
}

// zero words below index 0 of k_interp_w's sliding operand: the paired
// outputs of the Newton coefficients reach 127 words below an input block
constexpr int IPAD_W = 128;

__global__ __launch_bounds__(64) void k_interp_w(const ResJob* jobs, const int32_t* job_list, const int64_t* prefix,
                                                 int njobs, uint32_t* ws, uint32_t* zero_word) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *zero_word = 0u;  // abnormal counter, read by now
  extern __shared__ uint4 S4[];  // [IPAD_W + Dp] sliding operand, then [64] uniform operand
  uint32_t* S = reinterpret_cast<uint32_t*>(S4);
  const int64_t b = blockIdx.x;
  const int jj = find_job(prefix, njobs, b);
  const ResJob J = jobs[job_list[jj]];
  const int pi = (int)(b - prefix[jj]);
  const PrimeC c = g_primes[pi];
  const int n1 = J.D + 1;
  const int nblk = (n1 + 63) / 64;
  const int Dp = nblk * 64;
  const uint32_t* V = ws + J.pts_off + (int64_t)pi * n1;
  uint32_t* C = ws + J.val_off + (int64_t)pi * n1;
  uint32_t* Qg = ws + J.nq_off + (int64_t)pi * Dp;
  const uint32_t* IF = g_ifact + (int64_t)pi * (MAX_D + 1);
  const uint32_t* FB = g_fblk + (int64_t)pi * IW_NBLK * 64;
  const int lane = threadIdx.x;
  uint32_t* U = S + IPAD_W + Dp;  // 16-byte aligned: IPAD_W and Dp are multiples of 64
  uint32_t* K = U + 64;           // constants of the Newton blocks' iterations (128 words)
  // the uniform operand of the next Toeplitz sums (one wavefront: the
  // barriers only order its own LDS accesses)
  auto stage_u = [&](uint32_t v) {
    __syncthreads();
    U[lane] = v;
    __syncthreads();
  };
  for (int t = lane; t < IPAD_W + Dp; t += 64) {
    const int j = t - IPAD_W;
    uint32_t w = 0;
    if (j >= 0 && j < n1) {
      const uint32_t f = IF[j];
      w = (j & 1) ? mneg(f, c.p) : f;
    }
    S[t] = w;
  }
  __syncthreads();
  // u_{64 ib + lane} = v / (64 ib + lane)! from the loaded pair (v, 1/i!); the
  // loads of the next input block are issued before the current block's
  // Toeplitz sums, which hide their latency
  uint32_t vn = 0, fn = 0;
  auto load_u = [&](int ib) {
    const int i = 64 * ib + lane;
    vn = i < n1 ? V[i] : 0u;
    fn = i < n1 ? IF[i] : 0u;
  };
  auto uval = [&]() { return mmulc(canon(vn, c.p), fn, c.p, c.pinv); };
  for (int ob = 0; ob < nblk; ob += 2) {
    const int b0 = ob * 64;
    const uint32_t* w1 = S + IPAD_W + b0 + lane;
    uint32_t s1 = 0, s2 = 0;
    load_u(0);
    if (ob + 1 < nblk) {
      // lane l: outputs b0 + 2l and b0 + 2l + 1; the input block ob + 1
      // meets only the upper output block (the zeros below index 0 give the
      // lower lanes nothing)
      const int te = b0 + 2 * lane;
      uint32_t se = 0, so = 0;
      for (int ib = 0; ib <= ob + 1; ++ib) {
        stage_u(uval());
        if (ib <= ob) load_u(ib + 1);
        toeplitz64_pair(se, so, U, S + IPAD_W + te - 64 * ib, c);
      }
      // back to one output block per lane: b0 + lane and b0 + 64 + lane
      __syncthreads();
      reinterpret_cast<uint2*>(K)[lane] = make_uint2(se, so);
      __syncthreads();
      s1 = K[lane];
      s2 = K[64 + lane];
      Qg[b0 + lane] = newton_block2(s1, b0, 64, lane, c, U, K);
      Qg[b0 + 64 + lane] = newton_block2(s2, b0 + 64, min(64, n1 - b0 - 64), lane, c, U, K);
    } else {
      uint32_t dummy = 0;
      for (int ib = 0; ib <= ob; ++ib) {
        stage_u(uval());
        if (ib < ob) load_u(ib + 1);
        toeplitz64_w<false>(s1, dummy, U, w1 - 64 * ib, w1, c);
      }
      Qg[b0 + lane] = newton_block2(s1, b0, min(64, n1 - b0), lane, c, U, K);
    }
  }
  __syncthreads();
  // P = Q_{nblk-1}; P <- P F_j + Q_j for j = nblk-2 .. 0, in place from the top block down
  const int lastb = (nblk - 1) * 64;
  const int lastlen = n1 - lastb;
  for (int t = lane; t < IPAD_W + Dp; t += 64) {
    const int x = t - IPAD_W;
    S[t] = (x >= 0 && x < lastlen) ? Qg[lastb + x] : 0u;
  }
  __syncthreads();
  int dP = lastlen - 1;
  for (int j = nblk - 2; j >= 0; --j) {
    const int dN = dP + 64;
    const int nob = dN / 64 + 1;
    stage_u(FB[j * 64 + lane]);
    const uint32_t qj = Qg[j * 64 + lane];
    for (int ob = nob - 1; ob >= 0; ob -= 2) {
      if (ob >= 1) {
        // blocks ob - 1 and ob, lane l: outputs t = te and te + 1
        const int te = (ob - 1) * 64 + 2 * lane;
        uint32_t* pe = S + IPAD_W + te;  // P[t - i] = pe[-i]
        const uint2 x64 = *reinterpret_cast<const uint2*>(pe - 64);  // x^64 term of F_j
        uint32_t se = x64.x, so = x64.y;
        if (ob == 1 && lane < 32) {  // outputs below 64: + Q_j
          const uint2 q2 = *reinterpret_cast<const uint2*>(Qg + j * 64 + te);
          se = madd(se, q2.x, c.p);
          so = madd(so, q2.y, c.p);
        }
        toeplitz64_pair(se, so, U, pe, c);
        __syncthreads();  // every lane's reads of the old blocks before the new values land
        *reinterpret_cast<uint2*>(pe) = make_uint2(se, so);
        __syncthreads();
      } else {
        const uint32_t* p1 = S + IPAD_W + lane;  // P[t - i] = p1[-i]
        uint32_t s1 = madd(p1[-64], qj, c.p);    // x^64 term of F_j, + Q_j
        uint32_t dummy = 0;
        toeplitz64_w<false>(s1, dummy, U, p1, p1, c);
        __syncthreads();
        S[IPAD_W + lane] = s1;
        __syncthreads();
      }
    }
    dP = dN;
  }
  for (int t = lane; t < n1; t += 64) C[t] = from_mont(S[IPAD_W + t], c);
}

void launch_interp_w(const ResJob* jobs_d, const int32_t* job_list_d, const int64_t* prefix_d, int njobs,
                     int64_t nblocks, int max_D, uint32_t* ws, uint32_t* zero_word, hipStream_t s) {
  if (nblocks <= 0) return;
  const size_t lds = (size_t)(IPAD_W + (max_D + 64) / 64 * 64 + 64 + 128) * sizeof(uint32_t);
  hipLaunchKernelGGL(k_interp_w, dim3((unsigned)nblocks), dim3(64), lds, s, jobs_d, job_list_d, prefix_d, njobs,
                     ws, zero_word);
}

// ---------------------------------------------------------------------------
// Block-parallel interpolation (degree bounds below 64 IFF_J).
//   With G_j = x (x-1) ... (x - 64j + 1) the Newton form is P = sum_j G_j Q_j
//   (Q_j as above), so the blocks of 64 coefficients of P are independent
//   sums of Toeplitz products.  Two launches, each with one workgroup per
//   (resultant, prime, block):
//   k_interp_q:   Newton coefficients a_{64j..64j+63} (the convolution units
//                 over input blocks spread over the wavefronts, summed in LDS)
//                 and Q_j, stored in the workspace;
//   k_interp_out: coefficients 64 ob .. 64 ob + 63 of P as sum_{j >= ob} of
//                 G_j Q_j (one wavefront per j).
//   The G_j come from a table filled once per device.
// ---------------------------------------------------------------------------
constexpr int IFF_W = 32 * IFF_J * (IFF_J - 1) + IFF_J;  // words per prime: rows j < IFF_J of degree 64 j
__host__ __device__ constexpr int iff_off(int j) { return 32 * j * (j - 1) + j; }
constexpr int IBT = IFF_J;  // wavefronts per workgroup (one per input block or Newton block)

// Montgomery form of the coefficients of G_j for the first IFF_K primes
__device__ uint32_t g_ffact[(int64_t)IFF_K * IFF_W];

__global__ __launch_bounds__(256) void k_ffact_init() {
  __shared__ uint32_t buf[2][64 * IFF_J + 1];
  const int pi = blockIdx.x;
  const PrimeC c = g_primes[pi];
  uint32_t* out = g_ffact + (int64_t)pi * IFF_W;
  for (int m = threadIdx.x; m <= 64 * IFF_J; m += 256) buf[0][m] = m == 0 ? c.r1 : 0u;
  if (threadIdx.x == 0) out[iff_off(0)] = c.r1;
  __syncthreads();
  int cur = 0;
  for (int t = 0; t < 64 * (IFF_J - 1); ++t) {  // multiply by (x - t): degree t -> t + 1
    const uint32_t nt = to_mont(t == 0 ? 0u : c.p - (uint32_t)t, c);
    for (int m = threadIdx.x; m <= t + 1; m += 256) {
      const uint32_t lo = m >= 1 ? buf[cur][m - 1] : 0u;
      const uint32_t hi = m <= t ? buf[cur][m] : 0u;
      buf[cur ^ 1][m] = madd(lo, mmulc(nt, hi, c.p, c.pinv), c.p);
    }
    __syncthreads();
    cur ^= 1;
    if ((t + 1) % 64 == 0) {  // G_j complete, j = (t + 1) / 64
      const int j = (t + 1) / 64;
      for (int m = threadIdx.x; m <= t + 1; m += 256) out[iff_off(j) + m] = buf[cur][m];
    }
  }
}

__global__ __launch_bounds__(64 * IBT) void k_interp_q(const ResJob* jobs, const int64_t* prefix, int njobs,
                                                       uint32_t* ws, uint32_t* zero_word) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *zero_word = 0u;  // abnormal counter, read by now
  __shared__ __align__(16) uint32_t U[64 * IFF_J];  // v_i / i!
  __shared__ uint32_t Wp[IPAD + 64 * IFF_J];  // zeros, then (-1)^j / j!
  __shared__ uint32_t part[IFF_J][64];        // convolution units of this Newton block
  const int64_t b = blockIdx.x;
  const int jj = find_job(prefix, njobs, b);
  const ResJob J = jobs[jj];
  const int n1 = J.D + 1;
  const int nblk = (n1 + 63) / 64;
  const int64_t lb = b - prefix[jj];
  const int pi = (int)(lb / nblk);
  const int j = (int)(lb % nblk);             // Newton block
  const PrimeC c = g_primes[pi];
  const uint32_t* V = ws + J.pts_off + (int64_t)pi * n1;
  const uint32_t* IF = g_ifact + (int64_t)pi * (MAX_D + 1);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int top = 64 * (j + 1);               // inputs and weights below 64 (j + 1) are read
  for (int t = tid; t < IPAD + top; t += 64 * IBT) {
    const int i = t - IPAD;
    uint32_t w = 0;
    if (i >= 0 && i < n1) {
      const uint32_t f = IF[i];
      w = (i & 1) ? mneg(f, c.p) : f;
    }
    Wp[t] = w;
    if (t < top) U[t] = t < n1 ? mmulc(canon(V[t], c.p), IF[t], c.p, c.pinv) : 0u;
  }
  __syncthreads();
  // a_k, k = 64 j + lane: input block ib on wavefront ib
  if (wave <= j) part[wave][lane] = toeplitz64(0u, U + wave * 64, Wp + IPAD + 64 * (j - wave) + lane, c);
  __syncthreads();
  if (wave != 0) return;
  uint32_t a = 0;
  for (int ib = 0; ib <= j; ++ib) a = madd(a, part[ib][lane], c.p);
  // Q_j, coefficient of x^lane in lane
  const int b0 = 64 * j;
  const int len = min(64, n1 - b0);
  const uint32_t nk = to_mont(c.p - (uint32_t)(b0 + lane), c);  // -(b0 + lane)
  uint32_t q = lane == 0 ? bcast(a, len - 1) : 0u;
  for (int s = 0; s + 2 <= len; ++s) {  // Q <- Q (x - (b0 + kq)) + a_{b0 + kq}, kq = len - 2 - s
    const int kq = len - 2 - s;
    const uint32_t add = bcast(a, kq);
    const uint32_t qprev = lane_shr1(q) + (lane == 0 ? add : 0u);
    q = canon(redc((uint64_t)bcast(nk, kq) * q + ((uint64_t)qprev << 32), c.p, c.pinv), c.p);
  }
  ws[J.nq_off + (int64_t)pi * nblk * 64 + b0 + lane] = q;
}

__global__ __launch_bounds__(64 * IBT) void k_interp_out(const ResJob* jobs, const int64_t* prefix, int njobs,
                                                         uint32_t* ws) {
  __shared__ uint32_t Gs[IFF_J][128];   // coefficients 64 ob - 64 .. 64 ob + 63 of G_j
  __shared__ uint32_t outp[IFF_J][64];  // G_j Q_j on this block
  const int64_t b = blockIdx.x;
  const int jj = find_job(prefix, njobs, b);
  const ResJob J = jobs[jj];
  const int n1 = J.D + 1;
  const int nblk = (n1 + 63) / 64;
  const int64_t lb = b - prefix[jj];
  const int pi = (int)(lb / nblk);
  const int ob = (int)(lb % nblk);      // output block
  const PrimeC c = g_primes[pi];
  const uint32_t* GF = g_ffact + (int64_t)pi * IFF_W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = ob + wave;              // Newton block of this wavefront
  if (j < nblk) {
    for (int m = lane; m < 128; m += 64) {
      const int g = 64 * ob - 64 + m;
      Gs[wave][m] = (g >= 0 && g <= 64 * j) ? GF[iff_off(j) + g] : 0u;
    }
    const uint32_t q = ws[J.nq_off + (int64_t)pi * nblk * 64 + 64 * j + lane];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    outp[wave][lane] = toeplitz64_bc(0u, q, &Gs[wave][64 + lane], c);
  }
  __syncthreads();
  if (wave == 0) {
    uint32_t s = 0;
    for (int w = 0; w < nblk - ob; ++w) s = madd(s, outp[w][lane], c.p);
    const int t = 64 * ob + lane;
    if (t < n1) ws[J.val_off + (int64_t)pi * n1 + t] = from_mont(s, c);
  }
}

void launch_interp_blk(const ResJob* jobs_d, const int64_t* blk_prefix_d, int njobs, int64_t nblocks, uint32_t* ws,
                       uint32_t* zero_word, hipStream_t s) {
  if (nblocks <= 0) return;
  hipLaunchKernelGGL(k_interp_q, dim3((unsigned)nblocks), dim3(64 * IBT), 0, s, jobs_d, blk_prefix_d, njobs, ws,
                     zero_word);
  hipLaunchKernelGGL(k_interp_out, dim3((unsigned)nblocks), dim3(64 * IBT), 0, s, jobs_d, blk_prefix_d, njobs, ws);
}

size_t interp_lds_bytes(int max_D) {
  const size_t Dp = (size_t)((max_D + 1 + IB - 1) / IB) * IB;
  return (4 * Dp + 2 * IPAD) * sizeof(uint32_t);
}

void launch_interp(const ResJob* jobs_d, const int64_t* blk_prefix_d, int njobs, int64_t nblocks,
                   int max_D, uint32_t* ws, uint32_t* zero_word, hipStream_t s) {
  if (nblocks <= 0) return;
  hipLaunchKernelGGL(k_interp, dim3((unsigned)nblocks), dim3(INTERP_THREADS), interp_lds_bytes(max_D), s,
                     jobs_d, blk_prefix_d, njobs, ws, zero_word);
}

// ---------------------------------------------------------------------------
// (5) Chinese remaindering per coefficient.
//   digits: Garner's mixed-radix digits y_j, X = sum_j y_j P_j, with
//     y_i = (r_i - S_i) (P_i)^-1 mod p_i,  S_i = sum_{j<i} y_j P_j mod p_i.
//     One wavefront per coefficient, primes in blocks of 64 (lane l holds
//     prime 64 s + l of block s).  In block s the digits come one after
//     another: digit q is broadcast from lane q and folded into the later
//     primes of the block.  The finished block then goes to every later
//     block s2 at once, S_i += sum_q y_{64s+q} (P_{64s+q} mod p_i), sixteen
//     products per reduction.  S_i waits in digit slot i until digit i is
//     written there.  The 64 x 64 tiles of W = (P_j mod p_i) are staged in
//     LDS, double-buffered and shared by the block's wavefronts.
//   combine: X in binary by Horner over the digits; the balanced value is
//     X - M when X > (M-1)/2, decided on the digits ((M-1)/2 has digits
//     (p_j - 1)/2), written as L two's-complement limbs.
// ---------------------------------------------------------------------------
constexpr int CRT_TILE = 64 * 64;                          // words of one W tile
constexpr int CRT_PRE = CRT_TILE / (64 * CRT_COEF_PER_BLOCK);  // tile words fetched per thread

__global__ __launch_bounds__(64 * CRT_COEF_PER_BLOCK) void k_crt_digits(CrtTables tb, const ResJob* jobs,
                                                                        const int32_t* job_list,
                                                                        const int64_t* prefix,
                                                                        int njobs, uint32_t* ws) {
  __shared__ uint32_t wt[2][CRT_TILE];  // tile (s, s2): [q][l] = W[64 s + q][64 s2 + l]
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);
  const int jj = find_job(prefix, njobs, b);
  const ResJob J = jobs[job_list ? job_list[jj] : jj];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = (int)(b - prefix[jj]) * CRT_COEF_PER_BLOCK + wave;
  const bool active = t <= J.D;  // the block's waves share one job; idle ones still meet the barriers
  const int k = J.k;
  const int nsl = (k + 63) >> 6;
  const int n1 = J.D + 1;
  const uint32_t* V = ws + J.val_off;
  uint32_t* dig = ws + J.dig_off + (int64_t)(active ? t : 0) * k;
  if (active)
    for (int i = lane; i < k; i += 64) dig[i] = 0;  // the partial sums S_i start at zero
  uint32_t pre[CRT_PRE];
  auto fetch = [&](int s, int s2) {
#pragma unroll
    for (int e = 0; e < CRT_PRE; ++e) {
      const int x = threadIdx.x + e * 64 * CRT_COEF_PER_BLOCK;
      const int row = 64 * s + (x >> 6), col = 64 * s2 + (x & 63);
      pre[e] = (row < k && col < k) ? tb.wtab[(int64_t)row * tb.wstride + col] : 0u;
    }
  };
  fetch(0, 0);
  uint32_t ymine = 0;  // digit 64 s + lane of the current block
  const int ntiles = nsl * (nsl + 1) / 2;
  int s = 0, s2 = 0;
  for (int tau = 0; tau < ntiles; ++tau) {
    uint32_t* w = wt[tau & 1];
#pragma unroll
    for (int e = 0; e < CRT_PRE; ++e) w[threadIdx.x + e * 64 * CRT_COEF_PER_BLOCK] = pre[e];
    __syncthreads();
    int ns = s, ns2 = s2 + 1;  // the next tile, fetched while this one is worked on
    if (ns2 == nsl) { ++ns; ns2 = ns; }
    if (tau + 1 < ntiles) fetch(ns, ns2);
    const int i = 64 * s2 + lane;
    const bool ok = active && i < k;
    const PrimeC c = tb.primes[i < k ? i : 0];
    if (s2 == s) {  // digits of block s
      const int nq = min(64, k - 64 * s);
      const uint32_t g = tb.garner[i < k ? i : 0];
      const uint32_t r = ok ? V[(int64_t)i * n1 + t] : 0u;
      uint32_t S = ok ? dig[i] : 0u;
      for (int q = 0; q < nq; ++q) {
        const uint32_t cand = canon(redc((uint64_t)msub(r, S, c.p) * g, c.p, c.pinv), c.p);
        const uint32_t y = __builtin_amdgcn_readlane(cand, q);
        if (lane == q) ymine = cand;
        if (lane > q) S = madd(S, canon(redc((uint64_t)y * w[q * 64 + lane], c.p, c.pinv), c.p), c.p);
      }
      if (ok) dig[i] = ymine;
    } else {  // block s into block s2 > s (s is not the last block: 64 digits)
      uint32_t acc = ok ? dig[i] : 0u;  // < 2p from here on
#pragma unroll
      for (int q = 0; q < 64; q += 16) {
        // sixteen products y < 2^30 times W < p stay below 2^34 p < 2^64 (four
        // partial sums); with sum = hi 2^32 + lo, sum 2^-32 = hi + lo 2^-32,
        // where hi < 4p and the REDC of lo alone is at most p
        uint64_t part[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          part[u] = 0;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int qq = q + 4 * u + v;
            part[u] += (uint64_t)__builtin_amdgcn_readlane(ymine, qq) * w[qq * 64 + lane];
          }
        }
        const uint64_t sum = (part[0] + part[1]) + (part[2] + part[3]);
        uint32_t hi = (uint32_t)(sum >> 32);
        const uint32_t h2 = hi - 2 * c.p;
        hi = h2 < hi ? h2 : hi;  // [0, 4p) -> [0, 2p)
        uint32_t t = hi + redc((uint64_t)(uint32_t)sum, c.p, c.pinv);  // < 3p + 1
        const uint32_t t2 = t - 2 * c.p;
        t = t2 < t ? t2 : t;  // -> [0, 2p)
        acc += t;
        const uint32_t a2 = acc - 2 * c.p;
        acc = a2 < acc ? a2 : acc;  // [0, 4p) -> [0, 2p)
      }
      if (ok) dig[i] = canon(acc, c.p);
    }
    s = ns;
    s2 = ns2;
  }
}

// X = sum_j y_j P_j for the workgroup's CRT_COMB_PER_BLOCK coefficients,
// lanes over limbs: wavefront w of the CRT_COEF_PER_BLOCK takes limbs
// 64 w + 64 CRT_COEF_PER_BLOCK i + lane of every coefficient of the workgroup,
// so each limb of P_j is read once per workgroup.
// Limb l accumulates sum_j y_j P_j[l] (< 2^72) as lo (64 bits) + hi; its low
// word stays at limb l and the rest, a carry below 2^41, goes to limb l+1.
// Lane 0 of wavefront c then propagates the carries of coefficient c,
// subtracts M = P_k when X > (M-1)/2 (decided on the digits: (M-1)/2 has
// digits (p_j - 1)/2) and writes L two's-complement limbs.
__global__ __launch_bounds__(64 * CRT_COEF_PER_BLOCK) void k_crt_combine(CrtTables tb, const ResJob* jobs,
                                                                         const int32_t* job_list,
                                                                         const int64_t* prefix, int njobs,
                                                                         int lx_max, uint32_t* ws) {
  constexpr int C = CRT_COMB_PER_BLOCK;
  extern __shared__ uint32_t csm[];
  const int64_t b = blockIdx.x;
  const int jj = find_job(prefix, njobs, b);
  const ResJob J = jobs[job_list ? job_list[jj] : jj];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t0 = (int)(b - prefix[jj]) * C;
  const int nc = min(C, J.D + 1 - t0);  // coefficients of this block (>= 1)
  const int k = J.k;
  const int lx = lx_of(k);
  const uint32_t* d0 = ws + J.dig_off + (int64_t)t0 * k;  // digits of coefficient t0 + c at d0[c k + j]
  for (int l0 = 64 * wave; l0 < lx; l0 += 64 * CRT_COEF_PER_BLOCK) {
    const int l = l0 + lane;
    uint64_t lo[C];
    uint32_t hi[C];
#pragma unroll
    for (int c = 0; c < C; ++c) { lo[c] = 0; hi[c] = 0; }
    // P_j has at most 30 j / 32 + 1 limbs, so limbs >= l0 need j >= 32 l0 / 30 - 1
    int j0 = (32 * l0) / 30 - 1;
    if (j0 < 0) j0 = 0;
#pragma unroll 16
    for (int j = j0; j < k; ++j) {  // sixteen limb loads in flight per wavefront
      const uint32_t pl = l < tb.pstride ? tb.ptab[(int64_t)j * tb.pstride + l] : 0u;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const uint64_t pr = (uint64_t)(c < nc ? d0[c * k + j] : 0u) * pl;
        lo[c] += pr;
        hi[c] += lo[c] < pr ? 1u : 0u;
      }
    }
    if (l < lx) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        uint32_t* Xl = csm + c * 3 * lx_max;  // [lx] low words, then [2 lx] 64-bit carries as word pairs
        Xl[l] = (uint32_t)lo[c];
        const uint64_t cl = (lo[c] >> 32) | ((uint64_t)hi[c] << 32);
        Xl[lx_max + 2 * l] = (uint32_t)cl;
        Xl[lx_max + 2 * l + 1] = (uint32_t)(cl >> 32);
      }
    }
  }
  __syncthreads();
  if (wave >= nc) return;
  const int t = t0 + wave;
  const uint32_t* d = d0 + (int64_t)wave * k;
  const uint32_t* Xlo = csm + wave * 3 * lx_max;
  const uint32_t* Xc = Xlo + lx_max;
  if (lane != 0) return;
  const uint32_t* dt = d;
  int cmp = 0;
  for (int j = k - 1; j >= 0; --j) {
    const uint32_t h = (tb.primes[j].p - 1) >> 1;
    if (dt[j] != h) { cmp = dt[j] > h ? 1 : -1; break; }
  }
  const bool sub = cmp > 0;
  const uint32_t* M = tb.ptab + (int64_t)k * tb.pstride;
  uint32_t* out = ws + J.out_off + (int64_t)t * J.L;
  uint64_t carry = 0;
  int64_t borrow = 0;
  for (int l = 0; l < lx; ++l) {
    const uint64_t sv = (uint64_t)Xlo[l] + carry;
    uint32_t v = (uint32_t)sv;
    carry = (sv >> 32) + ((uint64_t)Xc[2 * l] | ((uint64_t)Xc[2 * l + 1] << 32));
    if (sub) {
      const int64_t dv = (int64_t)v - (int64_t)(l < tb.pstride ? M[l] : 0u) - borrow;
      borrow = dv < 0 ? 1 : 0;
      v = (uint32_t)(dv + (borrow << 32));
    }
    if (l < J.L) out[l] = v;
  }
  for (int l = lx; l < J.L; ++l) out[l] = sub ? 0xffffffffu : 0u;
}

// Chinese remaindering with few primes (k <= KC <= CRT_KS), the usual case of
// batched resultants: one lane per coefficient, so that every table constant
// is uniform across the wavefront (scalar loads) and no lane idles on a
// short prime list.
//   digits (Garner): y_i = (r_i - S_i) (P_i mod p_i)^-1 mod p_i with
//     S_i = sum_{j<i} y_j (P_j mod p_i), summed sixteen products per
//     reduction; the lane's digits wait in LDS (digit j at yl[64 j + lane]).
//   binary value: Horner's rule X <- X p_j + y_j from the top digit down in
//     LC registers, the multiply-add chain touching only the limbs X can
//     occupy so far (after digit j, X < P_k / P_j < 2^(30 (k - j))).
//   balanced result: X - M when X > (M-1)/2, decided on the digits on the
//     way down ((M-1)/2 has digits (p_j - 1)/2); L two's-complement limbs.
constexpr int CRT_KS = 128;                 // largest prime count of this path
__device__ __align__(64) uint32_t g_wts[CRT_KS * CRT_KS];  // [i][j] = Montgomery form of P_j mod p_i for j < i, else 0

__global__ void k_crt_small_init() {
  const int i = blockIdx.x;
  for (int j = threadIdx.x; j < CRT_KS; j += blockDim.x)
    g_wts[i * CRT_KS + j] = j < i ? g_wtab[(int64_t)j * KMAX + i] : 0u;
}

void launch_crt_small_init(hipStream_t s) {
  static_assert(CRT_KS <= KMAX, "small-path primes come from the table");
  hipLaunchKernelGGL(k_crt_small_init, dim3(CRT_KS), dim3(64), 0, s);
}

template <int KC>
__global__ __launch_bounds__(64) void k_crt_small(const ResJob* jobs, const int32_t* job_list, const int64_t* prefix,
                                                  int njobs, uint32_t* ws) {
  static_assert(KC <= CRT_KS && KC % 16 == 0, "prime capacity of the small path, whole groups of 16 digits");
  constexpr int LC = (30 * KC + 31) / 32 + 2;  // limbs of X (as lx_of)
  __shared__ uint32_t yl[KC * 64];
  const int64_t b = blockIdx.x;
  const int jj = find_job(prefix, njobs, b);
  const ResJob J = jobs[job_list[jj]];
  const int lane = threadIdx.x;
  const int t0 = (int)(b - prefix[jj]) * 64 + lane;
  const bool live = t0 <= J.D;
  const int t = live ? t0 : J.D;  // lanes past the last coefficient repeat it and store nothing
  const int k = J.k, n1 = J.D + 1;
  const uint32_t* V = ws + J.val_off + t;
  // Digits four at a time: the sums of rows i0..i0+3 over the digits before
  // i0 share each digit read (groups of sixteen: y_j < p_j and W < p_i, so
  // sixteen products stay below 2^64), then the block's own digits follow in
  // order with their products inside the block.  The digit slots start at
  // zero, so a group that reaches past i0 reads zeros for the digits not
  // computed yet (each lane reads only its own slots: no barrier).
  for (int j = 0; j < KC; ++j) yl[64 * j + lane] = 0u;
  // S < 2p, a sum below 2^64: S + a 2^-32 = S + hi + REDC(lo) with hi < 4p
  // taken below 2p and REDC(lo) <= p, back below 2p
  auto fold = [](uint32_t S, uint64_t a, const PrimeC& c) {
    uint32_t hi = (uint32_t)(a >> 32);
    const uint32_t h2 = hi - 2 * c.p;
    hi = h2 < hi ? h2 : hi;                                       // [0, 2p)
    uint32_t v = hi + redc((uint64_t)(uint32_t)a, c.p, c.pinv);  // < 3p + 1
    const uint32_t v2 = v - 2 * c.p;
    v = v2 < v ? v2 : v;  // [0, 2p)
    S += v;
    const uint32_t s2 = S - 2 * c.p;
    return s2 < S ? s2 : S;  // [0, 2p)
  };
  for (int i0 = 0; i0 < k; i0 += 4) {
    PrimeC cr[4];
    uint32_t S[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int r = 0; r < 4; ++r) cr[r] = g_primes[i0 + r];  // i0 + 3 < KC: rows of the table exist
    for (int j0 = 0; j0 < i0; j0 += 16) {
      uint32_t wv[4][16];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint4* w4 = reinterpret_cast<const uint4*>(g_wts + (i0 + r) * CRT_KS + j0);
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const uint4 x = w4[h];
          wv[r][4 * h] = x.x; wv[r][4 * h + 1] = x.y; wv[r][4 * h + 2] = x.z; wv[r][4 * h + 3] = x.w;
        }
      }
      uint64_t acc[4] = {0, 0, 0, 0};
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const uint64_t y = yl[64 * (j0 + u) + lane];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] += y * wv[r][u];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) S[r] = fold(S[r], acc[r], cr[r]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + r;
      if (i >= k) break;  // uniform
      uint64_t a = 0;
#pragma unroll
      for (int q = 0; q < r; ++q) a += (uint64_t)yl[64 * (i0 + q) + lane] * g_wts[i * CRT_KS + i0 + q];
      const uint32_t Sf = fold(S[r], a, cr[r]);
      const uint32_t rv = V[(int64_t)i * n1];
      yl[64 * i + lane] =
          canon(redc((uint64_t)msub(rv, canon2(Sf, cr[r].p), cr[r].p) * g_garner[i], cr[r].p, cr[r].pinv), cr[r].p);
    }
  }
  uint32_t X[LC];
#pragma unroll
  for (int l = 0; l < LC; ++l) X[l] = 0;
  int cmp = 0;  // sign of X - (M-1)/2, from the top digit down
  for (int j = k - 1; j >= 0; --j) {
    const uint32_t p = g_primes[j].p;
    const uint32_t y = yl[64 * j + lane];
    const uint32_t h = (p - 1) >> 1;
    if (cmp == 0 && y != h) cmp = y > h ? 1 : -1;
    const int len = (30 * (k - j) + 31) / 32 + 1;  // limbs X can occupy after this step (uniform)
    uint64_t carry = y;
#pragma unroll
    for (int l0 = 0; l0 < LC; l0 += 8) {
      if (l0 < len) {  // uniform: chunks above X's length are skipped (they hold zeros)
#pragma unroll
        for (int l = l0; l < l0 + 8 && l < LC; ++l) {
          const uint64_t v = (uint64_t)X[l] * p + carry;
          X[l] = (uint32_t)v;
          carry = v >> 32;
        }
      }
    }
  }
  const bool sub = cmp > 0;
  if (sub) {  // X - M, M = P_k (uniform limbs), two's complement over LC limbs
    const uint32_t* M = g_ptab + (int64_t)k * LPS;
    uint32_t borrow = 0;
#pragma unroll
    for (int l = 0; l < LC; ++l) {
      const uint64_t d = (uint64_t)X[l] - M[l] - borrow;
      X[l] = (uint32_t)d;
      borrow = (uint32_t)(d >> 63);
    }
  }
  if (!live) return;
  uint32_t* out = ws + J.out_off + (int64_t)t * J.L;
  const int L = J.L;
#pragma unroll
  for (int l = 0; l < LC; ++l)
    if (l < L) out[l] = X[l];
  for (int l = LC; l < L; ++l) out[l] = sub ? 0xffffffffu : 0u;
}

void launch_crt_small(int cls, const ResJob* jobs_d, const int32_t* job_list_d, const int64_t* prefix_d, int njobs,
                      int64_t nblocks, uint32_t* ws, hipStream_t s) {
  if (nblocks <= 0) return;
  const dim3 g((unsigned)nblocks), blk(64);
  switch (CRT_SMALL_K[cls]) {
    case 32: hipLaunchKernelGGL(k_crt_small<32>, g, blk, 0, s, jobs_d, job_list_d, prefix_d, njobs, ws); break;
    case 64: hipLaunchKernelGGL(k_crt_small<64>, g, blk, 0, s, jobs_d, job_list_d, prefix_d, njobs, ws); break;
    default: hipLaunchKernelGGL(k_crt_small<128>, g, blk, 0, s, jobs_d, job_list_d, prefix_d, njobs, ws); break;
  }
}

void launch_crt_digits(const CrtTables& tb, const ResJob* jobs_d, const int32_t* job_list_d, const int64_t* prefix_d,
                       int njobs, int64_t nblocks, uint32_t* ws, hipStream_t s) {
  if (nblocks <= 0) return;
  hipLaunchKernelGGL(k_crt_digits, dim3((unsigned)nblocks), dim3(64 * CRT_COEF_PER_BLOCK), 0, s, tb,
                     jobs_d, job_list_d, prefix_d, njobs, ws);
}

void launch_crt_combine(const CrtTables& tb, const ResJob* jobs_d, const int32_t* job_list_d, const int64_t* prefix_d,
                        int njobs, int64_t nblocks, int kmax, uint32_t* ws, hipStream_t s) {
  if (nblocks <= 0) return;
  const int lxm = lx_of(kmax);
  const size_t shmem = (size_t)CRT_COMB_PER_BLOCK * 3 * lxm * sizeof(uint32_t);
  static_assert((size_t)CRT_COMB_PER_BLOCK * 3 * ((30 * KMAX + 31) / 32 + 2) * 4 <= 160 * 1024,
                "combination buffers for the whole table fit the LDS of a CU");
  hipLaunchKernelGGL(k_crt_combine, dim3((unsigned)nblocks), dim3(64 * CRT_COEF_PER_BLOCK), shmem, s, tb, jobs_d,
                     job_list_d, prefix_d, njobs, lxm, ws);
}

CrtTables global_crt_tables() {
  static CrtTables cache[64];
  static bool have[64] = {false};
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev >= 0 && dev < 64 && have[dev]) return cache[dev];
  CrtTables t{};
  void* p = nullptr;
  (void)hipGetSymbolAddress(&p, HIP_SYMBOL(g_primes)); t.primes = (const PrimeC*)p;
  (void)hipGetSymbolAddress(&p, HIP_SYMBOL(g_garner)); t.garner = (const uint32_t*)p;
  (void)hipGetSymbolAddress(&p, HIP_SYMBOL(g_wtab)); t.wtab = (const uint32_t*)p;
  (void)hipGetSymbolAddress(&p, HIP_SYMBOL(g_ptab)); t.ptab = (const uint32_t*)p;
  t.wstride = KMAX;
  t.pstride = LPS;
  if (dev >= 0 && dev < 64) { cache[dev] = t; have[dev] = true; }
  return t;
}

void launch_ffact_init(hipStream_t s) {
  static_assert(IFF_K <= KMAX, "falling-factorial table covers table primes only");
  hipLaunchKernelGGL(k_ffact_init, dim3(IFF_K), dim3(256), 0, s);
}

}  // namespace snc
