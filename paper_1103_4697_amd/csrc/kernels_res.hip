// HIP kernels of the multi-modular resultant res_y(f, g) (Section 4,
// "Symbolic Speedups": modular and evaluation homomorphisms, one problem per
// (prime, point) over Z_p, interpolation and Chinese remaindering), written
// for gfx950: 64-wide wavefronts, full-rate 32-bit multiplies, LDS staging.
#include <hip/hip_runtime.h>

#include "snc_internal.hpp"

namespace snc {

// ---------------------------------------------------------------------------
// Constant tables (filled once per device by upload_tables)
// ---------------------------------------------------------------------------
__device__ PrimeC g_primes[KMAX];
__device__ uint32_t g_garner[KMAX];            // Montgomery form of (P_i mod p_i)^-1
__device__ uint32_t g_wtab[KMAX * KMAX];       // [j*KMAX + i] = Montgomery form of P_j mod p_i (j < i)
__device__ uint32_t g_ptab[(KMAX + 1) * LPS];  // row j: P_j = prod_{l<j} p_l, little-endian limbs

__global__ void k_interp(const ResJob* jobs, const int64_t* prefix, int njobs, uint32_t* ws);

// per-device kernel attributes (called once per device before any launch)
hipError_t configure_kernels() {
  return hipFuncSetAttribute((const void*)k_interp, hipFuncAttributeMaxDynamicSharedMemorySize,
                             160 * 1024);
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

// block index -> job index: largest jj with prefix[jj] <= b (prefix[0] = 0)
__device__ __forceinline__ int find_job(const int64_t* prefix, int njobs, int64_t b) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
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
                                                        uint32_t* wsw) {
  const int64_t b = blockIdx.x;
  const int jj = find_job(prefix, njobs, b);
  const ResJob J = jobs[jj];
  const int nb = (J.T + RED_THREADS - 1) / RED_THREADS;
  const int64_t lb = b - prefix[jj];
  const int pi = (int)(lb / nb);
  const int t = (int)(lb % nb) * RED_THREADS + threadIdx.x;
  if (t >= J.T) return;
  const PrimeC c = g_primes[pi];
  const uint32_t* limbs = ws + J.coef_off + (int64_t)t * J.nl;
  const uint32_t mask = (limbs[J.nl - 1] >> 31) ? 0xffffffffu : 0u;
  uint32_t acc = 0;
  for (int l = J.nl - 1; l >= 0; --l) {
    uint64_t v = (uint64_t)acc * c.r2 + (uint64_t)(limbs[l] ^ mask) * c.r2;
    acc = redc(v, c.p, c.pinv);
  }
  acc = canon(acc, c.p);
  if (mask) acc = mneg(madd(acc, c.r1, c.p), c.p);  // -(~x + 1)
  wsw[J.res_off + (int64_t)pi * J.T + t] = acc;
}

void launch_reduce(const ResJob* jobs_d, const int64_t* blk_prefix_d, int njobs, int64_t nblocks,
                   const uint32_t* ws, uint32_t* res_base, hipStream_t s) {
  if (nblocks <= 0) return;
  hipLaunchKernelGGL(k_reduce, dim3((unsigned)nblocks), dim3(RED_THREADS), 0, s, jobs_d,
                     blk_prefix_d, njobs, ws, res_base);
}

// ---------------------------------------------------------------------------
// (2)+(3) Evaluation at x_j = j fused with the univariate resultant mod p.
//
// One (prime, point) instance per lane: a wavefront holds 64 consecutive
// points of one prime, so every coefficient residue is uniform across the
// wavefront (scalar loads) and the 64 lanes run the same elimination in
// lockstep with no cross-lane traffic.  The values F_i(x_j), G_i(x_j) live
// in two register arrays, top-aligned (index 0 = leading coefficient).
//
// Elimination: Euclid's remainder sequence with the formal degrees m >= n,
// division-free.  One elementary step replaces X by lc(Y) X - lc(X) x^k Y,
// which cancels the leading term; s = deg X - deg Y + 1 of them give the
// pseudo-remainder prem = lc(Y)^s (X mod Y).  With
//   res(X, Y) = (-1)^{deg X deg Y} lc(Y)^{deg X - deg R} res(Y, R)
// and res(Y, c R) = c^{deg Y} res(Y, R), a remainder of the expected degree
// deg Y - 1 contributes the factor lc(Y)^{-s (deg Y - 1)}, collected in one
// denominator that is inverted once at the end.  The last step is
// res(X, c) = c^{deg X}.  A lane whose leading coefficients vanish at its
// point (formal degree not attained, or a remainder of lower degree) is
// queued for the general elimination below; the schedule stays uniform.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t horner_row(const uint32_t* coef, int len, uint32_t X,
                                               uint32_t p, uint32_t pinv) {
  uint32_t acc = 0;
#pragma nounroll
  for (int i = len - 1; i >= 0; --i) acc = mhorner(acc, X, coef[i], p, pinv);
  return acc;
}

// One remainder step X <- prem(X, Y) on the first C+1 entries of the
// register arrays (X of formal degree a <= C, Y of degree b >= 1, entries
// above each degree zero).  Branch-free inside an elementary step.
template <int N, int C>
__device__ __forceinline__ void rem_c(uint32_t (&X)[N + 1], const uint32_t (&Y)[N + 1], int a, int b,
                                      int s, bool& ok, uint32_t& den, const PrimeC& c) {
  const uint32_t lcY = canon(Y[0], c.p);
#pragma nounroll
  for (int e = 0; e < s; ++e) {
    const uint32_t nlX = c.p - canon(X[0], c.p);
#pragma unroll
    for (int i = 0; i < C; ++i) X[i] = mmul2(lcY, X[i + 1], nlX, Y[i + 1], c.p, c.pinv);
    X[C] = 0;
  }
  if (canon(X[0], c.p) == 0) ok = false;
  den = mmulc(den, mpow(lcY, (uint32_t)(s * (b - 1)), c), c.p, c.pinv);
}

// Remainder pairs (dividend B, divisor A) while the divisor degree bb stays
// >= C - 8, on arrays of width C; then the next narrower phase.
template <int N, int C>
__device__ __forceinline__ void elim_phases(uint32_t (&A)[N + 1], uint32_t (&B)[N + 1], int& a,
                                            int& bb, bool& ok, uint32_t& den, int& sg,
                                            const PrimeC& c) {
#pragma nounroll
  while (bb >= 2 && bb >= C - 8) {
    rem_c<N, C>(B, A, a, bb, 2, ok, den, c);  // B <- prem(B, A), degree bb-1
    sg ^= (a & bb & 1); a = bb; bb -= 1;
    rem_c<N, C>(A, B, a, bb, 2, ok, den, c);  // A <- prem(A, B), degree bb-1
    sg ^= (a & bb & 1); a = bb; bb -= 1;
  }
  if constexpr (C > 8) elim_phases<N, C - 8>(A, B, a, bb, ok, den, sg, c);
}

template <int N>
__global__ __launch_bounds__(EE_BLOCK) void k_eval_elim(const ResJob* jobs, const int32_t* job_list,
                                                        const int64_t* prefix, int njobs,
                                                        const RowDesc* rows, uint32_t* ws,
                                                        uint32_t* abn_count, AbnEntry* abn_list,
                                                        uint32_t abn_cap) {
  const int64_t b = blockIdx.x;
  const int jj = find_job(prefix, njobs, b);
  const int jid = job_list[jj];
  const ResJob J = jobs[jid];
  const int npb = (J.D + EE_BLOCK) / EE_BLOCK;
  const int64_t lb = b - prefix[jj];
  const int pi = (int)(lb / npb);
  const int j = (int)(lb % npb) * EE_BLOCK + threadIdx.x;
  if (j > J.D) return;
  const PrimeC c = g_primes[pi];
  const uint32_t* r = ws + J.res_off + (int64_t)pi * J.T;
  const uint32_t X = to_mont((uint32_t)j, c);
  // rows are padded to N+1 per operand (length 0 above the degree): no branches
  const RowDesc* ra = rows + J.rows_off;
  const RowDesc* rb = ra + J.rstride;  // J.rstride == N + 1 on this path
  uint32_t A[N + 1], B[N + 1];
#pragma unroll
  for (int t = 0; t <= N; ++t) A[t] = horner_row(r + ra[t].off, ra[t].len, X, c.p, c.pinv);
#pragma unroll
  for (int t = 0; t <= N; ++t) B[t] = horner_row(r + rb[t].off, rb[t].len, X, c.p, c.pinv);

  bool ok = canon(A[0], c.p) != 0;
  if (J.n >= 1 && canon(B[0], c.p) == 0) ok = false;
  uint32_t den = c.r1;
  int sg = J.sign;
  int a = J.m, bb = J.n;
  uint32_t res;
  if (bb < 1) {
    res = mpow(B[0], (uint32_t)a, c);
  } else {
    // first remainder: A <- prem(A, B) with s = m - n + 1 elementary steps
    rem_c<N, N>(A, B, a, bb, a - bb + 1, ok, den, c);
    sg ^= (a & bb & 1); a = bb; bb -= 1;
    // from here on: dividend B (degree a), divisor A (degree bb)
    elim_phases<N, N>(A, B, a, bb, ok, den, sg, c);
    if (bb == 1) {
      rem_c<N, 8>(B, A, a, bb, 2, ok, den, c);
      sg ^= (a & bb & 1); a = bb; bb -= 1;
      res = mpow(B[0], (uint32_t)a, c);
    } else {
      res = mpow(A[0], (uint32_t)a, c);
    }
  }
  res = mmulc(res, minv(den, c), c.p, c.pinv);
  if (sg) res = mneg(res, c.p);
  ws[J.val_off + (int64_t)pi * (J.D + 1) + j] = ok ? res : 0u;
  if (!ok) {
    uint32_t idx = atomicAdd(abn_count, 1u);
    if (idx < abn_cap) abn_list[idx] = AbnEntry{jid, pi, j, 0};
  }
}

static const int kClassCap[] = {8, 16, 32, 48, 64};

int fast_class_of(int maxy) {
  for (int i = 0; i < (int)(sizeof(kClassCap) / sizeof(int)); ++i)
    if (maxy <= kClassCap[i]) return i;
  return -1;
}
int fast_class_cap(int cls) { return kClassCap[cls]; }

void launch_eval_elim(int cls, const ResJob* jobs_d, const int32_t* job_list_d,
                      const int64_t* blk_prefix_d, int njobs, int64_t nblocks, const RowDesc* rows_d,
                      uint32_t* ws, uint32_t* abn_count, AbnEntry* abn_list, uint32_t abn_cap,
                      hipStream_t s) {
  if (nblocks <= 0) return;
  dim3 g((unsigned)nblocks), blk(EE_BLOCK);
  switch (kClassCap[cls]) {
    case 8: hipLaunchKernelGGL(k_eval_elim<8>, g, blk, 0, s, jobs_d, job_list_d, blk_prefix_d, njobs, rows_d, ws, abn_count, abn_list, abn_cap); break;
    case 16: hipLaunchKernelGGL(k_eval_elim<16>, g, blk, 0, s, jobs_d, job_list_d, blk_prefix_d, njobs, rows_d, ws, abn_count, abn_list, abn_cap); break;
    case 32: hipLaunchKernelGGL(k_eval_elim<32>, g, blk, 0, s, jobs_d, job_list_d, blk_prefix_d, njobs, rows_d, ws, abn_count, abn_list, abn_cap); break;
    case 48: hipLaunchKernelGGL(k_eval_elim<48>, g, blk, 0, s, jobs_d, job_list_d, blk_prefix_d, njobs, rows_d, ws, abn_count, abn_list, abn_cap); break;
    default: hipLaunchKernelGGL(k_eval_elim<64>, g, blk, 0, s, jobs_d, job_list_d, blk_prefix_d, njobs, rows_d, ws, abn_count, abn_list, abn_cap); break;
  }
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

__device__ void general_instance(const ResJob& J, const RowDesc* rows, uint32_t* ws, int pi, int j) {
  const PrimeC c = g_primes[pi];
  const uint32_t* r = ws + J.res_off + (int64_t)pi * J.T;
  const uint32_t X = to_mont((uint32_t)j, c);
  const RowDesc* ra = rows + J.rows_off;
  const RowDesc* rb = ra + J.rstride;
  uint32_t F[MAXY_GEN + 1], G[MAXY_GEN + 1];
  for (int t = 0; t <= J.m; ++t) F[J.m - t] = canon(horner_row(r + ra[t].off, ra[t].len, X, c.p, c.pinv), c.p);
  for (int t = 0; t <= J.n; ++t) G[J.n - t] = canon(horner_row(r + rb[t].off, rb[t].len, X, c.p, c.pinv), c.p);
  uint32_t res = res_general(F, J.m, G, J.n, c);
  if (J.sign) res = mneg(res, c.p);
  ws[J.val_off + (int64_t)pi * (J.D + 1) + j] = res;
}

__global__ void k_elim_general(const ResJob* jobs, const RowDesc* rows, uint32_t* ws,
                               const uint32_t* abn_count, const AbnEntry* list) {
  const uint32_t cnt = *abn_count;
  for (uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x; idx < cnt; idx += gridDim.x * blockDim.x) {
    const AbnEntry e = list[idx];
    const ResJob J = jobs[e.job];
    general_instance(J, rows, ws, e.prime, e.point);
  }
}

void launch_elim_general(const ResJob* jobs_d, const RowDesc* rows_d, uint32_t* ws,
                         const uint32_t* abn_count, const AbnEntry* abn_list, int nthreads,
                         hipStream_t s) {
  int blocks = (nthreads + 63) / 64;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_elim_general, dim3(blocks), dim3(64), 0, s, jobs_d, rows_d, ws, abn_count, abn_list);
}

__global__ void k_elim_general_all(const ResJob* jobs, const int32_t* job_list,
                                   const int64_t* prefix, int njobs, int64_t ninst,
                                   const RowDesc* rows, uint32_t* ws) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < ninst;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int jj = find_job(prefix, njobs, idx);
    const ResJob J = jobs[job_list[jj]];
    const int64_t li = idx - prefix[jj];
    general_instance(J, rows, ws, (int)(li / (J.D + 1)), (int)(li % (J.D + 1)));
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
//     (resultant, prime).  Newton coefficients of equispaced data are
//     a_k = (Delta^k v_0) / k! = sum_{i<=k} (v_i / i!) * ((-1)^{k-i} / (k-i)!),
//     a convolution that every thread evaluates independently; the Newton
//     form is then expanded by P <- P (x - k) + a_k, k = D..0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(INTERP_THREADS) void k_interp(const ResJob* jobs, const int64_t* prefix,
                                                           int njobs, uint32_t* ws) {
  extern __shared__ uint32_t sm[];
  const int64_t b = blockIdx.x;
  const int jj = find_job(prefix, njobs, b);
  const ResJob J = jobs[jj];
  const int pi = (int)(b - prefix[jj]);
  const PrimeC c = g_primes[pi];
  const int n1 = J.D + 1;
  uint32_t* V = ws + J.val_off + (int64_t)pi * n1;
  uint32_t* s0 = sm;
  uint32_t* s1 = sm + n1;
  uint32_t* s2 = sm + 2 * n1;
  const int tid = threadIdx.x;

  // factorials by an inclusive prefix product (Hillis-Steele, double-buffered)
  for (int t = tid; t < n1; t += INTERP_THREADS) s0[t] = t ? to_mont((uint32_t)t, c) : c.r1;
  __syncthreads();
  uint32_t* in = s0;
  uint32_t* out = s1;
  for (int off = 1; off < n1; off <<= 1) {
    for (int t = tid; t < n1; t += INTERP_THREADS)
      out[t] = t >= off ? mmulc(in[t], in[t - off], c.p, c.pinv) : in[t];
    __syncthreads();
    uint32_t* tmp = in; in = out; out = tmp;
  }
  // in = factorials; inverse factorials into s2
  for (int t = tid; t < n1; t += INTERP_THREADS) s2[t] = minv(in[t], c);
  __syncthreads();
  // u_i = v_i / i!  (s0),  w_j = (-1)^j / j!  (s1)
  for (int t = tid; t < n1; t += INTERP_THREADS) {
    const uint32_t inv = s2[t];
    s0[t] = mmulc(canon(V[t], c.p), inv, c.p, c.pinv);
    s1[t] = (t & 1) ? mneg(inv, c.p) : inv;
  }
  __syncthreads();
  // a_k = sum_{i<=k} u_i w_{k-i}, 64-bit lazy accumulation, reduce every 8 terms
  for (int kk = tid; kk < n1; kk += INTERP_THREADS) {
    uint32_t sum = 0;
    int i = 0;
    while (i <= kk) {
      uint64_t acc = 0;
      const int e = min(kk, i + 7);
      for (; i <= e; ++i) acc += (uint64_t)s0[i] * s1[kk - i];
      sum = madd(sum, canon(redc(acc, c.p, c.pinv), c.p), c.p);
    }
    s2[kk] = sum;
  }
  __syncthreads();
  // Newton form -> monomials: P <- P (x - k) + a_k
  in = s0;
  out = s1;
  if (tid == 0) in[0] = s2[J.D];
  __syncthreads();
  for (int kk = J.D - 1; kk >= 0; --kk) {
    const int len = J.D - kk;  // current length of P
    const uint32_t nk = mneg(to_mont((uint32_t)kk, c), c.p);
    const uint32_t ak = s2[kk];
    for (int t = tid; t <= len; t += INTERP_THREADS) {
      const uint32_t prev = t >= 1 ? in[t - 1] : 0u;
      const uint32_t cur = t < len ? in[t] : 0u;
      uint32_t q = canon(mmul2(c.r1, prev, nk, cur, c.p, c.pinv), c.p);
      if (t == 0) q = madd(q, ak, c.p);
      out[t] = q;
    }
    __syncthreads();
    uint32_t* tmp = in; in = out; out = tmp;
  }
  for (int t = tid; t < n1; t += INTERP_THREADS) V[t] = from_mont(in[t], c);
}

void launch_interp(const ResJob* jobs_d, const int64_t* blk_prefix_d, int njobs, int64_t nblocks,
                   int max_D, uint32_t* ws, hipStream_t s) {
  if (nblocks <= 0) return;
  size_t shmem = (size_t)3 * (max_D + 1) * sizeof(uint32_t);
  hipLaunchKernelGGL(k_interp, dim3((unsigned)nblocks), dim3(INTERP_THREADS), shmem, s, jobs_d,
                     blk_prefix_d, njobs, ws);
}

// ---------------------------------------------------------------------------
// (5) Chinese remaindering per coefficient.
//   digits: Garner's mixed-radix digits y_j, X = sum_j y_j P_j, with
//     y_i = (r_i - sum_{j<i} y_j P_j) (P_i)^-1 mod p_i.  One wavefront per
//     coefficient; lane l owns primes l, l+64, ...; digit j is broadcast
//     from its owner lane and every later prime folds it in.
//   combine: X in binary by Horner over the digits; the balanced value is
//     X - M when X > (M-1)/2, decided on the digits ((M-1)/2 has digits
//     (p_j - 1)/2), written as L two's-complement limbs.
// ---------------------------------------------------------------------------
constexpr int CRT_SLOTS = KMAX / 64;

__global__ __launch_bounds__(64 * CRT_COEF_PER_BLOCK) void k_crt_digits(CrtTables tb, const ResJob* jobs,
                                                                        const int64_t* prefix,
                                                                        int njobs, uint32_t* ws) {
  const int64_t b = blockIdx.x;
  const int jj = find_job(prefix, njobs, b);
  const ResJob J = jobs[jj];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = (int)(b - prefix[jj]) * CRT_COEF_PER_BLOCK + wave;
  if (t > J.D) return;
  const int k = J.k;
  const int n1 = J.D + 1;
  const uint32_t* V = ws + J.val_off;
  uint32_t* dig = ws + J.dig_off + (int64_t)t * k;
  uint32_t r[CRT_SLOTS], S[CRT_SLOTS];
#pragma unroll
  for (int s = 0; s < CRT_SLOTS; ++s) {
    const int i = lane + 64 * s;
    r[s] = 0; S[s] = 0;
    if (64 * s < k && i < k) r[s] = V[(int64_t)i * n1 + t];
  }
#pragma unroll
  for (int s = 0; s < CRT_SLOTS; ++s) {
    if (64 * s >= k) break;
    const int i0 = lane + 64 * s;
    const PrimeC c0 = tb.primes[i0 < k ? i0 : 0];
    const uint32_t g0 = tb.garner[i0 < k ? i0 : 0];
    for (int q = 0; q < 64; ++q) {
      const int j = 64 * s + q;
      if (j >= k) break;
      const uint32_t cand = canon(redc((uint64_t)msub(r[s], S[s], c0.p) * g0, c0.p, c0.pinv), c0.p);
      const uint32_t y = __builtin_amdgcn_readlane(cand, q);
      if (lane == q) dig[j] = y;
#pragma unroll
      for (int s2 = 0; s2 < CRT_SLOTS; ++s2) {
        if (64 * s2 >= k) break;
        if (64 * s2 + 63 <= j) continue;
        const int i = lane + 64 * s2;
        if (i > j && i < k) {
          const PrimeC ci = tb.primes[i];
          const uint32_t w = tb.wtab[(int64_t)j * tb.wstride + i];
          S[s2] = madd(S[s2], canon(redc((uint64_t)y * w, ci.p, ci.pinv), ci.p), ci.p);
        }
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_crt_combine(CrtTables tb, const ResJob* jobs, const int64_t* prefix,
                                                     int njobs, uint32_t* ws) {
  const int64_t b = blockIdx.x;
  const int jj = find_job(prefix, njobs, b);
  const ResJob J = jobs[jj];
  const int t = (int)(b - prefix[jj]) * 256 + threadIdx.x;
  if (t > J.D) return;
  const int k = J.k;
  const int lx = lx_of(k);
  const uint32_t* d = ws + J.dig_off + (int64_t)t * k;
  uint32_t* X = ws + J.acc_off + (int64_t)t * lx;
  int len = 1;
  X[0] = d[k - 1];
  for (int j = k - 2; j >= 0; --j) {
    const uint32_t p = tb.primes[j].p;
    uint64_t carry = d[j];
    for (int l = 0; l < len; ++l) {
      const uint64_t v = (uint64_t)X[l] * p + carry;
      X[l] = (uint32_t)v;
      carry = v >> 32;
    }
    if (carry) X[len++] = (uint32_t)carry;
  }
  for (int l = len; l < lx; ++l) X[l] = 0;
  int cmp = 0;
  for (int j = k - 1; j >= 0; --j) {
    const uint32_t h = (tb.primes[j].p - 1) >> 1;
    if (d[j] != h) { cmp = d[j] > h ? 1 : -1; break; }
  }
  uint32_t* out = ws + J.out_off + (int64_t)t * J.L;
  if (cmp > 0) {  // X - M, M = P_k
    const uint32_t* M = tb.ptab + (int64_t)k * tb.pstride;
    int64_t borrow = 0;
    for (int l = 0; l < lx; ++l) {
      const uint32_t ml = l < tb.pstride ? M[l] : 0u;
      int64_t v = (int64_t)X[l] - ml - borrow;
      borrow = v < 0;
      X[l] = (uint32_t)(v + (borrow << 32));
    }
  }
  for (int l = 0; l < J.L; ++l) out[l] = l < lx ? X[l] : ((cmp > 0) ? 0xffffffffu : 0u);
}

void launch_crt_digits(const CrtTables& tb, const ResJob* jobs_d, const int64_t* prefix_d, int njobs,
                       int64_t nblocks, uint32_t* ws, hipStream_t s) {
  if (nblocks <= 0) return;
  hipLaunchKernelGGL(k_crt_digits, dim3((unsigned)nblocks), dim3(64 * CRT_COEF_PER_BLOCK), 0, s, tb,
                     jobs_d, prefix_d, njobs, ws);
}

void launch_crt_combine(const CrtTables& tb, const ResJob* jobs_d, const int64_t* prefix_d, int njobs,
                        int64_t nblocks, uint32_t* ws, hipStream_t s) {
  if (nblocks <= 0) return;
  hipLaunchKernelGGL(k_crt_combine, dim3((unsigned)nblocks), dim3(256), 0, s, tb, jobs_d, prefix_d,
                     njobs, ws);
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

}  // namespace snc
