// Device code of the fused evaluation + elimination kernel (and the helpers
// it shares with the reduction and the general elimination).  Included by
// the kernel sources; each register class is instantiated in a translation
// unit of its own (eval_elim_c<N>.hip) so that they compile in parallel.
#pragma once
#include <hip/hip_runtime.h>

#include "snc_internal.hpp"

namespace snc {

// Width step of the elimination's register phases: a step of divisor degree
// b computes at most 3 entries beyond its b.  Steps of 8 measured the same on
// the degree-48 class and 4% slower on the degree-32 class; finer steps grow
// the code past what the instruction cache holds.
constexpr int EE_PHASE = 4;

// A zero that the compiler cannot see through.  An array entry set to a
// literal zero inside a loop and multiplied in the next iteration becomes a
// 64-bit loop value whose products take the full 64 x 32 multiply sequence
// (two multiply-adds and two moves instead of one multiply-add).
__device__ __forceinline__ uint32_t zero_v() {
  uint32_t z;
  asm("v_mov_b32 %0, 0" : "=v"(z));
  return z;
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

// signed coefficient of nl two's-complement limbs -> canonical Montgomery residue
// limb l of the coefficient at limbs[l stride] (limb-major: neighbouring
// lanes read neighbouring words)
__device__ __forceinline__ uint32_t reduce_limbs(const uint32_t* limbs, int nl, int64_t stride, const PrimeC& c) {
  const uint32_t mask = (limbs[(nl - 1) * stride] >> 31) ? 0xffffffffu : 0u;
  uint32_t acc = 0;
  for (int l = nl - 1; l >= 0; --l) {
    uint64_t v = (uint64_t)acc * c.r2 + (uint64_t)(limbs[l * stride] ^ mask) * c.r2;
    acc = redc(v, c.p, c.pinv);
  }
  acc = canon(acc, c.p);
  if (mask) acc = mneg(madd(acc, c.r1, c.p), c.p);  // -(~x + 1)
  return acc;
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
// one row q (0..3) of a row group
__device__ __forceinline__ uint32_t horner_grouped(const uint32_t* r, const RowDesc& d, int q, uint32_t X,
                                                   const PrimeC& c) {
  uint32_t acc = 0;
  for (int i = d.len - 1; i >= 0; --i) acc = mhorner(acc, X, r[d.off + ROWGRP * i + q], c.p, c.pinv);
  return acc;
}

// The N+1 rows of one operand evaluated at X, four rows at a time from the
// interleaved group layout: each 64-byte load holds four coefficients of
// four independent rows (instruction-level parallelism for a lone
// wavefront).  A chunk of four coefficients is one step of Horner's rule in
// x^4 with the powers x, x^2, x^3, x^4 kept per lane:
//   acc <- acc x^4 + v0 + v1 x + v2 x^2 + v3 x^3,
// four 64-bit multiply-adds and one reduction, v0 added to its result.  With
// canonical coefficients and powers and acc < 4p the sum stays below 7 p^2,
// the reduction below 2.75p and the result below 4p.  Group lengths are padded at the
// top with zeros, which keep an accumulator at zero.
struct alignas(16) HChunk {
  uint4 v[HCHUNK];
};
static_assert(HCHUNK == 4, "a chunk is four coefficients");

struct XPow {
  uint32_t x1, x2, x3, x4;  // Montgomery forms of x, x^2, x^3, x^4, canonical
};

__device__ __forceinline__ uint32_t hstep4(uint32_t acc, uint32_t v0, uint32_t v1, uint32_t v2, uint32_t v3,
                                           const XPow& xp, const PrimeC& c) {
  uint64_t t = (uint64_t)acc * xp.x4;
  t += (uint64_t)v1 * xp.x1;
  t += (uint64_t)v2 * xp.x2;
  t += (uint64_t)v3 * xp.x3;
  // v0 is added after the reduction, REDC(t + v0 2^32) = REDC(t) + v0: the
  // addition also moves the result out of the 64-bit register pair
  const uint32_t m = (uint32_t)t * c.pinv;
  return (uint32_t)((t + (uint64_t)m * c.p) >> 32) + v0;
}

__device__ __forceinline__ void horner_chunk(uint32_t& a0, uint32_t& a1, uint32_t& a2, uint32_t& a3,
                                             const HChunk& h, const XPow& xp, const PrimeC& c) {
  a0 = hstep4(a0, h.v[0].x, h.v[1].x, h.v[2].x, h.v[3].x, xp, c);
  a1 = hstep4(a1, h.v[0].y, h.v[1].y, h.v[2].y, h.v[3].y, xp, c);
  a2 = hstep4(a2, h.v[0].z, h.v[1].z, h.v[2].z, h.v[3].z, xp, c);
  a3 = hstep4(a3, h.v[0].w, h.v[1].w, h.v[2].w, h.v[3].w, xp, c);
}

// deg: the operand's y-degree.  The group that holds row 0 (index deg) is
// partial unless deg + 1 is a multiple of four; its missing rows would run
// the full length on zeros (that group has the longest rows of a dense
// polynomial), so it takes a loop over its rows that exist only.
template <int N>
__device__ __forceinline__ void eval_rows(uint32_t (&A)[N + 1], const uint32_t* r, const RowDesc* rd, int deg,
                                          const XPow& X, const PrimeC& c) {
#pragma unroll
  for (int t0 = 0; t0 <= N; t0 += ROWGRP) {
    const RowDesc d = rd[t0 / ROWGRP];
    const HChunk* q = reinterpret_cast<const HChunk*>(r + d.off);
    uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    const int nv = deg - t0 + 1;  // rows of the group that exist (uniform)
    if (nv >= ROWGRP) {
      for (int ch = d.len / HCHUNK - 1; ch >= 0; --ch) horner_chunk(a0, a1, a2, a3, q[ch], X, c);
    } else if (nv == 1) {
      for (int ch = d.len / HCHUNK - 1; ch >= 0; --ch) {
        const HChunk& h = q[ch];
        a0 = hstep4(a0, h.v[0].x, h.v[1].x, h.v[2].x, h.v[3].x, X, c);
      }
    } else if (nv == 2) {
      for (int ch = d.len / HCHUNK - 1; ch >= 0; --ch) {
        const HChunk& h = q[ch];
        a0 = hstep4(a0, h.v[0].x, h.v[1].x, h.v[2].x, h.v[3].x, X, c);
        a1 = hstep4(a1, h.v[0].y, h.v[1].y, h.v[2].y, h.v[3].y, X, c);
      }
    } else if (nv == 3) {
      for (int ch = d.len / HCHUNK - 1; ch >= 0; --ch) {
        const HChunk& h = q[ch];
        a0 = hstep4(a0, h.v[0].x, h.v[1].x, h.v[2].x, h.v[3].x, X, c);
        a1 = hstep4(a1, h.v[0].y, h.v[1].y, h.v[2].y, h.v[3].y, X, c);
        a2 = hstep4(a2, h.v[0].z, h.v[1].z, h.v[2].z, h.v[3].z, X, c);
      }
    }
    A[t0] = a0;
    if (t0 + 1 <= N) A[t0 + 1] = a1;
    if (t0 + 2 <= N) A[t0 + 2] = a2;
    if (t0 + 3 <= N) A[t0 + 3] = a3;
  }
}

// Lane state of the elimination: every remainder so far of its expected
// degree (EL_NORMAL); the first remainder whose leading coefficient vanished
// was zero altogether (EL_ZERO: the two polynomials share a factor of
// positive degree at this point, so the resultant is 0); or it was a
// non-zero remainder of lower degree (EL_ABN: the instance goes to the
// general elimination).  Only the first event counts: after a degree drop
// the uniform schedule no longer computes a remainder sequence.
constexpr int EL_NORMAL = 0, EL_ZERO = 1, EL_ABN = 2;

// Check of a new remainder X (entries 0..C, top-aligned) after a step.
// Lanes whose leading coefficient vanished scan the rest of it.  The scan
// sits behind a wavefront-uniform branch (a ballot of those lanes), which is
// almost never taken: a leading coefficient vanishes with probability about
// 1/p per step, so a normal step costs one comparison and no scan.  The
// leading coefficient is left canonical, which the next steps rely on.
template <int N, int C>
__device__ __forceinline__ void lead_check(uint32_t (&X)[N + 1], int& st, const PrimeC& c) {
  X[0] = canon(X[0], c.p);
  const bool z = X[0] == 0 && st == EL_NORMAL;
  if (__builtin_expect(__builtin_amdgcn_ballot_w64(z) != 0, 0)) {
    uint32_t nz = 0;
#pragma unroll
    for (int i = 1; i <= C; ++i) nz |= canon(X[i], c.p);
    if (z) st = nz ? EL_ABN : EL_ZERO;
  }
}

// One remainder X <- prem(X, Y) by s elementary steps on the first C+1
// entries of the register arrays (X of formal degree a <= C, Y of degree
// b >= 1, entries above each degree zero).  Branch-free inside an
// elementary step.  Returns lc(Y), canonical.
template <int N, int C>
__device__ __forceinline__ uint32_t rem_c(uint32_t (&X)[N + 1], const uint32_t (&Y)[N + 1], int s, int& st,
                                          const PrimeC& c) {
  const uint32_t lcY = canon(Y[0], c.p);
#pragma nounroll
  for (int e = 0; e < s; ++e) {
    const uint32_t nlX = c.p - canon(X[0], c.p);
#pragma unroll
    for (int i = 0; i < C; ++i)
      X[i] = redc_mv((uint64_t)lcY * X[i + 1] + (uint64_t)nlX * Y[i + 1], c.p, c.pinv);
    X[C] = zero_v();
  }
  lead_check<N, C>(X, st, c);
  return lcY;
}

// First remainder with a degree gap (s = deg X - deg Y + 1 elementary
// steps, deg Y = b < W): only the window X[0..W-2] meets Y; the entries
// above it are merely multiplied by lc(Y) and shifted down once per step.
// Those are kept unscaled and moved down one register per step, and an
// entry is scaled by lc(Y)^e when it enters the window at step e: one
// update of two products per window entry and one move per entry above,
// instead of the two-product update over the whole width.  The same
// residues as rem_c; after the s steps the entries above the window have
// all been shifted out (they are zero).
template <int N, int W>
__device__ __forceinline__ uint32_t rem_win(uint32_t (&X)[N + 1], const uint32_t (&Y)[N + 1], int s, int& st,
                                            const PrimeC& c) {
  const uint32_t lcY = canon(Y[0], c.p);
  uint32_t pw = c.r1;  // lc(Y)^e
#pragma nounroll
  for (int e = 0; e < s; ++e) {
    const uint32_t nlX = c.p - canon(X[0], c.p);
#pragma unroll
    for (int i = 0; i < W - 1; ++i)
      X[i] = redc_mv((uint64_t)lcY * X[i + 1] + (uint64_t)nlX * Y[i + 1], c.p, c.pinv);
    pw = mmulc(pw, lcY, c.p, c.pinv);
    X[W - 1] = redc_mv((uint64_t)pw * X[W], c.p, c.pinv);
#pragma unroll
    for (int i = W; i < N; ++i) X[i] = X[i + 1];
    X[N] = zero_v();
  }
  lead_check<N, W>(X, st, c);
  return lcY;
}

// rem_win on the narrowest window (N minus a multiple of 8, at least 8)
// with deg Y = b < W
template <int N, int C>
__device__ __forceinline__ uint32_t rem_win_fit(uint32_t (&X)[N + 1], const uint32_t (&Y)[N + 1], int s, int b,
                                                int& st, const PrimeC& c) {
  if constexpr (C - 8 >= 8) {
    if (b < C - 8) return rem_win_fit<N, C - 8>(X, Y, s, b, st, c);
  }
  return rem_win<N, C>(X, Y, s, st, c);
}

// The same remainder for deg X = deg Y + 1 (a normal step, s = 2) as one
// update with the two elementary steps fused:
//   X[i] <- a X[i+2] + b Y[i+2] + cc Y[i+1],  a = lc(Y)^2,  b = -lc(Y) lc(X),
//   cc = lc(X) Y[1] - lc(Y) X[1]
// (entries above C read as zero): 3 products and one reduction per entry
// instead of 4 and 2, the same residues.  Values stay below 4p; the leading
// coefficients X[0], Y[0] are canonical (every step's lead check, and the
// evaluation, leave them so).  With
// deg X <= K + 1 the new remainder (degree deg X - 2) has at most K
// entries: only those are computed, the entries K..C are set to zero.
template <int N, int C, int K>
__device__ __forceinline__ uint32_t rem2_c(uint32_t (&X)[N + 1], const uint32_t (&Y)[N + 1], int& st,
                                           const PrimeC& c) {
  static_assert(K <= C, "at most C entries");
  const uint32_t q0 = Y[0], p0 = X[0];
  const uint32_t a = mmulc(q0, q0, c.p, c.pinv);
  const uint32_t b = mmulc(q0, c.p - p0, c.p, c.pinv);
  // p0 Y[1] - q0 X[1] with one reduction: below 8 p^2, reduced below 3p
  const uint32_t cc = canon(redc((uint64_t)p0 * Y[1] + (uint64_t)(c.p - q0) * X[1], c.p, c.pinv), c.p);
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const uint32_t x2 = i + 2 <= C ? X[i + 2] : 0u;
    const uint32_t y2 = i + 2 <= C ? Y[i + 2] : 0u;
    X[i] = redc_mv((uint64_t)a * x2 + (uint64_t)b * y2 + (uint64_t)cc * Y[i + 1], c.p, c.pinv);
  }
#pragma unroll
  for (int i = K; i <= C; ++i) X[i] = zero_v();
  lead_check<N, C>(X, st, c);
  return q0;
}

// rem2_c on the narrowest width (a multiple of EE_PHASE, at least 8) that
// holds deg X = a
template <int N, int C>
__device__ __forceinline__ uint32_t rem2_fit(uint32_t (&X)[N + 1], const uint32_t (&Y)[N + 1], int a, int& st,
                                             const PrimeC& c) {
  if constexpr (C - EE_PHASE >= 8) {
    if (a <= C - EE_PHASE) return rem2_fit<N, C - EE_PHASE>(X, Y, a, st, c);
  }
  return rem2_c<N, C, C - 1>(X, Y, st, c);
}

// Scale factors of the normal steps.  A normal step with divisor degree b
// (s = 2) contributes y^{2(b-1)}, y = lc(divisor), and b drops by one per
// step, so with prefix products P_j = y_0 ... y_j the whole product is
// (P_0 P_1 ... P_J)^2 over the steps with b >= 2: two products per step, in
// straight-line code, instead of a power per step.  With y canonical the
// unreduced products keep P and Q below 2p (a product below 4p^2 reduces to
// below p^2 2^-30 + p < 2p), which is all the next products need.
__device__ __forceinline__ void scale_step(uint32_t y, int b, uint32_t& P, uint32_t& Q, const PrimeC& c) {
  const uint32_t Pn = mmul(P, y, c.p, c.pinv);
  const uint32_t Qn = mmul(Q, Pn, c.p, c.pinv);
  P = b >= 2 ? Pn : P;
  Q = b >= 2 ? Qn : Q;
}

// Remainder pairs (dividend B, divisor A) on arrays of width C, entered
// with deg B = a <= C, while the divisor degree bb stays >= C - EE_PHASE
// (the narrowest phase, C = 4, runs to the end); then the next narrower
// phase.  The pair's first step has a dividend of degree <= C, its second
// one of degree <= C - 1, so they compute C - 1 and C - 2 entries.
template <int N, int C>
__device__ __forceinline__ void elim_phases(uint32_t (&A)[N + 1], uint32_t (&B)[N + 1], int& a,
                                            int& bb, int& st, uint32_t& P, uint32_t& Q, int& sg,
                                            const PrimeC& c) {
  constexpr int nxt = C - EE_PHASE >= 4 ? C - EE_PHASE : 4;
  constexpr int lo = C > 4 ? nxt : 0;
#pragma nounroll
  while (bb >= 2 && bb >= lo) {
    scale_step(rem2_c<N, C, C - 1>(B, A, st, c), bb, P, Q, c);  // B <- prem(B, A), degree bb-1
    sg ^= (a & bb & 1); a = bb; bb -= 1;
    scale_step(rem2_c<N, C, C - 2>(A, B, st, c), bb, P, Q, c);  // A <- prem(A, B), degree bb-1
    sg ^= (a & bb & 1); a = bb; bb -= 1;
  }
  if constexpr (C > 4) elim_phases<N, nxt>(A, B, a, bb, st, P, Q, sg, c);
}

// One block of the evaluation: 64 consecutive points of one prime of one
// job, one (prime, point) instance per lane.
// LDSROWS: the wavefront first copies its prime's residues into LDS
// (coalesced) and reads the row chunks from there, so the reads pipeline;
// otherwise they are 64-byte scalar loads.  With reduce_in (LDSROWS only)
// the residues are reduced from the input limbs on the way into LDS, and the
// first point block of each prime also stores them for the general
// elimination: no separate reduction launch.  `staged` names the (job,
// prime) whose residues the LDS already holds (-1: none): consecutive
// blocks of one prime stage them once.
template <int N, bool LDSROWS>
__device__ __forceinline__ void eval_elim_block(int64_t b, const PrimeC* primes, const ResJob* jobs,
                                                const int32_t* job_list, const int64_t* prefix, int njobs,
                                                const RowDesc* rows, uint32_t* ws, uint32_t* abn_count,
                                                AbnEntry* abn_list, uint32_t abn_cap, int reduce_in, uint32_t* er,
                                                int64_t& staged) {
  const int jj = find_job(prefix, njobs, b);
  const int jid = job_list[jj];
  const ResJob J = jobs[jid];
  const int npb = (J.D + EE_BLOCK) / EE_BLOCK;
  const int64_t lb = b - prefix[jj];
  const int pi = (int)(lb / npb);
  const int j0 = (int)(lb % npb) * EE_BLOCK + threadIdx.x;
  const bool live = j0 <= J.D;  // lanes past the last point still help stage the rows
  const int j = live ? j0 : J.D;
  const PrimeC c = primes[pi];
  const uint32_t* r = ws + J.res_off + (int64_t)pi * J.T;
  if constexpr (LDSROWS) {
    const int64_t key = (int64_t)jid * KMAX + pi;
    if (key != staged) {  // uniform
      __syncthreads();    // the previous block's reads of the LDS rows are done
      if (reduce_in) {
        uint32_t* rg = ws + J.res_off + (int64_t)pi * J.T;
        const bool store = lb % npb == 0;
        for (int x = threadIdx.x; x < J.T; x += EE_BLOCK) {
          const uint32_t v = reduce_limbs(ws + J.coef_off + x, J.nl, J.T, c);
          er[x] = v;
          if (store) rg[x] = v;
        }
      } else {
        for (int x = threadIdx.x; x < J.T; x += EE_BLOCK) er[x] = r[x];
      }
      __syncthreads();
      staged = key;
    }
    r = er;
  }
  XPow X;
  X.x1 = to_mont((uint32_t)j, c);
  X.x2 = mmulc(X.x1, X.x1, c.p, c.pinv);
  X.x3 = mmulc(X.x2, X.x1, c.p, c.pinv);
  X.x4 = mmulc(X.x2, X.x2, c.p, c.pinv);
  // rows are padded to N+1 per operand (length 0 above the degree): no branches
  const RowDesc* ra = rows + J.rows_off;
  const RowDesc* rb = ra + J.rstride;  // J.rstride == N + 1 on this path
  uint32_t A[N + 1], B[N + 1];
  eval_rows<N>(A, r, ra, J.m, X, c);
  eval_rows<N>(B, r, rb, J.n, X, c);

  // formal degrees attained at this point, else the general elimination
  A[0] = canon(A[0], c.p);
  B[0] = canon(B[0], c.p);
  int st = A[0] != 0 ? EL_NORMAL : EL_ABN;
  if (J.n >= 1 && B[0] == 0) st = EL_ABN;
  uint32_t den = c.r1;
  int sg = J.sign;
  int a = J.m, bb = J.n;
  uint32_t res;
  if (bb < 1) {
    res = mpow(B[0], (uint32_t)a, c);
  } else {
    // first remainder: A <- prem(A, B) with s = m - n + 1 elementary steps,
    // scale lc(B)^{s (n - 1)}
    const int s0 = a - bb + 1;
    // (deg B = N only with deg A = N: the whole width meets B)
    const uint32_t y0 = s0 == 2   ? rem2_fit<N, N>(A, B, a, st, c)
                        : bb < N  ? rem_win_fit<N, N>(A, B, s0, bb, st, c)
                                  : rem_c<N, N>(A, B, s0, st, c);
    den = mpow(y0, (uint32_t)(s0 * (bb - 1)), c);
    sg ^= (a & bb & 1); a = bb; bb -= 1;
    // from here on: dividend B (degree a), divisor A (degree bb)
    uint32_t P = c.r1, Q = c.r1;
    elim_phases<N, N>(A, B, a, bb, st, P, Q, sg, c);
    den = mmulc(den, mmulc(Q, Q, c.p, c.pinv), c.p, c.pinv);
    if (bb == 1) {  // last step: divisor of degree 1, scale y^0
      rem2_c<N, 4, 1>(B, A, st, c);
      sg ^= (a & bb & 1); a = bb; bb -= 1;
      res = mpow(B[0], (uint32_t)a, c);
    } else {
      res = mpow(A[0], (uint32_t)a, c);
    }
  }
  res = mmulc(res, minv(den, c), c.p, c.pinv);
  if (sg) res = mneg(res, c.p);
  if (!live) return;
  // a zero remainder with a divisor of positive degree: res = 0; an
  // abnormal instance leaves a marker (never a residue) for the general pass
  ws[J.pts_off + (int64_t)pi * (J.D + 1) + j] = st == EL_NORMAL ? res : st == EL_ZERO ? 0u : ABN_MARK;
  if (st == EL_ABN) {
    uint32_t idx = atomicAdd(abn_count, 1u);
    if (idx < abn_cap) abn_list[idx] = AbnEntry{jid, pi, j, 0};
  }
}

// Work distribution of a launch.  chunk == 0: one workgroup per block,
// blocks renumbered so that one prime's blocks share an XCD.  chunk > 0: a
// persistent grid (sized to the occupancy of the variant) whose workgroups
// take `chunk` consecutive blocks at a time from the counter, which starts
// at zero; the class's jobs are listed most expensive first, so the last
// blocks to be taken are the cheapest.
struct EEWork {
  uint32_t* counter;
  int32_t chunk;
};

// WPE: minimum wavefronts per SIMD the register allocation is held to
// (1: unconstrained); the variants trade registers (and spills) for
// occupancy, and the autotuner picks one per register class.
template <int N, bool LDSROWS, int WPE>
__global__ __launch_bounds__(EE_BLOCK) __attribute__((amdgpu_waves_per_eu(WPE))) void k_eval_elim(
    const PrimeC* primes, const ResJob* jobs, const int32_t* job_list, const int64_t* prefix, int njobs,
    const RowDesc* rows, uint32_t* ws, uint32_t* abn_count, AbnEntry* abn_list, uint32_t abn_cap, int reduce_in,
    EEWork wk) {
  static_assert(EE_BLOCK == 64, "one wavefront per workgroup (the work counter is broadcast by readfirstlane)");
  extern __shared__ uint4 er4[];  // max T words (LDSROWS)
  uint32_t* er = reinterpret_cast<uint32_t*>(er4);
  int64_t staged = -1;
  if (wk.chunk == 0) {
    eval_elim_block<N, LDSROWS>(xcd_block(blockIdx.x, gridDim.x), primes, jobs, job_list, prefix, njobs, rows,
                                ws, abn_count, abn_list, abn_cap, reduce_in, er, staged);
    return;
  }
  const int64_t nb = prefix[njobs];
  for (;;) {
    uint32_t base = 0;
    if (threadIdx.x == 0) base = atomicAdd(wk.counter, (uint32_t)wk.chunk);
    base = __builtin_amdgcn_readfirstlane(base);
    if ((int64_t)base >= nb) break;
    const int64_t end = (int64_t)base + wk.chunk < nb ? (int64_t)base + wk.chunk : nb;
    for (int64_t b = base; b < end; ++b)
      eval_elim_block<N, LDSROWS>(b, primes, jobs, job_list, prefix, njobs, rows, ws, abn_count, abn_list,
                                  abn_cap, reduce_in, er, staged);
  }
}

// Launch of one register class NN: the variant's kernel (occupancy
// variants wpe 2..4 exist for the classes whose register arrays limit the
// occupancy, 32 and up, with the LDS rows; the others run wpe 1).
template <int NN>
constexpr bool ee_has_wpe_variants() { return NN >= 32; }

template <int NN, bool LDS>
static const void* ee_kernel_ptr(int wpe) {
  if constexpr (LDS && ee_has_wpe_variants<NN>()) {
    switch (wpe) {
      case 2: return (const void*)k_eval_elim<NN, true, 2>;
      case 3: return (const void*)k_eval_elim<NN, true, 3>;
      case 4: return (const void*)k_eval_elim<NN, true, 4>;
      default: break;
    }
  }
  return (const void*)k_eval_elim<NN, LDS, 1>;
}

template <int NN>
int eval_elim_grid_cls(int wpe, int max_T) {
  const bool in_lds = eval_elim_in_lds(max_T);
  const size_t lds = in_lds ? (size_t)max_T * sizeof(uint32_t) : 0;
  const void* k = in_lds ? ee_kernel_ptr<NN, true>(wpe) : ee_kernel_ptr<NN, false>(wpe);
  int per_cu = 0, dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, EE_BLOCK, lds) != hipSuccess) return 0;
  return per_cu * prop.multiProcessorCount;
}

// private (spill) bytes per lane of a variant's kernel, -1 if unknown
template <int NN>
int eval_elim_scratch_cls(int wpe, int max_T) {
  const void* k = eval_elim_in_lds(max_T) ? ee_kernel_ptr<NN, true>(wpe) : ee_kernel_ptr<NN, false>(wpe);
  hipFuncAttributes a;
  if (hipFuncGetAttributes(&a, k) != hipSuccess) return -1;
  return (int)a.localSizeBytes;
}

template <int NN>
void launch_eval_elim_cls(const EEVariant& v, uint32_t* counter, const PrimeC* primes, const ResJob* jobs_d,
                          const int32_t* job_list_d, const int64_t* blk_prefix_d, int njobs, int64_t nblocks,
                          int max_T, const RowDesc* rows_d, uint32_t* ws, uint32_t* abn_count, AbnEntry* abn_list,
                          uint32_t abn_cap, bool reduce_in, hipStream_t s) {
  if (nblocks <= 0) return;
  const bool persistent = v.chunk > 0 && v.grid > 0;
  const dim3 g((unsigned)(persistent ? (v.grid < nblocks ? v.grid : nblocks) : nblocks));
  const bool in_lds = eval_elim_in_lds(max_T);
  const size_t lds = in_lds ? (size_t)max_T * sizeof(uint32_t) : 0;
  const int red = reduce_in && in_lds ? 1 : 0;
  const EEWork wk{counter, persistent ? v.chunk : 0};
  const void* k = in_lds ? ee_kernel_ptr<NN, true>(v.wpe) : ee_kernel_ptr<NN, false>(v.wpe);
  void* args[] = {(void*)&primes, (void*)&jobs_d, (void*)&job_list_d, (void*)&blk_prefix_d, (void*)&njobs,
                  (void*)&rows_d, (void*)&ws, (void*)&abn_count, (void*)&abn_list, (void*)&abn_cap, (void*)&red,
                  (void*)&wk};
  (void)hipLaunchKernel(k, g, dim3(EE_BLOCK), args, lds, s);
}

// one translation unit per register class (eval_elim_c<NN>.hip) instantiates these
#define SNC_EVAL_ELIM_CLASS(NN)                                                                               \
  template int eval_elim_grid_cls<NN>(int, int);                                                              \
  template int eval_elim_scratch_cls<NN>(int, int);                                                           \
  template void launch_eval_elim_cls<NN>(const EEVariant&, uint32_t*, const PrimeC*, const ResJob*,           \
                                         const int32_t*, const int64_t*, int, int64_t, int, const RowDesc*,    \
                                         uint32_t*, uint32_t*, AbnEntry*, uint32_t, bool, hipStream_t);

}  // namespace snc
