// Device code of the register-resident Euclid mod p (one wavefront per
// (problem, prime)), shared by the gcd kernels of the modular gcd in Z[x]
// and the blocked Euclid of the square-free check (Section 2.1: gcd(R, R')).
#pragma once

#include <hip/hip_runtime.h>

#include "snc_internal.hpp"

namespace snc {

// where the fused check writes e and d: mapped host memory when given, else the workspace
__device__ __forceinline__ int32_t* fused_out(const GcdDesc& G, uint32_t* ws) {
  return G.ed_out ? G.ed_out : (int32_t*)ws;
}

// ---------------------------------------------------------------------------
// Register-resident variant: one wavefront per prime, degrees below 64*E.
// Polynomials are top-aligned (element i = coefficient of x^(deg-i)) and
// lane-blocked (element i in lane i/E, slot i%E), values lazy in [0, 4p).
// An elementary Euclid step X <- lc(Y) X - lc(X) x^(dX-dY) Y pairs X[i] with
// Y[i] (tops aligned) and shifts X down one element: E fused updates per
// lane plus one lane shift, no LDS and no barrier.  Leading coefficients are
// read from lane 0.  Exact division by the monic gcd is the same step with
// lc(Y) = 1 and the quotient coefficient as lc(X).
// ---------------------------------------------------------------------------
// the register Euclid runs on one wavefront: ordering its own LDS stores and
// loads across lanes needs no workgroup barrier (a wavefront's LDS operations
// complete in order), only that the compiler keeps them in program order
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t from_next_lane(uint32_t v) {  // lane l gets lane l+1 (0 for lane 63)
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130 /* wave_shl:1 */, 0xf, 0xf, true);
}
__device__ __forceinline__ uint32_t lead(uint32_t v0, uint32_t p) {
  return canon((uint32_t)__builtin_amdgcn_readfirstlane((int)v0), p);
}

template <int E>
__device__ __forceinline__ void reg_step(uint32_t (&X)[E], const uint32_t (&Y)[E], uint32_t lcY, uint32_t nlX,
                                         const PrimeC& c) {
  const uint32_t t0 = mmul2(lcY, X[0], nlX, Y[0], c.p, c.pinv);
#pragma unroll
  for (int s = 0; s + 1 < E; ++s) X[s] = mmul2(lcY, X[s + 1], nlX, Y[s + 1], c.p, c.pinv);
  X[E - 1] = from_next_lane(t0);
}

template <int E>
__device__ __forceinline__ void reg_shift(uint32_t (&X)[E]) {
  const uint32_t n0 = from_next_lane(X[0]);
#pragma unroll
  for (int s = 0; s + 1 < E; ++s) X[s] = X[s + 1];
  X[E - 1] = n0;
}

// drop vanishing leading coefficients: returns the degree
template <int E>
__device__ __forceinline__ int reg_trim(uint32_t (&X)[E], int d, const PrimeC& c) {
  while (d >= 0 && lead(X[0], c.p) == 0) { reg_shift<E>(X); --d; }
  return d;
}


// The normal remainder step (deg X = deg Y + 1) as one update: the pseudo-
// remainder lc(Y)^2 X - (lc(Y) lc(X) x + lc(Y) X_1 - lc(X) Y_1) Y, top-aligned
// at degree deg Y - 1, is R[i] = a X[i+2] + b Y[i+2] + cc Y[i+1] with
// a = lc(Y)^2, b = -lc(Y) lc(X), cc = lc(X) Y_1 - lc(Y) X_1.  Elements i+1,
// i+2 past the last slot come from the first two slots of the next lane.
template <int E>
__device__ __forceinline__ void reg_step2(uint32_t (&X)[E], const uint32_t (&Y)[E], uint32_t a, uint32_t b,
                                          uint32_t cc, const PrimeC& c) {
  static_assert(E >= 2, "two slots per lane");
  const uint32_t nx0 = from_next_lane(X[0]), nx1 = from_next_lane(X[1]);
  const uint32_t ny0 = from_next_lane(Y[0]), ny1 = from_next_lane(Y[1]);
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const uint32_t x2 = s + 2 < E ? X[s + 2] : (s + 2 == E ? nx0 : nx1);
    const uint32_t y2 = s + 2 < E ? Y[s + 2] : (s + 2 == E ? ny0 : ny1);
    const uint32_t y1 = s + 1 < E ? Y[s + 1] : ny0;
    X[s] = mmul3(a, x2, b, y2, cc, y1, c.p, c.pinv);
  }
}

// reduce X by Y until deg X < deg Y (Y fixed, deg Y >= 0)
template <int E>
__device__ __forceinline__ int reg_reduce(uint32_t (&X)[E], int dX, const uint32_t (&Y)[E], int dY,
                                          const PrimeC& c) {
  const uint32_t lcY = lead(Y[0], c.p);
  const uint32_t y1 = lead(Y[1], c.p);
  const uint32_t a = mmulc(lcY, lcY, c.p, c.pinv);
  while (dX >= dY) {
    const uint32_t lcX = lead(X[0], c.p);
    if (dX == dY + 1 && dY >= 1) {
      const uint32_t x1 = lead(X[1], c.p);
      const uint32_t b = mneg(mmulc(lcY, lcX, c.p, c.pinv), c.p);
      const uint32_t cc = msub(mmulc(lcX, y1, c.p, c.pinv), mmulc(lcY, x1, c.p, c.pinv), c.p);
      reg_step2<E>(X, Y, a, b, cc, c);
      dX = reg_trim<E>(X, dX - 2, c);
    } else {
      reg_step<E>(X, Y, lcY, c.p - lcX, c);
      dX = reg_trim<E>(X, dX - 1, c);
    }
  }
  return dX;
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

// Multipliers of the fused step from the top pairs (p0, p1) of the dividend
// and (q0, q1) of the divisor (p0, q0 canonical, p1, q1 below 4p), computed
// on the vector unit with lane 0's values (other lanes compute garbage that
// is never read) and then made uniform: cheaper than the same Montgomery
// products on the scalar unit.
__device__ __forceinline__ void step2_coefs(uint32_t p0, uint32_t p1, uint32_t q0, uint32_t q1, uint32_t& a,
                                            uint32_t& b, uint32_t& cc, const PrimeC& c) {
  a = uni(mmulc(q0, q0, c.p, c.pinv));
  b = uni(mmulc(q0, c.p - p0, c.p, c.pinv));  // -q0 p0 (p - p0 in (0, p])
  // p0 q1 - q0 p1 with one reduction: the sum stays below 8 p^2, its reduction below 3p
  cc = uni(canon(redc((uint64_t)p0 * q1 + (uint64_t)(c.p - q0) * p1, c.p, c.pinv), c.p));
}

// One normal remainder step X <- prem(X, Y) (multipliers a, b, cc) fused
// with the multipliers of the step after it, Y <- prem(Y, X): those come
// from the top pair (p0, p1) of Y, which this step leaves unchanged, and the
// new top pair of X.  The two top slots are updated first and the next
// multipliers computed from them, so that their dependent chain (products,
// reductions, broadcasts) overlaps the updates of the other slots instead of
// following them.  (nx0, nx1) and (ny0, ny1) are the first two slots of the
// next lane of X and Y: Y's carry over from the step that last changed Y, and
// X's are refreshed here for the steps after this one.  Returns the new
// leading coefficient of X (canonical, lane 0's value is the one used) and
// its second coefficient in x1; a, b, cc become the next step's multipliers.
template <int E>
__device__ __forceinline__ uint32_t reg_step2_next(uint32_t (&X)[E], const uint32_t (&Y)[E], uint32_t& nx0,
                                                   uint32_t& nx1, uint32_t ny0, uint32_t ny1, uint32_t& a,
                                                   uint32_t& b, uint32_t& cc, uint32_t p0, uint32_t p1,
                                                   uint32_t& x1, const PrimeC& c) {
  static_assert(E >= 2, "two slots per lane");
  auto slot = [&](int s) {
    const uint32_t x2 = s + 2 < E ? X[s + 2] : (s + 2 == E ? nx0 : nx1);
    const uint32_t y2 = s + 2 < E ? Y[s + 2] : (s + 2 == E ? ny0 : ny1);
    const uint32_t y1 = s + 1 < E ? Y[s + 1] : ny0;
    X[s] = mmul3(a, x2, b, y2, cc, y1, c.p, c.pinv);
  };
  slot(0);
  slot(1);
  const uint32_t x0 = canon(X[0], c.p);
  x1 = X[1];
  uint32_t na, nb, ncc;
  step2_coefs(p0, p1, x0, x1, na, nb, ncc, c);
#pragma unroll
  for (int s = 2; s < E; ++s) slot(s);
  nx0 = from_next_lane(X[0]);
  nx1 = from_next_lane(X[1]);
  a = na;
  b = nb;
  cc = ncc;
  return x0;
}

// Runs of normal remainder steps (each remainder one degree below its
// divisor) with fixed register roles: X <- prem(X, Y), then Y <- prem(Y, X).
// Each step hands the next one its multipliers (computed from the divisor's
// top pair, carried over from the step that produced it, and the new
// remainder's).  Returns at the first step that is not normal (the general
// loop takes over), or once both degrees are below dstop.
template <int E>
__device__ __forceinline__ void normal_run(uint32_t (&X)[E], int& dX, uint32_t (&Y)[E], int& dY, int dstop,
                                           const PrimeC& c) {
  if (dX != dY + 1 || dY < 1) return;
  // leading coefficients canonical, second coefficients lazy: every product
  // below pairs a canonical factor with one below 4p
  uint32_t x0 = canon(X[0], c.p), x1 = X[1];
  uint32_t y0 = canon(Y[0], c.p), y1 = Y[1];
  uint32_t nx0 = from_next_lane(X[0]), nx1 = from_next_lane(X[1]);
  uint32_t ny0 = from_next_lane(Y[0]), ny1 = from_next_lane(Y[1]);
  uint32_t a, b, cc;
  step2_coefs(x0, x1, y0, y1, a, b, cc, c);
  while (true) {
    x0 = reg_step2_next<E>(X, Y, nx0, nx1, ny0, ny1, a, b, cc, y0, y1, x1, c);
    dX -= 2;
    if (uni(x0) == 0) { dX = reg_trim<E>(X, dX, c); return; }
    if (dX < 1 || dY < dstop) return;
    y0 = reg_step2_next<E>(Y, X, ny0, ny1, nx0, nx1, a, b, cc, x0, x1, y1, c);
    dY -= 2;
    if (uni(y0) == 0) { dY = reg_trim<E>(Y, dY, c); return; }
    if (dY < 1 || dX < dstop) return;
  }
}

// Slots per lane of the register arrays, largest first.  The Euclid loop
// moves to the next smaller count once both remainders fit, so the work of a
// step follows the current degree instead of the input degree.
__host__ __device__ constexpr int next_slots(int E) {
  return E == 32 ? 24 : E == 24 ? 16 : E == 16 ? 12 : E == 12 ? 9 : E >= 3 && E <= 9 ? E - 1 : 0;
}

template <int E>
__device__ __forceinline__ void reg_store(const uint32_t (&X)[E], uint32_t* sm, int lane) {
#pragma unroll
  for (int s = 0; s < E; ++s) sm[lane * E + s] = X[s];
}

// elements 0..d from sm (element order), zeros above
template <int E>
__device__ __forceinline__ void reg_fetch(uint32_t (&X)[E], const uint32_t* sm, int d, int lane) {
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int i = lane * E + s;
    X[s] = i <= d ? sm[i] : 0u;
  }
}

// Euclid's remainder sequence from (X, Y); the last non-zero remainder
// (lazy, top-aligned) is left in sm[0..e] and e is returned.  sm holds
// 2 * 64 * E words.
template <int E>
__device__ __forceinline__ int euclid_levels(uint32_t (&X)[E], int dX, uint32_t (&Y)[E], int dY, uint32_t* sm, int lane,
                             const PrimeC& c) {
  constexpr int EN = next_slots(E);
  constexpr int dstop = 64 * EN;
  while (true) {
    normal_run<E>(X, dX, Y, dY, dstop, c);
    if (dY < 0) { reg_store<E>(X, sm, lane); return dX; }
    if (dX >= dY) dX = reg_reduce<E>(X, dX, Y, dY, c);
    if (dX < 0) { reg_store<E>(Y, sm, lane); return dY; }
    dY = reg_reduce<E>(Y, dY, X, dX, c);
    if constexpr (EN > 0) {
      if (dX < dstop && dY < dstop) {
        reg_store<E>(X, sm, lane);
        reg_store<E>(Y, sm + 64 * E, lane);
        wave_sync();
        uint32_t XN[EN], YN[EN];
        reg_fetch<EN>(XN, sm, dX, lane);
        reg_fetch<EN>(YN, sm + 64 * E, dY, lane);
        wave_sync();
        return euclid_levels<EN>(XN, dX, YN, dY, sm, lane, c);
      }
    }
  }
}

// coefficients 0..deg of a residue row, top-aligned, through LDS: consecutive
// lanes load consecutive words (each load instruction touches a few cache
// lines instead of one per lane), then every lane takes its block of E
template <int E>
__device__ __forceinline__ void reg_load_staged(uint32_t (&X)[E], const uint32_t* row, int deg, uint32_t* sm, int lane) {
  for (int t = lane; t <= deg; t += 64) sm[t] = row[t];
  wave_sync();
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int i = lane * E + s;
    X[s] = i <= deg ? sm[deg - i] : 0u;
  }
  wave_sync();
}

// load coefficients 0..deg of a residue row (scaled by sc) top-aligned
template <int E>
__device__ __forceinline__ void reg_load(uint32_t (&X)[E], const uint32_t* row, int deg, int lane) {
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int i = lane * E + s;
    X[s] = i <= deg ? row[deg - i] : 0u;
  }
}

}  // namespace snc
