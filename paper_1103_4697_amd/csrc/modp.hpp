// Arithmetic modulo a word-size prime for the modular resultant and gcd.
//
// The method of Section 4 ("Symbolic Speedups") maps the integer problem to
// many problems over prime fields Z_p.  Here every prime satisfies
// 2^29 < p < 2^30 and residues are kept in Montgomery form (v * 2^32 mod p).
//
// Lazy reduction: operands may be any value in [0, 3p).  With p < 2^30 the
// products used below stay within 64 bits and REDC maps them back into
// [0, 3p) without a final conditional subtraction:
//   redc(t) = (t + ((t mod 2^32) * pinv mod 2^32) * p) / 2^32,  pinv = -p^-1
//   t < 6 p^2      ->  redc(t) < 6p^2/2^32 + p < 2.5 p
//   t < 3 p^2 + p 2^32 -> redc(t) < 2.75 p
// Only leading coefficients (zero tests, scale factors) are brought to the
// canonical range [0, p).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

struct PrimeC {
  uint32_t p;     // the prime, 2^29 < p < 2^30
  uint32_t pinv;  // -p^-1 mod 2^32
  uint32_t r1;    // 2^32 mod p   (Montgomery form of 1)
  uint32_t r2;    // 2^64 mod p   (converts plain -> Montgomery)
};

__device__ __forceinline__ uint32_t redc(uint64_t t, uint32_t p, uint32_t pinv) {
  uint32_t m = (uint32_t)t * pinv;
  uint32_t r = (uint32_t)((t + (uint64_t)m * p) >> 32);
  // Opaque 32-bit result: keeps the compiler from carrying it as a 64-bit
  // value into the next product (which costs an extra 64x32 multiply-add).
  asm("" : "+v"(r));
  return r;
}

// redc whose result is copied into a register of its own.  The reduction's
// result is the high word of a 64-bit register pair; kernels that keep long
// arrays of residues in registers would otherwise hold each residue in half
// a pair (64-bit temporaries need aligned pairs), doubling their register
// use.  One extra move per reduction.
__device__ __forceinline__ uint32_t redc_mv(uint64_t t, uint32_t p, uint32_t pinv) {
  const uint32_t m = (uint32_t)t * pinv;
  const uint32_t r = (uint32_t)((t + (uint64_t)m * p) >> 32);
  uint32_t rr;
  asm volatile("v_mov_b32 %0, %1" : "=v"(rr) : "v"(r));
  return rr;
}

// a*b in Montgomery form, a,b in [0,3p) -> [0, 2p)
__device__ __forceinline__ uint32_t mmul(uint32_t a, uint32_t b, uint32_t p, uint32_t pinv) {
  return redc((uint64_t)a * b, p, pinv);
}

// a*b + c*d (Montgomery), a,c canonical-ish (<= p), b,d < 3p  ->  [0, 2.5p)
// (b,d < 4p -> [0, 3p))
__device__ __forceinline__ uint32_t mmul2(uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                                          uint32_t p, uint32_t pinv) {
  uint64_t t = (uint64_t)a * b + (uint64_t)c * d;
  return redc(t, p, pinv);
}

// a x + b y + c z with a, b, c canonical and x, y, z < 4p: the sum stays
// below 12 p^2 + 2^32 p < 2^64 (p < 2^30) and the result below 4p.
__device__ __forceinline__ uint32_t mmul3(uint32_t a, uint32_t x, uint32_t b, uint32_t y, uint32_t cc,
                                          uint32_t z, uint32_t p, uint32_t pinv) {
  const uint64_t t = (uint64_t)a * x + (uint64_t)b * y + (uint64_t)cc * z;
  return redc(t, p, pinv);
}

// Horner step acc*x + c (Montgomery; c canonical, enters as c * 2^32)
__device__ __forceinline__ uint32_t mhorner(uint32_t acc, uint32_t x, uint32_t c, uint32_t p,
                                            uint32_t pinv) {
  uint64_t t = (uint64_t)acc * x + ((uint64_t)c << 32);
  return redc(t, p, pinv);
}

// [0, 3p) -> [0, p)
__device__ __forceinline__ uint32_t canon(uint32_t x, uint32_t p) {
  uint32_t y = x - 2 * p;
  x = (y < x) ? y : x;  // unsigned min: keeps x when x < 2p (y wrapped)
  y = x - p;
  return (y < x) ? y : x;
}

// [0, 2p) -> [0, p)
__device__ __forceinline__ uint32_t canon2(uint32_t x, uint32_t p) {
  uint32_t y = x - p;
  return (y < x) ? y : x;
}

// canonical a, b -> canonical a + b, a - b, -a
__device__ __forceinline__ uint32_t madd(uint32_t a, uint32_t b, uint32_t p) { return canon2(a + b, p); }
__device__ __forceinline__ uint32_t msub(uint32_t a, uint32_t b, uint32_t p) { return canon2(a + p - b, p); }
__device__ __forceinline__ uint32_t mneg(uint32_t a, uint32_t p) { return a ? p - a : 0; }

// canonical Montgomery product
__device__ __forceinline__ uint32_t mmulc(uint32_t a, uint32_t b, uint32_t p, uint32_t pinv) {
  return canon2(mmul(a, b, p, pinv), p);
}

// plain -> Montgomery (v < 2^32)
__device__ __forceinline__ uint32_t to_mont(uint32_t v, const PrimeC& c) {
  return canon2(redc((uint64_t)v * c.r2, c.p, c.pinv), c.p) ;
}
// Montgomery -> plain canonical
__device__ __forceinline__ uint32_t from_mont(uint32_t v, const PrimeC& c) {
  return canon(redc((uint64_t)v, c.p, c.pinv), c.p);
}

// x^e (Montgomery, canonical result), e >= 0; e is usually uniform across
// the wavefront so the loop is scalar control flow.
__device__ __forceinline__ uint32_t mpow(uint32_t x, uint32_t e, const PrimeC& c) {
  uint32_t r = c.r1;
  x = canon(x, c.p);
  while (e) {
    if (e & 1u) r = mmulc(r, x, c.p, c.pinv);
    e >>= 1;
    if (e) x = mmulc(x, x, c.p, c.pinv);
  }
  return r;
}

// inverse by Fermat (x != 0 mod p)
__device__ __forceinline__ uint32_t minv(uint32_t x, const PrimeC& c) { return mpow(x, c.p - 2, c); }
