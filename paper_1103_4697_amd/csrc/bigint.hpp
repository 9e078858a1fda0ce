// Small host-side arbitrary-precision integers (sign + magnitude, 32-bit
// limbs, little endian).  Used on the host for what the modular path leaves
// there: contents and leading-coefficient gcds of gcd inputs, the final
// normalisation of a gcd, products of primes for the CRT tables, and exact
// coefficient bounds.  Division is Knuth's Algorithm D.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

namespace snc {

struct BigInt {
  bool neg = false;
  std::vector<uint32_t> mag;  // no leading zero limbs; empty = 0

  BigInt() = default;
  explicit BigInt(int64_t v) {
    neg = v < 0;
    uint64_t u = neg ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
    while (u) { mag.push_back((uint32_t)u); u >>= 32; }
  }
  static BigInt from_u64(uint64_t u) {
    BigInt r;
    while (u) { r.mag.push_back((uint32_t)u); u >>= 32; }
    return r;
  }
  bool is_zero() const { return mag.empty(); }
  void trim() {
    while (!mag.empty() && mag.back() == 0) mag.pop_back();
    if (mag.empty()) neg = false;
  }
  size_t bitlen() const {
    if (mag.empty()) return 0;
    return 32 * (mag.size() - 1) + (32 - __builtin_clz(mag.back()));
  }

  // two's complement limbs -> BigInt
  static BigInt from_twos(const uint32_t* limbs, int n) {
    BigInt r;
    bool ng = n > 0 && (limbs[n - 1] >> 31);
    r.mag.assign(limbs, limbs + n);
    if (ng) {  // magnitude = ~x + 1
      uint64_t carry = 1;
      for (auto& w : r.mag) { uint64_t t = (uint64_t)(~w) + carry; w = (uint32_t)t; carry = t >> 32; }
      r.neg = true;
    }
    r.trim();
    return r;
  }
  // BigInt -> two's complement limbs (n of them); false if it does not fit
  bool to_twos(uint32_t* out, int n) const {
    if ((int)mag.size() > n) return false;
    for (int i = 0; i < n; ++i) out[i] = i < (int)mag.size() ? mag[i] : 0;
    if (neg) {
      uint64_t carry = 1;
      for (int i = 0; i < n; ++i) { uint64_t t = (uint64_t)(~out[i]) + carry; out[i] = (uint32_t)t; carry = t >> 32; }
      if (n > 0 && !(out[n - 1] >> 31)) return false;
    } else if (n > 0 && (out[n - 1] >> 31)) {
      return false;
    }
    return true;
  }
  // minimal two's-complement limb count
  int twos_limbs() const {
    if (mag.empty()) return 1;
    size_t b = bitlen();
    // a negative power of two -2^(b-1) fits in b bits
    bool pow2 = neg;
    if (pow2) {
      for (size_t i = 0; i + 1 < mag.size(); ++i) if (mag[i]) { pow2 = false; break; }
      if (pow2 && (mag.back() & (mag.back() - 1))) pow2 = false;
    }
    size_t need = pow2 ? b : b + 1;
    return (int)((need + 31) / 32);
  }

  static int cmp_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
    if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
    for (size_t i = a.size(); i-- > 0;)
      if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
  }
  static std::vector<uint32_t> add_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
    const auto& x = a.size() >= b.size() ? a : b;
    const auto& y = a.size() >= b.size() ? b : a;
    std::vector<uint32_t> r(x.size() + 1);
    uint64_t c = 0;
    for (size_t i = 0; i < x.size(); ++i) {
      c += (uint64_t)x[i] + (i < y.size() ? y[i] : 0);
      r[i] = (uint32_t)c; c >>= 32;
    }
    r[x.size()] = (uint32_t)c;
    while (!r.empty() && r.back() == 0) r.pop_back();
    return r;
  }
  // |a| >= |b|
  static std::vector<uint32_t> sub_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
    std::vector<uint32_t> r(a.size());
    int64_t br = 0;
    for (size_t i = 0; i < a.size(); ++i) {
      int64_t t = (int64_t)a[i] - (i < b.size() ? b[i] : 0) - br;
      br = t < 0; r[i] = (uint32_t)(t + (br << 32));
    }
    while (!r.empty() && r.back() == 0) r.pop_back();
    return r;
  }
  friend BigInt operator+(const BigInt& a, const BigInt& b) {
    BigInt r;
    if (a.neg == b.neg) { r.mag = add_mag(a.mag, b.mag); r.neg = a.neg; }
    else {
      int c = cmp_mag(a.mag, b.mag);
      if (c == 0) return BigInt();
      if (c > 0) { r.mag = sub_mag(a.mag, b.mag); r.neg = a.neg; }
      else { r.mag = sub_mag(b.mag, a.mag); r.neg = b.neg; }
    }
    r.trim();
    return r;
  }
  BigInt operator-() const { BigInt r = *this; if (!r.is_zero()) r.neg = !r.neg; return r; }
  friend BigInt operator-(const BigInt& a, const BigInt& b) { return a + (-b); }
  friend BigInt operator*(const BigInt& a, const BigInt& b) {
    BigInt r;
    if (a.is_zero() || b.is_zero()) return r;
    r.mag.assign(a.mag.size() + b.mag.size(), 0);
    for (size_t i = 0; i < a.mag.size(); ++i) {
      uint64_t c = 0;
      for (size_t j = 0; j < b.mag.size(); ++j) {
        uint64_t t = (uint64_t)a.mag[i] * b.mag[j] + r.mag[i + j] + c;
        r.mag[i + j] = (uint32_t)t; c = t >> 32;
      }
      r.mag[i + b.mag.size()] = (uint32_t)c;
    }
    r.neg = a.neg != b.neg;
    r.trim();
    return r;
  }
  BigInt mul_small(uint32_t s) const {
    BigInt r; if (s == 0 || is_zero()) return r;
    r.mag.resize(mag.size() + 1);
    uint64_t c = 0;
    for (size_t i = 0; i < mag.size(); ++i) { uint64_t t = (uint64_t)mag[i] * s + c; r.mag[i] = (uint32_t)t; c = t >> 32; }
    r.mag[mag.size()] = (uint32_t)c; r.neg = neg; r.trim();
    return r;
  }
  // |x| mod s
  uint32_t mod_small(uint32_t s) const {
    uint64_t r = 0;
    for (size_t i = mag.size(); i-- > 0;) r = ((r << 32) | mag[i]) % s;
    return (uint32_t)r;
  }
  // x mod s in [0, s) for signed x
  uint32_t smod(uint32_t s) const {
    uint32_t r = mod_small(s);
    return (neg && r) ? s - r : r;
  }
  // truncated division of magnitudes (Knuth D); q = |a| / |b|, r = |a| mod |b|
  static void divmod_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b,
                         std::vector<uint32_t>& q, std::vector<uint32_t>& r) {
    if (cmp_mag(a, b) < 0) { q.clear(); r = a; return; }
    if (b.size() == 1) {
      q.assign(a.size(), 0);
      uint64_t rem = 0;
      for (size_t i = a.size(); i-- > 0;) { uint64_t cur = (rem << 32) | a[i]; q[i] = (uint32_t)(cur / b[0]); rem = cur % b[0]; }
      while (!q.empty() && q.back() == 0) q.pop_back();
      r.clear(); if (rem) r.push_back((uint32_t)rem);
      return;
    }
    int s = __builtin_clz(b.back());
    size_t n = b.size(), m = a.size() - n;
    std::vector<uint32_t> v(n), u(a.size() + 1);
    for (size_t i = n; i-- > 0;) v[i] = (b[i] << s) | (s && i ? (uint32_t)(b[i - 1] >> (32 - s)) : 0);
    u[a.size()] = s ? (uint32_t)(a.back() >> (32 - s)) : 0;
    for (size_t i = a.size(); i-- > 0;) u[i] = (a[i] << s) | (s && i ? (uint32_t)(a[i - 1] >> (32 - s)) : 0);
    q.assign(m + 1, 0);
    for (size_t j = m + 1; j-- > 0;) {
      uint64_t num = ((uint64_t)u[j + n] << 32) | u[j + n - 1];
      uint64_t qhat = num / v[n - 1], rhat = num % v[n - 1];
      while (qhat >= (1ull << 32) || qhat * v[n - 2] > ((rhat << 32) | u[j + n - 2])) {
        --qhat; rhat += v[n - 1];
        if (rhat >= (1ull << 32)) break;
      }
      int64_t borrow = 0; uint64_t carry = 0;
      for (size_t i = 0; i < n; ++i) {
        uint64_t p = qhat * v[i] + carry; carry = p >> 32;
        int64_t t = (int64_t)u[i + j] - (int64_t)(uint32_t)p - borrow;
        borrow = t < 0; u[i + j] = (uint32_t)(t + (borrow << 32));
      }
      int64_t t = (int64_t)u[j + n] - (int64_t)carry - borrow;
      borrow = t < 0; u[j + n] = (uint32_t)(t + (borrow << 32));
      if (borrow) {
        --qhat; uint64_t c = 0;
        for (size_t i = 0; i < n; ++i) { uint64_t s2 = (uint64_t)u[i + j] + v[i] + c; u[i + j] = (uint32_t)s2; c = s2 >> 32; }
        u[j + n] += (uint32_t)c;
      }
      q[j] = (uint32_t)qhat;
    }
    while (!q.empty() && q.back() == 0) q.pop_back();
    r.assign(n, 0);
    for (size_t i = 0; i < n; ++i) r[i] = (u[i] >> s) | (s ? (uint32_t)((uint64_t)u[i + 1] << (32 - s)) : 0);
    while (!r.empty() && r.back() == 0) r.pop_back();
  }
  // truncated division: a = q*b + r, |r| < |b|, sign(r) = sign(a)
  static void divmod(const BigInt& a, const BigInt& b, BigInt& q, BigInt& r) {
    divmod_mag(a.mag, b.mag, q.mag, r.mag);
    q.neg = a.neg != b.neg; r.neg = a.neg;
    q.trim(); r.trim();
  }
  // x * v for an unsigned 64-bit v (sign of x kept)
  static BigInt mul_u64(const BigInt& x, uint64_t v) {
    BigInt r = x.mul_small((uint32_t)v);
    const uint32_t hi = (uint32_t)(v >> 32);
    if (hi && !x.is_zero()) {
      BigInt t = x.mul_small(hi);
      t.mag.insert(t.mag.begin(), 0u);
      r = r + t;
    }
    return r;
  }
  // floor(|x| / 2^shift) truncated to 64 bits
  static uint64_t bits_at(const BigInt& x, size_t shift) {
    const size_t w = shift / 32, b = shift % 32;
    unsigned __int128 acc = 0;  // words w..w+2

    for (int i = 2; i >= 0; --i) {
      const size_t k = w + (size_t)i;
      acc = (acc << 32) | (k < x.mag.size() ? x.mag[k] : 0u);
    }
    return (uint64_t)(acc >> b);
  }
  static uint64_t mod_u64(const BigInt& x, uint64_t m) {
    unsigned __int128 r = 0;
    for (size_t i = x.mag.size(); i-- > 0;) r = ((r << 32) | x.mag[i]) % m;
    return (uint64_t)r;
  }
  // gcd by Lehmer's method: the leading 62 bits drive runs of Euclid steps
  // with 64-bit cofactors, applied to the full numbers as one linear
  // combination; a full division step when the run makes no progress.
  static BigInt gcd(BigInt a, BigInt b) {
    a.neg = b.neg = false;
    if (cmp_mag(a.mag, b.mag) < 0) std::swap(a, b);
    while (b.mag.size() > 2) {
      const size_t n = a.bitlen();
      const size_t shift = n > 62 ? n - 62 : 0;
      __int128 ah = (__int128)bits_at(a, shift), bh = (__int128)bits_at(b, shift);
      __int128 A = 1, B = 0, C = 0, D = 1;
      while (bh + C != 0 && bh + D != 0) {
        const __int128 q1 = (ah + A) / (bh + C), q2 = (ah + B) / (bh + D);
        if (q1 != q2) break;
        __int128 T = A - q1 * C; A = C; C = T;
        T = B - q1 * D; B = D; D = T;
        T = ah - q1 * bh; ah = bh; bh = T;
      }
      if (B == 0) {
        BigInt q, r;
        divmod(a, b, q, r);
        r.neg = false;
        a = std::move(b);
        b = std::move(r);
      } else {
        auto term = [](const BigInt& x, __int128 c) {
          BigInt t = mul_u64(x, (uint64_t)(c < 0 ? -c : c));
          return c < 0 ? -t : t;
        };
        BigInt na = term(a, A) + term(b, B);
        BigInt nb = term(a, C) + term(b, D);
        na.neg = nb.neg = false;
        a = std::move(na);
        b = std::move(nb);
      }
      if (cmp_mag(a.mag, b.mag) < 0) std::swap(a, b);
    }
    if (b.is_zero()) return a;
    uint64_t bb = 0;
    for (size_t i = b.mag.size(); i-- > 0;) bb = (bb << 32) | b.mag[i];
    uint64_t aa = mod_u64(a, bb);
    while (aa) { uint64_t t = bb % aa; bb = aa; aa = t; }
    return BigInt::from_u64(bb);
  }
  double log2_abs() const {  // approximate log2 |x|, -inf-ish for 0
    if (mag.empty()) return -1.0;
    size_t n = mag.size();
    double top = (double)mag[n - 1];
    if (n >= 2) top = top * 4294967296.0 + mag[n - 2];
    if (n >= 3) top = top * 4294967296.0 + mag[n - 3];
    int used = n >= 3 ? 3 : (int)n;
    return __builtin_log2(top) + 32.0 * (double)(n - used);
  }
  std::string to_string() const {  // decimal, for messages and tests
    if (mag.empty()) return "0";
    std::vector<uint32_t> m = mag; std::string s;
    while (!m.empty()) {
      uint64_t rem = 0;
      for (size_t i = m.size(); i-- > 0;) { uint64_t cur = (rem << 32) | m[i]; m[i] = (uint32_t)(cur / 1000000000u); rem = cur % 1000000000u; }
      while (!m.empty() && m.back() == 0) m.pop_back();
      char buf[16]; snprintf(buf, sizeof buf, m.empty() ? "%u" : "%09u", (unsigned)rem);
      s = std::string(buf) + s;
    }
    return neg ? "-" + s : s;
  }
};

}  // namespace snc
