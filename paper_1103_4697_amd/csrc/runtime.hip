// Host runtime of libsnc: the C ABI of snc.h for resultants, the modulus
// tables, planning (degree and coefficient bounds, number of primes),
// workspace layout and the launch sequence of the device pipeline.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "bigint.hpp"
#include "runtime_internal.hpp"
#include "snc.h"
#include "snc_internal.hpp"

namespace snc {

// ---------------------------------------------------------------------------
// Modulus table: the KMAX largest primes below 2^30, descending, with their
// Montgomery constants and the CRT tables derived from them.
// ---------------------------------------------------------------------------
static uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) { return (unsigned __int128)a * b % m; }
static uint64_t powmod64(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = mulmod64(r, a, m);
    a = mulmod64(a, a, m);
    e >>= 1;
  }
  return r;
}
// deterministic Miller-Rabin for n < 3,215,031,751 (bases 2, 3, 5, 7)
static bool is_prime_u32(uint32_t n) {
  if (n < 2) return false;
  for (uint32_t q : {2u, 3u, 5u, 7u}) {
    if (n % q == 0) return n == q;
  }
  uint32_t d = n - 1;
  int s = 0;
  while (!(d & 1)) { d >>= 1; ++s; }
  for (uint32_t a : {2u, 3u, 5u, 7u}) {
    uint64_t x = powmod64(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; ++r) {
      x = mulmod64(x, x, n);
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}

static uint32_t mont_of(uint64_t v, uint32_t p) { return (uint32_t)(((v % p) << 32) % p); }

const Tables& tables() {
  static Tables T;
  static std::once_flag once;
  std::call_once(once, [] {
    T.p.reserve(KMAX);
    for (uint32_t n = (1u << 30) - 1; (int)T.p.size() < KMAX; n -= 2)
      if (is_prime_u32(n)) T.p.push_back(n);
    T.pc.resize(KMAX);
    T.lg.assign(KMAX + 1, 0.0);
    for (int i = 0; i < KMAX; ++i) {
      uint32_t p = T.p[i], inv = p;
      for (int it = 0; it < 5; ++it) inv *= 2u - p * inv;
      T.pc[i].p = p;
      T.pc[i].pinv = 0u - inv;
      T.pc[i].r1 = (uint32_t)((1ull << 32) % p);
      T.pc[i].r2 = (uint32_t)mulmod64(T.pc[i].r1, T.pc[i].r1, p);
      T.lg[i + 1] = T.lg[i] + std::log2((double)p);
    }
    T.garner.assign(KMAX, 0);
    T.wtab.assign((size_t)KMAX * KMAX, 0);
    for (int i = 0; i < KMAX; ++i) {
      const uint32_t p = T.p[i];
      uint64_t run = 1;  // P_j mod p_i
      for (int j = 0; j < i; ++j) {
        T.wtab[(size_t)j * KMAX + i] = mont_of(run, p);
        run = mulmod64(run, T.p[j], p);
      }
      T.garner[i] = mont_of(powmod64(run, p - 2, p), p);
    }
    T.ptab.assign((size_t)(KMAX + 1) * LPS, 0);
    BigInt P = BigInt::from_u64(1);
    for (int j = 0; j <= KMAX; ++j) {
      for (size_t l = 0; l < P.mag.size() && (int)l < LPS; ++l) T.ptab[(size_t)j * LPS + l] = P.mag[l];
      if (j < KMAX) P = P.mul_small(T.p[j]);
    }
  });
  return T;
}

int ensure_device_tables(int device, std::string& err) {
  static std::mutex mu;
  static std::set<int> done;
  std::lock_guard<std::mutex> lk(mu);
  if (done.count(device)) return SNC_OK;
  const Tables& T = tables();
  hipError_t e = configure_kernels();
  if (e == hipSuccess) e = configure_gcd_kernels();
  if (e == hipSuccess) e = configure_ygcd_kernel();
  if (e != hipSuccess) { err = std::string("kernel attributes: ") + hipGetErrorString(e); return SNC_EDEVICE; }
  e = init_noalloc_scratch(device);
  if (e != hipSuccess) { err = std::string("scratch address: ") + hipGetErrorString(e); return SNC_EDEVICE; }
  upload_tables(T.pc.data(), T.garner.data(), T.wtab.data(), T.ptab.data(), nullptr);
  launch_ifact_init(nullptr);
  launch_crt_small_init(nullptr);
  e = hipDeviceSynchronize();
  if (e != hipSuccess) { err = std::string("table upload: ") + hipGetErrorString(e); return SNC_EDEVICE; }
  (void)global_crt_tables();
  done.insert(device);
  return SNC_OK;
}

// ---------------------------------------------------------------------------
// Planning
// ---------------------------------------------------------------------------
static bool coef_is_zero(const uint32_t* c, int nl) {
  for (int l = 0; l < nl; ++l) if (c[l]) return false;
  return true;
}

// log2 |c| of a non-zero two's-complement coefficient, from its top three
// magnitude limbs (the rest adds less than one unit of the third limb, which
// the caller's margin covers); no overflow at any size
static double coef_log2_abs(const uint32_t* c, int nl) {
  const bool neg = c[nl - 1] >> 31;
  std::vector<uint32_t> m(c, c + nl);
  if (neg) {  // magnitude = ~c + 1
    uint64_t carry = 1;
    for (int l = 0; l < nl; ++l) { uint64_t t = (uint64_t)(~c[l]) + carry; m[l] = (uint32_t)t; carry = t >> 32; }
  }
  int t = nl - 1;
  while (t > 0 && m[t] == 0) --t;
  double v = 0.0;
  int used = 0;
  for (int l = t; l >= 0 && used < 3; --l, ++used) v = v * 4294967296.0 + (double)m[l];
  return std::log2(v + 1.0) + 32.0 * (t + 1 - used);
}

// log2 of a sum of 2^x over xs (xs non-empty)
static double log2_sum_exp2(const std::vector<double>& xs) {
  double mx = xs[0];
  for (double x : xs) mx = std::max(mx, x);
  double s = 0.0;
  for (double x : xs) s += std::exp2(x - mx);
  return mx + std::log2(s);
}

int parse_bipoly(const snc_bipoly* f, Operand& op, std::string& err) {
  if (!f) { err = "null polynomial"; return SNC_EINVAL; }
  op = Operand();
  op.dy = f->dy; op.dx = f->dx; op.nl = f->nlimbs; op.limbs = f->limbs;
  if (f->dy < 0) { op.ydeg = -1; return SNC_OK; }
  if (f->dx < 0 || f->nlimbs < 1 || !f->limbs) { err = "invalid bivariate polynomial (dx < 0, nlimbs < 1 or NULL limbs)"; return SNC_EINVAL; }
  op.rowdeg.assign(f->dy + 1, -1);
  op.ydeg = -1;
  // log2 of S = sum_i ||f_i||_1^2, summed in the log domain (coefficients of any size)
  std::vector<double> rows2;  // 2 log2 ||f_i||_1 of the non-zero rows
  std::vector<double> lc;
  for (int i = 0; i <= f->dy; ++i) {
    lc.clear();
    for (int k = 0; k <= f->dx; ++k) {
      const uint32_t* c = f->limbs + ((size_t)i * (f->dx + 1) + k) * f->nlimbs;
      if (!coef_is_zero(c, f->nlimbs)) {
        op.rowdeg[i] = k;
        lc.push_back(coef_log2_abs(c, f->nlimbs));
      }
    }
    if (op.rowdeg[i] >= 0) {
      op.ydeg = i;
      rows2.push_back(2.0 * log2_sum_exp2(lc));
    }
  }
  op.rowdeg.resize(op.ydeg + 1);
  op.total_deg = -1;
  op.max_rowdeg = -1;
  for (int i = 0; i <= op.ydeg; ++i) {
    if (op.rowdeg[i] < 0) continue;
    op.total_deg = std::max(op.total_deg, i + op.rowdeg[i]);
    op.max_rowdeg = std::max(op.max_rowdeg, op.rowdeg[i]);
  }
  // rounding of the log-domain sums is far below 1e-9 bits per term; the margin makes it an upper bound
  op.log2S = op.ydeg >= 0 ? log2_sum_exp2(rows2) + 1e-9 * (1.0 + std::fabs(log2_sum_exp2(rows2))) : 0.0;
  return SNC_OK;
}

int plan_resultant(const Operand& F, const Operand& G, ResPlan& P, std::string& err) {
  P = ResPlan();
  if (F.ydeg < 0 || G.ydeg < 0) { P.trivial = 1; P.trivial_value = 0; return SNC_OK; }
  if (F.ydeg == 0 && G.ydeg == 0) { P.trivial = 1; P.trivial_value = 1; return SNC_OK; }
  const int m = F.ydeg, n = G.ydeg;
  P.swap = m < n;
  P.m = std::max(m, n);
  P.n = std::min(m, n);
  if (P.m > MAXY_GEN) { err = "y-degree above " + std::to_string(MAXY_GEN) + " is not supported"; return SNC_EINVAL; }
  const int64_t Dw = (int64_t)n * F.total_deg + (int64_t)m * G.total_deg - (int64_t)m * n;
  const int64_t Dr = (int64_t)n * F.max_rowdeg + (int64_t)m * G.max_rowdeg;
  int64_t D = std::max<int64_t>(0, std::min(Dw, Dr));
  if (D > MAX_D) { err = "degree bound " + std::to_string(D) + " exceeds the supported " + std::to_string(MAX_D); return SNC_EINVAL; }
  P.D = (int)D;
  // |coef| <= B = S_f^(n/2) S_g^(m/2); need prod p > 2B and L limbs of two's complement
  P.log2B = 0.5 * ((double)n * F.log2S + (double)m * G.log2S) + 1e-6;
  const Tables& T = tables();
  int k = 1;
  while (k <= KMAX && T.lg[k] <= P.log2B + 1.0 + 1e-6) ++k;
  if (k > KMAX) { err = "coefficient bound needs more than " + std::to_string(KMAX) + " primes"; return SNC_EINVAL; }
  P.k = k;
  P.L = (int)std::ceil((std::max(P.log2B, 0.0) + 2.0) / 32.0);
  if (P.L < 1) P.L = 1;
  P.nl = std::max(F.nl, G.nl);
  P.cls = fast_class_of(P.m);
  const int width = P.cls >= 0 ? fast_class_cap(P.cls) : P.m;
  P.rstride = (width + 1 + ROWGRP - 1) / ROWGRP;
  // residues per prime: rows top-down in groups of four, each group padded to its longest row
  // (rounded up to a whole number of 64-byte chunks)
  P.T = 0;
  for (const Operand* O : {&F, &G}) {
    const int deg = O->ydeg;
    for (int t0 = 0; t0 <= deg; t0 += ROWGRP) {
      int ml = 0;
      for (int q = 0; q < ROWGRP && t0 + q <= deg; ++q) ml = std::max(ml, O->rowdeg[deg - t0 - q] + 1);
      P.T += ROWGRP * padded_group_len(ml);
    }
  }
  return SNC_OK;
}

size_t job_region_words(const ResPlan& P) {
  const size_t n1 = (size_t)P.D + 1;
  return align_words((size_t)P.k * P.T) + align_words((size_t)P.k * n1) + align_words(n1 * P.k) +
         0;
}

}  // namespace snc

using namespace snc;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int snc_version(void) { return 100; }

const char* snc_status_str(int s) {
  switch (s) {
    case SNC_OK: return "ok";
    case SNC_EINVAL: return "invalid argument";
    case SNC_ERANGE: return "output buffer too small";
    case SNC_ENOMEM: return "workspace too small";
    case SNC_EDEVICE: return "device error";
    case SNC_EAGAIN: return "not finished";
    case SNC_EINTERNAL: return "internal error";
    case SNC_ENOTSUP: return "not supported";
    default: return "unknown status";
  }
}

uint32_t snc_prime(int32_t i) {
  if (i < 0 || i >= KMAX) return 0;
  return tables().p[i];
}

int snc_create(int device, snc_ctx** out) {
  if (!out) return SNC_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SNC_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return SNC_EDEVICE;
  snc_ctx* c = new snc_ctx();
  c->device = device;
  int st = ensure_device_tables(device, c->err);
  if (st != SNC_OK) { delete c; return st; }
  *out = c;
  return SNC_OK;
}

int snc_destroy(snc_ctx* c) {
  if (!c) return SNC_EINVAL;
  (void)hipSetDevice(c->device);
  c->release();
  delete c;
  return SNC_OK;
}

const char* snc_last_error(const snc_ctx* c) { return c ? c->err.c_str() : "null context"; }

int snc_set_timing(snc_ctx* c, int enable) {
  if (!c) return SNC_EINVAL;
  c->timing = enable != 0;
  return SNC_OK;
}

int snc_get_timing(const snc_ctx* c, const char** names, float* ms, int32_t* launches, int cap) {
  if (!c) return SNC_EINVAL;
  int n = (int)c->stage_ms.size();
  for (int i = 0; i < n && i < cap; ++i) {
    if (names) names[i] = c->stage_names[i];
    if (ms) ms[i] = c->stage_ms[i];
    if (launches) launches[i] = c->stage_launches[i];
  }
  return n;
}

int snc_set_tuning(snc_ctx* c, int mode) {
  if (!c || mode < 0 || mode > 2) return SNC_EINVAL;
  c->tune_mode = mode;
  return SNC_OK;
}

int snc_set_gcd_variant(snc_ctx* c, int variant) {
  if (!c || variant < 0 || variant > 2) return SNC_EINVAL;
  c->gcd_variant = variant;
  return SNC_OK;
}

int snc_set_eval_variant(snc_ctx* c, int32_t class_cap, int32_t wpe, int32_t chunk) {
  if (!c) return SNC_EINVAL;
  const int cls = fast_class_of(class_cap);
  if (cls < 0 || fast_class_cap(cls) != class_cap || wpe < 0 || wpe > EE_WPE_MAX || chunk < 0 || chunk > 64)
    return SNC_EINVAL;
  c->forced[cls] = EEVariant();
  c->forced[cls].wpe = 0;
  if (wpe > 0) {
    c->forced[cls].wpe = wpe;
    c->forced[cls].chunk = chunk;
  }
  return SNC_OK;
}

int snc_get_tuning(const snc_ctx* c, int32_t* info, float* ms, int cap, float* tune_ms) {
  if (!c) return SNC_EINVAL;
  const int n = (int)c->tune_report.size();
  for (int i = 0; i < n && i < cap; ++i) {
    const EETuneReport& r = c->tune_report[i];
    if (info) {
      int32_t* o = info + 6 * i;
      o[0] = r.cls_cap; o[1] = r.wpe; o[2] = r.chunk; o[3] = (int32_t)r.grid; o[4] = r.source; o[5] = r.candidates;
    }
    if (ms) { ms[2 * i] = r.best_ms; ms[2 * i + 1] = r.default_ms; }
  }
  if (tune_ms) *tune_ms = c->tune_ms;
  return n;
}

int snc_resultant_y_plan(const snc_bipoly* f, const snc_bipoly* g, snc_plan* out) {
  if (!out) return SNC_EINVAL;
  std::string err;
  Operand F, G;
  int st = parse_bipoly(f, F, err);
  if (st) return st;
  st = parse_bipoly(g, G, err);
  if (st) return st;
  ResPlan P;
  st = plan_resultant(F, G, P, err);
  if (st) return st;
  std::vector<ResPlan> plans{P};
  BatchLayout lay;
  layout_batch(plans, lay);
  out->deg_bound = P.trivial ? 0 : P.D;
  out->out_nlimbs = P.trivial ? 1 : P.L;
  out->nprimes = P.trivial ? 0 : P.k;
  out->reserved = 0;
  out->workspace_bytes = lay.dev.empty() ? 0 : lay.total_bytes;
  return SNC_OK;
}

int snc_resultant_y(snc_ctx* c, const snc_bipoly* f, const snc_bipoly* g, void* d_ws,
                    size_t ws_bytes, void* stream, snc_upoly* out) {
  if (!c || !out) return SNC_EINVAL;
  return run_resultants(c, 1, f, g, d_ws, ws_bytes, (hipStream_t)stream, out, /*graph=*/false);
}

int snc_resultant_y_batch_plan(int32_t n, const snc_bipoly* f, const snc_bipoly* g,
                               snc_plan* out_each, snc_plan* out_total) {
  if (n < 0 || (n > 0 && (!f || !g)) || !out_total) return SNC_EINVAL;
  std::vector<ResPlan> plans(n);
  std::string err;
  int maxD = 0, maxL = 1, maxk = 0;
  for (int i = 0; i < n; ++i) {
    Operand F, G;
    int st = parse_bipoly(&f[i], F, err);
    if (st) return st;
    st = parse_bipoly(&g[i], G, err);
    if (st) return st;
    st = plan_resultant(F, G, plans[i], err);
    if (st) return st;
    const ResPlan& P = plans[i];
    if (out_each) {
      out_each[i].deg_bound = P.trivial ? 0 : P.D;
      out_each[i].out_nlimbs = P.trivial ? 1 : P.L;
      out_each[i].nprimes = P.trivial ? 0 : P.k;
      out_each[i].reserved = 0;
      out_each[i].workspace_bytes = 0;
    }
    if (!P.trivial) { maxD = std::max(maxD, P.D); maxL = std::max(maxL, P.L); maxk = std::max(maxk, P.k); }
  }
  BatchLayout lay;
  layout_batch(plans, lay);
  out_total->deg_bound = maxD;
  out_total->out_nlimbs = maxL;
  out_total->nprimes = maxk;
  out_total->reserved = 0;
  out_total->workspace_bytes = lay.dev.empty() ? 0 : lay.total_bytes;
  return SNC_OK;
}

int snc_resultant_y_prepare(snc_ctx* c, int32_t n, const snc_bipoly* f, const snc_bipoly* g,
                            void* d_ws, size_t ws_bytes, void* stream, snc_prepared** out) {
  if (!c || !out || n < 0 || (n > 0 && (!f || !g))) return SNC_EINVAL;
  return prepare_resultants(c, n, f, g, d_ws, ws_bytes, (hipStream_t)stream, /*graph=*/true, out);
}

int snc_prepared_run(snc_prepared* p, void* stream, snc_upoly* out) {
  if (!p || (p->n > 0 && !out)) return SNC_EINVAL;
  return run_prepared(p, (hipStream_t)stream, out);
}

size_t snc_prepared_stage_bytes(const snc_prepared* p) { return p ? prepared_stage_bytes(p) : 0; }

int snc_prepared_submit(snc_prepared* p, void* d_stage, size_t stage_bytes, void* stream, int64_t* ticket) {
  if (!p || !ticket) return SNC_EINVAL;
  return submit_prepared(p, d_stage, stage_bytes, (hipStream_t)stream, ticket);
}

int snc_prepared_collect(snc_prepared* p, int64_t ticket, snc_upoly* out) {
  if (!p || (p->n > 0 && !out)) return SNC_EINVAL;
  return collect_prepared(p, ticket, out);
}

int snc_prepared_destroy(snc_prepared* p) {
  if (!p) return SNC_EINVAL;
  destroy_prepared(p);
  return SNC_OK;
}

int snc_resultant_y_batch(snc_ctx* c, int32_t n, const snc_bipoly* f, const snc_bipoly* g,
                          void* d_ws, size_t ws_bytes, void* stream, snc_upoly* out) {
  if (!c || n < 0 || (n > 0 && (!f || !g || !out))) return SNC_EINVAL;
  return run_resultants(c, n, f, g, d_ws, ws_bytes, (hipStream_t)stream, out, /*graph=*/true);
}

}  // extern "C"
