// Host side of the modular gcd in Z[x] (snc_gcd_z).
//
// a = cont(a) abar, b = cont(b) bbar; c = gcd(cont a, cont b); beta =
// gcd(lc abar, lc bbar).  For primes p dividing neither cont(a) nor cont(b)
// nor both leading coefficients (i.e. not beta) the device computes
// e_p = deg gcd(abar, bbar) mod p, the monic gcd mod p and the cofactors
// u_p, v_p; w_p = beta * monic gcd is formed when the selected primes are
// gathered (beta is only needed when the gcd is not a constant).  deg gcd over Q <= e_p for every such p, so e_p = 0
// for one prime proves gcd = c.  Otherwise the primes of minimal e_p are kept
// (the others are unlucky), w, u, v are lifted by Chinese remaindering with
// balanced residues, and the result is accepted only if
//   2 ||w||_1 ||u||_1 < M  and  2 ||w||_1 ||v||_1 < M      (M = prod p),
// which forces w u = beta abar and w v = beta bbar over Z, so pp(w) divides
// both and, having degree >= deg gcd, is the gcd.  Otherwise more primes are
// drawn.  The result is c * pp(w) with a positive leading coefficient.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "bigint.hpp"
#include "runtime_internal.hpp"
#include "snc.h"

namespace snc {
namespace {

// host/device phase timing of one gcd call (enabled with snc_set_timing)
struct GcdTimer {
  snc_ctx* c;
  hipStream_t s;
  bool on;
  std::chrono::steady_clock::time_point t0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float dev_ms = 0.f;
  GcdTimer(snc_ctx* c_, hipStream_t s_) : c(c_), s(s_), on(c_->timing) {
    if (on) { c->stage_names.clear(); c->stage_ms.clear(); c->stage_launches.clear(); t0 = std::chrono::steady_clock::now(); }
  }
  void host(const char* name) {
    if (!on) return;
    auto t = std::chrono::steady_clock::now();
    c->stage_names.push_back(name);
    c->stage_ms.push_back(std::chrono::duration<float, std::milli>(t - t0).count());
    c->stage_launches.push_back(0);
    t0 = t;
  }
  void dev_begin() {
    if (!on) return;
    if (!e0) { (void)hipEventCreate(&e0); (void)hipEventCreate(&e1); }
    (void)hipEventRecord(e0, s);
  }
  void dev_end(const char* name, int launches) {  // call after the stream was synchronised
    if (!on) return;
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    c->stage_names.push_back(name);
    c->stage_ms.push_back(ms);
    c->stage_launches.push_back(launches);
    t0 = std::chrono::steady_clock::now();
  }
  ~GcdTimer() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

struct UPoly {
  std::vector<BigInt> c;  // ascending, trimmed
  int deg() const { return (int)c.size() - 1; }
};

int parse_upoly(const snc_upoly* a, UPoly& P, int& nl, std::string& err) {
  if (!a) { err = "null polynomial"; return SNC_EINVAL; }
  P.c.clear();
  nl = 1;
  if (a->deg < 0) return SNC_OK;
  if (a->nlimbs < 1 || !a->limbs) { err = "invalid univariate polynomial (nlimbs < 1 or NULL limbs)"; return SNC_EINVAL; }
  nl = a->nlimbs;
  P.c.resize(a->deg + 1);
  for (int i = 0; i <= a->deg; ++i) P.c[i] = BigInt::from_twos(a->limbs + (size_t)i * nl, nl);
  while (!P.c.empty() && P.c.back().is_zero()) P.c.pop_back();
  return SNC_OK;
}

// |x| mod m for a 32-bit m with a table pw[i] = 2^(32 i) mod m (no divisions per limb)
uint32_t mod_by_table(const BigInt& x, const std::vector<uint64_t>& pw, uint32_t m) {
  unsigned __int128 acc = 0;
  for (size_t i = 0; i < x.mag.size(); ++i) acc += (unsigned __int128)x.mag[i] * pw[i];
  return (uint32_t)(acc % m);
}

BigInt content(const UPoly& P) {
  BigInt g;
  size_t i = 0;
  for (; i < P.c.size(); ++i) {
    g = BigInt::gcd(g, P.c[i]);
    if (g.mag.size() == 1) break;  // non-zero and one word: switch to the table reduction
  }
  if (g.mag.size() != 1) return g;
  // single-limb running gcd: reduce the remaining coefficients through a power table
  uint64_t gg = g.mag[0];
  size_t maxl = 1;
  for (const auto& x : P.c) maxl = std::max(maxl, x.mag.size());
  std::vector<uint64_t> pw(maxl);
  uint64_t table_for = 0;
  for (++i; i < P.c.size() && gg > 1; ++i) {
    if (table_for != gg) {
      uint64_t v = 1;
      for (size_t l = 0; l < maxl; ++l) { pw[l] = v; v = (v << 32) % gg; }
      table_for = gg;
    }
    uint64_t r = mod_by_table(P.c[i], pw, (uint32_t)gg);
    while (r) { uint64_t t = gg % r; gg = r; r = t; }
  }
  return BigInt::from_u64(gg);
}

// log2 of the 2-norm and of the 1-norm (approximate, used only for sizing)
void log2_norms(const UPoly& P, double& l2, double& l1) {
  double mx = -1e300;
  for (const auto& x : P.c) if (!x.is_zero()) mx = std::max(mx, x.log2_abs());
  double s2 = 0.0, s1 = 0.0;
  for (const auto& x : P.c) {
    if (x.is_zero()) continue;
    const double r = std::exp2(x.log2_abs() - mx);
    s2 += r * r;
    s1 += r;
  }
  l2 = mx + 0.5 * std::log2(std::max(s2, 1.0));
  l1 = mx + std::log2(std::max(s1, 1.0));
}

BigInt abs_big(BigInt x) { x.neg = false; return x; }

uint32_t powmod32(uint64_t a, uint64_t e, uint32_t p) {
  uint64_t r = 1;
  a %= p;
  while (e) {
    if (e & 1) r = r * a % p;
    a = a * a % p;
    e >>= 1;
  }
  return (uint32_t)r;
}
uint32_t mont32(uint64_t v, uint32_t p) { return (uint32_t)(((v % p) << 32) % p); }

struct GcdInfo {
  int trivial = 0;           // 1: result computed on the host
  UPoly triv;                // trivial result
  int da = 0, db = 0, nl = 1;
  BigInt ca, cb, c, beta, lca_bar, lcb_bar;
  bool have_beta = false;
  double l2a = 0, l2b = 0, l1a = 0, l1b = 0, lbeta = 0;
  int kmax = 0;
  int deg_bound = 0, out_nlimbs = 1;
};

UPoly normalise_sign(UPoly P) {
  if (!P.c.empty() && P.c.back().neg)
    for (auto& x : P.c) x = -x;
  return P;
}

double bits_needed_full(const GcdInfo& I, int e) {
  const double bw = I.lbeta + e + std::min(I.l2a, I.l2b) + std::log2(e + 1.0);
  const double bu = (I.da - e) + I.l2a + std::log2(I.da - e + 1.0);
  const double bv = (I.db - e) + I.l2b + std::log2(I.db - e + 1.0);
  return bw + std::max(bu, bv) + 2.0;
}

double bits_needed_opt(const GcdInfo& I) {
  return I.lbeta + std::max(I.l1a, I.l1b) + 2.0 * std::log2(std::max(I.da, I.db) + 1.0) + 32.0;
}

int primes_for_bits(double bits) { return (int)std::ceil(bits / 29.99) + 1; }

int analyse(const UPoly& A, const UPoly& B, int nla, int nlb, GcdInfo& I) {
  I = GcdInfo();
  I.nl = std::max(nla, nlb);
  if (A.c.empty() && B.c.empty()) { I.trivial = 1; I.deg_bound = 0; I.out_nlimbs = 1; return SNC_OK; }
  if (A.c.empty() || B.c.empty()) {
    I.trivial = 1;
    I.triv = normalise_sign(A.c.empty() ? B : A);
    I.deg_bound = I.triv.deg();
    int nl = 1;
    for (const auto& x : I.triv.c) nl = std::max(nl, x.twos_limbs());
    I.out_nlimbs = nl;
    return SNC_OK;
  }
  I.ca = content(A);
  I.cb = content(B);
  I.c = BigInt::gcd(I.ca, I.cb);
  if (A.deg() == 0 || B.deg() == 0) {
    I.trivial = 1;
    I.triv.c = {I.c};
    I.deg_bound = 0;
    I.out_nlimbs = I.c.twos_limbs();
    return SNC_OK;
  }
  I.da = A.deg();
  I.db = B.deg();
  BigInt q, r;
  BigInt::divmod(A.c.back(), I.ca, q, r);
  I.lca_bar = abs_big(q);
  BigInt::divmod(B.c.back(), I.cb, q, r);
  I.lcb_bar = abs_big(q);
  // beta divides both leading coefficients: bound its size by the smaller
  I.lbeta = std::min(I.lca_bar.log2_abs(), I.lcb_bar.log2_abs());
  log2_norms(A, I.l2a, I.l1a);
  log2_norms(B, I.l2b, I.l1b);
  const double lca = I.ca.log2_abs(), lcb = I.cb.log2_abs();
  I.l2a -= lca; I.l1a -= lca;
  I.l2b -= lcb; I.l1b -= lcb;
  // Mignotte: a factor of degree e of a has coefficients <= 2^e ||a||_2
  I.deg_bound = std::min(I.da, I.db);
  const double lo = std::min(I.l2a + lca, I.l2b + lcb);
  I.out_nlimbs = (int)std::ceil((I.deg_bound + lo + 3.0) / 32.0) + 1;
  double worst = 0.0;
  for (int e : {0, I.deg_bound}) worst = std::max(worst, bits_needed_full(I, e));
  I.kmax = std::min(KMAX, std::max(primes_for_bits(worst), primes_for_bits(bits_needed_opt(I))) + 12);
  return SNC_OK;
}

struct GcdLayout {
  size_t coef = 0, slot_prime = 0, slot_scale = 0, res = 0, e = 0, w = 0, u = 0, v = 0;   // words
  // CRT area (words)
  size_t primes = 0, garner = 0, wtab = 0, ptab = 0, jobs = 0, prefd = 0, prefc = 0, sel = 0, betas = 0;
  size_t wv = 0, uv = 0, vv = 0, dig = 0, out = 0;
  size_t header_words = 0, crt_header_words = 0, total_words = 0;
  int lpg = 0, lg = 0;
};

void layout_gcd(const GcdInfo& I, GcdLayout& L) {
  const int K = I.kmax, T = I.da + I.db + 2, wl = std::min(I.da, I.db) + 1;
  size_t w = 0;
  L.coef = w; w += align_words((size_t)T * I.nl);
  L.slot_prime = w; w += align_words(K);
  L.slot_scale = w; w += align_words((size_t)3 * K);
  L.header_words = w;
  L.res = w; w += align_words((size_t)K * T);
  L.e = w; w += align_words(K);
  L.w = w; w += align_words((size_t)K * wl);
  L.u = w; w += align_words((size_t)K * (I.da + 1));
  L.v = w; w += align_words((size_t)K * (I.db + 1));
  // CRT tables and jobs for up to K selected primes
  L.lpg = lx_of(K);
  L.lg = lx_of(K);
  const size_t crt0 = w;
  L.primes = w; w += align_words(sizeof(PrimeC) / 4 * K);
  L.garner = w; w += align_words(K);
  L.wtab = w; w += align_words((size_t)K * K);
  L.ptab = w; w += align_words((size_t)(K + 1) * L.lpg);
  L.jobs = w; w += align_words(3 * sizeof(ResJob) / 4);
  L.prefd = w; w += align_words(8);
  L.prefc = w; w += align_words(8);
  L.sel = w; w += align_words(K);
  L.betas = w; w += align_words(K);
  L.crt_header_words = w - crt0;
  const size_t nmax = (size_t)std::max(I.da, I.db) + 1;
  L.wv = w; w += align_words((size_t)K * wl);
  L.uv = w; w += align_words((size_t)K * (I.da + 1));
  L.vv = w; w += align_words((size_t)K * (I.db + 1));
  L.dig = w; w += align_words(3 * nmax * K);
  L.out = w; w += align_words(3 * nmax * L.lg);
  L.total_words = w;
}

int write_upoly(const UPoly& G, snc_upoly* out, std::string& err) {
  int need_nl = 1;
  for (const auto& x : G.c) need_nl = std::max(need_nl, x.twos_limbs());
  const int need_deg = std::max(G.deg(), 0);
  if (out->deg < need_deg || out->nlimbs < need_nl || !out->limbs) {
    out->deg = need_deg;
    out->nlimbs = need_nl;
    err = "output buffer too small";
    return SNC_ERANGE;
  }
  for (int i = 0; i <= G.deg(); ++i)
    if (!G.c[i].to_twos(out->limbs + (size_t)i * out->nlimbs, out->nlimbs)) { err = "output conversion"; return SNC_EINTERNAL; }
  out->deg = G.deg();
  return SNC_OK;
}

}  // namespace

#define HIPCHK(x)                                                              \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) {                                                    \
      ctx->err = std::string(#x) + ": " + hipGetErrorString(e_);               \
      return SNC_EDEVICE;                                                      \
    }                                                                          \
  } while (0)

// b = a' (formal derivative), with the limb count its coefficients need
void derivative(const UPoly& A, UPoly& B, int& nlb) {
  B.c.clear();
  nlb = 1;
  if (A.c.size() <= 1) return;
  B.c.resize(A.c.size() - 1);
  for (size_t i = 0; i + 1 < A.c.size(); ++i) {
    B.c[i] = A.c[i + 1].mul_small((uint32_t)(i + 1));
    nlb = std::max(nlb, B.c[i].twos_limbs());
  }
}

static int gcd_core(snc_ctx* ctx, GcdTimer& tm, const UPoly& A, const UPoly& B, int nla, int nlb, void* d_ws,
                    size_t ws_bytes, hipStream_t stream, snc_upoly* out);

static int gcd_impl(snc_ctx* ctx, const snc_upoly* a, const snc_upoly* b, void* d_ws, size_t ws_bytes,
                    hipStream_t stream, snc_upoly* out) {
  HIPCHK(hipSetDevice(ctx->device));
  GcdTimer tm(ctx, stream);
  UPoly A, B;
  int nla = 1, nlb = 1;
  int st = parse_upoly(a, A, nla, ctx->err);
  if (!st) st = parse_upoly(b, B, nlb, ctx->err);
  if (st) return st;
  tm.host("gcd_parse");
  return gcd_core(ctx, tm, A, B, nla, nlb, d_ws, ws_bytes, stream, out);
}

static int gcd_deriv_impl(snc_ctx* ctx, const snc_upoly* a, void* d_ws, size_t ws_bytes, hipStream_t stream,
                          snc_upoly* out) {
  HIPCHK(hipSetDevice(ctx->device));
  GcdTimer tm(ctx, stream);
  UPoly A, B;
  int nla = 1, nlb = 1;
  int st = parse_upoly(a, A, nla, ctx->err);
  if (st) return st;
  derivative(A, B, nlb);
  tm.host("gcd_parse");
  return gcd_core(ctx, tm, A, B, nla, nlb, d_ws, ws_bytes, stream, out);
}

static int gcd_core(snc_ctx* ctx, GcdTimer& tm, const UPoly& A, const UPoly& B, int nla, int nlb, void* d_ws,
                    size_t ws_bytes, hipStream_t stream, snc_upoly* out) {
  GcdInfo I;
  int st = analyse(A, B, nla, nlb, I);
  if (st) return st;
  tm.host("gcd_contents");
  if (I.trivial) return write_upoly(I.triv, out, ctx->err);
  if (out->deg < I.deg_bound || out->nlimbs < I.out_nlimbs || !out->limbs) {
    out->deg = I.deg_bound;
    out->nlimbs = I.out_nlimbs;
    ctx->err = "output buffer too small";
    return SNC_ERANGE;
  }
  GcdLayout L;
  layout_gcd(I, L);
  if (!d_ws || ws_bytes < L.total_words * 4) {
    ctx->err = "workspace of " + std::to_string(ws_bytes) + " bytes, need " + std::to_string(L.total_words * 4);
    return SNC_ENOMEM;
  }
  uint32_t* ws = (uint32_t*)d_ws;
  const Tables& TB = tables();
  const int T = I.da + I.db + 2, wl = std::min(I.da, I.db) + 1;
  const int K = I.kmax;
  if (ctx->stage_in((L.header_words + L.crt_header_words) * 4) ||
      ctx->stage_out((size_t)std::max<size_t>(K, 3 * ((size_t)std::max(I.da, I.db) + 1) * L.lg) * 4)) {
    ctx->err = "pinned staging allocation failed";
    return SNC_EDEVICE;
  }
  // upload block: packed coefficients, then the slot tables (grown per round)
  uint32_t* h = (uint32_t*)ctx->h_in;
  for (int i = 0; i < T; ++i) {
    const BigInt& x = i <= I.da ? A.c[i] : B.c[i - I.da - 1];
    if (!x.to_twos(h + L.coef + (size_t)i * I.nl, I.nl)) { ctx->err = "input conversion"; return SNC_EINTERNAL; }
  }
  int32_t* slot_prime = (int32_t*)(h + L.slot_prime);
  uint32_t* slot_scale = h + L.slot_scale;
  GcdDesc G{};
  G.da = I.da; G.db = I.db; G.nl = I.nl; G.wl = wl;
  G.coef_off = (int64_t)L.coef; G.slot_prime_off = (int64_t)L.slot_prime; G.slot_scale_off = (int64_t)L.slot_scale;
  G.res_off = (int64_t)L.res; G.e_off = (int64_t)L.e; G.w_off = (int64_t)L.w; G.u_off = (int64_t)L.u; G.v_off = (int64_t)L.v;

  int next_prime = 0;  // next table index to try
  int ns = 0;          // slots filled
  std::vector<int32_t> e_host;
  int target = std::min(K, std::max(3, primes_for_bits(bits_needed_opt(I)) + 2));
  bool full_tried = false;
  for (int round = 0; round < 64; ++round) {
    const int first = ns;
    while (ns < target && next_prime < KMAX) {
      const uint32_t p = TB.p[next_prime];
      const uint32_t cam = I.ca.mod_small(p), cbm = I.cb.mod_small(p);
      const bool lc_ok = I.lca_bar.mod_small(p) != 0 || I.lcb_bar.mod_small(p) != 0;  // p does not divide beta
      if (cam && cbm && lc_ok) {
        slot_prime[ns] = next_prime;
        slot_scale[3 * ns + 0] = cam == 1 ? 1u : powmod32(cam, p - 2, p);
        slot_scale[3 * ns + 1] = cbm == 1 ? 1u : powmod32(cbm, p - 2, p);
        slot_scale[3 * ns + 2] = 0;
        ++ns;
      }
      ++next_prime;
    }
    if (ns == first) { ctx->err = "gcd: ran out of primes before the result certified"; return SNC_EINTERNAL; }
    tm.host("gcd_select_primes");
    HIPCHK(hipMemcpyAsync(ws, h, L.header_words * 4, hipMemcpyHostToDevice, stream));
    G.slot0 = first;
    tm.dev_begin();
    launch_gcd_reduce(G, ns - first, ws, stream);
    tm.dev_end("gcd_reduce", ns - first);
    tm.dev_begin();
    launch_gcd_euclid(G, ns - first, ws, stream);
    HIPCHK(hipGetLastError());
    tm.dev_end("gcd_euclid", ns - first);
    HIPCHK(hipMemcpyAsync(ctx->h_out, ws + L.e, (size_t)ns * 4, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    tm.host("gcd_d2h_sync");
    e_host.assign((int32_t*)ctx->h_out, (int32_t*)ctx->h_out + ns);
    for (int s = 0; s < ns; ++s) {
      if (e_host[s] < 0 || e_host[s] > std::min(I.da, I.db)) {
        ctx->err = "gcd: degree " + std::to_string(e_host[s]) + " out of range for prime slot " + std::to_string(s);
        return SNC_EINTERNAL;
      }
    }
    const int emin = *std::min_element(e_host.begin(), e_host.end());
    if (emin == 0) {
      UPoly R;
      R.c = {I.c};
      return write_upoly(R, out, ctx->err);
    }
    if (!I.have_beta) {
      I.beta = BigInt::gcd(I.lca_bar, I.lcb_bar);
      I.have_beta = true;
    }
    std::vector<int32_t> sel;
    for (int s = 0; s < ns; ++s) if (e_host[s] == emin) sel.push_back(s);
    const int ks = (int)sel.size();
    if (ks < primes_for_bits(bits_needed_opt(I))) {  // too few lucky-looking primes yet
      target = std::min(K, ns + primes_for_bits(bits_needed_opt(I)) - ks + 2);
      if (target <= ns) { ctx->err = "gcd: prime budget exhausted"; return SNC_EINTERNAL; }
      continue;
    }
    // CRT tables for the selected primes, staged after the slot tables
    uint32_t* hc = (uint32_t*)ctx->h_in + L.header_words;
    const size_t crt0 = L.primes;
    auto at = [&](size_t word) { return hc + (word - crt0); };
    PrimeC* pc = (PrimeC*)at(L.primes);
    std::vector<uint32_t> q(ks);
    for (int j = 0; j < ks; ++j) { q[j] = TB.p[slot_prime[sel[j]]]; pc[j] = TB.pc[slot_prime[sel[j]]]; }
    uint32_t* garner = at(L.garner);
    uint32_t* wtab = at(L.wtab);
    for (int i = 0; i < ks; ++i) {
      uint64_t run = 1;
      for (int j = 0; j < i; ++j) {
        wtab[(size_t)j * ks + i] = mont32(run, q[i]);
        run = run * q[j] % q[i];
      }
      garner[i] = mont32(powmod32(run, q[i] - 2, q[i]), q[i]);
    }
    uint32_t* ptab = at(L.ptab);
    std::memset(ptab, 0, (size_t)(ks + 1) * L.lpg * 4);
    BigInt Pr = BigInt::from_u64(1);
    for (int j = 0; j <= ks; ++j) {
      for (size_t l = 0; l < Pr.mag.size() && (int)l < L.lpg; ++l) ptab[(size_t)j * L.lpg + l] = Pr.mag[l];
      if (j < ks) Pr = Pr.mul_small(q[j]);
    }
    const BigInt M = Pr;
    const int lens[3] = {emin + 1, I.da - emin + 1, I.db - emin + 1};
    const size_t vals[3] = {L.wv, L.uv, L.vv};
    ResJob* jb = (ResJob*)at(L.jobs);
    int64_t* pd = (int64_t*)at(L.prefd);
    int64_t* pcb = (int64_t*)at(L.prefc);
    pd[0] = pcb[0] = 0;
    const size_t nmax = (size_t)std::max(I.da, I.db) + 1;
    for (int t = 0; t < 3; ++t) {
      std::memset(&jb[t], 0, sizeof(ResJob));
      jb[t].D = lens[t] - 1;
      jb[t].k = ks;
      jb[t].L = L.lg;
      jb[t].val_off = (int64_t)vals[t];
      jb[t].dig_off = (int64_t)(L.dig + t * nmax * ks);
      jb[t].acc_off = 0;
      jb[t].out_off = (int64_t)(L.out + t * nmax * L.lg);
      pd[t + 1] = pd[t] + (lens[t] + CRT_COEF_PER_BLOCK - 1) / CRT_COEF_PER_BLOCK;
      pcb[t + 1] = pcb[t] + (lens[t] + CRT_COEF_PER_BLOCK - 1) / CRT_COEF_PER_BLOCK;
    }
    int32_t* hsel = (int32_t*)at(L.sel);
    for (int j = 0; j < ks; ++j) hsel[j] = sel[j];
    uint32_t* hbeta = at(L.betas);
    for (int j = 0; j < ks; ++j) hbeta[j] = I.beta.mod_small(q[j]);
    HIPCHK(hipMemcpyAsync(ws + crt0, hc, L.crt_header_words * 4, hipMemcpyHostToDevice, stream));
    launch_gcd_gather(G, (const int32_t*)(ws + L.sel), ws + L.betas, (const PrimeC*)(ws + L.primes), ks, emin, ws,
                      (int64_t)L.wv, (int64_t)L.uv, (int64_t)L.vv, stream);
    CrtTables tb{(const PrimeC*)(ws + L.primes), ws + L.garner, ws + L.wtab, ws + L.ptab, ks, L.lpg};
    launch_crt_digits(tb, (const ResJob*)(ws + L.jobs), (const int64_t*)(ws + L.prefd), 3, pd[3], ws, stream);
    launch_crt_combine(tb, (const ResJob*)(ws + L.jobs), (const int64_t*)(ws + L.prefc), 3, pcb[3], ks, ws, stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(ctx->h_out, ws + L.out, 3 * nmax * L.lg * 4, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    const uint32_t* ho = (const uint32_t*)ctx->h_out;
    UPoly W, U, V;
    UPoly* polys[3] = {&W, &U, &V};
    BigInt n1[3];
    for (int t = 0; t < 3; ++t) {
      polys[t]->c.resize(lens[t]);
      for (int i = 0; i < lens[t]; ++i) {
        polys[t]->c[i] = BigInt::from_twos(ho + t * nmax * L.lg + (size_t)i * L.lg, L.lg);
        n1[t] = n1[t] + abs_big(polys[t]->c[i]);
      }
    }
    const BigInt two = BigInt::from_u64(2);
    const bool ok = BigInt::cmp_mag((two * n1[0] * n1[1]).mag, M.mag) < 0 &&
                    BigInt::cmp_mag((two * n1[0] * n1[2]).mag, M.mag) < 0 &&
                    !W.c.back().is_zero() && !W.c.back().neg;
    if (ok) {
      // result: c * pp(w)
      BigInt cw = content(W);
      UPoly R;
      R.c.resize(W.c.size());
      for (size_t i = 0; i < W.c.size(); ++i) {
        BigInt qq, rr;
        BigInt::divmod(W.c[i], cw, qq, rr);
        R.c[i] = I.c * qq;
      }
      return write_upoly(normalise_sign(R), out, ctx->err);
    }
    // not certified: either too few primes for the true sizes, or all unlucky
    int want = primes_for_bits(bits_needed_full(I, emin));
    if (!full_tried && want > ks) {
      target = std::min(K, ns + (want - ks) + 2);
      full_tried = true;
    } else {
      target = std::min(K, ns + std::max(4, ks / 2));
    }
    if (target <= ns) { ctx->err = "gcd: prime budget exhausted before the result certified"; return SNC_EINTERNAL; }
  }
  ctx->err = "gcd: too many rounds";
  return SNC_EINTERNAL;
}

}  // namespace snc

using namespace snc;

static int gcd_plan(const UPoly& A, const UPoly& B, int nla, int nlb, snc_plan* out) {
  GcdInfo I;
  const int st = analyse(A, B, nla, nlb, I);
  if (st) return st;
  out->deg_bound = I.deg_bound;
  out->out_nlimbs = I.out_nlimbs;
  out->nprimes = I.trivial ? 0 : I.kmax;
  out->reserved = 0;
  if (I.trivial) {
    out->workspace_bytes = 0;
  } else {
    GcdLayout L;
    layout_gcd(I, L);
    out->workspace_bytes = L.total_words * 4;
  }
  return SNC_OK;
}

extern "C" {

int snc_gcd_z_plan(const snc_upoly* a, const snc_upoly* b, snc_plan* out) {
  if (!out) return SNC_EINVAL;
  std::string err;
  UPoly A, B;
  int nla = 1, nlb = 1;
  int st = parse_upoly(a, A, nla, err);
  if (!st) st = parse_upoly(b, B, nlb, err);
  if (st) return st;
  return gcd_plan(A, B, nla, nlb, out);
}

int snc_gcd_z_deriv_plan(const snc_upoly* a, snc_plan* out) {
  if (!out) return SNC_EINVAL;
  std::string err;
  UPoly A, B;
  int nla = 1, nlb = 1;
  int st = parse_upoly(a, A, nla, err);
  if (st) return st;
  derivative(A, B, nlb);
  return gcd_plan(A, B, nla, nlb, out);
}

int snc_gcd_z_deriv(snc_ctx* ctx, const snc_upoly* a, void* d_ws, size_t ws_bytes, void* stream, snc_upoly* out) {
  if (!ctx || !out) return SNC_EINVAL;
  return gcd_deriv_impl(ctx, a, d_ws, ws_bytes, (hipStream_t)stream, out);
}

int snc_gcd_z(snc_ctx* ctx, const snc_upoly* a, const snc_upoly* b, void* d_ws, size_t ws_bytes,
              void* stream, snc_upoly* out) {
  if (!ctx || !out) return SNC_EINVAL;
  return gcd_impl(ctx, a, b, d_ws, ws_bytes, (hipStream_t)stream, out);
}

}  // extern "C"
