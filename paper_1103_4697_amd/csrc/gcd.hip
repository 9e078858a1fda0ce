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
#include <climits>
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

// content of a polynomial given as two's-complement limbs: big-integer gcds
// only while the running gcd exceeds one word, then each coefficient is
// reduced straight from its limbs (x = U - 2^(32 n) when negative)
BigInt content_limbs(const snc_upoly& a) {
  const int nl = a.nlimbs;
  BigInt g;
  int i = 0;
  for (; i <= a.deg; ++i) {
    g = BigInt::gcd(g, BigInt::from_twos(a.limbs + (size_t)i * nl, nl));
    if (g.mag.size() == 1) break;
  }
  if (g.mag.size() != 1) return g;
  const uint32_t m = g.mag[0];
  uint64_t gg = m;
  std::vector<uint64_t> pw(nl + 1);
  uint64_t v = 1;
  for (int l = 0; l <= nl; ++l) { pw[l] = v; v = (v << 32) % m; }
  for (++i; i <= a.deg && gg > 1; ++i) {
    const uint32_t* c = a.limbs + (size_t)i * nl;
    unsigned __int128 acc = 0;
    for (int l = 0; l < nl; ++l) acc += (unsigned __int128)c[l] * pw[l];
    uint64_t r = (uint64_t)(acc % m);
    if (c[nl - 1] >> 31) r = (r + m - pw[nl]) % m;
    r %= gg;  // gg divides m
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

void trim(UPoly& P) {
  while (!P.c.empty() && P.c.back().is_zero()) P.c.pop_back();
}

// exact quotient num / den of integers known to divide; false if they do not
bool div_exact(const BigInt& num, const BigInt& den, BigInt& q) {
  BigInt r;
  BigInt::divmod(num, den, q, r);
  return r.is_zero();
}

// every coefficient times mul, divided exactly by den
bool scale_exact(const UPoly& A, const BigInt& mul, const BigInt& den, UPoly& Q) {
  Q.c.resize(A.c.size());
  for (size_t j = 0; j < A.c.size(); ++j)
    if (!div_exact(A.c[j] * mul, den, Q.c[j])) return false;
  trim(Q);
  return true;
}

// cofactors A / G, B / G of a gcd computed on the host (a zero or constant operand)
bool trivial_cofactors(const UPoly& A, const UPoly& B, const UPoly& G, UPoly& qa, UPoly& qb) {
  qa.c.clear();
  qb.c.clear();
  if (G.c.empty()) return A.c.empty() && B.c.empty();  // gcd(0, 0) = 0: cofactors 0
  if (G.deg() == 0) {
    const BigInt one = BigInt::from_u64(1);
    return scale_exact(A, one, G.c[0], qa) && scale_exact(B, one, G.c[0], qb);
  }
  // G = +-(the non-zero operand), the other one is zero
  const UPoly& N = A.c.empty() ? B : A;
  UPoly& qn = A.c.empty() ? qb : qa;
  qn.c = {BigInt::from_u64(1)};
  if (N.c.back().neg != G.c.back().neg) qn.c[0] = -qn.c[0];
  return true;
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

// raw2, raw1: log2 of the 2- and 1-norms of a and b when already known from
// their limbs (NULL: computed here)
int analyse(const UPoly& A, const UPoly& B, int nla, int nlb, GcdInfo& I, const double* raw2 = nullptr,
            const double* raw1 = nullptr) {
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
  if (raw2 && raw1) {
    I.l2a = raw2[0]; I.l1a = raw1[0];
    I.l2b = raw2[1]; I.l1b = raw1[1];
  } else {
    log2_norms(A, I.l2a, I.l1a);
    log2_norms(B, I.l2b, I.l1b);
  }
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

// b = a' (formal derivative)
void derivative(const UPoly& A, UPoly& B) {
  B.c.clear();
  if (A.c.size() <= 1) return;
  B.c.resize(A.c.size() - 1);
  for (size_t i = 0; i + 1 < A.c.size(); ++i) B.c[i] = A.c[i + 1].mul_small((uint32_t)(i + 1));
}

// ---------------------------------------------------------------------------
// Sizes read from the limbs alone, without big-integer arithmetic: trimmed
// degrees and log2 of the norms and leading coefficients, each coefficient
// taken from its top three magnitude limbs.  They are the sizes of a and b
// themselves, not of their primitive parts, so every bound derived from them
// is at least the one the contents would give.  The plan and the run both
// size the work from these, and the first round of primes is launched on
// them before the host has parsed the inputs or computed any content.
// ---------------------------------------------------------------------------
struct Quick {
  int da = -1, db = -1, nla = 1, nlb = 1, nl = 1;
  bool deriv = false, trivial = false;
  double l2[2] = {0, 0}, l1[2] = {0, 0}, llc[2] = {0, 0};
  int deg_bound = 0, out_nlimbs = 1, kmax = 0, target0 = 0;
};

// |x| ~ m 2^ex for a two's-complement coefficient (m from the top three limbs of |x|); m = 0 for x = 0
void coef_size(const uint32_t* c, int nl, double& m, int& ex) {
  const bool neg = c[nl - 1] >> 31;
  int z = 0;  // lowest non-zero limb: |x| = ~x + 1 carries up to it
  if (neg) while (z < nl && c[z] == 0) ++z;
  auto mag = [&](int i) -> uint32_t { return !neg ? c[i] : i < z ? 0u : i == z ? 0u - c[i] : ~c[i]; };
  int t = nl - 1;
  while (t >= 0 && mag(t) == 0) --t;
  if (t < 0) { m = 0.0; ex = 0; return; }
  double v = (double)mag(t);
  int used = 1;
  for (int k = 1; k <= 2 && t - k >= 0; ++k, ++used) v = v * 4294967296.0 + (double)mag(t - k);
  m = v;
  ex = 32 * (t + 1 - used);
}

bool zero_coef(const uint32_t* c, int nl) {
  for (int l = 0; l < nl; ++l) if (c[l]) return false;
  return true;
}

int trimmed_degree(const snc_upoly* a) {
  int d = a->deg;
  while (d >= 0 && zero_coef(a->limbs + (size_t)d * a->nlimbs, a->nlimbs)) --d;
  return d;
}

// log2 of the 2-norm, 1-norm and leading coefficient of the first deg+1
// coefficients (times j+1 for coefficient j when mult: the derivative's)
void limb_norms(const uint32_t* limbs, int nl, int deg, bool mult, double& l2, double& l1, double& llc) {
  std::vector<double> m(deg + 1);
  std::vector<int> ex(deg + 1);
  int emax = INT_MIN;
  for (int j = 0; j <= deg; ++j) {
    coef_size(limbs + (size_t)(mult ? j + 1 : j) * nl, nl, m[j], ex[j]);
    if (mult) m[j] *= (double)(j + 1);
    if (m[j] > 0.0) emax = std::max(emax, ex[j]);
  }
  const int E = emax + 128;  // m < 2^111, so every scaled term is below 1
  double s2 = 0.0, s1 = 0.0;
  for (int j = 0; j <= deg; ++j) {
    if (m[j] == 0.0) continue;
    const double r = std::ldexp(m[j], ex[j] - E);
    s2 += r * r;
    s1 += r;
  }
  l2 = E + 0.5 * std::log2(s2);
  l1 = E + std::log2(s1);
  llc = std::log2(m[deg]) + ex[deg];
}

int check_upoly(const snc_upoly* a, std::string& err) {
  if (!a) { err = "null polynomial"; return SNC_EINVAL; }
  if (a->deg >= 0 && (a->nlimbs < 1 || !a->limbs)) {
    err = "invalid univariate polynomial (nlimbs < 1 or NULL limbs)";
    return SNC_EINVAL;
  }
  return SNC_OK;
}

int quick_scan(const snc_upoly* a, const snc_upoly* b, bool deriv, Quick& Q, std::string& err) {
  Q = Quick();
  Q.deriv = deriv;
  int st = check_upoly(a, err);
  if (!st && !deriv) st = check_upoly(b, err);
  if (st) return st;
  Q.nla = a->deg >= 0 ? a->nlimbs : 1;
  Q.da = trimmed_degree(a);
  if (deriv) {
    Q.nlb = Q.nla;
    Q.db = Q.da >= 1 ? Q.da - 1 : -1;
  } else {
    Q.nlb = b->deg >= 0 ? b->nlimbs : 1;
    Q.db = trimmed_degree(b);
  }
  Q.nl = deriv ? Q.nla : std::max(Q.nla, Q.nlb);
  if (std::max(Q.da, Q.db) > GCD_MAX_DEG) {
    err = "gcd: degree " + std::to_string(std::max(Q.da, Q.db)) + " exceeds the supported " +
          std::to_string(GCD_MAX_DEG);
    return SNC_EINVAL;
  }
  Q.trivial = Q.da <= 0 || Q.db <= 0;
  if (Q.trivial) return SNC_OK;
  limb_norms(a->limbs, a->nlimbs, Q.da, false, Q.l2[0], Q.l1[0], Q.llc[0]);
  if (deriv) limb_norms(a->limbs, a->nlimbs, Q.db, true, Q.l2[1], Q.l1[1], Q.llc[1]);
  else limb_norms(b->limbs, b->nlimbs, Q.db, false, Q.l2[1], Q.l1[1], Q.llc[1]);
  GcdInfo sz;  // the size fields only
  sz.da = Q.da; sz.db = Q.db;
  sz.l2a = Q.l2[0]; sz.l1a = Q.l1[0]; sz.l2b = Q.l2[1]; sz.l1b = Q.l1[1];
  sz.lbeta = std::min(Q.llc[0], Q.llc[1]);
  // Mignotte: a factor of degree e of a has coefficients <= 2^e ||a||_2
  Q.deg_bound = std::min(Q.da, Q.db);
  Q.out_nlimbs = (int)std::ceil((Q.deg_bound + std::min(Q.l2[0], Q.l2[1]) + 3.0) / 32.0) + 1;
  double worst = 0.0;
  for (int e : {0, Q.deg_bound}) worst = std::max(worst, bits_needed_full(sz, e));
  Q.kmax = std::min(KMAX, std::max(primes_for_bits(worst), primes_for_bits(bits_needed_opt(sz))) + 12);
  Q.target0 = std::min(Q.kmax, std::max(3, primes_for_bits(bits_needed_opt(sz)) + 2));
  return SNC_OK;
}

// ---------------------------------------------------------------------------
// Batched driver.  n problems share one workspace and advance in rounds.  In a
// round every unfinished problem draws its next primes; one upload, one
// reduction launch, one Euclid launch per register class and one download
// serve all of them.  The first round starts from the limbs as given, and
// the host parses the inputs and computes contents while it runs; primes
// dividing a content are then set aside.  Problems whose minimal-degree
// primes suffice are lifted (gather, CRT digits and combination per problem,
// one upload and one download in all) and certified; the others draw more
// primes in the next round.
// ---------------------------------------------------------------------------
struct GcdProb {
  const snc_upoly* a = nullptr;
  const snc_upoly* b = nullptr;
  Quick Q;
  UPoly A, B;
  GcdInfo I;
  snc_upoly* out = nullptr;
  UPoly* cofa = nullptr;  // optional: a / gcd and b / gcd (exact), host big integers
  UPoly* cofb = nullptr;
  bool done = false, parsed = false;
  int K = 0, T = 0, wl = 0, lg = 0, cls = 0;
  size_t nmax = 0;
  GcdDesc G{};
  std::vector<uint8_t> usable;  // per slot, known after the round that computed it
  // word offsets into the workspace
  size_t coef = 0, slot_prime = 0, e = 0;
  size_t res = 0, w = 0, u = 0, v = 0;
  size_t primes = 0, garner = 0, wtab = 0, ptab = 0, jobs = 0, prefd = 0, prefc = 0, sel = 0, scales = 0;
  size_t wv = 0, uv = 0, vv = 0, dig = 0, outw = 0;
  // round state
  int ns = 0, next_prime = 0, target = 0, first = 0;
  bool full_tried = false;
};

struct GcdBatchLayout {
  size_t descs = 0, items = 0, item_cap = 0;
  size_t hdr_end = 0;                  // [0, hdr_end): descriptors, work items, inputs, slot tables
  size_t e_begin = 0, e_end = 0;       // gcd degree of every slot
  size_t crt_begin = 0, crt_end = 0;   // CRT tables and jobs
  size_t out_begin = 0, out_end = 0;   // lifted w, u, v
  size_t total = 0;                    // words
};

// Offsets of every problem (trivial ones take no space); the same function
// sizes the plan and places the run.
void layout_batch(std::vector<GcdProb>& P, GcdBatchLayout& L) {
  size_t w = 0;
  L.descs = w; w += align_words(sizeof(GcdDesc) / 4 * P.size());
  L.item_cap = 0;
  for (const auto& p : P) if (!p.Q.trivial) L.item_cap += (size_t)p.Q.kmax;
  L.items = w; w += align_words(2 * L.item_cap);
  for (auto& p : P) {
    if (p.Q.trivial) continue;
    p.K = p.Q.kmax;
    p.T = p.Q.da + p.Q.db + 2;
    p.wl = std::min(p.Q.da, p.Q.db) + 1;
    p.nmax = (size_t)std::max(p.Q.da, p.Q.db) + 1;
    p.lg = lx_of(p.K);
    p.cls = gcd_reg_slots(std::max(p.Q.da, p.Q.db));
    p.coef = w; w += align_words((size_t)(p.Q.deriv ? p.Q.da + 1 : p.T) * p.Q.nl);
    p.slot_prime = w; w += align_words(p.K);
  }
  L.hdr_end = w;
  L.e_begin = w;
  for (auto& p : P) if (!p.Q.trivial) { p.e = w; w += align_words(p.K); }
  L.e_end = w;
  L.crt_begin = w;
  for (auto& p : P) {
    if (p.Q.trivial) continue;
    const size_t K = p.K;
    p.primes = w; w += align_words(sizeof(PrimeC) / 4 * K);
    p.garner = w; w += align_words(K);
    p.wtab = w; w += align_words(K * K);
    p.ptab = w; w += align_words((K + 1) * p.lg);
    p.jobs = w; w += align_words(3 * sizeof(ResJob) / 4);
    p.prefd = w; w += align_words(8);
    p.prefc = w; w += align_words(8);
    p.sel = w; w += align_words(K);
    p.scales = w; w += align_words(3 * K);
  }
  L.crt_end = w;
  L.out_begin = w;
  for (auto& p : P) if (!p.Q.trivial) { p.outw = w; w += align_words(3 * p.nmax * p.lg); }
  L.out_end = w;
  for (auto& p : P) {
    if (p.Q.trivial) continue;
    const size_t K = p.K;
    p.res = w; w += align_words(K * p.T);
    p.w = w; w += align_words(K * p.wl);
    p.u = w; w += align_words(K * (p.Q.da + 1));
    p.v = w; w += align_words(K * (p.Q.db + 1));
    p.wv = w; w += align_words(K * p.wl);
    p.uv = w; w += align_words(K * (p.Q.da + 1));
    p.vv = w; w += align_words(K * (p.Q.db + 1));
    p.dig = w; w += align_words(3 * p.nmax * K);
  }
  L.total = w;
}

// big-integer form of a and b (b = a' when deriv) and their contents
int parse_analyse(GcdProb& p, std::string& err) {
  int nla = 1, nlb = 1;
  int st = parse_upoly(p.a, p.A, nla, err);
  if (st) return st;
  if (p.Q.deriv) derivative(p.A, p.B);
  else st = parse_upoly(p.b, p.B, nlb, err);
  if (st) return st;
  st = p.Q.trivial ? analyse(p.A, p.B, nla, nlb, p.I) : analyse(p.A, p.B, nla, nlb, p.I, p.Q.l2, p.Q.l1);
  p.parsed = true;
  return st;
}

// rows 0..deg of a limb array into nl-limb rows (sign-extended)
void pack_rows(const snc_upoly* a, int deg, int nl, uint32_t* dst) {
  for (int i = 0; i <= deg; ++i) {
    const uint32_t* src = a->limbs + (size_t)i * a->nlimbs;
    const uint32_t ext = (src[a->nlimbs - 1] >> 31) ? 0xffffffffu : 0u;
    uint32_t* d = dst + (size_t)i * nl;
    for (int l = 0; l < nl; ++l) d[l] = l < a->nlimbs ? src[l] : ext;
  }
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

// Chinese remaindering tables and jobs of one problem for its selected slots
// (written into the staging copy of its CRT area); returns M = prod q.
static BigInt stage_crt(GcdProb& p, const std::vector<int32_t>& sel, int emin, const int32_t* slot_prime,
                        uint32_t* h) {
  const Tables& TB = tables();
  const int ks = (int)sel.size();
  PrimeC* pc = (PrimeC*)(h + p.primes);
  std::vector<uint32_t> q(ks);
  for (int j = 0; j < ks; ++j) { q[j] = TB.p[slot_prime[sel[j]]]; pc[j] = TB.pc[slot_prime[sel[j]]]; }
  uint32_t* garner = h + p.garner;
  uint32_t* wtab = h + p.wtab;
  for (int i = 0; i < ks; ++i) {
    uint64_t run = 1;
    for (int j = 0; j < i; ++j) {
      wtab[(size_t)j * ks + i] = mont32(run, q[i]);
      run = run * q[j] % q[i];
    }
    garner[i] = mont32(powmod32(run, q[i] - 2, q[i]), q[i]);
  }
  uint32_t* ptab = h + p.ptab;
  std::memset(ptab, 0, (size_t)(ks + 1) * p.lg * 4);
  BigInt Pr = BigInt::from_u64(1);
  for (int j = 0; j <= ks; ++j) {
    for (size_t l = 0; l < Pr.mag.size() && (int)l < p.lg; ++l) ptab[(size_t)j * p.lg + l] = Pr.mag[l];
    if (j < ks) Pr = Pr.mul_small(q[j]);
  }
  const int lens[3] = {emin + 1, p.Q.da - emin + 1, p.Q.db - emin + 1};
  const size_t vals[3] = {p.wv, p.uv, p.vv};
  ResJob* jb = (ResJob*)(h + p.jobs);
  int64_t* pd = (int64_t*)(h + p.prefd);
  int64_t* pcb = (int64_t*)(h + p.prefc);
  pd[0] = pcb[0] = 0;
  for (int t = 0; t < 3; ++t) {
    std::memset(&jb[t], 0, sizeof(ResJob));
    jb[t].D = lens[t] - 1;
    jb[t].k = ks;
    jb[t].L = p.lg;
    jb[t].val_off = (int64_t)vals[t];
    jb[t].dig_off = (int64_t)(p.dig + t * p.nmax * ks);
    jb[t].acc_off = 0;
    jb[t].pts_off = 0;
    jb[t].nq_off = 0;
    jb[t].out_off = (int64_t)(p.outw + t * p.nmax * p.lg);
    pd[t + 1] = pd[t] + (lens[t] + CRT_COEF_PER_BLOCK - 1) / CRT_COEF_PER_BLOCK;
    pcb[t + 1] = pcb[t] + (lens[t] + CRT_COMB_PER_BLOCK - 1) / CRT_COMB_PER_BLOCK;
  }
  int32_t* hsel = (int32_t*)(h + p.sel);
  uint32_t* hsc = h + p.scales;
  for (int j = 0; j < ks; ++j) {
    hsel[j] = sel[j];
    hsc[3 * j + 0] = p.I.beta.mod_small(q[j]);
    hsc[3 * j + 1] = powmod32(p.I.ca.mod_small(q[j]), q[j] - 2, q[j]);
    hsc[3 * j + 2] = powmod32(p.I.cb.mod_small(q[j]), q[j] - 2, q[j]);
  }
  return Pr;
}

// Quick scans are done; this runs every problem.
static int gcd_batch(snc_ctx* ctx, GcdTimer& tm, std::vector<GcdProb>& P, void* d_ws, size_t ws_bytes,
                     hipStream_t stream) {
  const int n = (int)P.size();
  bool short_out = false;
  for (auto& p : P) {
    if (p.Q.trivial) {  // a zero or constant operand: on the host
      int st = parse_analyse(p, ctx->err);
      if (st) return st;
      if (!p.I.trivial) { ctx->err = "gcd: size scan and analysis disagree"; return SNC_EINTERNAL; }
      st = write_upoly(p.I.triv, p.out, ctx->err);
      if (st == SNC_ERANGE) { short_out = true; continue; }
      if (st) return st;
      if (p.cofa && !trivial_cofactors(p.A, p.B, p.I.triv, *p.cofa, *p.cofb)) {
        ctx->err = "gcd: inexact cofactor";
        return SNC_EINTERNAL;
      }
      p.done = true;
    } else if (p.out->deg < p.Q.deg_bound || p.out->nlimbs < p.Q.out_nlimbs || !p.out->limbs) {
      p.out->deg = p.Q.deg_bound;
      p.out->nlimbs = p.Q.out_nlimbs;
      short_out = true;
    }
  }
  if (short_out) { ctx->err = "output buffer too small"; return SNC_ERANGE; }
  int active = 0;
  for (auto& p : P) active += !p.done;
  if (!active) return SNC_OK;

  GcdBatchLayout L;
  layout_batch(P, L);
  if (!d_ws || ws_bytes < L.total * 4) {
    ctx->err = "workspace of " + std::to_string(ws_bytes) + " bytes, need " + std::to_string(L.total * 4);
    return SNC_ENOMEM;
  }
  uint32_t* ws = (uint32_t*)d_ws;
  if (ctx->stage_in(L.crt_end * 4) || ctx->stage_out((L.out_end - L.e_begin) * 4)) {
    ctx->err = "pinned staging allocation failed";
    return SNC_EDEVICE;
  }
  uint32_t* h = (uint32_t*)ctx->h_in;                  // mirrors ws[0, crt_end)
  const uint32_t* ho = (const uint32_t*)ctx->h_out;    // mirrors ws[e_begin, out_end)
  GcdDesc* descs = (GcdDesc*)(h + L.descs);
  for (int i = 0; i < n; ++i) {
    GcdProb& p = P[i];
    if (p.done) continue;
    pack_rows(p.a, p.Q.da, p.Q.nl, h + p.coef);
    if (!p.Q.deriv) pack_rows(p.b, p.Q.db, p.Q.nl, h + p.coef + (size_t)(p.Q.da + 1) * p.Q.nl);
    GcdDesc& G = p.G;
    G.da = p.Q.da; G.db = p.Q.db; G.nl = p.Q.nl; G.wl = p.wl; G.deriv = p.Q.deriv ? 1 : 0; G.fused = 0; G.vals = nullptr; G.vstride = 0; G.d_off = 0;
    G.ed_out = nullptr;
    G.coef_off = (int64_t)p.coef; G.slot_prime_off = (int64_t)p.slot_prime;
    G.res_off = (int64_t)p.res; G.e_off = (int64_t)p.e; G.w_off = (int64_t)p.w; G.u_off = (int64_t)p.u;
    G.v_off = (int64_t)p.v;
    descs[i] = G;
    p.target = p.Q.target0;
    p.usable.assign(p.K, 0);
  }
  tm.host("gcd_pack");
  const Tables& TB = tables();
  int32_t* items = (int32_t*)(h + L.items);
  const GcdDesc* descs_d = (const GcdDesc*)(ws + L.descs);
  const int32_t* items_d = (const int32_t*)(ws + L.items);

  for (int round = 0; round < 64 && active; ++round) {
    // 1. next primes of every unfinished problem; before the contents are
    //    known (first round) every table prime is drawn, later only primes
    //    dividing neither content
    int max_rows = 0, max_nl = 1;
    for (auto& p : P) {
      if (p.done) continue;
      p.first = p.ns;
      int32_t* slot_prime = (int32_t*)(h + p.slot_prime);
      while (p.ns < p.target && p.next_prime < KMAX) {
        const uint32_t q = TB.p[p.next_prime];
        if (!p.parsed || (p.I.ca.mod_small(q) && p.I.cb.mod_small(q))) slot_prime[p.ns++] = p.next_prime;
        ++p.next_prime;
      }
      if (p.ns == p.first) { ctx->err = "gcd: ran out of primes before the result certified"; return SNC_EINTERNAL; }
      max_rows = std::max(max_rows, p.Q.deriv ? p.Q.da + 1 : p.T);
      max_nl = std::max(max_nl, p.Q.nl);
    }
    // work items grouped by register class, one launch per class
    struct Range { int cls, off, cnt, maxd; };
    std::vector<Range> ranges;
    int nitems = 0;
    for (int cls : {2, 4, 6, 9, 12, 16, 24, 32, 0}) {
      Range r{cls, nitems, 0, 0};
      for (int i = 0; i < n; ++i) {
        GcdProb& p = P[i];
        if (p.done || p.cls != cls) continue;
        for (int s = p.first; s < p.ns; ++s) { items[2 * nitems] = i; items[2 * nitems + 1] = s; ++nitems; }
        r.maxd = std::max(r.maxd, std::max(p.Q.da, p.Q.db));
      }
      r.cnt = nitems - r.off;
      if (r.cnt) ranges.push_back(r);
    }
    tm.host("gcd_select_primes");
    HIPCHK(hipMemcpyAsync(ws, h, L.hdr_end * 4, hipMemcpyHostToDevice, stream));
    tm.dev_begin();
    launch_gcd_reduce(descs_d, items_d, nitems, max_rows, max_nl, ws, stream);
    tm.dev_end("gcd_reduce", nitems);
    tm.dev_begin();
    for (const Range& r : ranges) launch_gcd_euclid(descs_d, items_d + 2 * r.off, r.cnt, r.cls, r.maxd, ws, stream);
    HIPCHK(hipGetLastError());
    tm.dev_end("gcd_euclid", nitems);
    HIPCHK(hipMemcpyAsync(ctx->h_out, ws + L.e_begin, (L.e_end - L.e_begin) * 4, hipMemcpyDeviceToHost, stream));
    if (round == 0) {  // while the device works: big integers and contents
      for (auto& p : P) {
        if (p.done) continue;
        const int st = parse_analyse(p, ctx->err);
        if (st) return st;
        if (p.I.trivial || p.I.da != p.Q.da || p.I.db != p.Q.db) {
          ctx->err = "gcd: size scan and analysis disagree";
          return SNC_EINTERNAL;
        }
      }
      tm.host("gcd_parse_contents");
    }
    HIPCHK(hipStreamSynchronize(stream));
    tm.host("gcd_d2h_sync");

    // 2. decide per problem: constant gcd, more primes, or lift
    std::vector<int> lift;
    std::vector<std::vector<int32_t>> sels(n);
    std::vector<int> emins(n, -1);
    std::vector<BigInt> Ms(n);
    for (int i = 0; i < n; ++i) {
      GcdProb& p = P[i];
      if (p.done) continue;
      const int32_t* e_host = (const int32_t*)(ho + (p.e - L.e_begin));
      const int32_t* slot_prime = (const int32_t*)(h + p.slot_prime);
      int emin = INT32_MAX;
      for (int s = 0; s < p.ns; ++s) {
        if (s >= p.first) {
          const int32_t es = e_host[s];
          if (es != GCD_SLOT_UNUSABLE && (es < 0 || es > std::min(p.Q.da, p.Q.db))) {
            ctx->err = "gcd: degree " + std::to_string(es) + " out of range for prime slot " + std::to_string(s);
            return SNC_EINTERNAL;
          }
          const uint32_t q = TB.p[slot_prime[s]];
          p.usable[s] = es != GCD_SLOT_UNUSABLE && p.I.ca.mod_small(q) && p.I.cb.mod_small(q);
        }
        if (p.usable[s]) emin = std::min(emin, (int)e_host[s]);
      }
      if (emin == INT32_MAX) {  // no usable prime yet
        p.target = std::min(p.K, p.ns + 4);
        if (p.target <= p.ns) { ctx->err = "gcd: prime budget exhausted"; return SNC_EINTERNAL; }
        continue;
      }
      if (emin == 0) {  // a usable prime with a constant gcd: the gcd is the content
        UPoly R;
        R.c = {p.I.c};
        const int st = write_upoly(R, p.out, ctx->err);
        if (st) return st;
        const BigInt one = BigInt::from_u64(1);
        if (p.cofa && !(scale_exact(p.A, one, p.I.c, *p.cofa) && scale_exact(p.B, one, p.I.c, *p.cofb))) {
          ctx->err = "gcd: inexact cofactor";
          return SNC_EINTERNAL;
        }
        p.done = true;
        --active;
        continue;
      }
      if (!p.I.have_beta) {
        p.I.beta = BigInt::gcd(p.I.lca_bar, p.I.lcb_bar);
        p.I.have_beta = true;
      }
      std::vector<int32_t> sel;
      for (int s = 0; s < p.ns; ++s) if (p.usable[s] && e_host[s] == emin) sel.push_back(s);
      const int ks = (int)sel.size();
      const int need = primes_for_bits(bits_needed_opt(p.I));
      if (ks < need) {  // too few lucky-looking primes yet
        p.target = std::min(p.K, p.ns + need - ks + 2);
        if (p.target <= p.ns) { ctx->err = "gcd: prime budget exhausted"; return SNC_EINTERNAL; }
        continue;
      }
      Ms[i] = stage_crt(p, sel, emin, slot_prime, h);
      sels[i] = std::move(sel);
      emins[i] = emin;
      lift.push_back(i);
    }
    if (lift.empty()) continue;

    // 3. lift w, u, v of those problems and certify
    HIPCHK(hipMemcpyAsync(ws + L.crt_begin, h + L.crt_begin, (L.crt_end - L.crt_begin) * 4, hipMemcpyHostToDevice,
                          stream));
    for (int i : lift) {
      GcdProb& p = P[i];
      const int ks = (int)sels[i].size();
      launch_gcd_gather(p.G, (const int32_t*)(ws + p.sel), ws + p.scales, (const PrimeC*)(ws + p.primes), ks,
                        emins[i], ws, (int64_t)p.wv, (int64_t)p.uv, (int64_t)p.vv, stream);
      CrtTables tb{(const PrimeC*)(ws + p.primes), ws + p.garner, ws + p.wtab, ws + p.ptab, ks, p.lg};
      const int64_t* pd = (const int64_t*)(h + p.prefd);
      launch_crt_digits(tb, (const ResJob*)(ws + p.jobs), nullptr, (const int64_t*)(ws + p.prefd), 3, pd[3], ws, stream);
      const int64_t* pc = (const int64_t*)(h + p.prefc);
      launch_crt_combine(tb, (const ResJob*)(ws + p.jobs), nullptr, (const int64_t*)(ws + p.prefc), 3, pc[3], ks, ws,
                         stream);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync((uint8_t*)ctx->h_out + (L.out_begin - L.e_begin) * 4, ws + L.out_begin,
                          (L.out_end - L.out_begin) * 4, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    tm.host("gcd_lift");
    for (int i : lift) {
      GcdProb& p = P[i];
      const int emin = emins[i];
      const int ks = (int)sels[i].size();
      const int lens[3] = {emin + 1, p.Q.da - emin + 1, p.Q.db - emin + 1};
      const uint32_t* hq = ho + (p.outw - L.e_begin);
      UPoly W, U, V;
      UPoly* polys[3] = {&W, &U, &V};
      BigInt n1[3];
      for (int t = 0; t < 3; ++t) {
        polys[t]->c.resize(lens[t]);
        for (int j = 0; j < lens[t]; ++j) {
          polys[t]->c[j] = BigInt::from_twos(hq + t * p.nmax * p.lg + (size_t)j * p.lg, p.lg);
          n1[t] = n1[t] + abs_big(polys[t]->c[j]);
        }
      }
      const BigInt two = BigInt::from_u64(2);
      const BigInt& M = Ms[i];
      const bool ok = BigInt::cmp_mag((two * n1[0] * n1[1]).mag, M.mag) < 0 &&
                      BigInt::cmp_mag((two * n1[0] * n1[2]).mag, M.mag) < 0 &&
                      !W.c.back().is_zero() && !W.c.back().neg;
      if (ok) {  // result: c * pp(w)
        const BigInt cw = content(W);
        UPoly R;
        R.c.resize(W.c.size());
        for (size_t j = 0; j < W.c.size(); ++j) {
          BigInt qq, rr;
          BigInt::divmod(W.c[j], cw, qq, rr);
          R.c[j] = p.I.c * qq;
        }
        const int st = write_upoly(normalise_sign(R), p.out, ctx->err);
        if (st) return st;
        if (p.cofa) {
          // beta abar = w u with w = cw pp(w) and gcd = c pp(w) (lc(w) = beta > 0):
          // a / gcd = u cont(a) cw / (c beta), b / gcd = v cont(b) cw / (c beta)
          const BigInt den = p.I.c * p.I.beta;
          if (!(scale_exact(U, p.I.ca * cw, den, *p.cofa) && scale_exact(V, p.I.cb * cw, den, *p.cofb))) {
            ctx->err = "gcd: inexact cofactor";
            return SNC_EINTERNAL;
          }
        }
        p.done = true;
        --active;
        continue;
      }
      // not certified: too few primes for the true sizes, or all unlucky
      const int want = primes_for_bits(bits_needed_full(p.I, emin));
      if (!p.full_tried && want > ks) {
        p.target = std::min(p.K, p.ns + (want - ks) + 2);
        p.full_tried = true;
      } else {
        p.target = std::min(p.K, p.ns + std::max(4, ks / 2));
      }
      if (p.target <= p.ns) { ctx->err = "gcd: prime budget exhausted before the result certified"; return SNC_EINTERNAL; }
    }
    tm.host("gcd_certify");
  }
  if (active) { ctx->err = "gcd: too many rounds"; return SNC_EINTERNAL; }
  return SNC_OK;
}

static int gcd_run(snc_ctx* ctx, int n, const snc_upoly* a, const snc_upoly* b, bool deriv, void* d_ws,
                   size_t ws_bytes, hipStream_t stream, snc_upoly* out, UPoly* cofa = nullptr,
                   UPoly* cofb = nullptr) {
  HIPCHK(hipSetDevice(ctx->device));
  GcdTimer tm(ctx, stream);
  std::vector<GcdProb> P(n);
  for (int i = 0; i < n; ++i) {
    P[i].a = &a[i];
    P[i].b = deriv ? nullptr : &b[i];
    P[i].out = &out[i];
    if (cofa && cofb) { P[i].cofa = &cofa[i]; P[i].cofb = &cofb[i]; }
    const int st = quick_scan(P[i].a, P[i].b, deriv, P[i].Q, ctx->err);
    if (st) return st;
  }
  tm.host("gcd_scan");
  return gcd_batch(ctx, tm, P, d_ws, ws_bytes, stream);
}

static int gcd_plan(int n, const snc_upoly* a, const snc_upoly* b, bool deriv, snc_plan* each, snc_plan* total) {
  std::string err;
  std::vector<GcdProb> P(n);
  for (int i = 0; i < n; ++i) {
    P[i].a = &a[i];
    P[i].b = deriv ? nullptr : &b[i];
    int st = quick_scan(P[i].a, P[i].b, deriv, P[i].Q, err);
    if (!st && P[i].Q.trivial) st = parse_analyse(P[i], err);  // exact size of a host result
    if (st) return st;
  }
  GcdBatchLayout L;
  layout_batch(P, L);
  int needs_device = 0;
  if (total) *total = snc_plan{};
  for (int i = 0; i < n; ++i) {
    const Quick& Q = P[i].Q;
    snc_plan pl{};
    if (Q.trivial) {
      pl.deg_bound = P[i].I.deg_bound;
      pl.out_nlimbs = P[i].I.out_nlimbs;
    } else {
      pl.deg_bound = Q.deg_bound;
      pl.out_nlimbs = Q.out_nlimbs;
      pl.nprimes = Q.kmax;
      std::vector<GcdProb> one(1);
      one[0].Q = Q;
      GcdBatchLayout L1;
      layout_batch(one, L1);
      pl.workspace_bytes = L1.total * 4;
      needs_device = 1;
    }
    if (each) each[i] = pl;
    if (total) {
      total->deg_bound = std::max(total->deg_bound, pl.deg_bound);
      total->out_nlimbs = std::max(total->out_nlimbs, pl.out_nlimbs);
      total->nprimes += pl.nprimes;
    }
  }
  if (total) total->workspace_bytes = needs_device ? L.total * 4 : 0;
  return SNC_OK;
}

// ---------------------------------------------------------------------------
// Resultant and gcd(R, R') in one pass (the projection step, Section 2.1).
// The interpolation leaves R mod p for the resultant's own primes; the
// Euclid kernel runs on those residues (b = R' formed from them) right after
// the interpolation while the Chinese remaindering runs on a second stream,
// and reports e_p and the degree
// d_p of R mod p.  A prime with d_p = deg R does not divide lc(R), so
// e_p >= deg gcd(R, R'); e_p = 0 for one such prime proves that the gcd is
// gcd(cont R, cont R').  The host computes the contents from R while the
// Euclid runs.  Without such a prime the full modular gcd of R follows.
// ---------------------------------------------------------------------------

// sizes of the gcd(R, R') problem bounded by the resultant's bounds: |R_i| <= B, |R'_i| <= D B
static void sqfree_bound(const ResPlan& P, Quick& Q) {
  Q = Quick();
  Q.deriv = true;
  Q.da = P.trivial ? 0 : P.D;
  Q.db = Q.da - 1;
  Q.nla = Q.nlb = Q.nl = P.L;
  Q.trivial = Q.da <= 0;
  if (Q.trivial) { Q.deg_bound = 0; Q.out_nlimbs = P.L; return; }
  const double lb = std::max(P.log2B, 0.0), ln = std::log2((double)P.D + 1.0), ld = std::log2((double)P.D);
  Q.l2[0] = lb + 0.5 * ln; Q.l1[0] = lb + ln; Q.llc[0] = lb;
  Q.l2[1] = Q.l2[0] + ld; Q.l1[1] = Q.l1[0] + ld; Q.llc[1] = lb + ld;
  GcdInfo sz;
  sz.da = Q.da; sz.db = Q.db;
  sz.l2a = Q.l2[0]; sz.l1a = Q.l1[0]; sz.l2b = Q.l2[1]; sz.l1b = Q.l1[1];
  sz.lbeta = std::min(Q.llc[0], Q.llc[1]);
  Q.deg_bound = Q.db;
  Q.out_nlimbs = std::max(P.L, (int)std::ceil((Q.deg_bound + std::min(Q.l2[0], Q.l2[1]) + 3.0) / 32.0) + 1);
  double worst = 0.0;
  for (int e : {0, Q.deg_bound}) worst = std::max(worst, bits_needed_full(sz, e));
  Q.kmax = std::min(KMAX, std::max(primes_for_bits(worst), primes_for_bits(bits_needed_opt(sz))) + 12);
  Q.target0 = std::min(Q.kmax, std::max(3, primes_for_bits(bits_needed_opt(sz)) + 2));
}

struct SqfreeLayout {
  size_t descs = 0, items = 0, slotp = 0, e = 0, d = 0, fused = 0;  // words
  size_t fallback_words = 0;                                         // full gcd of one R
  std::vector<size_t> job_base;                                      // first e/d entry of each device job
};

static void sqfree_layout(const snc_prepared* pr, SqfreeLayout& S, std::vector<Quick>* bounds) {
  const BatchLayout& lay = pr->lay;
  size_t w = 0, nk = 0;
  S.job_base.clear();
  for (const ResJob& J : lay.jobs) { S.job_base.push_back(nk); nk += J.k; }
  S.descs = w; w += align_words(sizeof(GcdDesc) / 4 * std::max<size_t>(lay.jobs.size(), 1));
  S.items = w; w += align_words(2 * std::max<size_t>(nk, 1));
  S.slotp = w; w += align_words(KMAX);
  S.e = w; w += align_words(std::max<size_t>(nk, 1));
  S.d = w; w += align_words(std::max<size_t>(nk, 1));
  S.fused = w;
  S.fallback_words = 0;
  if (bounds) bounds->assign(pr->n, Quick());
  for (int i = 0; i < pr->n; ++i) {
    Quick Q;
    sqfree_bound(pr->P[i], Q);
    if (bounds) (*bounds)[i] = Q;
    if (Q.trivial) continue;
    std::vector<GcdProb> one(1);
    one[0].Q = Q;
    GcdBatchLayout L1;
    layout_batch(one, L1);
    S.fallback_words = std::max(S.fallback_words, L1.total);
  }
}

int prepared_sqfree_plan(const snc_prepared* pr, snc_plan* each, snc_plan* total) {
  SqfreeLayout S;
  std::vector<Quick> B;
  sqfree_layout(pr, S, &B);
  for (int i = 0; i < pr->n; ++i) {
    snc_plan pl{};
    pl.deg_bound = std::max(B[i].deg_bound, 0);
    pl.out_nlimbs = B[i].out_nlimbs;
    pl.nprimes = B[i].trivial ? 0 : B[i].kmax;
    if (each) each[i] = pl;
    if (total) {
      total->deg_bound = std::max(total->deg_bound, pl.deg_bound);
      total->out_nlimbs = std::max(total->out_nlimbs, pl.out_nlimbs);
    }
  }
  if (total) total->workspace_bytes = std::max<size_t>(S.fallback_words * 4, 256);
  return SNC_OK;
}

// descriptors, work items by register class and slot -> prime of the Euclid
// on the resultant's primes, uploaded once into the prepared workspace (its
// projection-step region), and the pinned buffer for e and d
static int sqfree_setup(snc_prepared* pr, const SqfreeLayout& S, hipStream_t stream) {
  snc_ctx* ctx = pr->c;
  const BatchLayout& lay = pr->lay;
  if (S.fused > lay.sq_words) { ctx->err = "projection-step region too small"; return SNC_EINTERNAL; }
  const size_t e_words = S.fused - S.e;
  int32_t* ed_dev = nullptr;
  if (!pr->h_ed) {
    if (hipHostMalloc(&pr->h_ed, std::max<size_t>(e_words * 4, 4), hipHostMallocMapped) != hipSuccess) {
      pr->h_ed = nullptr;
      ctx->err = "pinned staging allocation failed";
      return SNC_EDEVICE;
    }
  }
  HIPCHK(hipHostGetDevicePointer((void**)&ed_dev, pr->h_ed, 0));
  const int64_t base = (int64_t)(lay.sq_off / 4);
  std::vector<uint32_t> hf(S.e, 0u);
  GcdDesc* descs = (GcdDesc*)(hf.data() + S.descs);
  int32_t* items = (int32_t*)(hf.data() + S.items);
  int32_t* slotp = (int32_t*)(hf.data() + S.slotp);
  for (int q = 0; q < KMAX; ++q) slotp[q] = q;
  const int NJ = (int)lay.jobs.size();
  for (int j = 0; j < NJ; ++j) {
    const ResJob& J = lay.jobs[j];
    GcdDesc& G = descs[j];
    G = GcdDesc{};
    G.da = J.D; G.db = J.D - 1; G.nl = 1; G.wl = J.D; G.deriv = 1; G.fused = 1;
    G.vals = (const uint32_t*)pr->ws + J.val_off;
    G.vstride = J.D + 1;
    G.slot_prime_off = base + (int64_t)S.slotp;
    G.e_off = (int64_t)S.job_base[j];                  // relative to ed_out
    G.d_off = (int64_t)(S.d - S.e + S.job_base[j]);
    G.ed_out = ed_dev;
  }
  pr->sq_ranges.clear();
  int nitems = 0;
  for (int cls : {2, 4, 6, 9, 12, 16, 24, 32, 0}) {
    const int off = nitems;
    int maxd = 0;
    for (int j = 0; j < NJ; ++j) {
      const ResJob& J = lay.jobs[j];
      if (J.D < 1 || gcd_reg_slots(J.D) != cls) continue;
      for (int q = 0; q < J.k; ++q) { items[2 * nitems] = j; items[2 * nitems + 1] = q; ++nitems; }
      maxd = std::max(maxd, J.D);
    }
    if (nitems > off) pr->sq_ranges.insert(pr->sq_ranges.end(), {cls, off, nitems - off, maxd});
  }
  if (ctx->stage_in(S.e * 4)) { ctx->err = "pinned staging allocation failed"; return SNC_EDEVICE; }
  std::memcpy(ctx->h_in, hf.data(), S.e * 4);
  HIPCHK(hipMemcpyAsync(pr->ws + lay.sq_off, ctx->h_in, S.e * 4, hipMemcpyHostToDevice, stream));
  HIPCHK(hipStreamSynchronize(stream));
  pr->sq_ready = true;
  return SNC_OK;
}

// the projection step's layout and per-pair bounds, made on its first run
struct SqCache {
  SqfreeLayout S;
  std::vector<Quick> B;
};

int run_prepared_sqfree(snc_prepared* pr, void* d_gws, size_t gws_bytes, hipStream_t stream, snc_upoly* R,
                        snc_upoly* Gout) {
  snc_ctx* ctx = pr->c;
  const int n = pr->n;
  const BatchLayout& lay = pr->lay;
  if (!pr->sq_cache) {
    auto sc = std::make_shared<SqCache>();
    sqfree_layout(pr, sc->S, &sc->B);
    pr->sq_cache = sc;
  }
  const SqCache& SC = *static_cast<const SqCache*>(pr->sq_cache.get());
  const SqfreeLayout& S = SC.S;
  const std::vector<Quick>& B = SC.B;
  bool short_out = false;
  for (int i = 0; i < n; ++i) {
    const int need_deg = std::max(B[i].deg_bound, 0);
    if (Gout[i].deg < need_deg || Gout[i].nlimbs < B[i].out_nlimbs || !Gout[i].limbs) {
      Gout[i].deg = need_deg;
      Gout[i].nlimbs = B[i].out_nlimbs;
      short_out = true;
    }
  }
  if (short_out) { ctx->err = "gcd output buffer too small"; return SNC_ERANGE; }
  const size_t need = std::max<size_t>(S.fallback_words * 4, 256);
  if (!d_gws || gws_bytes < need) {
    ctx->err = "gcd workspace of " + std::to_string(gws_bytes) + " bytes, need " + std::to_string(need);
    return SNC_ENOMEM;
  }
  HIPCHK(hipSetDevice(ctx->device));
  uint32_t* gws = (uint32_t*)d_gws;
  if (!lay.dev.empty() && !pr->sq_ready) {
    const int st = sqfree_setup(pr, S, stream);
    if (st) return st;
  }
  uint32_t* ws = (uint32_t*)pr->ws;
  const int64_t base = (int64_t)(lay.sq_off / 4);
  int nitems = 0;
  for (size_t r = 0; r < pr->sq_ranges.size(); r += 4) nitems += pr->sq_ranges[r + 2];
  // with timing on: events around the Euclid launches
  const bool timing = ctx->timing;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (timing) {
    ctx->stage_names.clear(); ctx->stage_ms.clear(); ctx->stage_launches.clear();
    HIPCHK(hipEventCreate(&t0));
    HIPCHK(hipEventCreate(&t1));
  }
  // the Euclid and the download of e and d, following the interpolation
  auto euclid = [&](hipStream_t s) -> int {
    if (!nitems) return SNC_OK;
    const GcdDesc* descs_d = (const GcdDesc*)(ws + base + S.descs);
    const int32_t* items_d = (const int32_t*)(ws + base + S.items);
    if (timing) HIPCHK(hipEventRecord(t0, s));
    for (size_t r = 0; r < pr->sq_ranges.size(); r += 4) {
      const int* q = &pr->sq_ranges[r];  // register class, first item, items, largest degree
      const bool blocked = ctx->gcd_variant == 2 && gcd_lehmer_class(q[0]);
      if (blocked)
        launch_gcd_lehmer(descs_d, items_d + 2 * q[1], q[2], q[0], ws, s);
      else
        launch_gcd_euclid(descs_d, items_d + 2 * q[1], q[2], q[0], q[3], ws, s);
    }
    HIPCHK(hipGetLastError());
    if (timing) HIPCHK(hipEventRecord(t1, s));
    return SNC_OK;  // e and d land in mapped host memory: no download
  };
  // while the Euclid runs: cont R, which is also gcd(cont R, cont R') since
  // cont R divides every i R_i
  std::vector<BigInt> cont(n);
  auto contents = [&]() {
    for (int i = 0; i < n; ++i)
      if (R[i].deg >= 1) cont[i] = content_limbs(R[i]);
  };
  int st = run_prepared_fork(pr, stream, euclid, contents, R);
  if (st) return st;
  float euclid_ms = 0.f;
  if (timing) {
    if (nitems && !lay.dev.empty()) HIPCHK(hipEventElapsedTime(&euclid_ms, t0, t1));
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
  }
  const int32_t* ed = (const int32_t*)pr->h_ed;
  std::vector<int> job_of(n, -1);
  for (int j = 0; j < (int)lay.dev.size(); ++j) job_of[lay.dev[j]] = j;
  int full = 0;
  for (int i = 0; i < n; ++i) {
    const int dR = R[i].deg;
    const int j = job_of[i];
    bool done = false;
    if (j >= 0 && dR >= 1 && nitems) {
      const ResJob& J = lay.jobs[j];
      const int32_t* e = ed + S.job_base[j];
      const int32_t* d = ed + (S.d - S.e) + S.job_base[j];
      for (int q = 0; q < J.k && !done; ++q) done = d[q] == dR && e[q] == 0;
    }
    if (done) {
      UPoly G1;
      G1.c = {cont[i]};
      st = write_upoly(G1, &Gout[i], ctx->err);
      if (st) return st;
      continue;
    }
    // the full modular gcd of R (also the host-only cases: R zero or constant)
    st = gcd_run(ctx, 1, &R[i], nullptr, true, gws, gws_bytes, stream, &Gout[i]);
    if (st) return st;
    if (dR >= 1) ++full;
  }
  if (timing) {  // the Euclid on the resultant's primes, and the pairs that needed the full gcd
    if (!full) { ctx->stage_names.clear(); ctx->stage_ms.clear(); ctx->stage_launches.clear(); }
    ctx->stage_names.push_back("sqfree_euclid");
    ctx->stage_ms.push_back(euclid_ms);
    ctx->stage_launches.push_back(nitems);
    ctx->stage_names.push_back("sqfree_full_gcd");
    ctx->stage_ms.push_back(0.f);
    ctx->stage_launches.push_back(full);
  }
  return SNC_OK;
}

// ---------------------------------------------------------------------------
// Square-free factorisation by Yun's algorithm (Section 2.1: the square-free
// part of R and the multiplicities of its roots).  With P the primitive part
// of a (positive leading coefficient):
//   g = gcd(P, P'),  b_1 = P / g,  c_1 = P' / g;
//   for i = 1, 2, ...: d_i = c_i - b_i',  f_i = gcd(b_i, d_i),
//                      b_{i+1} = b_i / f_i,  c_{i+1} = d_i / f_i,
// until b_i is constant; P = prod f_i^i, the f_i square-free and pairwise
// coprime.  Every step is one modular gcd (the batched driver above) and
// its exact quotients are the cofactors that the driver's certificate
// already lifted, so no division of polynomials is done.
// ---------------------------------------------------------------------------
static void to_limbs(const UPoly& A, std::vector<uint32_t>& buf, snc_upoly& u) {
  int nl = 1;
  for (const auto& x : A.c) nl = std::max(nl, x.twos_limbs());
  buf.assign(std::max<size_t>(A.c.size(), 1) * nl, 0u);
  for (size_t j = 0; j < A.c.size(); ++j) (void)A.c[j].to_twos(buf.data() + j * nl, nl);
  u = snc_upoly{buf.data(), A.deg(), nl};
}

static UPoly poly_sub(const UPoly& A, const UPoly& B) {
  UPoly R;
  R.c.resize(std::max(A.c.size(), B.c.size()));
  for (size_t j = 0; j < R.c.size(); ++j) {
    if (j < A.c.size() && j < B.c.size()) R.c[j] = A.c[j] - B.c[j];
    else if (j < A.c.size()) R.c[j] = A.c[j];
    else R.c[j] = -B.c[j];
  }
  trim(R);
  return R;
}

// gcd(a, b) and the exact cofactors a / gcd, b / gcd
static int gcd_with_cofactors(snc_ctx* ctx, const UPoly& a, const UPoly& b, void* d_ws, size_t ws_bytes,
                              hipStream_t stream, UPoly& g, UPoly& qa, UPoly& qb) {
  std::vector<uint32_t> la, lb;
  snc_upoly ua, ub;
  to_limbs(a, la, ua);
  to_limbs(b, lb, ub);
  snc_plan pl{};
  int st = gcd_plan(1, &ua, &ub, false, nullptr, &pl);
  if (st) return st;
  std::vector<uint32_t> lo((size_t)(std::max(pl.deg_bound, 0) + 1) * pl.out_nlimbs, 0u);
  snc_upoly uo{lo.data(), pl.deg_bound, pl.out_nlimbs};
  st = gcd_run(ctx, 1, &ua, &ub, false, d_ws, ws_bytes, stream, &uo, &qa, &qb);
  if (st) return st;
  int nl = 1;
  return parse_upoly(&uo, g, nl, ctx->err);
}

// ---- content in y: h = gcd(f_0, f_1, ...) of the rows of f in Z[x] ----
// The rows are paired and their gcds taken in one batch per level of a
// binary tree (a level of constants finishes on the host).
static int bipoly_rows(const snc_bipoly* f, std::vector<UPoly>& rows, std::string& err) {
  rows.clear();
  if (!f) { err = "null polynomial"; return SNC_EINVAL; }
  if (f->dy < 0) return SNC_OK;
  if (f->dx < 0 || f->nlimbs < 1 || !f->limbs) { err = "bivariate polynomial: bad sizes"; return SNC_EINVAL; }
  for (int i = 0; i <= f->dy; ++i) {
    snc_upoly v{const_cast<uint32_t*>(f->limbs) + (size_t)i * (f->dx + 1) * f->nlimbs, f->dx, f->nlimbs};
    UPoly r;
    int nl = 1;
    const int st = parse_upoly(&v, r, nl, err);
    if (st) return st;
    if (!r.c.empty()) rows.push_back(std::move(r));
  }
  return SNC_OK;
}

// one level: the gcds of rows 2i and 2i+1 (an odd last row is carried)
static int content_level(snc_ctx* ctx, const std::vector<UPoly>& rows, void* d_ws, size_t ws_bytes,
                         hipStream_t stream, std::vector<UPoly>* next, size_t* ws_need) {
  const int np = (int)rows.size() / 2;
  std::vector<std::vector<uint32_t>> la(np), lb(np), lo(np);
  std::vector<snc_upoly> ua(np), ub(np), uo(np);
  for (int i = 0; i < np; ++i) {
    to_limbs(rows[2 * i], la[i], ua[i]);
    to_limbs(rows[2 * i + 1], lb[i], ub[i]);
  }
  std::vector<snc_plan> each(np);
  snc_plan tot{};
  int st = gcd_plan(np, ua.data(), ub.data(), false, each.data(), &tot);
  if (st) return st;
  if (ws_need) *ws_need = tot.workspace_bytes;
  if (!next) return SNC_OK;
  if (tot.workspace_bytes > ws_bytes) {
    ctx->err = "content_y: a level of the row gcds needs " + std::to_string(tot.workspace_bytes) +
               " bytes of workspace";
    return SNC_ENOMEM;
  }
  for (int i = 0; i < np; ++i) {
    lo[i].assign((size_t)(std::max(each[i].deg_bound, 0) + 1) * each[i].out_nlimbs, 0u);
    uo[i] = snc_upoly{lo[i].data(), each[i].deg_bound, each[i].out_nlimbs};
  }
  st = gcd_run(ctx, np, ua.data(), ub.data(), false, d_ws, ws_bytes, stream, uo.data());
  if (st) return st;
  next->assign(np, UPoly());
  for (int i = 0; i < np; ++i) {
    int nl = 1;
    st = parse_upoly(&uo[i], (*next)[i], nl, ctx->err);
    if (st) return st;
  }
  if (rows.size() % 2) next->push_back(rows.back());
  return SNC_OK;
}

// gcd of the non-zero polynomials in rows (consumed), positive leading coefficient
static int content_rows(snc_ctx* ctx, std::vector<UPoly>& rows, void* d_ws, size_t ws_bytes, hipStream_t stream,
                        UPoly& h) {
  int st = SNC_OK;
  h = UPoly();
  if (rows.empty()) return SNC_OK;  // f = 0
  while (rows.size() > 1) {
    std::vector<UPoly> next;
    st = content_level(ctx, rows, d_ws, ws_bytes, stream, &next, nullptr);
    if (st) return st;
    rows.swap(next);
  }
  h = std::move(rows[0]);
  if (h.c.back().neg)
    for (auto& x : h.c) x = -x;
  return SNC_OK;
}

static int content_y_run(snc_ctx* ctx, const snc_bipoly* f, void* d_ws, size_t ws_bytes, hipStream_t stream,
                         UPoly& h) {
  std::vector<UPoly> rows;
  const int st = bipoly_rows(f, rows, ctx->err);
  if (st) return st;
  return content_rows(ctx, rows, d_ws, ws_bytes, stream, h);
}

// degree and size bounds of the content and the workspace of the first level
static int content_y_plan(const snc_bipoly* f, snc_plan* out) {
  std::string err;
  std::vector<UPoly> rows;
  int st = bipoly_rows(f, rows, err);
  if (st) return st;
  *out = snc_plan{};
  out->out_nlimbs = 1;
  if (rows.empty()) return SNC_OK;
  // h divides the row of least degree: Mignotte bounds its coefficients by 2^deg ||row||_1
  size_t best = 0;
  for (size_t i = 1; i < rows.size(); ++i)
    if (rows[i].deg() < rows[best].deg()) best = i;
  int nl = 1;
  for (const auto& x : rows[best].c) nl = std::max(nl, x.twos_limbs());
  out->deg_bound = rows[best].deg();
  out->out_nlimbs = nl + (out->deg_bound + (int)std::ceil(std::log2(out->deg_bound + 2.0))) / 32 + 1;
  size_t need = 0;
  if (rows.size() > 1) {
    st = content_level(nullptr, rows, nullptr, 0, nullptr, nullptr, &need);
    if (st) return st;
  }
  out->workspace_bytes = need;
  return SNC_OK;
}

// ---- FastLift's Q = res_y(f_x / h, f_y / h), h = gcd(f_x, f_y) ----------
// rows of f in y with their positions (zero rows kept, trailing ones dropped)
static int bipoly_all_rows(const snc_bipoly* f, std::vector<UPoly>& rows, std::string& err) {
  rows.clear();
  if (!f) { err = "null polynomial"; return SNC_EINVAL; }
  if (f->dy < 0) return SNC_OK;
  if (f->dx < 0 || f->nlimbs < 1 || !f->limbs) { err = "bivariate polynomial: bad sizes"; return SNC_EINVAL; }
  rows.resize(f->dy + 1);
  for (int i = 0; i <= f->dy; ++i) {
    snc_upoly v{const_cast<uint32_t*>(f->limbs) + (size_t)i * (f->dx + 1) * f->nlimbs, f->dx, f->nlimbs};
    int nl = 1;
    const int st = parse_upoly(&v, rows[i], nl, err);
    if (st) return st;
  }
  while (!rows.empty() && rows.back().c.empty()) rows.pop_back();
  return SNC_OK;
}

static void partials(const std::vector<UPoly>& f, std::vector<UPoly>& fx, std::vector<UPoly>& fy) {
  fx.assign(f.size(), UPoly());
  for (size_t i = 0; i < f.size(); ++i) derivative(f[i], fx[i]);
  while (!fx.empty() && fx.back().c.empty()) fx.pop_back();
  fy.assign(f.size() > 1 ? f.size() - 1 : 0, UPoly());
  for (size_t i = 1; i < f.size(); ++i)
    for (const auto& x : f[i].c) fy[i - 1].c.push_back(x.mul_small((uint32_t)i));
}

// degree in y of gcd(a(x0, y), b(x0, y)) mod p, or -1 when a leading
// coefficient in y vanishes at x0 mod p (the point says nothing)
static int ygcd_degree_mod(const std::vector<UPoly>& a, const std::vector<UPoly>& b, uint32_t p, uint32_t x0) {
  auto at = [&](const std::vector<UPoly>& f) {
    std::vector<uint64_t> v(f.size(), 0);
    for (size_t i = 0; i < f.size(); ++i) {
      uint64_t acc = 0;
      for (size_t k = f[i].c.size(); k-- > 0;) acc = (acc * x0 + f[i].c[k].smod(p)) % p;
      v[i] = acc;
    }
    return v;
  };
  std::vector<uint64_t> A = at(a), B = at(b);
  if (A.empty() || B.empty() || A.back() == 0 || B.back() == 0) return -1;
  auto inv = [&](uint64_t x) {
    uint64_t r = 1, e = p - 2;
    while (e) { if (e & 1) r = r * x % p; x = x * x % p; e >>= 1; }
    return r;
  };
  while (!B.empty()) {
    while (A.size() >= B.size()) {  // A <- A mod B
      const uint64_t q = A.back() * inv(B.back()) % p;
      const size_t s = A.size() - B.size();
      for (size_t i = 0; i < B.size(); ++i) A[s + i] = (A[s + i] + p - q * B[i] % p) % p;
      while (!A.empty() && A.back() == 0) A.pop_back();
      if (A.empty()) break;
    }
    std::swap(A, B);
  }
  return (int)A.size() - 1;
}

// degree of gcd(a mod p, b mod p), or -1 when a leading coefficient vanishes mod p
static int gcd_degree_mod(const UPoly& a, const UPoly& b, uint32_t p) {
  auto red = [&](const UPoly& f) {
    std::vector<uint64_t> v(f.c.size());
    for (size_t k = 0; k < f.c.size(); ++k) v[k] = f.c[k].smod(p);
    return v;
  };
  std::vector<uint64_t> A = red(a), B = red(b);
  if (A.empty() || B.empty() || A.back() == 0 || B.back() == 0) return -1;
  auto inv = [&](uint64_t x) {
    uint64_t r = 1, e = p - 2;
    while (e) { if (e & 1) r = r * x % p; x = x * x % p; e >>= 1; }
    return r;
  };
  while (!B.empty()) {
    while (A.size() >= B.size()) {
      const uint64_t q = A.back() * inv(B.back()) % p;
      const size_t s = A.size() - B.size();
      for (size_t i = 0; i < B.size(); ++i) A[s + i] = (A[s + i] + p - q * B[i] % p) % p;
      while (!A.empty() && A.back() == 0) A.pop_back();
      if (A.empty()) break;
    }
    std::swap(A, B);
  }
  return (int)A.size() - 1;
}

// exact quotient of polynomials in Z[x]; false if h does not divide a
static bool poly_divexact(const UPoly& a, const UPoly& h, UPoly& q) {
  q.c.assign(a.c.size() >= h.c.size() ? a.c.size() - h.c.size() + 1 : 0, BigInt());
  UPoly r = a;
  while (r.c.size() >= h.c.size() && !r.c.empty()) {
    const size_t s = r.c.size() - h.c.size();
    BigInt c;
    if (!div_exact(r.c.back(), h.c.back(), c)) return false;
    q.c[s] = c;
    for (size_t i = 0; i < h.c.size(); ++i) r.c[s + i] = r.c[s + i] - c * h.c[i];
    trim(r);
  }
  trim(q);
  return r.c.empty();
}

// rows -> limbs of a snc_bipoly view (buf keeps the limbs)
static snc_bipoly bipoly_of(const std::vector<UPoly>& rows, std::vector<uint32_t>& buf) {
  if (rows.empty()) return snc_bipoly{nullptr, -1, 0, 1};
  int nl = 1, dx = 0;
  for (const auto& r : rows) {
    dx = std::max(dx, r.deg());
    for (const auto& x : r.c) nl = std::max(nl, x.twos_limbs());
  }
  buf.assign(rows.size() * (size_t)(dx + 1) * nl, 0u);
  for (size_t i = 0; i < rows.size(); ++i)
    for (size_t k = 0; k < rows[i].c.size(); ++k)
      (void)rows[i].c[k].to_twos(buf.data() + (i * (size_t)(dx + 1) + k) * nl, nl);
  return snc_bipoly{buf.data(), (int32_t)rows.size() - 1, dx, nl};
}

static int content_rows_multi(snc_ctx* ctx, std::vector<std::vector<UPoly>>& rows, void* d_ws, size_t ws_bytes,
                              hipStream_t stream, std::vector<UPoly>& h, size_t* first_need);

// ---- bivariate gcd in Z[x, y] (FastLift's h = gcd(f_x, f_y) when it depends on y) ----
// Brown's dense modular method on the device (k_ygcd per (prime, point),
// the interpolation and Chinese-remainder kernels of the resultant per
// coefficient in y), certified by exact division on the host.
static int poly_gcd1(snc_ctx* ctx, const UPoly& a, const UPoly& b, void* d_ws, size_t ws_bytes, hipStream_t stream,
                     UPoly& g) {
  if (a.c.empty() && b.c.empty()) { g = UPoly(); return SNC_OK; }
  std::vector<uint32_t> la, lb;
  snc_upoly ua, ub;
  to_limbs(a, la, ua);
  to_limbs(b, lb, ub);
  snc_plan pl{};
  int st = gcd_plan(1, &ua, &ub, false, nullptr, &pl);
  if (st) return st;
  if (pl.workspace_bytes > ws_bytes) { ctx->err = "bivariate gcd: a gcd in Z[x] needs " + std::to_string(pl.workspace_bytes) + " bytes of workspace"; return SNC_ENOMEM; }
  std::vector<uint32_t> lo((size_t)(std::max(pl.deg_bound, 0) + 1) * pl.out_nlimbs, 0u);
  snc_upoly uo{lo.data(), pl.deg_bound, pl.out_nlimbs};
  st = gcd_run(ctx, 1, &ua, &ub, false, d_ws, ws_bytes, stream, &uo);
  if (st) return st;
  int nl = 1;
  return parse_upoly(&uo, g, nl, ctx->err);
}

// a / h in Z[x][y] (rows in y): long division in y with exact divisions in Z[x]; false if inexact
static bool bivariate_divexact(const std::vector<UPoly>& a, const std::vector<UPoly>& h, std::vector<UPoly>& q) {
  std::vector<UPoly> r = a;
  while (!r.empty() && r.back().c.empty()) r.pop_back();
  const int dh = (int)h.size() - 1;
  q.assign(r.size() >= h.size() ? r.size() - h.size() + 1 : 0, UPoly());
  while (!r.empty() && (int)r.size() - 1 >= dh) {
    const int sft = (int)r.size() - 1 - dh;
    UPoly c;
    if (!poly_divexact(r.back(), h.back(), c)) return false;
    for (int i = 0; i <= dh; ++i) {
      UPoly prod;
      prod.c.assign(c.c.size() + h[i].c.size() - 1, BigInt());
      if (c.c.empty() || h[i].c.empty()) prod.c.clear();
      for (size_t u = 0; u < c.c.size(); ++u)
        for (size_t v = 0; v < h[i].c.size(); ++v) prod.c[u + v] = prod.c[u + v] + c.c[u] * h[i].c[v];
      trim(prod);
      r[sft + i] = poly_sub(r[sft + i], prod);
    }
    q[sft] = std::move(c);
    while (!r.empty() && r.back().c.empty()) r.pop_back();
  }
  while (!q.empty() && q.back().c.empty()) q.pop_back();
  return r.empty();
}

// P(x) -> P(x - s)
static void taylor_shift_back(UPoly& P, int64_t s) {
  const int n = P.deg();
  if (n < 1 || s == 0) return;
  const uint32_t m = (uint32_t)(s < 0 ? -s : s);
  for (int i = 0; i < n; ++i)
    for (int j = n - 1; j >= i; --j) {
      const BigInt t = P.c[j + 1].mul_small(m);
      P.c[j] = s > 0 ? P.c[j] - t : P.c[j] + t;  // c_j += (-s) c_{j+1}
    }
}

static uint64_t eval_mod(const UPoly& P, uint64_t x, uint32_t p) {
  uint64_t acc = 0;
  for (size_t k = P.c.size(); k-- > 0;) acc = (acc * x + P.c[k].smod(p)) % p;
  return acc;
}

static int max_rowdeg(const std::vector<UPoly>& R) {
  int d = 0;
  for (const auto& r : R) d = std::max(d, r.deg());
  return d;
}

// device part of one attempt: images at x = j + shift for the first k primes,
// then (if the gcd degree e > 0 is the same at every image) W's coefficients
// 0..e in x by interpolation and Chinese remaindering
struct YgcdLayout {
  size_t jr = 0, jobs = 0, pref_red = 0, pref_ip = 0, pref_crt = 0, pref_crt2 = 0, list_crt = 0, zero = 0, e_out = 0;
  size_t coef = 0, res = 0, regions = 0, total = 0;
  int64_t n1 = 0, L = 1, job_words = 0;
};

static void ygcd_layout(int k, int T, int nl, int Dx, int emax, YgcdLayout& Y) {
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  Y = YgcdLayout();
  Y.n1 = Dx + 1;
  Y.L = (30 * (int64_t)k + 31) / 32 + 1;
  const int nj = emax + 1;
  size_t off = 0;
  Y.jr = off; off = al(off + sizeof(ResJob));
  Y.jobs = off; off = al(off + sizeof(ResJob) * nj);
  Y.pref_red = off; off = al(off + 16);
  Y.pref_ip = off; off = al(off + 8 * (nj + 1));
  Y.pref_crt = off; off = al(off + 8 * (nj + 1));
  Y.pref_crt2 = off; off = al(off + 8 * (nj + 1));
  Y.list_crt = off; off = al(off + 4 * nj);
  Y.zero = off; off = al(off + 4);
  Y.e_out = off; off = al(off + 4 * (size_t)k * Y.n1);
  Y.coef = off; off = al(off + 4 * (size_t)T * nl);
  Y.res = off; off = al(off + 4 * (size_t)T * k);
  Y.regions = off;
  const size_t nqw = (size_t)k * ((Y.n1 + 63) / 64) * 64;
  Y.job_words = (int64_t)(align_words((size_t)k * Y.n1) * 2 + align_words(nqw) + align_words((size_t)Y.n1 * k) +
                          align_words((size_t)Y.n1 * Y.L));
  Y.total = Y.regions + 4 * (size_t)Y.job_words * nj;
}

static int bivariate_gcd_run(snc_ctx* ctx, const std::vector<UPoly>& A, const std::vector<UPoly>& B, void* d_ws,
                             size_t ws_bytes, hipStream_t stream, std::vector<UPoly>& H) {
  H.clear();
  // contents in y and primitive parts
  std::vector<std::vector<UPoly>> rows(2);
  for (const auto& r : A) if (!r.c.empty()) rows[0].push_back(r);
  for (const auto& r : B) if (!r.c.empty()) rows[1].push_back(r);
  std::vector<UPoly> cont;
  int st = content_rows_multi(ctx, rows, d_ws, ws_bytes, stream, cont, nullptr);
  if (st) return st;
  UPoly c;
  st = poly_gcd1(ctx, cont[0], cont[1], d_ws, ws_bytes, stream, c);
  if (st) return st;
  std::vector<UPoly> Ap(A.size()), Bp(B.size());
  for (size_t i = 0; i < A.size(); ++i)
    if (!A[i].c.empty() && !poly_divexact(A[i], cont[0], Ap[i])) { ctx->err = "bivariate gcd: content"; return SNC_EINTERNAL; }
  for (size_t i = 0; i < B.size(); ++i)
    if (!B[i].c.empty() && !poly_divexact(B[i], cont[1], Bp[i])) { ctx->err = "bivariate gcd: content"; return SNC_EINTERNAL; }
  const int mA = (int)Ap.size() - 1, mB = (int)Bp.size() - 1;
  if (mA == 0 || mB == 0) { H = {c}; return SNC_OK; }  // a primitive part of y-degree 0 is 1
  UPoly gam;
  st = poly_gcd1(ctx, Ap.back(), Bp.back(), d_ws, ws_bytes, stream, gam);
  if (st) return st;
  const int dxA = max_rowdeg(Ap), dxB = max_rowdeg(Bp);
  const int Dx = gam.deg() + std::min(dxA, dxB);
  const int emax = std::min(mA, mB);
  if (Dx > MAX_D || std::max(mA, mB) > MAXY_GEN) { ctx->err = "bivariate gcd: degrees beyond the supported range"; return SNC_ENOTSUP; }
  // residues layout: A rows, B rows (dense rectangles), gamma
  const int offA = 0, offB = (mA + 1) * (dxA + 1), offG = offB + (mB + 1) * (dxB + 1);
  const int T = offG + gam.deg() + 1;
  int nl = 1;
  for (const auto* P : {&Ap, &Bp})
    for (const auto& r : *P) for (const auto& x : r.c) nl = std::max(nl, x.twos_limbs());
  for (const auto& x : gam.c) nl = std::max(nl, x.twos_limbs());
  std::vector<uint32_t> coef((size_t)T * nl, 0u);  // limb-major [nl][T]
  auto put = [&](int t, const BigInt& v) {
    std::vector<uint32_t> tmp(nl);
    (void)v.to_twos(tmp.data(), nl);
    for (int l = 0; l < nl; ++l) coef[(size_t)l * T + t] = tmp[l];
  };
  for (int i = 0; i <= mA; ++i) for (size_t k2 = 0; k2 < Ap[i].c.size(); ++k2) put(offA + i * (dxA + 1) + (int)k2, Ap[i].c[k2]);
  for (int i = 0; i <= mB; ++i) for (size_t k2 = 0; k2 < Bp[i].c.size(); ++k2) put(offB + i * (dxB + 1) + (int)k2, Bp[i].c[k2]);
  for (size_t k2 = 0; k2 < gam.c.size(); ++k2) put(offG + (int)k2, gam.c[k2]);
  // first prime count: coefficients of A, B and gamma, with room for the growth of a factor
  double bits = 0;
  for (const auto* P : {&Ap, &Bp})
    for (const auto& r : *P) for (const auto& x : r.c) bits = std::max(bits, (double)x.bitlen());
  for (const auto& x : gam.c) bits = std::max(bits, (double)x.bitlen());
  const Tables& Tb = tables();
  auto primes_for = [&](double b) { int k = 1; while (k < KMAX && Tb.lg[k] <= b + 2.0) ++k; return k; };
  int k = std::max(2, primes_for(bits + Dx + emax + std::log2((double)Dx + 2.0) * (emax + 1) + 16.0));
  int64_t shift = 0;
  const CrtTables tb = global_crt_tables();
  HIPCHK(hipSetDevice(ctx->device));
  for (int attempt = 0; attempt < 12; ++attempt) {
    // points whose leading coefficients or gamma vanish mod a prime are avoided by shifting the point set
    for (int tries = 0; tries < 64; ++tries) {
      bool ok = true;
      for (int i = 0; i < k && ok; ++i) {
        const uint32_t p = Tb.p[i];
        for (int j = 0; j <= Dx && ok; ++j) {
          const uint64_t x = ((uint64_t)j + (uint64_t)shift) % p;
          ok = eval_mod(Ap.back(), x, p) && eval_mod(Bp.back(), x, p) && eval_mod(gam, x, p);
        }
      }
      if (ok) break;
      shift += Dx + 1 + 7 * tries;
    }
    YgcdLayout Y;
    ygcd_layout(k, T, nl, Dx, emax, Y);
    if (Y.total > ws_bytes) {
      ctx->err = "bivariate gcd: " + std::to_string(k) + " primes need " + std::to_string(Y.total) + " bytes of workspace";
      return SNC_ENOMEM;
    }
    uint8_t* ws = (uint8_t*)d_ws;
    // upload block: the reduction job, the coefficient limbs
    std::vector<uint8_t> hdr(Y.regions, 0);
    ResJob jr{};
    jr.k = k; jr.T = T; jr.nl = nl;
    jr.coef_off = (int64_t)(Y.coef / 4);
    jr.res_off = (int64_t)(Y.res / 4);
    std::memcpy(hdr.data() + Y.jr, &jr, sizeof jr);
    const int64_t pr[2] = {0, (int64_t)k * ((T + 255) / 256)};
    std::memcpy(hdr.data() + Y.pref_red, pr, sizeof pr);
    std::memcpy(hdr.data() + Y.coef, coef.data(), coef.size() * 4);
    HIPCHK(hipMemcpyAsync(ws, hdr.data(), Y.regions, hipMemcpyHostToDevice, stream));
    launch_reduce((const ResJob*)(ws + Y.jr), (const int64_t*)(ws + Y.pref_red), 1, pr[1], (const uint32_t*)ws,
                  (uint32_t*)ws, nullptr, stream);
    YGcdArgs ya{};
    ya.primes = tb.primes; ya.res = (const uint32_t*)(ws + Y.res); ya.T = T; ya.k = k; ya.npts = (int)Y.n1;
    ya.mA = mA; ya.dxA = dxA; ya.offA = offA; ya.mB = mB; ya.dxB = dxB; ya.offB = offB;
    ya.offG = offG; ya.dg = gam.deg(); ya.emax = emax; ya.cap = std::max(mA, mB); ya.shift = (uint32_t)shift;
    ya.e_out = (int32_t*)(ws + Y.e_out);
    ya.w = (uint32_t*)ws;
    ya.w_off = (int64_t)(Y.regions / 4);  // pts region of job i at regions + i job_words
    ya.w_stride = Y.job_words;
    launch_ygcd(ya, stream);
    HIPCHK(hipGetLastError());
    std::vector<int32_t> e((size_t)k * Y.n1);
    HIPCHK(hipMemcpyAsync(e.data(), ws + Y.e_out, e.size() * 4, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    const int emin = *std::min_element(e.begin(), e.end());
    const int emx = *std::max_element(e.begin(), e.end());
    if (emin < 0 || emin != emx) { shift += Dx + 1; continue; }  // a bad or unlucky image: other points
    if (emin == 0) { H = {c}; return SNC_OK; }                     // the primitive parts are coprime
    // interpolation and Chinese remaindering of W's coefficients 0..emin (jobs 0..emin)
    const int nj = emin + 1;
    std::vector<ResJob> jobs(nj);
    for (int i = 0; i < nj; ++i) {
      ResJob& J = jobs[i];
      std::memset(&J, 0, sizeof J);
      J.D = Dx; J.k = k; J.L = (int)Y.L; J.nl = 1;
      int64_t w = (int64_t)(Y.regions / 4) + (int64_t)i * Y.job_words;
      J.pts_off = w; w += (int64_t)align_words((size_t)k * Y.n1);
      J.val_off = w; w += (int64_t)align_words((size_t)k * Y.n1);
      J.nq_off = w; w += (int64_t)align_words((size_t)k * ((Y.n1 + 63) / 64) * 64);
      J.dig_off = w; w += (int64_t)align_words((size_t)Y.n1 * k);
      J.out_off = w;
    }
    const bool blk = interp_blk_fits(Dx, k);
    std::vector<int64_t> pip(nj + 1, 0), pcr(nj + 1, 0), pcc(nj + 1, 0);
    const int cc = crt_small_class(k);
    for (int i = 0; i < nj; ++i) {
      pip[i + 1] = pip[i] + (blk ? (int64_t)k * ((Y.n1 + 63) / 64) : k);
      pcr[i + 1] = pcr[i] + (cc >= 0 ? (Y.n1 + 63) / 64 : (Y.n1 + CRT_COEF_PER_BLOCK - 1) / CRT_COEF_PER_BLOCK);
      pcc[i + 1] = pcc[i] + (Y.n1 + CRT_COMB_PER_BLOCK - 1) / CRT_COMB_PER_BLOCK;
    }
    std::vector<int32_t> lst(nj);
    for (int i = 0; i < nj; ++i) lst[i] = i;
    HIPCHK(hipMemcpyAsync(ws + Y.jobs, jobs.data(), sizeof(ResJob) * nj, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(ws + Y.pref_ip, pip.data(), 8 * (nj + 1), hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(ws + Y.pref_crt, pcr.data(), 8 * (nj + 1), hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(ws + Y.pref_crt2, pcc.data(), 8 * (nj + 1), hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(ws + Y.list_crt, lst.data(), 4 * nj, hipMemcpyHostToDevice, stream));
    const ResJob* jd = (const ResJob*)(ws + Y.jobs);
    uint32_t* zero = (uint32_t*)(ws + Y.zero);
    if (blk) launch_interp_blk(jd, (const int64_t*)(ws + Y.pref_ip), nj, pip[nj], (uint32_t*)ws, zero, stream);
    else launch_interp(jd, (const int64_t*)(ws + Y.pref_ip), nj, pip[nj], Dx, (uint32_t*)ws, zero, stream);
    if (cc >= 0) {
      launch_crt_small(cc, jd, (const int32_t*)(ws + Y.list_crt), (const int64_t*)(ws + Y.pref_crt), nj, pcr[nj],
                       (uint32_t*)ws, stream);
    } else {
      launch_crt_digits(tb, jd, (const int32_t*)(ws + Y.list_crt), (const int64_t*)(ws + Y.pref_crt), nj, pcr[nj],
                        (uint32_t*)ws, stream);
      launch_crt_combine(tb, jd, (const int32_t*)(ws + Y.list_crt), (const int64_t*)(ws + Y.pref_crt2), nj, pcc[nj],
                         k, (uint32_t*)ws, stream);
    }
    HIPCHK(hipGetLastError());
    std::vector<uint32_t> outl((size_t)nj * Y.n1 * Y.L);
    for (int i = 0; i < nj; ++i)
      HIPCHK(hipMemcpyAsync(outl.data() + (size_t)i * Y.n1 * Y.L, ws + 4 * (size_t)jobs[i].out_off,
                            4 * (size_t)Y.n1 * Y.L, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    std::vector<UPoly> W(nj);
    for (int i = 0; i < nj; ++i) {
      W[i].c.resize(Y.n1);
      for (int64_t t = 0; t < Y.n1; ++t)
        W[i].c[t] = BigInt::from_twos(outl.data() + ((size_t)i * Y.n1 + t) * Y.L, (int)Y.L);
      trim(W[i]);
      taylor_shift_back(W[i], shift);
    }
    // h0 = pp_y(W): W's rows divided by their gcd in Z[x]
    std::vector<std::vector<UPoly>> wr(1);
    for (const auto& r : W) if (!r.c.empty()) wr[0].push_back(r);
    std::vector<UPoly> wc;
    st = content_rows_multi(ctx, wr, d_ws, ws_bytes, stream, wc, nullptr);
    if (st) return st;
    std::vector<UPoly> h0(nj), qa, qb;
    bool good = !wc[0].c.empty();
    for (int i = 0; i < nj && good; ++i)
      good = W[i].c.empty() || poly_divexact(W[i], wc[0], h0[i]);
    if (good && bivariate_divexact(Ap, h0, qa) && bivariate_divexact(Bp, h0, qb)) {
      H.resize(nj);
      for (int i = 0; i < nj; ++i) {
        // H_i = c h0_i
        H[i].c.assign(h0[i].c.empty() ? 0 : h0[i].c.size() + c.c.size() - 1, BigInt());
        for (size_t u = 0; u < h0[i].c.size(); ++u)
          for (size_t v = 0; v < c.c.size(); ++v) H[i].c[u + v] = H[i].c[u + v] + h0[i].c[u] * c.c[v];
        trim(H[i]);
      }
      if (!H.back().c.empty() && H.back().c.back().neg)
        for (auto& r : H) for (auto& x : r.c) x = -x;
      return SNC_OK;
    }
    k = std::min(KMAX, 2 * k);  // too few primes for W's coefficients
  }
  ctx->err = "bivariate gcd: no certified result";
  return SNC_EINTERNAL;
}

// workspace of the bivariate gcd's device pass with up to four times the first prime count
static size_t bivariate_gcd_ws(const std::vector<UPoly>& A, const std::vector<UPoly>& B) {
  const int mA = (int)A.size() - 1, mB = (int)B.size() - 1;
  if (mA < 1 || mB < 1) return 0;
  const int dxA = max_rowdeg(A), dxB = max_rowdeg(B);
  const int Dx = std::max(dxA, dxB) + std::min(dxA, dxB);
  double bits = 0;
  int nl = 1;
  for (const auto* P : {&A, &B})
    for (const auto& r : *P) for (const auto& x : r.c) { bits = std::max(bits, (double)x.bitlen()); nl = std::max(nl, x.twos_limbs()); }
  const Tables& Tb = tables();
  int k = 1;
  const int emax = std::min(mA, mB);
  while (k < KMAX && Tb.lg[k] <= bits + Dx + emax + std::log2((double)Dx + 2.0) * (emax + 1) + 18.0) ++k;
  k = std::min(KMAX, 4 * std::max(k, 2));
  const int T = (mA + 1) * (dxA + 1) + (mB + 1) * (dxB + 1) + Dx + 1;
  YgcdLayout Y;
  ygcd_layout(k, T, nl + 1, Dx, emax, Y);
  return Y.total;
}

static int fastlift_q_run(snc_ctx* ctx, const snc_bipoly* f, void* d_ws, size_t ws_bytes, hipStream_t stream,
                          snc_upoly* out) {
  std::vector<UPoly> rows, fx, fy;
  int st = bipoly_all_rows(f, rows, ctx->err);
  if (st) return st;
  partials(rows, fx, fy);
  if (fx.empty() || fy.empty()) {  // f_x = 0 or f_y = 0: h = the other one, Q of a constant (or 0)
    ctx->err = "fastlift Q: f_x or f_y is zero (f constant in x or in y)";
    return SNC_ENOTSUP;
  }
  // certify deg_y gcd(f_x, f_y) = 0 at a (prime, point)
  const Tables& T = tables();
  bool ydeg0 = false;
  for (int a = 0, tries = 0; a < 64 && tries < 4 && !ydeg0; ++a) {
    const int d = ygcd_degree_mod(fx, fy, T.p[a], (uint32_t)(a + 2));
    if (d < 0) continue;
    ++tries;
    ydeg0 = d == 0;
  }
  if (!ydeg0) {  // h depends on y: the bivariate modular gcd, then exact division of f_x and f_y
    std::vector<UPoly> H, qx, qy;
    st = bivariate_gcd_run(ctx, fx, fy, d_ws, ws_bytes, stream, H);
    if (st) return st;
    if (!bivariate_divexact(fx, H, qx) || !bivariate_divexact(fy, H, qy)) {
      ctx->err = "fastlift Q: h does not divide f_x, f_y";
      return SNC_EINTERNAL;
    }
    std::vector<uint32_t> bx, by;
    const snc_bipoly px = bipoly_of(qx, bx), py = bipoly_of(qy, by);
    return snc_resultant_y(ctx, &px, &py, d_ws, ws_bytes, stream, out);
  }
  // h in Z[x]: the gcd of every row of f_x and f_y
  std::vector<UPoly> all;
  for (const auto* v : {&fx, &fy})
    for (const auto& r : *v)
      if (!r.c.empty()) all.push_back(r);
  // two rows with a constant gcd mod p make h an integer: the gcd of all coefficients
  bool integer_h = false;
  if (all.size() >= 2)
    for (int a = 0, tries = 0; a < 16 && tries < 3 && !integer_h; ++a) {
      const int d = gcd_degree_mod(all[0], all[1], T.p[a]);
      if (d < 0) continue;
      ++tries;
      integer_h = d == 0;
    }
  UPoly h;
  if (integer_h) {
    BigInt g;
    for (const auto& r : all)
      for (const auto& x : r.c) g = BigInt::gcd(g, x);
    g.neg = false;
    h.c = {g};
  } else {
    st = content_rows(ctx, all, d_ws, ws_bytes, stream, h);
    if (st) return st;
  }
  const bool unit = h.deg() == 0 && h.c[0].mag.size() == 1 && h.c[0].mag[0] == 1;
  if (!unit) {
    for (auto* v : {&fx, &fy})
      for (auto& r : *v) {
        UPoly q;
        if (!poly_divexact(r, h, q)) { ctx->err = "fastlift Q: content does not divide a row"; return SNC_EINTERNAL; }
        r = std::move(q);
      }
  }
  std::vector<uint32_t> bx, by;
  const snc_bipoly px = bipoly_of(fx, bx), py = bipoly_of(fy, by);
  return snc_resultant_y(ctx, &px, &py, d_ws, ws_bytes, stream, out);
}

static int fastlift_q_plan(const snc_bipoly* f, snc_plan* out) {
  std::string err;
  std::vector<UPoly> rows, fx, fy;
  int st = bipoly_all_rows(f, rows, err);
  if (st) return st;
  partials(rows, fx, fy);
  *out = snc_plan{};
  out->out_nlimbs = 1;
  if (fx.empty() || fy.empty()) return SNC_OK;
  std::vector<uint32_t> bx, by;
  const snc_bipoly px = bipoly_of(fx, bx), py = bipoly_of(fy, by);
  st = snc_resultant_y_plan(&px, &py, out);
  if (st) return st;
  std::vector<UPoly> all;
  for (const auto* v : {&fx, &fy})
    for (const auto& r : *v)
      if (!r.c.empty()) all.push_back(r);
  size_t need = 0;
  if (all.size() > 1) {
    st = content_level(nullptr, all, nullptr, 0, nullptr, nullptr, &need);
    if (st) return st;
  }
  // a y-dependent h: the bivariate gcd's device pass (its plan, a bound for up to four times its first primes)
  out->workspace_bytes = std::max({out->workspace_bytes, need, bivariate_gcd_ws(fx, fy)});
  return SNC_OK;
}

struct SqfResult {
  BigInt content;
  std::vector<UPoly> f;
  std::vector<int> m;
};

static int sqfree_run(snc_ctx* ctx, const snc_upoly* a, void* d_ws, size_t ws_bytes, hipStream_t stream,
                      SqfResult& R) {
  R = SqfResult();
  UPoly A;
  int nl = 1;
  int st = parse_upoly(a, A, nl, ctx->err);
  if (st) return st;
  if (A.c.empty()) return SNC_OK;  // zero: content 0, no factors
  R.content = content(A);
  if (A.c.back().neg) R.content = -R.content;
  if (A.deg() == 0) return SNC_OK;
  UPoly P, dP;
  if (!scale_exact(A, BigInt::from_u64(1), R.content, P)) { ctx->err = "sqfree: content"; return SNC_EINTERNAL; }
  derivative(P, dP);
  UPoly g, b, c;
  st = gcd_with_cofactors(ctx, P, dP, d_ws, ws_bytes, stream, g, b, c);
  if (st) return st;
  for (int i = 1; b.deg() > 0; ++i) {
    if (i > P.deg()) { ctx->err = "sqfree: multiplicity above the degree"; return SNC_EINTERNAL; }
    UPoly db;
    derivative(b, db);
    const UPoly d = poly_sub(c, db);
    UPoly f, bn, cn;
    st = gcd_with_cofactors(ctx, b, d, d_ws, ws_bytes, stream, f, bn, cn);
    if (st) return st;
    if (f.deg() > 0) { R.f.push_back(f); R.m.push_back(i); }
    b = std::move(bn);
    c = std::move(cn);
  }
  return SNC_OK;
}

// sizes of a gcd problem from bounds: degrees da, db, coefficients below 2^ba, 2^bb
static void bound_quick(int da, int db, double ba, double bb, Quick& Q) {
  Q = Quick();
  Q.da = da;
  Q.db = db;
  Q.nla = (int)std::ceil((ba + 1.0) / 32.0) + 1;
  Q.nlb = (int)std::ceil((bb + 1.0) / 32.0) + 1;
  Q.nl = std::max(Q.nla, Q.nlb);
  Q.trivial = da <= 0 || db <= 0;
  if (Q.trivial) { Q.deg_bound = 0; Q.out_nlimbs = Q.nl; return; }
  const double la = std::log2(da + 1.0), lbn = std::log2(db + 1.0);
  Q.l2[0] = ba + 0.5 * la; Q.l1[0] = ba + la; Q.llc[0] = ba;
  Q.l2[1] = bb + 0.5 * lbn; Q.l1[1] = bb + lbn; Q.llc[1] = bb;
  GcdInfo sz;
  sz.da = da; sz.db = db;
  sz.l2a = Q.l2[0]; sz.l1a = Q.l1[0]; sz.l2b = Q.l2[1]; sz.l1b = Q.l1[1];
  sz.lbeta = std::min(Q.llc[0], Q.llc[1]);
  Q.deg_bound = std::min(da, db);
  Q.out_nlimbs = (int)std::ceil((Q.deg_bound + std::min(Q.l2[0], Q.l2[1]) + 3.0) / 32.0) + 1;
  double worst = 0.0;
  for (int e : {0, Q.deg_bound}) worst = std::max(worst, bits_needed_full(sz, e));
  Q.kmax = std::min(KMAX, std::max(primes_for_bits(worst), primes_for_bits(bits_needed_opt(sz))) + 12);
  Q.target0 = std::min(Q.kmax, std::max(3, primes_for_bits(bits_needed_opt(sz)) + 2));
}


// ---- arrangement batches: every curve and every pair of a set (Section 3) ----
// The contents in y of all curves come from one binary tree: per level, the
// rows of every curve are paired and all pairs of all curves go to one
// batched gcd submission (an odd last row is carried to the next level).
// first_need (if set): only the workspace of the first level is computed.
static int content_rows_multi(snc_ctx* ctx, std::vector<std::vector<UPoly>>& rows, void* d_ws, size_t ws_bytes,
                              hipStream_t stream, std::vector<UPoly>& h, size_t* first_need) {
  const size_t n = rows.size();
  for (;;) {
    std::vector<int> owner;
    std::vector<std::vector<uint32_t>> la, lb, lo;
    std::vector<snc_upoly> ua, ub, uo;
    for (size_t i = 0; i < n; ++i)
      for (size_t q = 0; q + 1 < rows[i].size(); q += 2) owner.push_back((int)i);
    const int np = (int)owner.size();
    if (np == 0) break;
    la.resize(np); lb.resize(np); lo.resize(np); ua.resize(np); ub.resize(np); uo.resize(np);
    {
      int t = 0;
      for (size_t i = 0; i < n; ++i)
        for (size_t q = 0; q + 1 < rows[i].size(); q += 2, ++t) {
          to_limbs(rows[i][q], la[t], ua[t]);
          to_limbs(rows[i][q + 1], lb[t], ub[t]);
        }
    }
    std::vector<snc_plan> each(np);
    snc_plan tot{};
    int st = gcd_plan(np, ua.data(), ub.data(), false, each.data(), &tot);
    if (st) return st;
    if (first_need) { *first_need = tot.workspace_bytes; return SNC_OK; }
    if (tot.workspace_bytes > ws_bytes) {
      ctx->err = "contents: a level of the row gcds needs " + std::to_string(tot.workspace_bytes) +
                 " bytes of workspace";
      return SNC_ENOMEM;
    }
    for (int t = 0; t < np; ++t) {
      lo[t].assign((size_t)(std::max(each[t].deg_bound, 0) + 1) * each[t].out_nlimbs, 0u);
      uo[t] = snc_upoly{lo[t].data(), each[t].deg_bound, each[t].out_nlimbs};
    }
    st = gcd_run(ctx, np, ua.data(), ub.data(), false, d_ws, ws_bytes, stream, uo.data());
    if (st) return st;
    std::vector<std::vector<UPoly>> next(n);
    int t = 0;
    for (size_t i = 0; i < n; ++i) {
      for (size_t q = 0; q + 1 < rows[i].size(); q += 2, ++t) {
        UPoly g;
        int nl = 1;
        st = parse_upoly(&uo[t], g, nl, ctx->err);
        if (st) return st;
        next[i].push_back(std::move(g));
      }
      if (rows[i].size() % 2) next[i].push_back(std::move(rows[i].back()));
    }
    rows.swap(next);
  }
  if (first_need) { *first_need = 0; return SNC_OK; }
  h.assign(n, UPoly());
  for (size_t i = 0; i < n; ++i) {
    if (rows[i].empty()) continue;  // f_i = 0
    h[i] = std::move(rows[i][0]);
    if (h[i].c.back().neg)
      for (auto& x : h[i].c) x = -x;
  }
  return SNC_OK;
}

// non-zero rows of each curve (the input of the content tree)
static int curves_rows(int n, const snc_bipoly* f, std::vector<std::vector<UPoly>>& rows, std::string& err) {
  rows.assign(n, {});
  for (int i = 0; i < n; ++i) {
    const int st = bipoly_rows(&f[i], rows[i], err);
    if (st) { err = "curve " + std::to_string(i) + ": " + err; return st; }
  }
  return SNC_OK;
}

// bound on a curve's content: it divides the row of least degree (Mignotte)
static void content_bound(const std::vector<UPoly>& rows, snc_plan& out) {
  out = snc_plan{};
  out.out_nlimbs = 1;
  if (rows.empty()) return;
  size_t best = 0;
  for (size_t i = 1; i < rows.size(); ++i)
    if (rows[i].deg() < rows[best].deg()) best = i;
  int nl = 1;
  for (const auto& x : rows[best].c) nl = std::max(nl, x.twos_limbs());
  out.deg_bound = rows[best].deg();
  out.out_nlimbs = nl + (out.deg_bound + (int)std::ceil(std::log2(out.deg_bound + 2.0))) / 32 + 1;
}

static int sqfree_plan(const snc_upoly* a, snc_plan* out) {
  std::string err;
  int st = check_upoly(a, err);
  if (st) return st;
  *out = snc_plan{};
  const int d = trimmed_degree(a);
  out->deg_bound = std::max(d, 0);
  out->out_nlimbs = a->deg >= 0 ? a->nlimbs : 1;
  out->workspace_bytes = 256;
  if (d < 1) return SNC_OK;
  snc_plan p0{};  // the first step, gcd(a, a'), on a's own sizes
  st = gcd_plan(1, a, nullptr, true, nullptr, &p0);
  if (st) return st;
  // later steps: b_i divides a, d_i = c_i - b_i' with c_i dividing a' (Mignotte: a factor of degree e
  // of a has coefficients below 2^e ||a||_2)
  double l2 = 0, l1 = 0, llc = 0;
  limb_norms(a->limbs, a->nlimbs, d, false, l2, l1, llc);
  const double ba = d + l2 + 1.0, bd = d + l2 + 2.0 * std::log2(d + 1.0) + 2.0;
  Quick Q;
  bound_quick(d, d - 1, ba, bd, Q);
  size_t w1 = 0;
  if (!Q.trivial) {
    std::vector<GcdProb> one(1);
    one[0].Q = Q;
    GcdBatchLayout L1;
    layout_batch(one, L1);
    w1 = L1.total * 4;
  }
  out->workspace_bytes = std::max<size_t>({p0.workspace_bytes, w1, 256});
  out->out_nlimbs = std::max(out->out_nlimbs, (int)std::ceil((ba + 1.0) / 32.0) + 1);
  return SNC_OK;
}

}  // namespace snc


// A prepared arrangement: the contents of the curves (computed at
// preparation), the primitive parts f_i / cont_y(f_i) and their
// y-derivatives as operand limbs, and the resultant pairs
//   (f~_i, d f~_i / dy) for every curve, then (f~_i, f~_j) for i < j,
// run as one prepared resultant batch.
struct snc_arrangement {
  snc_ctx* c = nullptr;
  int n = 0;
  std::vector<snc::UPoly> h;                    // contents
  std::vector<std::vector<uint32_t>> limbs;     // 2n operands: f~_i, then d f~_i / dy
  std::vector<snc_bipoly> ops;
  std::vector<snc_bipoly> F, G;                 // n + n(n-1)/2 pairs
  snc_prepared* prep = nullptr;
  void* prep_ws = nullptr;
  size_t prep_bytes = 0;
};

using namespace snc;

extern "C" {

int snc_gcd_z_plan(const snc_upoly* a, const snc_upoly* b, snc_plan* out) {
  if (!out || !a || !b) return SNC_EINVAL;
  return gcd_plan(1, a, b, false, nullptr, out);
}

int snc_gcd_z(snc_ctx* ctx, const snc_upoly* a, const snc_upoly* b, void* d_ws, size_t ws_bytes,
              void* stream, snc_upoly* out) {
  if (!ctx || !out || !a || !b) return SNC_EINVAL;
  return gcd_run(ctx, 1, a, b, false, d_ws, ws_bytes, (hipStream_t)stream, out);
}

int snc_gcd_z_batch_plan(int32_t n, const snc_upoly* a, const snc_upoly* b, snc_plan* out_each,
                         snc_plan* out_total) {
  if (n < 0 || (n > 0 && (!a || !b)) || !out_total) return SNC_EINVAL;
  return gcd_plan(n, a, b, false, out_each, out_total);
}

int snc_gcd_z_batch(snc_ctx* ctx, int32_t n, const snc_upoly* a, const snc_upoly* b, void* d_ws, size_t ws_bytes,
                    void* stream, snc_upoly* out) {
  if (!ctx || n < 0 || (n > 0 && (!a || !b || !out))) return SNC_EINVAL;
  if (n == 0) return SNC_OK;
  return gcd_run(ctx, n, a, b, false, d_ws, ws_bytes, (hipStream_t)stream, out);
}

int snc_prepared_sqfree_plan(const snc_prepared* prep, snc_plan* gcd_each, snc_plan* gcd_total) {
  if (!prep || !gcd_total) return SNC_EINVAL;
  *gcd_total = snc_plan{};
  return prepared_sqfree_plan(prep, gcd_each, gcd_total);
}

int snc_prepared_run_sqfree(snc_prepared* prep, void* d_gws, size_t gws_bytes, void* stream, snc_upoly* R,
                            snc_upoly* G) {
  if (!prep || !R || !G) return SNC_EINVAL;
  return run_prepared_sqfree(prep, d_gws, gws_bytes, (hipStream_t)stream, R, G);
}

int snc_prepared_sqfree_degrees(const snc_prepared* prep, int pair, int32_t* d, int32_t* e, int cap) {
  if (!prep || pair < 0 || pair >= prep->n || cap < 0 || (cap > 0 && (!d || !e))) return SNC_EINVAL;
  if (!prep->sq_cache || !prep->h_ed) return SNC_EINVAL;  // no projection step has run
  const SqfreeLayout& S = static_cast<const SqCache*>(prep->sq_cache.get())->S;
  const BatchLayout& lay = prep->lay;
  for (int j = 0; j < (int)lay.dev.size(); ++j) {
    if (lay.dev[j] != pair) continue;
    const ResJob& J = lay.jobs[j];
    if (J.D < 1) return 0;
    const int32_t* ed = (const int32_t*)prep->h_ed;
    for (int q = 0; q < std::min(J.k, cap); ++q) {
      e[q] = ed[S.job_base[j] + q];
      d[q] = ed[(S.d - S.e) + S.job_base[j] + q];
    }
    return J.k;
  }
  return 0;  // a trivial pair: no Euclid
}

int snc_gcd_z_deriv_plan(const snc_upoly* a, snc_plan* out) {
  if (!out || !a) return SNC_EINVAL;
  return gcd_plan(1, a, nullptr, true, nullptr, out);
}

int snc_fastlift_q_plan(const snc_bipoly* f, snc_plan* out) {
  if (!f || !out) return SNC_EINVAL;
  return fastlift_q_plan(f, out);
}

int snc_fastlift_q(snc_ctx* ctx, const snc_bipoly* f, void* d_ws, size_t ws_bytes, void* stream, snc_upoly* out) {
  if (!ctx || !f || !out) return SNC_EINVAL;
  HIPCHK(hipSetDevice(ctx->device));
  return fastlift_q_run(ctx, f, d_ws, ws_bytes, (hipStream_t)stream, out);
}

int snc_content_y_plan(const snc_bipoly* f, snc_plan* out) {
  if (!f || !out) return SNC_EINVAL;
  return content_y_plan(f, out);
}

int snc_content_y(snc_ctx* ctx, const snc_bipoly* f, void* d_ws, size_t ws_bytes, void* stream, snc_upoly* out) {
  if (!ctx || !f || !out) return SNC_EINVAL;
  HIPCHK(hipSetDevice(ctx->device));
  UPoly h;
  const int st = content_y_run(ctx, f, d_ws, ws_bytes, (hipStream_t)stream, h);
  if (st) return st;
  if (h.c.empty()) {
    out->deg = -1;
    return SNC_OK;
  }
  return write_upoly(h, out, ctx->err);
}

int snc_sqfree_plan(const snc_upoly* a, snc_plan* out) {
  if (!a || !out) return SNC_EINVAL;
  return sqfree_plan(a, out);
}

int snc_sqfree(snc_ctx* ctx, const snc_upoly* a, void* d_ws, size_t ws_bytes, void* stream, int32_t nlimbs,
               uint32_t* content, uint32_t* limbs, int32_t cap_coefs, int32_t* degs, int32_t* mults,
               int32_t max_factors, int32_t* nfactors) {
  if (!ctx || !a || !content || !nfactors || nlimbs < 1 || cap_coefs < 0 || max_factors < 0) return SNC_EINVAL;
  if (max_factors > 0 && (!degs || !mults)) return SNC_EINVAL;
  if (cap_coefs > 0 && !limbs) return SNC_EINVAL;
  HIPCHK(hipSetDevice(ctx->device));
  SqfResult R;
  int st = sqfree_run(ctx, a, d_ws, ws_bytes, (hipStream_t)stream, R);
  if (st) return st;
  *nfactors = (int32_t)R.f.size();
  size_t need = 0;
  for (const auto& f : R.f) need += f.c.size();
  if ((int32_t)R.f.size() > max_factors || need > (size_t)cap_coefs) {
    ctx->err = "sqfree: output capacity too small (" + std::to_string(R.f.size()) + " factors, " +
               std::to_string(need) + " coefficients)";
    return SNC_ERANGE;
  }
  if (!R.content.to_twos(content, nlimbs)) { ctx->err = "sqfree: content exceeds nlimbs"; return SNC_ERANGE; }
  size_t pos = 0;
  for (size_t i = 0; i < R.f.size(); ++i) {
    degs[i] = R.f[i].deg();
    mults[i] = R.m[i];
    for (const auto& x : R.f[i].c) {
      if (!x.to_twos(limbs + pos * nlimbs, nlimbs)) { ctx->err = "sqfree: coefficient exceeds nlimbs"; return SNC_ERANGE; }
      ++pos;
    }
  }
  return SNC_OK;
}

int snc_content_y_batch_plan(int32_t n, const snc_bipoly* f, snc_plan* out_each, snc_plan* out_total) {
  if (n < 0 || (n > 0 && !f) || !out_total) return SNC_EINVAL;
  std::string err;
  std::vector<std::vector<UPoly>> rows;
  int st = curves_rows(n, f, rows, err);
  if (st) return st;
  *out_total = snc_plan{};
  out_total->out_nlimbs = 1;
  for (int i = 0; i < n; ++i) {
    snc_plan b;
    content_bound(rows[i], b);
    if (out_each) out_each[i] = b;
    out_total->deg_bound = std::max(out_total->deg_bound, b.deg_bound);
    out_total->out_nlimbs = std::max(out_total->out_nlimbs, b.out_nlimbs);
  }
  size_t need = 0;
  std::vector<UPoly> h;
  st = content_rows_multi(nullptr, rows, nullptr, 0, nullptr, h, &need);
  if (st) return st;
  out_total->workspace_bytes = need;
  return SNC_OK;
}

static int write_upoly(snc_ctx* ctx, const UPoly& P, snc_upoly* out) {
  int nl = 1;
  for (const auto& x : P.c) nl = std::max(nl, x.twos_limbs());
  if (out->deg < P.deg() || out->nlimbs < nl || (!P.c.empty() && !out->limbs)) {
    out->deg = P.deg();
    out->nlimbs = nl;
    ctx->err = "output buffer too small";
    return SNC_ERANGE;
  }
  for (size_t k = 0; k < P.c.size(); ++k) (void)P.c[k].to_twos(out->limbs + k * out->nlimbs, out->nlimbs);
  out->deg = P.deg();
  return SNC_OK;
}

int snc_content_y_batch(snc_ctx* ctx, int32_t n, const snc_bipoly* f, void* d_ws, size_t ws_bytes, void* stream,
                        snc_upoly* out) {
  if (!ctx || n < 0 || (n > 0 && (!f || !out))) return SNC_EINVAL;
  std::vector<std::vector<UPoly>> rows;
  int st = curves_rows(n, f, rows, ctx->err);
  if (st) return st;
  std::vector<UPoly> h;
  st = content_rows_multi(ctx, rows, d_ws, ws_bytes, (hipStream_t)stream, h, nullptr);
  if (st) return st;
  int range = SNC_OK;
  for (int i = 0; i < n; ++i)
    if (write_upoly(ctx, h[i], &out[i]) == SNC_ERANGE) range = SNC_ERANGE;
  return range;
}

int snc_arrangement_prepare(snc_ctx* ctx, int32_t n, const snc_bipoly* curves, void* d_ws, size_t ws_bytes,
                            void* stream, snc_arrangement** out) {
  if (!ctx || !out || n < 0 || (n > 0 && !curves)) return SNC_EINVAL;
  *out = nullptr;
  std::vector<std::vector<UPoly>> rows;
  int st = curves_rows(n, curves, rows, ctx->err);
  if (st) return st;
  auto* A = new snc_arrangement();
  A->c = ctx;
  A->n = n;
  st = content_rows_multi(ctx, rows, d_ws, ws_bytes, (hipStream_t)stream, A->h, nullptr);
  if (st) { delete A; return st; }
  A->limbs.resize(2 * (size_t)n);
  A->ops.resize(2 * (size_t)n);
  for (int i = 0; i < n; ++i) {
    std::vector<UPoly> all, prim, dprim;
    st = bipoly_all_rows(&curves[i], all, ctx->err);
    if (st) { delete A; return st; }
    prim.resize(all.size());
    for (size_t r = 0; r < all.size(); ++r) {
      if (all[r].c.empty()) continue;
      if (!poly_divexact(all[r], A->h[i], prim[r])) {
        ctx->err = "arrangement: the content of curve " + std::to_string(i) + " does not divide a row";
        delete A;
        return SNC_EINTERNAL;
      }
    }
    while (!prim.empty() && prim.back().c.empty()) prim.pop_back();
    dprim.resize(prim.size() > 1 ? prim.size() - 1 : 0);
    for (size_t r = 1; r < prim.size(); ++r)
      for (const auto& x : prim[r].c) dprim[r - 1].c.push_back(x.mul_small((uint32_t)r));
    while (!dprim.empty() && dprim.back().c.empty()) dprim.pop_back();
    A->ops[i] = bipoly_of(prim, A->limbs[i]);
    A->ops[n + i] = bipoly_of(dprim, A->limbs[n + i]);
  }
  for (int i = 0; i < n; ++i) { A->F.push_back(A->ops[i]); A->G.push_back(A->ops[n + i]); }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) { A->F.push_back(A->ops[i]); A->G.push_back(A->ops[j]); }
  *out = A;
  return SNC_OK;
}

int snc_arrangement_plan(const snc_arrangement* A, snc_plan* content_each, snc_plan* res_each, snc_plan* res_total) {
  if (!A || !res_total) return SNC_EINVAL;
  if (content_each)
    for (int i = 0; i < A->n; ++i) {
      int nl = 1;
      for (const auto& x : A->h[i].c) nl = std::max(nl, x.twos_limbs());
      content_each[i] = snc_plan{};
      content_each[i].deg_bound = std::max(A->h[i].deg(), 0);
      content_each[i].out_nlimbs = nl;
    }
  return snc_resultant_y_batch_plan((int32_t)A->F.size(), A->F.data(), A->G.data(), res_each, res_total);
}

int snc_arrangement_run(snc_arrangement* A, void* d_ws, size_t ws_bytes, void* stream, snc_upoly* contents,
                        snc_upoly* resultants) {
  if (!A || (A->n > 0 && (!contents || !resultants))) return SNC_EINVAL;
  snc_ctx* ctx = A->c;
  int range = SNC_OK;
  for (int i = 0; i < A->n; ++i)
    if (write_upoly(ctx, A->h[i], &contents[i]) == SNC_ERANGE) range = SNC_ERANGE;
  if (range) return range;
  if (A->prep && (A->prep_ws != d_ws || A->prep_bytes != ws_bytes)) {
    destroy_prepared(A->prep);
    A->prep = nullptr;
  }
  if (!A->prep) {
    const int st = prepare_resultants(ctx, (int)A->F.size(), A->F.data(), A->G.data(), d_ws, ws_bytes,
                                      (hipStream_t)stream, /*graph=*/true, &A->prep);
    if (st) return st;
    A->prep_ws = d_ws;
    A->prep_bytes = ws_bytes;
  }
  return run_prepared(A->prep, (hipStream_t)stream, resultants);
}

int snc_arrangement_destroy(snc_arrangement* A) {
  if (!A) return SNC_EINVAL;
  if (A->prep) destroy_prepared(A->prep);
  delete A;
  return SNC_OK;
}

int snc_gcd_z_deriv(snc_ctx* ctx, const snc_upoly* a, void* d_ws, size_t ws_bytes, void* stream, snc_upoly* out) {
  if (!ctx || !out || !a) return SNC_EINVAL;
  return gcd_run(ctx, 1, a, nullptr, true, d_ws, ws_bytes, (hipStream_t)stream, out);
}

}  // extern "C"
