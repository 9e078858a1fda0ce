// Blocked Euclid for the square-free check of a resultant at high degree
// (Section 2.1, "Projection Phase": whether gcd(R, R') mod p is constant
// decides that R is square-free; Section 4, "Symbolic Speedups": the gcd
// follows the modular scheme of the resultant).  One workgroup of eight
// wavefronts per (problem, prime) instead of one wavefront.
//
// A run of normal remainder steps (each remainder one degree below its
// divisor, the generic case) is decided by the top coefficients alone: the
// multipliers of a block of s <= 31 steps depend only on the top 2s + 2
// coefficients of the two remainders, and the block acts on the full
// remainders as one 2x2 matrix M of polynomials of degree <= s:
//   (P', Q') = M (P, Q),  P-step: row_P <- a row_P + (b x + c) row_Q,
//                         Q-step: row_Q <- a row_Q + (b x + c) row_P,
// with the pseudo-remainder multipliers a = q0^2, b = -q0 n0,
// c = n0 q1 - q0 n1 of the dividend's top pair (n0, n1) and the divisor's
// (q0, q1).  Roles of the wavefronts in a block:
//   0  (leader)          the steps on the top 64 coefficients of P and Q
//                        (one per lane), publishing each step's multipliers;
//   1  (matrix builder)  M from the multipliers as they are published;
//   2..7 (followers)     the previous block's M applied to the full
//                        remainders in LDS: 64 products per coefficient.
// Between blocks all eight wavefronts compute the leader's next window (the
// top 64 coefficients of M times the remainders) as partial sums over four
// chunks of M's coefficients.  A step whose remainder loses its leading
// coefficient, or a divisor degree below LW_TAIL, ends the blocks: the
// remainders are brought up to date and wavefront 0 finishes with the
// register-resident Euclid.  Only the degrees leave the kernel: d = deg R
// mod p and e = deg gcd(R, R') mod p, as from the one-wavefront kernel.
//
// On gfx950 the leader's step costs about 460 cycles, as much as a whole step
// of the one-wavefront kernel: both are bound by the dependent chain of a
// step (the multipliers, one Montgomery product level, then the new top pair,
// another level, each with its reductions and cross-lane broadcasts), not by
// the O(deg) work the blocks move off the critical path.  The kernel is
// therefore an option (snc_set_gcd_variant 2), not the default.
#include <hip/hip_runtime.h>

#include "gcd_reg.hpp"
#include "snc_internal.hpp"

namespace snc {

namespace {

constexpr int LW_WAVES = 8;
constexpr int LW_THREADS = 64 * LW_WAVES;
constexpr int LW_STEPS = 31;      // steps per block: the window's 64 coefficients cover 2 * 31 + 2
constexpr int LW_TAIL = 16;       // no step with a divisor below this degree inside a block
constexpr int LW_PAD = 32;        // zero words below index 0 of every remainder (M has 32 coefficients)
constexpr int LW_OVER = 128;      // outputs past the nominal degree (zeros), covering earlier contents
constexpr int LW_SPIN = 1 << 16;  // bound of the matrix builder's waits for a step (a step takes < 1 us)

struct LwLayout {  // word offsets into the dynamic LDS
  int len;    // words per remainder after its pad
  int arr;    // [2 buffers][2 slots][LW_PAD + len], coefficient t of a remainder at LW_PAD + t
  int mrec;   // [2][128]: a block's M (canonical Montgomery), row P then row Q, each [M_.P (32) | M_.Q (32)]
  int coefs;  // [LW_STEPS][4]: a, b, c and a tag per step of the running block
  int part;   // [4][128]: partial sums of the leader's next window
  int ctl;    // [2]: per block parity, steps | abnormal << 8 | (block + 1) << 16; [2]: a wait ran out
  int sm;     // [2 * 64 * E]: level switches of the register Euclid
  int total;
};

__host__ __device__ constexpr LwLayout lw_layout(int E) {
  LwLayout L{};
  L.len = 64 * E + LW_OVER;
  L.arr = 0;
  L.mrec = L.arr + 4 * (LW_PAD + L.len);
  L.coefs = L.mrec + 2 * 128;
  L.part = L.coefs + 4 * LW_STEPS;
  L.ctl = L.part + 4 * 128;
  L.sm = L.ctl + 4;
  L.total = L.sm + 2 * 64 * E;
  return L;
}

static_assert((LW_PAD % 4) == 0 && (lw_layout(2).len % 4) == 0, "remainders start on 16-byte boundaries");

// Words the leader and the matrix builder exchange while both run: volatile
// and explicitly in LDS (a generic volatile pointer becomes FLAT accesses,
// whose stores need not become visible in order); a wavefront's LDS
// operations complete in order, so a reader that sees a step's tag sees the
// multipliers written before it.
typedef __attribute__((address_space(3))) volatile uint32_t lds_vu32;
__device__ __forceinline__ lds_vu32* lds_v(uint32_t* p) { return (lds_vu32*)p; }

__device__ __forceinline__ uint32_t* lw_poly(uint32_t* lds, const LwLayout& L, int buf, int slot) {
  return lds + L.arr + (2 * buf + slot) * (LW_PAD + L.len) + LW_PAD;
}

__device__ __forceinline__ uint32_t lane_prev(uint32_t v) {  // lane l gets lane l-1 (0 for lane 0)
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x138 /* wave_shr:1 */, 0xf, 0xf, true);
}

__device__ __forceinline__ uint32_t lw_bcast(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

// S 2^-32 mod p for a sum S < 2^64 of up to sixteen products of canonical
// values: S = hi 2^32 + lo with hi < 16 p^2 / 2^32 < 4p, taken below 2p,
// plus REDC(lo) <= p; the result is canonical.
__device__ __forceinline__ uint32_t lw_fold(uint64_t S, const PrimeC& c) {
  uint32_t hi = (uint32_t)(S >> 32);
  const uint32_t h2 = hi - 2 * c.p;
  hi = h2 < hi ? h2 : hi;
  return canon(hi + redc((uint64_t)(uint32_t)S, c.p, c.pinv), c.p);
}

// Block state every wavefront keeps (uniform).
struct LwBlock {
  int dP, dQ;  // nominal degrees of P and Q at the block's start
  int pslot;   // slot of P in the block's input buffer
  int s;       // steps of the block
  bool abn;    // the block's last step left a vanishing leading coefficient
  __device__ int dPo() const { return dP - 2 * ((s + 1) >> 1); }
  __device__ int dQo() const { return dQ - 2 * (s >> 1); }
};

// M (at Mrec) applied to the remainders of buffer ib (P in slot B.pslot)
// into buffer ob (P's image in the same slot): coefficients 0 .. nominal
// degree + LW_OVER, four consecutive coefficients per lane, tasks of 64
// lanes over wavefronts w0, w0 + nw, ... (a task's row of M is uniform).
__device__ void lw_apply(uint32_t* lds, const LwLayout& L, const LwBlock& B, const uint32_t* Mrec, int ib, int ob,
                         int w0, int nw, int wave, int lane, int over, const PrimeC& c) {
  const uint32_t* Pi = lw_poly(lds, L, ib, B.pslot);
  const uint32_t* Qi = lw_poly(lds, L, ib, 1 - B.pslot);
  uint32_t* Po = lw_poly(lds, L, ob, B.pslot);
  uint32_t* Qo = lw_poly(lds, L, ob, 1 - B.pslot);
  const int nP = min(L.len - 1, B.dPo() + over) + 1;  // outputs 0 .. nP-1 (nP <= len, a multiple of 4 or less)
  const int nQ = min(L.len - 1, B.dQo() + over) + 1;
  const int gP = (nP + 3) >> 2, gQ = (nQ + 3) >> 2;
  const int tP = (gP + 63) >> 6, tQ = (gQ + 63) >> 6;
  for (int task = wave - w0; task < tP + tQ; task += nw) {  // uniform: wave, tasks and rows
    const bool isQ = task >= tP;
    const int gl = isQ ? gQ : gP;
    const int graw = (isQ ? task - tP : task) * 64 + lane;
    // every lane loads its word of the row and computes (a lane past the last
    // group repeats the last one): the broadcasts below read all 64 lanes, so
    // nothing they depend on may sit under a lane-dependent branch
    const uint32_t rv = Mrec[(isQ ? 64 : 0) + lane];  // lane i: M_.P[i] (i < 32), M_.Q[i - 32]
    const int g = min(graw, gl - 1);
    const int m0 = 4 * g;
    uint32_t pv[36], qv[36];  // coefficients m0 - 32 .. m0 + 3
#pragma unroll
    for (int u = 0; u < 9; ++u) {
      const uint4 a = *(const uint4*)(Pi + m0 - 32 + 4 * u);
      const uint4 b = *(const uint4*)(Qi + m0 - 32 + 4 * u);
      pv[4 * u] = a.x; pv[4 * u + 1] = a.y; pv[4 * u + 2] = a.z; pv[4 * u + 3] = a.w;
      qv[4 * u] = b.x; qv[4 * u + 1] = b.y; qv[4 * u + 2] = b.z; qv[4 * u + 3] = b.w;
    }
    uint32_t out[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) out[r] = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // coefficients i of M in [16h, 16h + 16)
      uint64_t sp[4] = {0, 0, 0, 0}, sq[4] = {0, 0, 0, 0};
#pragma unroll
      for (int i = 16 * h; i < 16 * h + 16; ++i) {
        const uint64_t mp = lw_bcast(rv, i), mq = lw_bcast(rv, 32 + i);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          sp[r] += mp * pv[32 + r - i];
          sq[r] += mq * qv[32 + r - i];
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) out[r] = canon(out[r] + lw_fold(sp[r], c) + lw_fold(sq[r], c), c.p);
    }
    uint32_t* dst = isQ ? Qo : Po;
    if (graw < gl) *(uint4*)(dst + m0) = make_uint4(out[0], out[1], out[2], out[3]);
  }
}

// The register Euclid from the remainders P (degree <= dP) and Q in LDS, on
// the fewest slots per lane that hold them; returns the gcd's degree.
template <int E>
__device__ int lw_tail(const uint32_t* P, int dP, const uint32_t* Q, int dQ, uint32_t* sm, int lane,
                       const PrimeC& c) {
  constexpr int EN = next_slots(E);
  if constexpr (EN > 0) {
    if (max(dP, dQ) < 64 * EN) return lw_tail<EN>(P, dP, Q, dQ, sm, lane, c);
  }
  uint32_t X[E], Y[E];
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int i = lane * E + s;
    X[s] = i <= dP ? P[dP - i] : 0u;
    Y[s] = i <= dQ ? Q[dQ - i] : 0u;
  }
  const int dX = reg_trim<E>(X, dP, c);
  const int dY = reg_trim<E>(Y, dQ, c);
  if (dX < 0 && dY < 0) return -1;
  return euclid_levels<E>(X, dX, Y, dY, sm, lane, c);
}

template <int E>
__global__ __launch_bounds__(LW_THREADS) void k_gcd_lehmer(const GcdDesc* descs, const int32_t* items,
                                                           const PrimeC* primes, uint32_t* ws) {
  constexpr LwLayout L = lw_layout(E);
  extern __shared__ uint32_t lds[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform role branches and task loops
  const GcdDesc G = descs[items[2 * blockIdx.x]];
  const int slot = items[2 * blockIdx.x + 1];
  const int pidx = ((const int32_t*)(ws + G.slot_prime_off))[slot];
  const PrimeC c = primes[pidx];
  const int da = G.da;
  int32_t* outp = fused_out(G, ws);
  uint32_t* ctl = lds + L.ctl;

  // R and R' (Montgomery, ascending) into buffer 0; everything else zero
  for (int t = tid; t < L.sm; t += LW_THREADS) lds[t] = 0u;
  __syncthreads();
  {
    const uint32_t* va = G.vals + (int64_t)slot * G.vstride;
    uint32_t* X0 = lw_poly(lds, L, 0, 0);
    uint32_t* Y0 = lw_poly(lds, L, 0, 1);
    for (int t = tid; t <= da; t += LW_THREADS) {
      const uint32_t x = to_mont(va[t], c);
      X0[t] = x;
      if (t >= 1) Y0[t - 1] = mmulc(x, to_mont((uint32_t)t, c), c.p, c.pinv);
    }
  }
  __syncthreads();
  LwBlock B;
  B.pslot = 0;
  B.s = 0;
  B.abn = false;
  {
    const uint32_t* X0 = lw_poly(lds, L, 0, 0);
    const uint32_t* Y0 = lw_poly(lds, L, 0, 1);
    int dP = da;
    while (dP >= 0 && uni(X0[dP]) == 0) --dP;
    int dQ = da - 1;
    while (dQ >= 0 && uni(Y0[dQ]) == 0) --dQ;
    B.dP = dP;  // uniform (every lane read the same words): the block loop branches on the scalar unit
    B.dQ = dQ;
  }
  if (tid == 0) outp[G.d_off + slot] = B.dP;
  if (B.dP < 0) {
    if (tid == 0) outp[G.e_off + slot] = -1;
    return;
  }
  if (wave == 0) __builtin_amdgcn_s_setprio(3);  // the leader's steps are the critical path

  int cur = 0;  // buffer of the latest complete remainders (a block behind the leader while the followers run)
  LwBlock prev;  // the block before, whose M the followers apply
  prev.s = 0;
  bool have_prev = false;
  bool blocks = B.dP == B.dQ + 1 && B.dQ >= LW_TAIL;
  int k = 0;
  while (blocks) {
    const int par = k & 1;
    uint32_t* Mk = lds + L.mrec + 128 * par;
    if (wave == 0) {
      // ---- leader: window (top-aligned, element j in lane j) ----
      uint32_t Pw, Qw;
      if (k == 0) {
        const uint32_t* P = lw_poly(lds, L, cur, B.pslot);
        const uint32_t* Q = lw_poly(lds, L, cur, 1 - B.pslot);
        Pw = lane <= B.dP ? P[B.dP - lane] : 0u;
        Qw = lane <= B.dQ ? Q[B.dQ - lane] : 0u;
      } else {
        const uint32_t* pt = lds + L.part;
        Pw = canon(pt[lane] + pt[128 + lane] + pt[256 + lane] + pt[384 + lane], c.p);
        Qw = canon(pt[64 + lane] + pt[192 + lane] + pt[320 + lane] + pt[448 + lane], c.p);
      }
      uint32_t P1 = from_next_lane(Pw), P2 = from_next_lane(P1);
      uint32_t Q1 = from_next_lane(Qw), Q2 = from_next_lane(Q1);
      uint32_t p0 = uni(Pw), p1 = uni(P1), q0 = uni(Qw), q1 = uni(Q1);  // window values are canonical here
      int cdP = B.dP, cdQ = B.dQ, s = 0;
      bool abn = false;
      const uint32_t tag0 = (uint32_t)((k + 1) << 8);
      // multipliers of A <- prem(A, D) from the dividend's top pair (n0, n1)
      // and the divisor's (d0, d1), one Montgomery product in each of lanes
      // 0, 1, 2: a = d0^2, b = -d0 n0, c = n0 d1 - d0 n1 (the sum below 8 p^2);
      // lanes 0..2 publish them, then lane 0 the step's tag
      // per-lane operand masks (selects without branches)
      const uint32_t m0 = lane == 0 ? ~0u : 0u, m1 = lane == 1 ? ~0u : 0u, m2 = lane == 2 ? ~0u : 0u;
      auto coefs = [&](uint32_t n0, uint32_t n1, uint32_t d0, uint32_t d1, uint32_t& ma, uint32_t& mb,
                       uint32_t& mc) {
        const uint32_t u1 = (n0 & m2) | (d0 & ~m2);
        const uint32_t v1 = (d0 & m0) | ((c.p - n0) & m1) | (d1 & ~(m0 | m1));
        const uint32_t u2 = (c.p - d0) & m2;
        const uint32_t r = canon(redc((uint64_t)u1 * v1 + (uint64_t)u2 * n1, c.p, c.pinv), c.p);
        ma = lw_bcast(r, 0);
        mb = lw_bcast(r, 1);
        mc = lw_bcast(r, 2);
        lds_vu32* cw = lds_v(lds + L.coefs + 4 * s);
        if (lane < 3) cw[lane] = r;
        if (lane == 0) cw[3] = tag0 | (uint32_t)(s + 1);
      };
      while (true) {
        // P <- prem(P, Q)
        if (s >= LW_STEPS || cdQ < LW_TAIL) break;
        uint32_t ma, mb, mc;
        coefs(p0, p1, q0, q1, ma, mb, mc);
        Pw = mmul3(ma, P2, mb, Q2, mc, Q1, c.p, c.pinv);
        P1 = from_next_lane(Pw);
        P2 = from_next_lane(P1);
        p0 = uni(canon(Pw, c.p));  // uniform: the loop branches on the scalar unit
        p1 = uni(P1);
        cdP -= 2;
        ++s;
        if (p0 == 0) { abn = true; break; }
        // Q <- prem(Q, P)
        if (s >= LW_STEPS || cdP < LW_TAIL) break;
        coefs(q0, q1, p0, p1, ma, mb, mc);
        Qw = mmul3(ma, Q2, mb, P2, mc, P1, c.p, c.pinv);
        Q1 = from_next_lane(Qw);
        Q2 = from_next_lane(Q1);
        q0 = uni(canon(Qw, c.p));
        q1 = uni(Q1);
        cdQ -= 2;
        ++s;
        if (q0 == 0) { abn = true; break; }
      }
      if (lane == 0) *lds_v(ctl + par) = (uint32_t)(s | (abn ? 256 : 0) | ((k + 1) << 16));
    } else if (wave == 1) {
      // ---- matrix builder: M from the published multipliers ----
      uint32_t rowP = lane == 0 ? c.r1 : 0u;   // [M_PP | M_PQ]
      uint32_t rowQ = lane == 32 ? c.r1 : 0u;  // [M_QP | M_QQ]
      const uint32_t want = (uint32_t)(k + 1);
      for (int t = 0;; ++t) {
        uint4 cf;
        bool end = false;
        for (int spin = 0;; ++spin) {
          lds_vu32* cp = lds_v(lds + L.coefs + 4 * t);
          // the tag first, then the multipliers; uniform copies keep the loop
          // (and the lane shifts in it) on the whole wavefront
          if (uni(cp[3]) == ((want << 8) | (uint32_t)(t + 1))) {
            cf = make_uint4(uni(cp[0]), uni(cp[1]), uni(cp[2]), 0u);
            break;
          }
          const uint32_t ew = uni(*lds_v(ctl + par));
          if ((ew >> 16) == want && (int)(ew & 255) <= t) { end = true; break; }
          if (spin >= LW_SPIN) { end = true; ctl[2] = 1u; break; }
          __builtin_amdgcn_s_sleep(1);
        }
        if (end) break;
        if ((t & 1) == 0)
          rowP = mmul3(cf.x, rowP, cf.y, lane_prev(rowQ), cf.z, rowQ, c.p, c.pinv);
        else
          rowQ = mmul3(cf.x, rowQ, cf.y, lane_prev(rowP), cf.z, rowP, c.p, c.pinv);
      }
      Mk[lane] = canon(rowP, c.p);
      Mk[64 + lane] = canon(rowQ, c.p);
      ctl[par ^ 1] = 0u;  // the next block's end word (the block before read it long ago)
    } else if (have_prev) {
      // ---- followers: the previous block's M on the full remainders ----
      lw_apply(lds, L, prev, lds + L.mrec + 128 * (par ^ 1), cur, cur ^ 1, 2, LW_WAVES - 2, wave, lane, LW_OVER, c);
    }
    __syncthreads();
    // the block's outcome (all wavefronts)
    {
      const uint32_t ew = uni(ctl[par]);
      B.s = (int)(ew & 255);
      B.abn = (ew & 256) != 0;
    }
    if (have_prev) cur ^= 1;  // the followers brought the remainders up to the block's start
    const int dPo = B.dPo(), dQo = B.dQo();
    const bool odd = (B.s & 1) != 0;
    const int nP = odd ? dQo : dPo, nQ = odd ? dPo : dQo;  // degrees of the next P and Q
    const bool more = !B.abn && B.s > 0 && nQ >= LW_TAIL;
    if (more) {
      // partial sums of the next window: thread (chunk, output); outputs 0..63
      // the next P's top coefficients, 64..127 the next Q's
      const int o = tid & 127, ch = tid >> 7;
      const bool forP = o < 64;
      const int j = o & 63;
      const bool qrow = forP ? odd : !odd;
      const int m = (forP ? nP : nQ) - j;
      uint32_t acc = 0;
      if (m >= 0) {
        const int col = ch >> 1, i0 = 16 * (ch & 1);
        const uint32_t* Mr = Mk + (qrow ? 64 : 0) + 32 * col + i0;
        const uint32_t* src = lw_poly(lds, L, cur, col == 0 ? B.pslot : 1 - B.pslot) + m - i0;
        uint64_t S = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) S += (uint64_t)Mr[i] * src[-i];
        acc = lw_fold(S, c);
      }
      lds[L.part + 128 * ch + o] = acc;
    } else {
      // last block: its M on the full remainders (every wavefront)
      lw_apply(lds, L, B, Mk, cur, cur ^ 1, 0, LW_WAVES, wave, lane, 0, c);
    }
    __syncthreads();
    prev = B;
    have_prev = true;
    B.dP = nP;
    B.dQ = nQ;
    B.pslot = odd ? 1 - B.pslot : B.pslot;
    B.s = 0;
    ++k;
    if (!more) {
      cur ^= 1;
      blocks = false;
    }
  }
  if (wave != 0) return;
  if (k > 0) __builtin_amdgcn_s_setprio(0);
  const int e = lw_tail<E>(lw_poly(lds, L, cur, B.pslot), B.dP, lw_poly(lds, L, cur, 1 - B.pslot), B.dQ,
                           lds + L.sm, lane, c);
  if (lane == 0) outp[G.e_off + slot] = ctl[2] ? GCD_SLOT_UNUSABLE : e;
}

}  // namespace

size_t gcd_lehmer_lds_bytes(int slots) { return (size_t)lw_layout(slots).total * sizeof(uint32_t); }

bool gcd_lehmer_class(int slots) { return slots == 6 || slots == 9 || slots == 12 || slots == 16; }

void launch_gcd_lehmer(const GcdDesc* descs, const int32_t* items, int nitems, int slots, uint32_t* ws,
                       hipStream_t s) {
  if (nitems <= 0) return;
  const PrimeC* primes = global_crt_tables().primes;
  const size_t lds = gcd_lehmer_lds_bytes(slots);
  switch (slots) {
#define SNC_GCD_LW(E) \
    case E: hipLaunchKernelGGL(k_gcd_lehmer<E>, dim3(nitems), dim3(LW_THREADS), lds, s, descs, items, primes, ws); return;
    SNC_GCD_LW(6) SNC_GCD_LW(9) SNC_GCD_LW(12) SNC_GCD_LW(16)
#undef SNC_GCD_LW
    default: break;
  }
}

}  // namespace snc
