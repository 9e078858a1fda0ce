// Workspace layout and launch sequence of the resultant pipeline, shared by
// the single-resultant call (direct launches, optional per-stage timing) and
// the batched call (one captured HIP graph per batch shape, replayed).
#include <hip/hip_runtime.h>

#include <atomic>
#include <functional>
#include <thread>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "runtime_internal.hpp"

int snc_ctx::stage_in(size_t bytes) {
  if (bytes <= h_in_bytes) return SNC_OK;
  if (h_in) (void)hipHostFree(h_in);
  h_in = nullptr;
  size_t nb = std::max(bytes, h_in_bytes * 2);
  if (hipHostMalloc(&h_in, nb, hipHostMallocDefault) != hipSuccess) { h_in_bytes = 0; h_in = nullptr; return SNC_EDEVICE; }
  h_in_bytes = nb;
  return SNC_OK;
}

int snc_ctx::stage_out(size_t bytes) {
  if (bytes <= h_out_bytes) return SNC_OK;
  if (h_out) (void)hipHostFree(h_out);
  h_out = nullptr;
  size_t nb = std::max(bytes, h_out_bytes * 2);
  if (hipHostMalloc(&h_out, nb, hipHostMallocDefault) != hipSuccess) { h_out_bytes = 0; h_out = nullptr; return SNC_EDEVICE; }
  h_out_bytes = nb;
  return SNC_OK;
}

void snc_ctx::release() {
  if (gexec) (void)hipGraphExecDestroy(gexec);
  gexec = nullptr;
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  cap_stream = nullptr;
  if (side_stream) (void)hipStreamDestroy(side_stream);
  side_stream = nullptr;
  if (ev_mid) (void)hipEventDestroy(ev_mid);
  ev_mid = nullptr;
  if (fork_stream) (void)hipStreamDestroy(fork_stream);
  fork_stream = nullptr;
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  ev_fork = nullptr;
  if (ev_join) (void)hipEventDestroy(ev_join);
  ev_join = nullptr;
  for (auto e : events) (void)hipEventDestroy(e);
  events.clear();
  if (h_in) (void)hipHostFree(h_in);
  if (h_out) (void)hipHostFree(h_out);
  h_in = h_out = nullptr;
  h_in_bytes = h_out_bytes = 0;
}

namespace snc {

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

void layout_batch(const std::vector<ResPlan>& plans, BatchLayout& lay) {
  lay = BatchLayout();
  for (int i = 0; i < (int)plans.size(); ++i)
    if (!plans[i].trivial) lay.dev.push_back(i);
  const int NJ = (int)lay.dev.size();
  lay.jobs.resize(NJ);
  size_t off = 0;
  lay.jobs_off = off; off = align256(off + sizeof(ResJob) * NJ);
  int nrows = 0;
  for (int j = 0; j < NJ; ++j) nrows += 2 * plans[lay.dev[j]].rstride;
  lay.n_rows = nrows;
  lay.rows_off = off; off = align256(off + sizeof(RowDesc) * nrows);
  lay.pref_red = off; off = align256(off + 8 * (NJ + 1));
  lay.pref_interp = off; off = align256(off + 8 * (NJ + 1));
  lay.pref_interp_blk = off; off = align256(off + 8 * (NJ + 1));
  lay.pref_crtd = off; off = align256(off + 8 * (NJ + 1));
  lay.pref_crtc = off; off = align256(off + 8 * (NJ + 1));
  // one lane per coefficient pays off only when the batch's few-prime coefficients fill the device
  // (a wavefront per CU); otherwise the lanes go over the primes of each coefficient
  int64_t small_coefs = 0;
  for (int j = 0; j < NJ; ++j)
    if (crt_small_class(plans[lay.dev[j]].k) >= 0) small_coefs += plans[lay.dev[j]].D + 1;
  lay.crt_small_on = small_coefs >= CRT_SMALL_MIN_COEFS;
  for (int j = 0; j < NJ; ++j) {
    const int cc = lay.crt_small_on ? crt_small_class(plans[lay.dev[j]].k) : -1;
    if (cc >= 0) lay.n_crts_jobs[cc]++; else lay.n_crtb_jobs++;
  }
  for (int c = 0; c < NCRT_SMALL; ++c) {
    lay.pref_crts[c] = off; off = align256(off + 8 * (lay.n_crts_jobs[c] + 1));
    lay.list_crts[c] = off; off = align256(off + 4 * std::max(lay.n_crts_jobs[c], 1));
  }
  lay.list_crtb = off; off = align256(off + 4 * std::max(lay.n_crtb_jobs, 1));
  lay.pref_inst = off; off = align256(off + 8 * (NJ + 1));
  lay.pref_iw = off; off = align256(off + 8 * (NJ + 1));
  lay.list_iw = off; off = align256(off + 4 * std::max(NJ, 1));
  for (int j = 0; j < NJ; ++j) {
    const ResPlan& P = plans[lay.dev[j]];
    if (P.cls >= 0) lay.n_ee_jobs[P.cls]++; else lay.n_gen_jobs++;
  }
  for (int c = 0; c < NCLS; ++c) {
    lay.pref_ee[c] = off; off = align256(off + 8 * (lay.n_ee_jobs[c] + 1));
    lay.list_ee[c] = off; off = align256(off + 4 * std::max(lay.n_ee_jobs[c], 1));
  }
  lay.pref_gen = off; off = align256(off + 8 * (lay.n_gen_jobs + 1));
  lay.list_gen = off; off = align256(off + 4 * std::max(lay.n_gen_jobs, 1));
  lay.coef_off = off;
  size_t cw = 0;
  for (int j = 0; j < NJ; ++j) { const ResPlan& P = plans[lay.dev[j]]; cw += (size_t)P.T * P.nl; }
  lay.coef_words = cw;
  off = align256(off + 4 * cw);
  lay.header_bytes = off;
  // per-job device regions
  size_t w = off / 4;
  size_t coefw = lay.coef_off / 4;
  int rows = 0;
  for (int j = 0; j < NJ; ++j) {
    const ResPlan& P = plans[lay.dev[j]];
    ResJob& J = lay.jobs[j];
    std::memset(&J, 0, sizeof J);
    J.m = P.m; J.n = P.n;
    J.sign = (P.swap && ((P.m * P.n) & 1)) ? 1 : 0;
    J.D = P.D; J.k = P.k; J.T = P.T; J.L = P.L; J.nl = P.nl;
    J.rows_off = rows; J.rstride = P.rstride;
    rows += 2 * P.rstride;
    J.coef_off = (int64_t)coefw; coefw += (size_t)P.T * P.nl;
    const size_t n1 = (size_t)P.D + 1;
    J.res_off = (int64_t)w; w += align_words((size_t)P.k * P.T);
    J.val_off = (int64_t)w; w += align_words((size_t)P.k * n1);
    J.pts_off = (int64_t)w; w += align_words((size_t)P.k * n1);
    J.nq_off = (int64_t)w; w += align_words((size_t)P.k * ((n1 + 63) / 64) * 64);
    J.dig_off = (int64_t)w; w += align_words(n1 * P.k);
    J.acc_off = (int64_t)w;  // unused: the combine step keeps its accumulators in LDS
    lay.nb_red += (int64_t)P.k * ((P.T + 255) / 256);
    lay.nb_interp += P.k;
    lay.nb_interp_blk += (int64_t)P.k * ((n1 + 63) / 64);
    const int cc = lay.crt_small_on ? crt_small_class(P.k) : -1;
    if (cc >= 0) {
      lay.nb_crts[cc] += (int64_t)((n1 + 63) / 64);
    } else {
      lay.nb_crtd += (int64_t)((n1 + CRT_COEF_PER_BLOCK - 1) / CRT_COEF_PER_BLOCK);
      lay.nb_crtc += (int64_t)((n1 + CRT_COMB_PER_BLOCK - 1) / CRT_COMB_PER_BLOCK);
    }
    lay.max_k = std::max(lay.max_k, P.k);
    if (P.cls >= 0) {
      lay.nb_ee[P.cls] += (int64_t)P.k * ((n1 + EE_BLOCK - 1) / EE_BLOCK);
      lay.max_T_ee[P.cls] = std::max(lay.max_T_ee[P.cls], P.T);
    }
    else lay.n_gen_inst += (int64_t)P.k * n1;
    lay.total_inst += (int64_t)P.k * n1;
    lay.max_D = std::max(lay.max_D, P.D);
  }
  lay.interp_blk = NJ > 0 && interp_blk_fits(lay.max_D, lay.max_k);
  // many (resultant, prime) pairs: one wavefront each, no barriers between wavefronts
  int64_t npairs = 0;
  for (const ResJob& J : lay.jobs) npairs += J.k;
  lay.interp_w = NJ > 0 && !lay.interp_blk && lay.max_D <= IW_MAXD && npairs >= IW_MIN_PAIRS;
  // every job on the evaluation kernel's LDS variant: it reduces the inputs itself
  lay.reduce_in_eval = NJ > 0 && lay.n_gen_jobs == 0;
  for (int c = 0; c < NCLS; ++c)
    if (lay.n_ee_jobs[c] && !eval_elim_in_lds(lay.max_T_ee[c])) lay.reduce_in_eval = false;
  lay.abn_count_off = w * 4; w += 64;
  lay.ee_counter_off = w * 4; w += 64;
  lay.abn_list_off = w * 4;
  lay.abn_cap = abn_list_cap(lay.total_inst);
  w += align_words((size_t)lay.abn_cap * (sizeof(AbnEntry) / 4));
  lay.out_off = w * 4;
  size_t ow = 0;
  for (int j = 0; j < NJ; ++j) {
    const ResPlan& P = plans[lay.dev[j]];
    lay.jobs[j].out_off = (int64_t)(w + ow);
    ow += ((size_t)P.D + 1) * P.L;
  }
  lay.out_words = ow;
  w += align_words(ow);
  size_t nk = 0;
  for (const ResJob& J : lay.jobs) nk += J.k;
  lay.sq_off = w * 4;
  lay.sq_words = align_words(sizeof(GcdDesc) / 4 * std::max<size_t>(NJ, 1)) + align_words(2 * std::max<size_t>(nk, 1)) +
                 align_words(KMAX) + 2 * align_words(std::max<size_t>(nk, 1));
  w += lay.sq_words;
  lay.total_bytes = w * 4;
}

struct StageTimer {
  snc_ctx* c;
  hipStream_t s;
  bool on;
  int n = 0;
  void start() {
    if (!on) return;
    c->stage_names.clear(); c->stage_ms.clear(); c->stage_launches.clear();
    mark(nullptr, 0);
  }
  void mark(const char* name, int launches) {
    if (!on) return;
    if ((int)c->events.size() <= n) {
      hipEvent_t e;
      (void)hipEventCreate(&e);
      c->events.push_back(e);
    }
    (void)hipEventRecord(c->events[n], s);
    if (name) { c->stage_names.push_back(name); c->stage_launches.push_back(launches); }
    ++n;
  }
  void finish() {
    if (!on) return;
    for (int i = 1; i < n; ++i) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, c->events[i - 1], c->events[i]);
      c->stage_ms.push_back(ms);
    }
  }
};

// Device launch sequence for a laid-out batch (everything after the upload).
// part: PIPE_ALL, PIPE_TO_INTERP (reduction .. interpolation) or PIPE_CRT
void launch_pipeline(const BatchLayout& lay, uint8_t* ws, hipStream_t s, StageTimer* tm, int part,
                     const PipeFork& fk) {
  uint32_t* wsw = (uint32_t*)ws;
  const ResJob* jobs = (const ResJob*)(ws + lay.jobs_off);
  const RowDesc* rows = (const RowDesc*)(ws + lay.rows_off);
  const int NJ = (int)lay.jobs.size();
  uint32_t* abn_count = (uint32_t*)(ws + lay.abn_count_off);
  AbnEntry* abn_list = (AbnEntry*)(ws + lay.abn_list_off);
  if (part != PIPE_CRT) {
  // the counter is cleared by the previous run's interpolation (and at preparation)
  if (!lay.reduce_in_eval) launch_reduce(jobs, (const int64_t*)(ws + lay.pref_red), NJ, lay.nb_red, wsw, wsw, abn_count, s);
  if (tm) tm->mark("reduce", lay.reduce_in_eval ? 0 : 1);
  // one stage per register class (names: eval_elim_<width>), then the
  // jobs above the register classes
  static const char* const kEEStage[NCLS] = {"eval_elim_8", "eval_elim_16", "eval_elim_32", "eval_elim_40",
                                             "eval_elim_48", "eval_elim_64"};
  uint32_t* ee_counters = (uint32_t*)(ws + lay.ee_counter_off);
  bool persistent = false;
  for (int c = 0; c < NCLS; ++c) persistent |= lay.n_ee_jobs[c] && lay.ee_var[c].chunk > 0;
  if (persistent) launch_zero_u32(ee_counters, NCLS, s);  // a kernel, not a memset node
  for (int c = 0; c < NCLS; ++c) {
    if (!lay.n_ee_jobs[c]) continue;
    launch_eval_elim(c, lay.ee_var[c], ee_counters + c, jobs, (const int32_t*)(ws + lay.list_ee[c]),
                     (const int64_t*)(ws + lay.pref_ee[c]), lay.n_ee_jobs[c], lay.nb_ee[c], lay.max_T_ee[c], rows,
                     wsw, abn_count, abn_list, lay.abn_cap, lay.reduce_in_eval, s);
    if (tm) tm->mark(kEEStage[c], 1);
  }
  if (lay.n_gen_jobs) {
    launch_elim_general_all(jobs, (const int32_t*)(ws + lay.list_gen), (const int64_t*)(ws + lay.pref_gen),
                            lay.n_gen_jobs, lay.n_gen_inst, rows, wsw, s);
    if (tm) tm->mark("eval_elim_general", 1);
  }
  launch_elim_general(jobs, rows, wsw, abn_count, abn_list, lay.abn_cap, (const int64_t*)(ws + lay.pref_inst), NJ,
                      s);
  if (tm) tm->mark("elim_general", 1);
  if (lay.interp_blk)
    launch_interp_blk(jobs, (const int64_t*)(ws + lay.pref_interp_blk), NJ, lay.nb_interp_blk, wsw, abn_count, s);
  else if (lay.interp_w)
    launch_interp_w(jobs, (const int32_t*)(ws + lay.list_iw), (const int64_t*)(ws + lay.pref_iw), NJ, lay.nb_interp,
                    lay.max_D, wsw, abn_count, s);
  else
    launch_interp(jobs, (const int64_t*)(ws + lay.pref_interp), NJ, lay.nb_interp, lay.max_D, wsw, abn_count, s);
  if (tm) tm->mark("interp", 1);
  }
  if (part == PIPE_TO_INTERP) return;
  static const char* const kCrtStage[NCRT_SMALL] = {"crt_small_32", "crt_small_64", "crt_small_128"};
  // The class with the most primes has the fewest, longest workgroups (one
  // round on the device, each bound by its own latency): on a branch it runs
  // beside the other classes instead of after them.
  int nsmall = 0, top = -1;
  for (int c = 0; c < NCRT_SMALL; ++c)
    if (lay.n_crts_jobs[c]) { ++nsmall; top = c; }
  const bool branch = fk.stream && !tm && nsmall >= 2;
  if (branch) {
    (void)hipEventRecord(fk.fork, s);
    (void)hipStreamWaitEvent(fk.stream, fk.fork, 0);
    launch_crt_small(top, jobs, (const int32_t*)(ws + lay.list_crts[top]), (const int64_t*)(ws + lay.pref_crts[top]),
                     lay.n_crts_jobs[top], lay.nb_crts[top], wsw, fk.stream);
  }
  for (int c = 0; c < NCRT_SMALL; ++c) {
    if (!lay.n_crts_jobs[c] || (branch && c == top)) continue;
    launch_crt_small(c, jobs, (const int32_t*)(ws + lay.list_crts[c]), (const int64_t*)(ws + lay.pref_crts[c]),
                     lay.n_crts_jobs[c], lay.nb_crts[c], wsw, s);
    if (tm) tm->mark(kCrtStage[c], 1);
  }
  if (branch) {
    (void)hipEventRecord(fk.join, fk.stream);
    (void)hipStreamWaitEvent(s, fk.join, 0);
  }
  if (lay.n_crtb_jobs) {
    const CrtTables tb = global_crt_tables();
    const int32_t* lb = (const int32_t*)(ws + lay.list_crtb);
    launch_crt_digits(tb, jobs, lb, (const int64_t*)(ws + lay.pref_crtd), lay.n_crtb_jobs, lay.nb_crtd, wsw, s);
    if (tm) tm->mark("crt_digits", 1);
    launch_crt_combine(tb, jobs, lb, (const int64_t*)(ws + lay.pref_crtc), lay.n_crtb_jobs, lay.nb_crtc, lay.max_k,
                       wsw, s);
    if (tm) tm->mark("crt_combine", 1);
  }
}

// Essential lane-operations of one evaluation block (64 instances): Horner
// in x^4 (1.5 per coefficient), the fused remainder steps (5 per entry of
// each remainder), the first remainder's elementary steps and the final
// powers and inversion.
static int64_t eval_block_cost(const ResPlan& P) {
  const int64_t m = P.m, n = P.n;
  return 3 * (int64_t)P.T / 2 + 5 * n * (n + 1) / 2 + 4 * n * std::max<int64_t>(m - n - 1, 0) + 300;
}

// Fill the upload block: job descriptors, row descriptors, block prefixes,
// class job lists and the packed input coefficients.
void fill_header(const BatchLayout& lay, const std::vector<ResPlan>& plans, const std::vector<Operand>& F,
                 const std::vector<Operand>& G, uint8_t* h) {
  const int NJ = (int)lay.dev.size();
  std::memcpy(h + lay.jobs_off, lay.jobs.data(), sizeof(ResJob) * NJ);
  RowDesc* rows = (RowDesc*)(h + lay.rows_off);
  uint32_t* coef = (uint32_t*)(h + lay.coef_off);
  int64_t* pr = (int64_t*)(h + lay.pref_red);
  int64_t* pi = (int64_t*)(h + lay.pref_interp);
  int64_t* pib = (int64_t*)(h + lay.pref_interp_blk);
  int64_t* pd = (int64_t*)(h + lay.pref_crtd);
  int64_t* pc = (int64_t*)(h + lay.pref_crtc);
  int64_t* pn = (int64_t*)(h + lay.pref_inst);
  int64_t* pe[NCLS];
  int32_t* le[NCLS];
  int ne[NCLS] = {0};
  for (int c = 0; c < NCLS; ++c) {
    pe[c] = (int64_t*)(h + lay.pref_ee[c]);
    le[c] = (int32_t*)(h + lay.list_ee[c]);
    pe[c][0] = 0;
  }
  int64_t* ps[NCRT_SMALL];
  int32_t* ls[NCRT_SMALL];
  int ns[NCRT_SMALL] = {0};
  for (int c = 0; c < NCRT_SMALL; ++c) {
    ps[c] = (int64_t*)(h + lay.pref_crts[c]);
    ls[c] = (int32_t*)(h + lay.list_crts[c]);
    ps[c][0] = 0;
  }
  int32_t* lbig = (int32_t*)(h + lay.list_crtb);
  int nbig = 0;
  std::vector<std::pair<int64_t, int>> by_cost[NCLS];  // (work per block, job) per register class
  int64_t* pg = (int64_t*)(h + lay.pref_gen);
  int32_t* lg = (int32_t*)(h + lay.list_gen);
  int ng = 0;
  pg[0] = 0;
  pr[0] = pi[0] = pib[0] = pd[0] = pc[0] = pn[0] = 0;
  size_t cw = 0;
  for (int j = 0; j < NJ; ++j) {
    const int idx = lay.dev[j];
    const ResPlan& P = plans[idx];
    const ResJob& J = lay.jobs[j];
    const Operand& A = P.swap ? G[idx] : F[idx];
    const Operand& B = P.swap ? F[idx] : G[idx];
    RowDesc* ra = rows + J.rows_off;
    int off = 0;
    auto emit = [&](const Operand& O, RowDesc* rd, int deg) {
      for (int g = 0; g < P.rstride; ++g) {
        rd[g].off = 0; rd[g].len = 0;
        const int t0 = g * ROWGRP;
        if (t0 > deg) continue;
        int ml = 0;
        for (int q = 0; q < ROWGRP && t0 + q <= deg; ++q) ml = std::max(ml, O.rowdeg[deg - t0 - q] + 1);
        ml = padded_group_len(ml);
        rd[g].off = off; rd[g].len = ml;
        for (int kx = 0; kx < ml; ++kx) {
          for (int q = 0; q < ROWGRP; ++q) {
            uint32_t* dst = coef + cw + (size_t)(off + ROWGRP * kx + q);  // limb l at dst[l T]
            const int row = deg - t0 - q;
            if (t0 + q > deg || kx > O.rowdeg[row]) {
              for (int l = 0; l < P.nl; ++l) dst[(size_t)l * P.T] = 0u;
              continue;
            }
            const uint32_t* src = O.limbs + ((size_t)row * (O.dx + 1) + kx) * O.nl;
            const uint32_t ext = (src[O.nl - 1] >> 31) ? 0xffffffffu : 0u;
            for (int l = 0; l < P.nl; ++l) dst[(size_t)l * P.T] = l < O.nl ? src[l] : ext;
          }
        }
        off += ROWGRP * ml;
      }
    };
    emit(A, ra, P.m);
    emit(B, ra + P.rstride, P.n);
    cw += (size_t)P.T * P.nl;
    const int64_t n1 = P.D + 1;
    pr[j + 1] = pr[j] + (int64_t)P.k * ((P.T + 255) / 256);
    pi[j + 1] = pi[j] + P.k;
    pib[j + 1] = pib[j] + (int64_t)P.k * ((P.D + 1 + 63) / 64);
    const int cc = lay.crt_small_on ? crt_small_class(P.k) : -1;
    if (cc >= 0) {
      ls[cc][ns[cc]] = j;
      ps[cc][ns[cc] + 1] = ps[cc][ns[cc]] + (n1 + 63) / 64;
      ns[cc]++;
    } else {
      lbig[nbig] = j;
      pd[nbig + 1] = pd[nbig] + (n1 + CRT_COEF_PER_BLOCK - 1) / CRT_COEF_PER_BLOCK;
      pc[nbig + 1] = pc[nbig] + (n1 + CRT_COMB_PER_BLOCK - 1) / CRT_COMB_PER_BLOCK;
      nbig++;
    }
    pn[j + 1] = pn[j] + (int64_t)P.k * n1;
    if (P.cls >= 0) {
      by_cost[P.cls].push_back({eval_block_cost(P), j});
    } else {
      lg[ng] = j;
      pg[ng + 1] = pg[ng] + (int64_t)P.k * n1;
      ng++;
    }
  }
  // the one-wavefront interpolation's jobs by degree bound, largest first (the
  // longest wavefronts start first)
  {
    std::vector<int> ord(NJ);
    for (int j = 0; j < NJ; ++j) ord[j] = j;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return lay.jobs[x].D > lay.jobs[y].D; });
    int32_t* li = (int32_t*)(h + lay.list_iw);
    int64_t* pw = (int64_t*)(h + lay.pref_iw);
    pw[0] = 0;
    for (int t = 0; t < NJ; ++t) {
      li[t] = ord[t];
      pw[t + 1] = pw[t] + lay.jobs[ord[t]].k;
    }
  }
  // a class's jobs most expensive first: a persistent launch hands out the
  // cheapest blocks last (the order does not change any result)
  for (int c = 0; c < NCLS; ++c) {
    std::stable_sort(by_cost[c].begin(), by_cost[c].end(),
                     [](const std::pair<int64_t, int>& x, const std::pair<int64_t, int>& y) { return x.first > y.first; });
    for (const auto& e : by_cost[c]) {
      const ResJob& J = lay.jobs[e.second];
      le[c][ne[c]] = e.second;
      pe[c][ne[c] + 1] = pe[c][ne[c]] + (int64_t)J.k * ((J.D + 1 + EE_BLOCK - 1) / EE_BLOCK);
      ne[c]++;
    }
  }
}


#define HIPCHK(x)                                                                     \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) {                                                           \
      c->err = std::string(#x) + ": " + hipGetErrorString(e_);                        \
      return SNC_EDEVICE;                                                             \
    }                                                                                 \
  } while (0)

int prepare_resultants(snc_ctx* c, int n, const snc_bipoly* f, const snc_bipoly* g, void* d_ws,
                       size_t ws_bytes, hipStream_t stream, bool use_graph, snc_prepared** outp) {
  *outp = nullptr;
  HIPCHK(hipSetDevice(c->device));
  std::vector<Operand> F(n), G(n);
  snc_prepared* pr = new snc_prepared();
  pr->c = c;
  pr->n = n;
  pr->use_graph = use_graph;
  pr->P.resize(n);
  for (int i = 0; i < n; ++i) {
    int st = parse_bipoly(&f[i], F[i], c->err);
    if (!st) st = parse_bipoly(&g[i], G[i], c->err);
    if (!st) st = plan_resultant(F[i], G[i], pr->P[i], c->err);
    if (st) { c->err = "pair " + std::to_string(i) + ": " + c->err; delete pr; return st; }
  }
  layout_batch(pr->P, pr->lay);
  const BatchLayout& lay = pr->lay;
  if (!lay.dev.empty()) {
    if (!d_ws || ws_bytes < lay.total_bytes) {
      c->err = "workspace of " + std::to_string(ws_bytes) + " bytes, need " + std::to_string(lay.total_bytes);
      delete pr;
      return SNC_ENOMEM;
    }
    pr->ws = (uint8_t*)d_ws;
    if (c->stage_in(lay.header_bytes)) { c->err = "pinned staging allocation failed"; delete pr; return SNC_EDEVICE; }
    if (hipHostMalloc(&pr->h_out, std::max<size_t>(lay.out_words * 4, 4), hipHostMallocDefault) != hipSuccess) {
      pr->h_out = nullptr;
      c->err = "pinned staging allocation failed";
      delete pr;
      return SNC_EDEVICE;
    }
    fill_header(lay, pr->P, F, G, (uint8_t*)c->h_in);
    StageTimer tm{c, stream, c->timing && !use_graph};
    tm.start();
    hipError_t e = hipMemcpyAsync(pr->ws, c->h_in, lay.header_bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) {
      // launch variants of the evaluation kernel: measured for a batched graph, looked up otherwise
      const int st = choose_eval_variants(c, pr->lay, pr->ws, stream, use_graph);
      if (st) { destroy_prepared(pr); return st; }
    }
    if (e == hipSuccess) {  // the abnormal-instance counter starts at zero; each run's interpolation clears it
      launch_zero_u32((uint32_t*)(pr->ws + lay.abn_count_off), 1, stream);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) { c->err = std::string("input upload: ") + hipGetErrorString(e); destroy_prepared(pr); return SNC_EDEVICE; }
  }
  *outp = pr;
  return SNC_OK;
}

// output sizes and the host-only (trivial) results; false with SNC_ERANGE sizes written back
static bool prepared_outputs(snc_prepared* pr, snc_upoly* out) {
  const std::vector<ResPlan>& P = pr->P;
  bool range_err = false;
  for (int i = 0; i < pr->n; ++i) {
    const int need_deg = P[i].trivial ? (P[i].trivial_value ? 0 : -1) : P[i].D;
    const int need_nl = P[i].trivial ? 1 : P[i].L;
    if (out[i].deg < need_deg || out[i].nlimbs < need_nl || (need_deg >= 0 && !out[i].limbs)) {
      out[i].deg = need_deg;
      out[i].nlimbs = need_nl;
      range_err = true;
    }
  }
  if (range_err) { pr->c->err = "output buffer too small"; return false; }
  for (int i = 0; i < pr->n; ++i) {
    if (!P[i].trivial) continue;
    if (P[i].trivial_value) {
      for (int l = 0; l < out[i].nlimbs; ++l) out[i].limbs[l] = l == 0 ? 1u : 0u;
      out[i].deg = 0;
    } else {
      out[i].deg = -1;
    }
  }
  return true;
}

// the whole pipeline on `stream`, as a HIP graph captured on first use
static int launch_prepared_all(snc_prepared* pr, hipStream_t stream, StageTimer& tm) {
  const int part = PIPE_ALL;
  snc_ctx* c = pr->c;
  // with timing on, the same launches go straight to the stream between
  // events (a replayed graph cannot be timed per stage)
  if (!pr->use_graph || tm.on) {
    launch_pipeline(pr->lay, pr->ws, stream, tm.on ? &tm : nullptr, part);
    HIPCHK(hipGetLastError());
    return SNC_OK;
  }
  hipGraphExec_t& gx = pr->gexec;
  if (!gx) {
    if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    if (!c->fork_stream) HIPCHK(hipStreamCreateWithFlags(&c->fork_stream, hipStreamNonBlocking));
    if (!c->ev_fork) HIPCHK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    if (!c->ev_join) HIPCHK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    PipeFork fk;
    fk.stream = c->fork_stream;
    fk.fork = c->ev_fork;
    fk.join = c->ev_join;
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    launch_pipeline(pr->lay, pr->ws, c->cap_stream, nullptr, part, fk);
    HIPCHK(hipStreamEndCapture(c->cap_stream, &graph));
    hipError_t e = hipGraphInstantiate(&gx, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) { gx = nullptr; c->err = std::string("graph instantiate: ") + hipGetErrorString(e); return SNC_EDEVICE; }
  }
  HIPCHK(hipGraphLaunch(gx, stream));
  return SNC_OK;
}

// results of jobs j0 .. j1-1 with j = tid mod nthr from the staged output block into out
static void collect_jobs(const snc_prepared* pr, const uint32_t* ho, snc_upoly* out, int j0, int j1, int tid,
                         int nthr) {
  const BatchLayout& lay = pr->lay;
  const size_t base = lay.out_off / 4;
  for (int j = j0 + tid; j < j1; j += nthr) {
    const int i = lay.dev[j];
    const ResJob& J = lay.jobs[j];
    const uint32_t* src = ho + (J.out_off - base);
    int deg = -1;
    for (int t = J.D; t >= 0 && deg < 0; --t)
      for (int l = 0; l < J.L; ++l)
        if (src[(size_t)t * J.L + l]) { deg = t; break; }
    const int stride = out[i].nlimbs;
    if (stride == J.L) {
      std::memcpy(out[i].limbs, src, sizeof(uint32_t) * (size_t)(deg + 1) * J.L);
    } else {
      for (int t = 0; t <= deg; ++t) {
        const uint32_t* s = src + (size_t)t * J.L;
        uint32_t* d = out[i].limbs + (size_t)t * stride;
        const uint32_t ext = (s[J.L - 1] >> 31) ? 0xffffffffu : 0u;
        for (int l = 0; l < stride; ++l) d[l] = l < J.L ? s[l] : ext;
      }
    }
    out[i].deg = deg;
  }
}

static void prepared_collect(snc_prepared* pr, snc_upoly* out) {
  collect_jobs(pr, (const uint32_t*)pr->h_out, out, 0, (int)pr->lay.dev.size(), 0, 1);
}

// Download and collection of a large output block in chunks: the copy of
// chunk c+1 runs while host threads widen chunk c into the caller's buffers.
constexpr size_t COLLECT_CHUNKED_WORDS = (size_t)1 << 20;
constexpr int COLLECT_CHUNKS = 8;

// job ranges of about equal output words (the jobs' output regions are consecutive)
static std::vector<int> chunk_bounds(const BatchLayout& lay) {
  const int NJ = (int)lay.dev.size();
  std::vector<int> bnd{0};
  const size_t per = (lay.out_words + COLLECT_CHUNKS - 1) / COLLECT_CHUNKS;
  size_t acc = 0;
  for (int j = 0; j < NJ; ++j) {
    acc += (size_t)(lay.jobs[j].D + 1) * lay.jobs[j].L;
    if (acc >= per * bnd.size() && j + 1 < NJ && (int)bnd.size() < COLLECT_CHUNKS) bnd.push_back(j + 1);
  }
  bnd.push_back(NJ);
  return bnd;
}

// downloads of the output block from src (device, laid out as the
// workspace's output region) to dst (pinned host) in the chunks of bnd on
// stream, one event recorded after each
static int enqueue_chunks(const snc_prepared* pr, const std::vector<int>& bnd, const uint8_t* src, void* dst,
                          std::vector<hipEvent_t>& ev, hipStream_t stream) {
  snc_ctx* c = pr->c;
  const BatchLayout& lay = pr->lay;
  const int NJ = (int)lay.dev.size();
  const int nch = (int)bnd.size() - 1;
  while ((int)ev.size() < nch) {
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ev.push_back(e);
  }
  const size_t base = lay.out_off / 4;
  for (int ch = 0; ch < nch; ++ch) {
    const size_t w0 = lay.jobs[bnd[ch]].out_off - base;
    const size_t w1 = bnd[ch + 1] < NJ ? lay.jobs[bnd[ch + 1]].out_off - base : lay.out_words;
    HIPCHK(hipMemcpyAsync((uint32_t*)dst + w0, src + w0 * 4, (w1 - w0) * 4, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipEventRecord(ev[ch], stream));
  }
  return SNC_OK;
}

// host threads widen each chunk of ho into the caller's buffers as soon as
// its event has completed
static int widen_chunks(snc_prepared* pr, const std::vector<int>& bnd, const std::vector<hipEvent_t>& ev,
                        const uint32_t* ho, snc_upoly* out) {
  snc_ctx* c = pr->c;
  const int nch = (int)bnd.size() - 1;
  const unsigned hc = std::thread::hardware_concurrency();
  const int nthr = (int)std::max(1u, std::min(8u, hc / 2));
  std::atomic<int> ready{0};
  std::vector<std::thread> workers;
  for (int t = 1; t < nthr; ++t)
    workers.emplace_back([&, t] {
      for (int ch = 0; ch < nch; ++ch) {
        while (ready.load(std::memory_order_acquire) <= ch) {
          if (ready.load(std::memory_order_acquire) < 0) return;
          std::this_thread::yield();
        }
        collect_jobs(pr, ho, out, bnd[ch], bnd[ch + 1], t, nthr);
      }
    });
  hipError_t err = hipSuccess;
  for (int ch = 0; ch < nch; ++ch) {
    err = hipEventSynchronize(ev[ch]);
    if (err != hipSuccess) { ready.store(-1, std::memory_order_release); break; }
    ready.store(ch + 1, std::memory_order_release);
    collect_jobs(pr, ho, out, bnd[ch], bnd[ch + 1], 0, nthr);
  }
  for (auto& w : workers) w.join();
  if (err != hipSuccess) { c->err = std::string("result download: ") + hipGetErrorString(err); return SNC_EDEVICE; }
  return SNC_OK;
}

static int download_collect_chunked(snc_prepared* pr, hipStream_t stream, snc_upoly* out) {
  const std::vector<int> bnd = chunk_bounds(pr->lay);
  const int st = enqueue_chunks(pr, bnd, pr->ws + pr->lay.out_off, pr->h_out, pr->d2h_ev, stream);
  if (st) return st;
  return widen_chunks(pr, bnd, pr->d2h_ev, (const uint32_t*)pr->h_out, out);
}

int run_prepared(snc_prepared* pr, hipStream_t stream, snc_upoly* out) {
  snc_ctx* c = pr->c;
  if (!prepared_outputs(pr, out)) return SNC_ERANGE;
  if (pr->lay.dev.empty()) return SNC_OK;
  HIPCHK(hipSetDevice(c->device));
  StageTimer tm{c, stream, c->timing};
  tm.start();
  int st = launch_prepared_all(pr, stream, tm);
  if (st) return st;
  if (!tm.on && pr->lay.out_words >= COLLECT_CHUNKED_WORDS) return download_collect_chunked(pr, stream, out);
  HIPCHK(hipMemcpyAsync(pr->h_out, pr->ws + pr->lay.out_off, pr->lay.out_words * 4, hipMemcpyDeviceToHost, stream));
  tm.mark("d2h", 1);
  HIPCHK(hipStreamSynchronize(stream));
  tm.finish();
  prepared_collect(pr, out);
  return SNC_OK;
}

size_t prepared_stage_bytes(const snc_prepared* pr) {
  return pr->lay.dev.empty() ? 0 : 2 * align_words(pr->lay.out_words) * 4;
}

int submit_prepared(snc_prepared* pr, void* d_stage, size_t stage_bytes, hipStream_t stream, int64_t* ticket) {
  snc_ctx* c = pr->c;
  const size_t need = prepared_stage_bytes(pr);
  if (stage_bytes < need || (need && !d_stage)) {
    c->err = "snc_prepared_submit: staging buffer of " + std::to_string(stage_bytes) + " bytes, " +
             std::to_string(need) + " needed (snc_prepared_stage_bytes)";
    return SNC_ENOMEM;
  }
  int s = (int)(pr->next_ticket & 1);
  if (pr->slot_ticket[s] >= 0) s ^= 1;
  if (pr->slot_ticket[s] >= 0) {
    c->err = "snc_prepared_submit: two runs are outstanding; collect one first";
    return SNC_EAGAIN;
  }
  HIPCHK(hipSetDevice(c->device));
  const size_t bytes = pr->lay.out_words * 4;
  if (bytes && !pr->slot_host[s]) {
    HIPCHK(hipHostMalloc(&pr->slot_host[s], bytes, hipHostMallocDefault));
    HIPCHK(hipEventCreateWithFlags(&pr->slot_copied[s], hipEventDisableTiming));
  }
  if (!c->side_stream) HIPCHK(hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking));
  if (!pr->lay.dev.empty()) {
    uint8_t* slot = (uint8_t*)d_stage + (size_t)s * (need / 2);
    StageTimer tm{c, stream, false};
    const int st = launch_prepared_all(pr, stream, tm);
    if (st) return st;
    // the output region goes to the slot on the device (a short copy on
    // this stream), and from there to the host on the side stream, so the
    // next run's kernels can start right after this copy
    HIPCHK(hipMemcpyAsync(slot, pr->ws + pr->lay.out_off, bytes, hipMemcpyDeviceToDevice, stream));
    HIPCHK(hipEventRecord(pr->slot_copied[s], stream));
    HIPCHK(hipStreamWaitEvent(c->side_stream, pr->slot_copied[s], 0));
    const int st2 = enqueue_chunks(pr, chunk_bounds(pr->lay), slot, pr->slot_host[s], pr->slot_ev[s], c->side_stream);
    if (st2) return st2;
  }
  pr->slot_ticket[s] = pr->next_ticket;
  *ticket = pr->next_ticket++;
  return SNC_OK;
}

int collect_prepared(snc_prepared* pr, int64_t ticket, snc_upoly* out) {
  snc_ctx* c = pr->c;
  const int s = ticket >= 0 && pr->slot_ticket[0] == ticket ? 0 : ticket >= 0 && pr->slot_ticket[1] == ticket ? 1 : -1;
  if (s < 0) {
    c->err = "snc_prepared_collect: ticket " + std::to_string(ticket) + " is not an outstanding run";
    return SNC_EINVAL;
  }
  if (!prepared_outputs(pr, out)) return SNC_ERANGE;
  int st = SNC_OK;
  if (!pr->lay.dev.empty()) {
    HIPCHK(hipSetDevice(c->device));
    st = widen_chunks(pr, chunk_bounds(pr->lay), pr->slot_ev[s], (const uint32_t*)pr->slot_host[s], out);
  }
  pr->slot_ticket[s] = -1;
  return st;
}

int run_prepared_fork(snc_prepared* pr, hipStream_t stream, const std::function<int(hipStream_t)>& branch,
                      const std::function<void()>& on_results, snc_upoly* out) {
  snc_ctx* c = pr->c;
  if (!prepared_outputs(pr, out)) return SNC_ERANGE;
  if (pr->lay.dev.empty()) { on_results(); return SNC_OK; }
  HIPCHK(hipSetDevice(c->device));
  if (!c->side_stream) HIPCHK(hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking));
  // the side stream runs on this device only: a device-scope release suffices
  if (!c->ev_mid) HIPCHK(hipEventCreateWithFlags(&c->ev_mid, hipEventDisableTiming | hipEventReleaseToDevice));
  // plain launches: the host queues the whole step (both streams) while the
  // first kernels run, which measured slightly faster than replaying graphs here
  launch_pipeline(pr->lay, pr->ws, stream, nullptr, PIPE_TO_INTERP);
  HIPCHK(hipGetLastError());
  // the branch is queued on this stream right behind the interpolation, so
  // it starts without a cross-stream wait; the Chinese remaindering and the
  // download of the results go to the side stream
  HIPCHK(hipEventRecord(c->ev_mid, stream));
  const int st = branch(stream);
  if (st) return st;
  HIPCHK(hipStreamWaitEvent(c->side_stream, c->ev_mid, 0));
  launch_pipeline(pr->lay, pr->ws, c->side_stream, nullptr, PIPE_CRT);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(pr->h_out, pr->ws + pr->lay.out_off, pr->lay.out_words * 4, hipMemcpyDeviceToHost,
                        c->side_stream));
  HIPCHK(hipStreamSynchronize(c->side_stream));
  prepared_collect(pr, out);
  on_results();
  HIPCHK(hipStreamSynchronize(stream));
  return SNC_OK;
}

int run_resultants(snc_ctx* c, int n, const snc_bipoly* f, const snc_bipoly* g, void* d_ws,
                   size_t ws_bytes, hipStream_t stream, snc_upoly* out, bool use_graph) {
  snc_prepared* pr = nullptr;
  int st = prepare_resultants(c, n, f, g, d_ws, ws_bytes, stream, use_graph, &pr);
  if (st) return st;
  st = run_prepared(pr, stream, out);
  destroy_prepared(pr);
  return st;
}

void destroy_prepared(snc_prepared* pr) {
  if (!pr) return;
  for (int s = 0; s < 2; ++s) {
    // an uncollected run's download must end before its buffers go
    if (pr->slot_ticket[s] >= 0 && !pr->slot_ev[s].empty()) (void)hipEventSynchronize(pr->slot_ev[s].back());
    if (pr->slot_host[s]) (void)hipHostFree(pr->slot_host[s]);
    if (pr->slot_copied[s]) (void)hipEventDestroy(pr->slot_copied[s]);
    for (hipEvent_t e : pr->slot_ev[s]) (void)hipEventDestroy(e);
  }
  if (pr->gexec) (void)hipGraphExecDestroy(pr->gexec);
  if (pr->h_out) (void)hipHostFree(pr->h_out);
  if (pr->h_ed) (void)hipHostFree(pr->h_ed);
  for (hipEvent_t e : pr->d2h_ev) (void)hipEventDestroy(e);
  delete pr;
}

}  // namespace snc
