// Host-side structures of the runtime: parsed operands, plans, workspace
// layout and the context object behind the opaque snc_ctx handle.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "snc.h"
#include "snc_internal.hpp"

namespace snc {

constexpr int NCLS = 6;        // register classes of the fused evaluate+eliminate kernel

struct Tables {
  std::vector<uint32_t> p;       // primes, descending below 2^30
  std::vector<PrimeC> pc;        // Montgomery constants
  std::vector<double> lg;        // lg[k] = sum_{i<k} log2 p_i
  std::vector<uint32_t> garner;  // Montgomery form of (P_i mod p_i)^-1
  std::vector<uint32_t> wtab;    // [j*KMAX+i] Montgomery form of P_j mod p_i
  std::vector<uint32_t> ptab;    // [(KMAX+1)][LPS] limbs of P_j
};
const Tables& tables();
int ensure_device_tables(int device, std::string& err);
// device address of the fixed scratch array of snc_resultant_y_noalloc,
// looked up once per device with that device current
hipError_t init_noalloc_scratch(int device);

struct Operand {
  int dy = -1, dx = -1, nl = 1;
  const uint32_t* limbs = nullptr;
  int ydeg = -1;               // y-degree over Z[x], -1 for zero
  std::vector<int> rowdeg;     // x-degree per row (-1 zero row), size ydeg+1
  int total_deg = -1, max_rowdeg = -1;
  double log2S = 0.0;          // upper bound on log2(sum_i ||f_i||_1^2)
};

struct ResPlan {
  int trivial = 0, trivial_value = 0;   // f or g zero -> 0; both constant in y -> 1
  int swap = 0;                         // A = g (m < n)
  int m = 0, n = 0, D = 0, k = 0, L = 1, T = 0, nl = 1, cls = -1, rstride = 0;
  double log2B = 0.0;
};

inline size_t align_words(size_t w) { return (w + 63) & ~(size_t)63; }  // 256-byte sections

struct BatchLayout {
  std::vector<int> dev;              // plan index of each device job
  std::vector<ResJob> jobs;          // device job descriptors (offsets filled)
  size_t jobs_off = 0, rows_off = 0, coef_off = 0;        // bytes
  size_t pref_red = 0, pref_interp = 0, pref_crtd = 0, pref_crtc = 0, pref_gen = 0;  // bytes
  size_t pref_interp_blk = 0;        // bytes: block prefix of the block-parallel interpolation
  size_t pref_inst = 0;              // bytes: instance prefix k (D+1) over the jobs
  bool interp_blk = false;           // every job fits the block-parallel interpolation
  bool interp_w = false;             // one-wavefront interpolation (many (resultant, prime) pairs)
  size_t pref_iw = 0, list_iw = 0;   // bytes: its job list (degree bound descending) and block prefix
  bool reduce_in_eval = false;       // the evaluation kernel reduces the inputs (no reduction launch)
  size_t pref_ee[NCLS] = {0}, list_ee[NCLS] = {0}, list_gen = 0;                   // bytes
  // Chinese remaindering: the small-prime classes (one lane per coefficient)
  // and the jobs with more primes (pref_crtd / pref_crtc over list_crtb)
  size_t pref_crts[NCRT_SMALL] = {0}, list_crts[NCRT_SMALL] = {0}, list_crtb = 0;  // bytes
  int64_t nb_crts[NCRT_SMALL] = {0};
  int n_crts_jobs[NCRT_SMALL] = {0}, n_crtb_jobs = 0;
  bool crt_small_on = false;         // the few-prime jobs take k_crt_small (enough coefficients)
  EEVariant ee_var[NCLS];            // launch variant of each register class (autotuner, or the defaults)
  size_t ee_counter_off = 0;         // bytes: the NCLS work counters of persistent evaluation launches
  size_t header_bytes = 0;
  size_t abn_count_off = 0, abn_list_off = 0;              // bytes
  uint32_t abn_cap = 0;
  size_t out_off = 0, out_words = 0;                       // bytes / words
  size_t sq_off = 0, sq_words = 0;  // bytes / words: gcd(R, R') descriptors, work items, e and d
  size_t total_bytes = 0;
  int64_t nb_red = 0, nb_interp = 0, nb_crtd = 0, nb_crtc = 0, n_gen_inst = 0, nb_interp_blk = 0;
  int64_t nb_ee[NCLS] = {0};
  int n_ee_jobs[NCLS] = {0}, n_gen_jobs = 0, n_rows = 0, max_D = 0, max_k = 0;
  int max_T_ee[NCLS] = {0};  // largest residue count per prime among a class's jobs
  int64_t total_inst = 0;
  size_t coef_words = 0;
};

void layout_batch(const std::vector<ResPlan>& plans, BatchLayout& lay);
size_t job_region_words(const ResPlan& P);
int parse_bipoly(const snc_bipoly* f, Operand& op, std::string& err);
int plan_resultant(const Operand& F, const Operand& G, ResPlan& P, std::string& err);

}  // namespace snc

// One register class's choice by the evaluation autotuner on a prepared batch.
struct EETuneReport {
  int32_t cls_cap = 0;       // register class (largest y-degree)
  int32_t wpe = 1, chunk = 0;
  int64_t grid = 0;          // persistent workgroups (chunk > 0)
  int32_t source = 0;        // 0 defaults, 1 measured now, 2 from the cache, 3 forced
  float best_ms = 0.f;       // measured time of the chosen variant (source 1)
  float default_ms = 0.f;    // measured time of the default variant (source 1)
  int32_t candidates = 0;    // variants timed
};

struct snc_ctx {
  int device = 0;
  std::string err;
  bool timing = false;
  // evaluation autotuner: 0 off (defaults, cache lookups only), 1 tune classes the cache lacks, 2 retune
  int tune_mode = 1;
  int gcd_variant = 0;  // Euclid of the square-free check: 0 automatic (one wavefront), 1 one wavefront, 2 blocked
  snc::EEVariant forced[snc::NCLS];  // wpe > 0: variant forced for every launch of that class (0: none)
  std::vector<EETuneReport> tune_report;  // the last batched preparation's choices
  float tune_ms = 0.f;                    // host wall time spent tuning in that preparation
  std::vector<const char*> stage_names;
  std::vector<float> stage_ms;
  std::vector<int> stage_launches;
  std::vector<hipEvent_t> events;
  // pinned host staging
  void* h_in = nullptr;
  size_t h_in_bytes = 0;
  void* h_out = nullptr;
  size_t h_out_bytes = 0;
  // captured pipeline of the last batch shape
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<int64_t> gkey;
  // second stream (default priority) and event for work beside the pipeline
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_mid = nullptr;
  // branch of the captured pipeline (default priority): the small-prime CRT
  // class with the most primes runs beside the other classes
  hipStream_t fork_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  snc_ctx() {
    for (auto& f : forced) f.wpe = 0;
  }
  int stage_in(size_t bytes);
  int stage_out(size_t bytes);
  void release();
};

// A batch of resultants whose inputs have been planned and uploaded into a
// device workspace; running it launches only the device pipeline.
struct snc_prepared {
  snc_ctx* c = nullptr;
  int n = 0;
  bool use_graph = false;
  std::vector<snc::ResPlan> P;
  snc::BatchLayout lay;
  uint8_t* ws = nullptr;
  void* h_out = nullptr;
  hipGraphExec_t gexec = nullptr;    // whole pipeline
  std::vector<hipEvent_t> d2h_ev;    // chunks of the result download (large batches)
  // projection step (resultant and gcd(R, R')): the Euclid descriptors are
  // uploaded into the workspace on the first run
  void* h_ed = nullptr;              // mapped pinned memory the Euclid writes e and d to
  bool sq_ready = false;
  std::shared_ptr<void> sq_cache;    // the projection step's plan, built on the first run
  std::vector<int> sq_ranges;        // (register class, first item, items, largest degree) per launch
  // pipelined runs (snc_prepared_submit / _collect): two staging slots of the
  // output block, on the device (the caller's staging buffer) and in pinned
  // host memory
  void* slot_host[2] = {nullptr, nullptr};
  int64_t slot_ticket[2] = {-1, -1};            // the run a slot holds, -1 free
  hipEvent_t slot_copied[2] = {nullptr, nullptr};  // output region copied into the slot
  std::vector<hipEvent_t> slot_ev[2];           // download chunks of the slot
  int64_t next_ticket = 0;
};

namespace snc {
enum { PIPE_ALL = 0, PIPE_TO_INTERP = 1, PIPE_CRT = 2 };
struct StageTimer;
// upload block of a laid-out batch: job and row descriptors, block
// prefixes, class job lists and the packed input limbs (header_bytes)
void fill_header(const BatchLayout& lay, const std::vector<ResPlan>& plans, const std::vector<Operand>& F,
                 const std::vector<Operand>& G, uint8_t* h);
// Stream and events of a branch beside the main stream (all null: no branch).
struct PipeFork {
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
// device launch sequence of a laid-out batch whose header is in ws (tm may be
// null); with a branch (fk.stream set, tm null) the small-prime CRT class
// with the most primes runs on the branch beside the other classes
void launch_pipeline(const BatchLayout& lay, uint8_t* ws, hipStream_t s, StageTimer* tm, int part,
                     const PipeFork& fk = PipeFork());
// launch variants of the evaluation kernel for a laid-out batch whose header is on the device:
// forced variants, then (tune true) measured ones for the classes the cache lacks, else cached
// choices or the defaults; fills lay.ee_var and the context's report
int choose_eval_variants(snc_ctx* c, BatchLayout& lay, uint8_t* ws, hipStream_t s, bool tune);
int prepare_resultants(snc_ctx* c, int n, const snc_bipoly* f, const snc_bipoly* g, void* d_ws,
                       size_t ws_bytes, hipStream_t stream, bool use_graph, snc_prepared** outp);
int run_prepared(snc_prepared* pr, hipStream_t stream, snc_upoly* out);
// pipelined runs: submit enqueues a run and the download of its results
// into a free staging slot (SNC_EAGAIN when both hold uncollected runs);
// collect waits for a ticket's download and widens it into out
size_t prepared_stage_bytes(const snc_prepared* pr);
int submit_prepared(snc_prepared* pr, void* d_stage, size_t stage_bytes, hipStream_t stream, int64_t* ticket);
int collect_prepared(snc_prepared* pr, int64_t ticket, snc_upoly* out);
// the pipeline with a second branch after the interpolation: branch(stream)
// enqueues work that follows the interpolation on `stream` while the Chinese
// remaindering and the download of the results run on the side stream;
// on_results() runs on the host once the results are in out, while the
// branch may still run; returns with all work complete.
int run_prepared_fork(snc_prepared* pr, hipStream_t stream, const std::function<int(hipStream_t)>& branch,
                      const std::function<void()>& on_results, snc_upoly* out);
void destroy_prepared(snc_prepared* pr);
int run_resultants(snc_ctx* c, int n, const snc_bipoly* f, const snc_bipoly* g, void* d_ws,
                   size_t ws_bytes, hipStream_t stream, snc_upoly* out, bool use_graph);
}
