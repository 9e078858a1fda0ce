// Autotuner of the evaluation + elimination kernel (the batched resultant's
// dominant stage).  For each register class a batch uses it chooses:
//   wpe   -- the minimum wavefronts per SIMD the kernel's register allocation
//            is held to (1 = unconstrained, 2, 3, 4): more resident
//            wavefronts hide the latency of the dependent 64-bit
//            multiply-add chains, fewer registers spill the arrays;
//   chunk -- 0 for one workgroup per block of 64 points, else a persistent
//            grid (as many workgroups as fit on the device) taking `chunk`
//            blocks at a time from a work counter, blocks of one prime
//            sharing the residues staged in LDS.
// Every variant computes the same residues; only the time differs.  Each
// candidate is timed on the batch's own class launch (best of two, HIP
// events on the batch's stream); of the variants within 5% of the fastest
// the one with the fewest spilled bytes per lane is kept per (register
// class, LDS variant, size bucket = log2 of the class's block count) in a
// per-device table, which is also appended to a cache file
// ($SNC_TUNE_DIR, else $HOME/.cache/snc) and read back by later processes.
#include <hip/hip_runtime.h>

#include <sys/stat.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "runtime_internal.hpp"

namespace snc {

namespace {

constexpr float EE_TUNE_TIE = 0.05f;  // relative time difference taken as a tie

std::mutex g_mu;
std::map<std::string, EEVariant> g_table;  // "device|cls|lds|bucket" -> variant (grid recomputed)
std::set<std::string> g_loaded;            // devices whose cache file has been read

std::string device_tag(const hipDeviceProp_t& prop) {
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  return arch + "_" + std::to_string(prop.multiProcessorCount) + "cu";
}

std::string cache_path(const std::string& tag) {
  std::string dir;
  if (const char* d = std::getenv("SNC_TUNE_DIR"); d && *d) {
    dir = d;
  } else if (const char* h = std::getenv("HOME"); h && *h) {
    dir = std::string(h) + "/.cache/snc";
  } else {
    return "";
  }
  return dir + "/eval_elim_" + tag + "_r" + std::to_string(EE_KERNEL_REV) + ".tune";
}

void mkdirs(const std::string& file) {
  for (size_t i = 1; i < file.size(); ++i)
    if (file[i] == '/') (void)mkdir(file.substr(0, i).c_str(), 0755);
}

std::string key_of(const std::string& tag, int cls, int lds, int bucket) {
  return tag + "|" + std::to_string(cls) + "|" + std::to_string(lds) + "|" + std::to_string(bucket);
}

// cache lines: "cls lds bucket wpe chunk"; later lines win
void load_cache(const std::string& tag) {
  if (g_loaded.count(tag)) return;
  g_loaded.insert(tag);
  const std::string path = cache_path(tag);
  if (path.empty()) return;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  int cls, lds, bucket, wpe, chunk;
  while (std::fscanf(f, "%d %d %d %d %d", &cls, &lds, &bucket, &wpe, &chunk) == 5) {
    if (cls < 0 || cls >= NCLS || wpe < 1 || wpe > EE_WPE_MAX || chunk < 0 || chunk > 64) continue;
    EEVariant v;
    v.wpe = wpe;
    v.chunk = chunk;
    g_table[key_of(tag, cls, lds, bucket)] = v;
  }
  std::fclose(f);
}

void append_cache(const std::string& tag, int cls, int lds, int bucket, const EEVariant& v) {
  const std::string path = cache_path(tag);
  if (path.empty()) return;
  mkdirs(path);
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;  // an unwritable cache only costs a retune in the next process
  std::fprintf(f, "%d %d %d %d %d\n", cls, lds, bucket, v.wpe, v.chunk);
  std::fclose(f);
}

int size_bucket(int64_t nblocks) {
  int b = 0;
  while ((int64_t(1) << (b + 1)) <= nblocks) ++b;
  return b;
}

}  // namespace

#define TUNECHK(x)                                                      \
  do {                                                                  \
    hipError_t e_ = (x);                                                \
    if (e_ != hipSuccess) {                                             \
      c->err = std::string("autotune: ") + #x + ": " + hipGetErrorString(e_); \
      st = SNC_EDEVICE;                                                 \
      goto done;                                                        \
    }                                                                   \
  } while (0)

int choose_eval_variants(snc_ctx* c, BatchLayout& lay, uint8_t* ws, hipStream_t s, bool tune) {
  c->tune_report.clear();
  c->tune_ms = 0.f;
  bool any = false;
  for (int k = 0; k < NCLS; ++k) any |= lay.n_ee_jobs[k] > 0;
  if (!any) return SNC_OK;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) {
    c->err = "autotune: device query failed";
    return SNC_EDEVICE;
  }
  const std::string tag = device_tag(prop);
  const auto t0 = std::chrono::steady_clock::now();
  int st = SNC_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool reduced = false, measured = false;
  uint32_t* wsw = (uint32_t*)ws;
  const ResJob* jobs = (const ResJob*)(ws + lay.jobs_off);
  const RowDesc* rows = (const RowDesc*)(ws + lay.rows_off);
  uint32_t* abn_count = (uint32_t*)(ws + lay.abn_count_off);
  AbnEntry* abn_list = (AbnEntry*)(ws + lay.abn_list_off);
  uint32_t* counters = (uint32_t*)(ws + lay.ee_counter_off);
  std::lock_guard<std::mutex> lk(g_mu);
  load_cache(tag);
  for (int cls = 0; cls < NCLS; ++cls) {
    if (!lay.n_ee_jobs[cls]) continue;
    EETuneReport rep;
    rep.cls_cap = fast_class_cap(cls);
    const int lds = eval_elim_in_lds(lay.max_T_ee[cls]) ? 1 : 0;
    const int bucket = size_bucket(lay.nb_ee[cls]);
    const std::string key = key_of(tag, cls, lds, bucket);
    EEVariant v;
    if (c->forced[cls].wpe > 0) {
      v = c->forced[cls];
      rep.source = 3;
    } else if (c->tune_mode != 2 && g_table.count(key)) {
      v = g_table[key];
      rep.source = 2;
    } else if (tune && c->tune_mode != 0) {
      if (!e0) {
        TUNECHK(hipEventCreate(&e0));
        TUNECHK(hipEventCreate(&e1));
      }
      if (!lay.reduce_in_eval && !reduced) {  // residues for the variants that read them
        launch_reduce(jobs, (const int64_t*)(ws + lay.pref_red), (int)lay.jobs.size(), lay.nb_red, wsw, wsw,
                      abn_count, s);
        reduced = true;
      }
      float best = -1.f, def = -1.f;
      EEVariant bestv;
      std::vector<std::pair<EEVariant, float>> timed;
      for (int wpe = 1; wpe <= EE_WPE_MAX; ++wpe) {
        for (int chunk : {0, 1, 4}) {
          EEVariant cand;
          cand.wpe = wpe;
          cand.chunk = chunk;
          if (chunk > 0) {
            cand.grid = eval_elim_grid(cls, wpe, lay.max_T_ee[cls]);
            if (cand.grid <= 0) continue;
          }
          float ms_best = -1.f;
          for (int rep_i = 0; rep_i < 2; ++rep_i) {
            launch_zero_u32(abn_count, 1, s);
            launch_zero_u32(counters + cls, 1, s);
            TUNECHK(hipEventRecord(e0, s));
            launch_eval_elim(cls, cand, counters + cls, jobs, (const int32_t*)(ws + lay.list_ee[cls]),
                             (const int64_t*)(ws + lay.pref_ee[cls]), lay.n_ee_jobs[cls], lay.nb_ee[cls],
                             lay.max_T_ee[cls], rows, wsw, abn_count, abn_list, lay.abn_cap, lay.reduce_in_eval, s);
            TUNECHK(hipGetLastError());
            TUNECHK(hipEventRecord(e1, s));
            TUNECHK(hipEventSynchronize(e1));
            float ms = 0.f;
            TUNECHK(hipEventElapsedTime(&ms, e0, e1));
            if (ms_best < 0.f || ms < ms_best) ms_best = ms;
          }
          ++rep.candidates;
          if (wpe == 1 && chunk == 0) def = ms_best;
          if (best < 0.f || ms_best < best) { best = ms_best; bestv = cand; }
          timed.emplace_back(cand, ms_best);
        }
      }
      // Among the variants within EE_TUNE_TIE of the fastest, the one that
      // spills least: a kernel timed alone does not show what its spill
      // traffic costs the kernels after it, whose data it evicts from the
      // L2 and the last-level cache.  Measured on the 512-pair batch: the
      // degree-40 class at four wavefronts per SIMD (280 spilled bytes per
      // lane, 1.8 GB written per step) ran 3% faster alone than at three
      // (60 bytes, 0.18 GB), but the interpolation after it ran 8% slower
      // and the whole step 3% slower.
      {
        int best_scr = eval_elim_scratch(cls, bestv.wpe, lay.max_T_ee[cls]);
        for (const auto& tv : timed) {
          if (tv.second > best * (1.f + EE_TUNE_TIE)) continue;
          const int scr = eval_elim_scratch(cls, tv.first.wpe, lay.max_T_ee[cls]);
          if (scr >= 0 && best_scr >= 0 && scr < best_scr) {
            best_scr = scr;
            bestv = tv.first;
            rep.best_ms = tv.second;
          }
        }
      }
      v = bestv;
      v.grid = 0;
      if (rep.best_ms <= 0.f) rep.best_ms = best;
      rep.default_ms = def;
      rep.source = 1;
      measured = true;
      g_table[key] = v;
      append_cache(tag, cls, lds, bucket, v);
    } else {
      rep.source = 0;  // defaults: wpe 1, one workgroup per block
    }
    if (v.chunk > 0) {
      v.grid = eval_elim_grid(cls, v.wpe, lay.max_T_ee[cls]);
      if (v.grid <= 0) v.chunk = 0;  // no occupancy figure: one workgroup per block
    }
    lay.ee_var[cls] = v;
    rep.wpe = v.wpe;
    rep.chunk = v.chunk;
    rep.grid = v.grid;
    c->tune_report.push_back(rep);
  }
  if (reduced || measured) {
    launch_zero_u32(abn_count, 1, s);  // the runs start from an empty abnormal list
    if (hipStreamSynchronize(s) != hipSuccess) { c->err = "autotune: synchronize failed"; st = SNC_EDEVICE; }
  }
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  c->tune_ms = (float)std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

}  // namespace snc
