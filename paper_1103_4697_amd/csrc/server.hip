// Serving: a request loop over resultant and gcd jobs with continuous
// batching on one GPU.
//
// The caller hands the server one device pool.  Requests are copied at
// submission and planned on the host (their device footprint is the plan's
// workspace size).  Worker threads, each with its own context and HIP stream,
// take work from the queue: a free worker collects the waiting requests of
// the kind at the head of the queue that fit into the free pool bytes and
// slots and runs them as one batch (resultants: every stage launched once
// over all of them; gcds: one batched gcd submission).  A
// request that arrives while others are on the GPU is admitted as soon as
// pool bytes and a slot free up, and its work overlaps with the in-flight
// work on the other streams.  Results are kept until the caller polls them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "runtime_internal.hpp"
#include "snc.h"

namespace snc {
namespace {

using Clock = std::chrono::steady_clock;

double secs(Clock::time_point t) {
  return std::chrono::duration<double>(t.time_since_epoch()).count();
}

struct Request {
  uint64_t ticket = 0;
  int kind = 0;  // 0: resultant, 1: gcd
  // copied inputs
  std::vector<uint32_t> fl, gl;
  snc_bipoly f{}, g{};
  snc_upoly a{}, b{};
  size_t footprint = 0;  // device bytes
  int out_deg = 0, out_nl = 1;
  // result
  std::vector<uint32_t> res;
  int res_deg = -1, res_nl = 1;
  int status = SNC_EAGAIN;
  std::string err;
  Clock::time_point t_submit, t_done;
};

// First-fit allocator over [0, bytes) of the pool (256-byte granularity).
struct PoolAlloc {
  size_t bytes = 0;
  std::map<size_t, size_t> free_;  // offset -> size
  void init(size_t b) { bytes = b; free_.clear(); if (b) free_[0] = b; }
  bool alloc(size_t n, size_t& off) {
    n = (n + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        off = it->first;
        const size_t rest = it->second - n;
        free_.erase(it);
        if (rest) free_[off + n] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) & ~(size_t)255;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) { it->second += nx->second; free_.erase(nx); }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) { pv->second += it->second; free_.erase(it); }
    }
  }
};

}  // namespace
}  // namespace snc

using namespace snc;

struct snc_server {
  int device = 0;
  uint8_t* pool = nullptr;
  size_t pool_bytes = 0;
  int max_slots = 1;
  std::mutex mu;
  std::condition_variable cv;      // work available / shutdown
  std::condition_variable cv_done; // request finished
  std::deque<uint64_t> queue;      // tickets waiting for admission
  std::map<uint64_t, Request*> reqs;
  std::map<uint64_t, std::pair<double, double>> times;  // ticket -> (submitted, finished), seconds
  PoolAlloc alloc;
  int slots_used = 0;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::vector<std::thread> workers;
  std::atomic<int64_t> completed{0};
};

namespace snc {
namespace {

size_t round256(size_t n) { return (n + 255) & ~(size_t)255; }

// Device bytes of a batch of requests of one kind: its joint workspace.
size_t batch_bytes(const std::vector<Request*>& batch, int kind, size_t fallback) {
  if (kind == 1) {
    std::vector<snc_upoly> as(batch.size()), bs(batch.size());
    for (size_t i = 0; i < batch.size(); ++i) { as[i] = batch[i]->a; bs[i] = batch[i]->b; }
    snc_plan tot{};
    if (snc_gcd_z_batch_plan((int32_t)batch.size(), as.data(), bs.data(), nullptr, &tot) != SNC_OK) return fallback;
    return std::max<size_t>(tot.workspace_bytes, 256);
  }
  std::vector<ResPlan> plans(batch.size());
  std::string err;
  for (size_t i = 0; i < batch.size(); ++i) {
    Operand F, G;
    parse_bipoly(&batch[i]->f, F, err);
    parse_bipoly(&batch[i]->g, G, err);
    plan_resultant(F, G, plans[i], err);
  }
  BatchLayout lay;
  layout_batch(plans, lay);
  return std::max<size_t>(lay.total_bytes, 256);
}

// Finish a request that cannot run (lock held).
void fail_request(snc_server* s, Request* r, int status, const std::string& msg) {
  const auto now = Clock::now();
  r->status = status;
  r->err = msg;
  r->t_done = now;
  s->times[r->ticket] = {secs(r->t_submit), secs(now)};
  s->completed += 1;
}

// Take work for one worker: a batch of admitted requests of one kind.
// Called with the lock held; returns false if nothing could be admitted.
// The head request is probed with its own footprint (a batch of one needs
// no more), later ones with headroom for the joint header; a batch whose
// joint workspace does not fit shrinks to its head request, which waits
// only while other work holds pool bytes (it fits an empty pool, else it
// fails with SNC_ENOMEM).
bool take_work(snc_server* s, std::vector<Request*>& batch, size_t& off, size_t& bytes, bool& failed) {
  batch.clear();
  failed = false;
  if (s->queue.empty() || s->slots_used >= s->max_slots) return false;
  const int kind = s->reqs[s->queue.front()]->kind;
  // grow a batch of the first request's kind while the summed footprint and the slots allow
  size_t total = 0;
  for (auto it = s->queue.begin(); it != s->queue.end();) {
    Request* r = s->reqs[*it];
    if (r->kind != kind) { ++it; continue; }
    if (s->slots_used + (int)batch.size() >= s->max_slots) break;
    size_t probe = 0;
    const size_t want = batch.empty() ? r->footprint : total + r->footprint + 65536;
    if (!s->alloc.alloc(want, probe)) break;
    s->alloc.release(probe, want);
    total += r->footprint;
    batch.push_back(r);
    it = s->queue.erase(it);
  }
  if (batch.empty()) return false;
  while (true) {
    bytes = batch_bytes(batch, kind, total);
    if (s->alloc.alloc(bytes, off)) break;
    if (batch.size() > 1) {
      // give back all but the head, in their order
      for (size_t i = batch.size() - 1; i >= 1; --i) s->queue.push_front(batch[i]->ticket);
      batch.resize(1);
      continue;
    }
    if (round256(bytes) > s->pool_bytes) {
      fail_request(s, batch[0], SNC_ENOMEM, "request workspace of " + std::to_string(bytes) +
                                                 " bytes exceeds the pool of " + std::to_string(s->pool_bytes));
      failed = true;
    } else {
      s->queue.push_front(batch[0]->ticket);  // in-flight work frees pool bytes and notifies
    }
    batch.clear();
    return false;
  }
  s->slots_used += (int)batch.size();
  return true;
}

void worker_main(snc_server* s) {
  (void)hipSetDevice(s->device);
  snc_ctx* c = nullptr;
  if (snc_create(s->device, &c) != SNC_OK) return;
  hipStream_t st = nullptr;
  (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  std::vector<Request*> batch;
  std::vector<snc_upoly> outs;
  std::vector<snc_bipoly> fs, gs;
  while (true) {
    size_t off = 0, bytes = 0;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      bool failed = false;
      s->cv.wait(lk, [&] {
        if (s->stop) return true;
        while (true) {  // after a request failed, the next one may be admitted
          if (take_work(s, batch, off, bytes, failed)) return true;
          if (!failed) return false;
          s->cv_done.notify_all();
        }
      });
      if (batch.empty() && s->stop) break;
    }
    void* ws = s->pool + off;
    // results are written before the status is published under the lock
    std::vector<int> status(batch.size(), SNC_EINTERNAL);
    if (batch[0]->kind == 1) {
      const int n = (int)batch.size();
      std::vector<snc_upoly> as(n), bs(n), os(n);
      std::vector<std::vector<uint32_t>> bufs(n);
      for (int i = 0; i < n; ++i) {
        as[i] = batch[i]->a; bs[i] = batch[i]->b;
        bufs[i].assign((size_t)(batch[i]->out_deg + 1) * batch[i]->out_nl, 0u);
        os[i] = snc_upoly{bufs[i].data(), batch[i]->out_deg, batch[i]->out_nl};
      }
      int stt = snc_gcd_z_batch(c, n, as.data(), bs.data(), ws, bytes, st, os.data());
      if (stt == SNC_OK) {
        for (int i = 0; i < n; ++i) status[i] = SNC_OK;
      } else {
        // isolate the failing request: each alone in the same workspace
        for (int i = 0; i < n; ++i) {
          os[i] = snc_upoly{bufs[i].data(), batch[i]->out_deg, batch[i]->out_nl};
          status[i] = snc_gcd_z(c, &as[i], &bs[i], ws, bytes, st, &os[i]);
          if (status[i] != SNC_OK) batch[i]->err = snc_last_error(c);
        }
      }
      for (int i = 0; i < n; ++i)
        if (status[i] == SNC_OK) {
          batch[i]->res.swap(bufs[i]);
          batch[i]->res_deg = os[i].deg;
          batch[i]->res_nl = os[i].nlimbs;
        }
    } else {
      const int n = (int)batch.size();
      fs.resize(n); gs.resize(n); outs.resize(n);
      std::vector<std::vector<uint32_t>> bufs(n);
      for (int i = 0; i < n; ++i) {
        fs[i] = batch[i]->f; gs[i] = batch[i]->g;
        bufs[i].assign((size_t)(batch[i]->out_deg + 1) * batch[i]->out_nl, 0u);
        outs[i] = snc_upoly{bufs[i].data(), batch[i]->out_deg, batch[i]->out_nl};
      }
      const int stt = run_resultants(c, n, fs.data(), gs.data(), ws, bytes, st, outs.data(), /*graph=*/false);
      for (int i = 0; i < n; ++i) {
        Request* r = batch[i];
        status[i] = stt;
        if (stt == SNC_OK) { r->res.swap(bufs[i]); r->res_deg = outs[i].deg; r->res_nl = outs[i].nlimbs; }
        else r->err = c->err;
      }
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      const auto now = Clock::now();
      for (size_t i = 0; i < batch.size(); ++i) {
        Request* r = batch[i];
        r->t_done = now;
        r->status = status[i];
        s->times[r->ticket] = {secs(r->t_submit), secs(now)};
      }
      s->alloc.release(off, bytes);
      s->slots_used -= (int)batch.size();
      s->completed += (int64_t)batch.size();
    }
    s->cv.notify_all();
    s->cv_done.notify_all();
  }
  (void)hipStreamDestroy(st);
  snc_destroy(c);
}

}  // namespace
}  // namespace snc

extern "C" {

int snc_server_create(snc_ctx* ctx, void* d_pool, size_t pool_bytes, int32_t max_slots, int32_t nstreams,
                      snc_server** out) {
  if (!ctx || !out || !d_pool || pool_bytes < 256 || max_slots < 1 || nstreams < 1 || nstreams > 16)
    return SNC_EINVAL;
  snc_server* s = new snc_server();
  s->device = ctx->device;
  s->pool = (uint8_t*)d_pool;
  s->pool_bytes = pool_bytes;
  s->max_slots = max_slots;
  s->alloc.init(pool_bytes);
  for (int i = 0; i < nstreams; ++i) s->workers.emplace_back(worker_main, s);
  *out = s;
  return SNC_OK;
}

static int submit(snc_server* s, Request* r, uint64_t* ticket) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (round256(r->footprint) > s->pool_bytes) { delete r; return SNC_ENOMEM; }
  r->ticket = s->next_ticket++;
  r->t_submit = Clock::now();
  s->reqs[r->ticket] = r;
  s->queue.push_back(r->ticket);
  *ticket = r->ticket;
  s->cv.notify_one();
  return SNC_OK;
}

int snc_submit_resultant_y(snc_server* s, const snc_bipoly* f, const snc_bipoly* g, uint64_t* ticket) {
  if (!s || !f || !g || !ticket) return SNC_EINVAL;
  Request* r = new Request();
  r->kind = 0;
  auto copy = [](const snc_bipoly* p, std::vector<uint32_t>& v, snc_bipoly& d) {
    d = *p;
    if (p->dy >= 0 && p->limbs) {
      v.assign(p->limbs, p->limbs + (size_t)(p->dy + 1) * (p->dx + 1) * p->nlimbs);
      d.limbs = v.data();
    }
  };
  copy(f, r->fl, r->f);
  copy(g, r->gl, r->g);
  snc_plan pl{};
  int st = snc_resultant_y_plan(&r->f, &r->g, &pl);
  if (st) { delete r; return st; }
  r->footprint = pl.workspace_bytes;
  r->out_deg = pl.deg_bound;
  r->out_nl = pl.out_nlimbs;
  return submit(s, r, ticket);
}

int snc_submit_gcd_z(snc_server* s, const snc_upoly* a, const snc_upoly* b, uint64_t* ticket) {
  if (!s || !a || !b || !ticket) return SNC_EINVAL;
  Request* r = new Request();
  r->kind = 1;
  auto copy = [](const snc_upoly* p, std::vector<uint32_t>& v, snc_upoly& d) {
    d = *p;
    if (p->deg >= 0 && p->limbs) {
      v.assign(p->limbs, p->limbs + (size_t)(p->deg + 1) * p->nlimbs);
      d.limbs = v.data();
    }
  };
  copy(a, r->fl, r->a);
  copy(b, r->gl, r->b);
  snc_plan pl{};
  int st = snc_gcd_z_plan(&r->a, &r->b, &pl);
  if (st) { delete r; return st; }
  r->footprint = pl.workspace_bytes;
  r->out_deg = pl.deg_bound;
  r->out_nl = pl.out_nlimbs;
  return submit(s, r, ticket);
}

int snc_poll(snc_server* s, uint64_t ticket, snc_upoly* out) {
  if (!s || !out) return SNC_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return SNC_EINVAL;
  Request* r = it->second;
  if (r->status == SNC_EAGAIN) return SNC_EAGAIN;
  if (r->status != SNC_OK) {
    const int st = r->status;
    delete r;
    s->reqs.erase(it);
    return st;
  }
  const int need_deg = std::max(r->res_deg, 0);
  if (out->deg < need_deg || out->nlimbs < r->res_nl || (r->res_deg >= 0 && !out->limbs)) {
    out->deg = need_deg;
    out->nlimbs = r->res_nl;
    return SNC_ERANGE;  // the result stays available
  }
  for (int i = 0; i <= r->res_deg; ++i) {
    const uint32_t* src = r->res.data() + (size_t)i * r->res_nl;
    uint32_t* dst = out->limbs + (size_t)i * out->nlimbs;
    const uint32_t ext = (src[r->res_nl - 1] >> 31) ? 0xffffffffu : 0u;
    for (int l = 0; l < out->nlimbs; ++l) dst[l] = l < r->res_nl ? src[l] : ext;
  }
  out->deg = r->res_deg;
  delete r;
  s->reqs.erase(it);
  return SNC_OK;
}

int snc_request_times(snc_server* s, uint64_t ticket, double* submit_s, double* done_s) {
  if (!s) return SNC_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->times.find(ticket);
  if (it == s->times.end()) return s->reqs.count(ticket) ? SNC_EAGAIN : SNC_EINVAL;
  if (submit_s) *submit_s = it->second.first;
  if (done_s) *done_s = it->second.second;
  return SNC_OK;
}

int snc_server_wait(snc_server* s, int64_t completed_at_least, double timeout_s) {
  if (!s) return SNC_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  const bool ok = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                      [&] { return s->completed >= completed_at_least; });
  return ok ? SNC_OK : SNC_EAGAIN;
}

int snc_server_destroy(snc_server* s) {
  if (!s) return SNC_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    // drop requests that were never admitted
    for (uint64_t t : s->queue) {
      auto it = s->reqs.find(t);
      if (it != s->reqs.end()) { delete it->second; s->reqs.erase(it); }
    }
    s->queue.clear();
  }
  s->cv.notify_all();
  for (auto& w : s->workers) w.join();
  for (auto& kv : s->reqs) delete kv.second;
  delete s;
  return SNC_OK;
}

}  // extern "C"
