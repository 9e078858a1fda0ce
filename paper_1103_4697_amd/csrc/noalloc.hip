// One resultant with no allocation: snc_resultant_y_noalloc.
//
// The same pipeline of launches as snc_resultant_y (reduction, evaluation and
// elimination, interpolation, Chinese remaindering), with its device
// workspace taken from a fixed array in device memory instead of a caller
// workspace, the upload block built in a fixed host array, and the results
// downloaded straight into the caller's output buffer.  The call makes no
// device or pinned allocation and creates no stream, event or graph: for
// callers that cannot allocate.
//
// The array is a module global: each device holds one copy from the first
// load of the library until the process ends, every call on a device shares
// it and it keeps the last call's contents.  Nothing read by the pipeline
// depends on its earlier contents except the abnormal-instance counter,
// which is cleared (by a kernel) before the launches.  Calls that overlap on
// one device race on the array; the host part of a call is serialised by a
// mutex, which the call holds until its results are on the host.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "runtime_internal.hpp"
#include "snc.h"

namespace snc {

constexpr int NOALLOC_MAX_DEVICES = 64;
constexpr size_t NOALLOC_HEADER_BYTES = (size_t)8 << 20;  // host upload block

static __device__ __align__(256) uint8_t scratch[SNC_NOALLOC_SCRATCH_BYTES];

// device address of `scratch` per device, looked up once at set-up with the
// device current (the host-side name is not a device address)
static uint8_t* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {nullptr};
static uint8_t g_header[NOALLOC_HEADER_BYTES];
static std::mutex g_noalloc_mu;

hipError_t init_noalloc_scratch(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = (uint8_t*)p;
  return hipSuccess;
}

}  // namespace snc

using namespace snc;

extern "C" int snc_resultant_y_noalloc(snc_ctx* c, const snc_bipoly* f, const snc_bipoly* g, void* stream,
                                       snc_upoly* out) {
  if (!c || !out) return SNC_EINVAL;
  std::vector<Operand> F(1), G(1);
  std::vector<ResPlan> P(1);
  int st = parse_bipoly(f, F[0], c->err);
  if (!st) st = parse_bipoly(g, G[0], c->err);
  if (!st) st = plan_resultant(F[0], G[0], P[0], c->err);
  if (st) return st;
  const ResPlan& pl = P[0];
  // output sizes first (SNC_ERANGE writes the required sizes back)
  const int need_deg = pl.trivial ? (pl.trivial_value ? 0 : -1) : pl.D;
  const int need_nl = pl.trivial ? 1 : pl.L;
  if (out->deg < need_deg || out->nlimbs < need_nl || (need_deg >= 0 && !out->limbs)) {
    out->deg = need_deg;
    out->nlimbs = need_nl;
    c->err = "output buffer too small";
    return SNC_ERANGE;
  }
  if (pl.trivial) {
    if (pl.trivial_value) {
      for (int l = 0; l < out->nlimbs; ++l) out->limbs[l] = l == 0 ? 1u : 0u;
      out->deg = 0;
    } else {
      out->deg = -1;
    }
    return SNC_OK;
  }
  BatchLayout lay;
  layout_batch(P, lay);
  if (lay.total_bytes > SNC_NOALLOC_SCRATCH_BYTES) {
    c->err = "snc_resultant_y_noalloc: the pair needs " + std::to_string(lay.total_bytes) +
             " bytes of device scratch, the fixed array holds " + std::to_string((size_t)SNC_NOALLOC_SCRATCH_BYTES);
    return SNC_ENOMEM;
  }
  if (lay.header_bytes > NOALLOC_HEADER_BYTES) {
    c->err = "snc_resultant_y_noalloc: upload block of " + std::to_string(lay.header_bytes) +
             " bytes exceeds the fixed host array of " + std::to_string(NOALLOC_HEADER_BYTES);
    return SNC_ENOMEM;
  }
  if (c->device < 0 || c->device >= NOALLOC_MAX_DEVICES || !g_scratch_ptr[c->device]) {
    c->err = "snc_resultant_y_noalloc: no scratch address for this device (context not set up)";
    return SNC_EDEVICE;
  }
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  auto fail = [&](const char* what, hipError_t e) {
    c->err = std::string("snc_resultant_y_noalloc: ") + what + ": " + hipGetErrorString(e);
    return SNC_EDEVICE;
  };
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return fail("set device", e);
  uint8_t* ws = g_scratch_ptr[c->device];
  fill_header(lay, P, F, G, g_header);
  e = hipMemcpyAsync(ws, g_header, lay.header_bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail("upload", e);
  // the only state a run reads before writing it: cleared by a kernel
  launch_zero_u32((uint32_t*)(ws + lay.abn_count_off), 1, s);
  launch_pipeline(lay, ws, s, nullptr, PIPE_ALL);
  e = hipGetLastError();
  if (e != hipSuccess) return fail("launch", e);
  // [D+1][L] limbs straight into the caller's buffer, which holds at least
  // (D+1) * nlimbs >= (D+1) * L words; widened to the caller's stride below
  const ResJob& J = lay.jobs[0];
  const size_t n1 = (size_t)J.D + 1;
  e = hipMemcpyAsync(out->limbs, ws + (size_t)J.out_off * 4, n1 * J.L * 4, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return fail("download", e);
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail("synchronize", e);
  // widen in place from the top coefficient and the top limb down: the
  // destination of every word lies at or above its source, and the sources
  // below it are still unread
  const int S = out->nlimbs, L = J.L;
  uint32_t* buf = out->limbs;
  for (int64_t t = (int64_t)n1 - 1; t >= 0 && S != L; --t) {
    const uint32_t ext = (buf[t * L + L - 1] >> 31) ? 0xffffffffu : 0u;
    for (int l = S - 1; l >= L; --l) buf[t * S + l] = ext;
    for (int l = L - 1; l >= 0; --l) buf[t * S + l] = buf[t * L + l];
  }
  int deg = -1;
  for (int64_t t = (int64_t)n1 - 1; t >= 0 && deg < 0; --t)
    for (int l = 0; l < S; ++l)
      if (buf[t * S + l]) { deg = (int)t; break; }
  out->deg = deg;
  return SNC_OK;
}
