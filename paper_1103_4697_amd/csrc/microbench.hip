// Throughput ceilings of the integer operations the modular kernels are made
// of, measured on the device they run on: Montgomery products, 32-bit low
// multiplies and 64-bit multiply-adds, each in eight independent chains per
// lane so that issue, not latency, bounds them.  The roofline of the
// resultant and gcd kernels is stated against these rates beside the
// nominal int32 VALU peak.
#include <hip/hip_runtime.h>

#include <string>

#include "runtime_internal.hpp"

namespace snc {

constexpr int MB_THREADS = 256;
constexpr int MB_CHAINS = 8;

template <int KIND>
__global__ __launch_bounds__(MB_THREADS) void k_microbench(uint32_t* out, int iters, uint32_t y, PrimeC c) {
  const uint32_t t = blockIdx.x * MB_THREADS + threadIdx.x;
  uint32_t a[MB_CHAINS];
  uint64_t w[MB_CHAINS];
#pragma unroll
  for (int i = 0; i < MB_CHAINS; ++i) {
    a[i] = (t * 2654435761u + (uint32_t)i * 40503u) % c.p;
    w[i] = a[i];
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < MB_CHAINS; ++i) {
      if constexpr (KIND == SNC_MB_MONTGOMERY) a[i] = mmul(a[i], y, c.p, c.pinv);   // [0, 2p) stays in range
      else if constexpr (KIND == SNC_MB_MUL_LO) a[i] = a[i] * y;
      else w[i] = (uint64_t)(uint32_t)w[i] * y + (w[i] >> 32);                       // v_mad_u64_u32
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < MB_CHAINS; ++i) s ^= KIND == SNC_MB_MAD_U64 ? (uint32_t)w[i] ^ (uint32_t)(w[i] >> 32) : a[i];
  out[t] = s;
}

}  // namespace snc

using namespace snc;

extern "C" int snc_microbench(snc_ctx* c, int kind, int32_t iters, void* d_buf, size_t buf_bytes, void* stream,
                              double* ops_per_s) {
  if (!c || !ops_per_s || iters < 1 || kind < 0 || kind > 2) return SNC_EINVAL;
  hipDeviceProp_t prop;
  if (hipSetDevice(c->device) != hipSuccess || hipGetDeviceProperties(&prop, c->device) != hipSuccess) {
    c->err = "device query failed";
    return SNC_EDEVICE;
  }
  // sixteen wavefronts per CU
  const int blocks = prop.multiProcessorCount * 16 * 64 / MB_THREADS;
  const size_t need = (size_t)blocks * MB_THREADS * sizeof(uint32_t);
  if (!d_buf || buf_bytes < need) {
    c->err = "microbench buffer of " + std::to_string(buf_bytes) + " bytes, need " + std::to_string(need);
    return SNC_ENOMEM;
  }
  std::string err;
  if (int st = ensure_device_tables(c->device, err)) { c->err = err; return st; }
  const PrimeC pc = tables().pc[0];
  const uint32_t y = pc.r2 % pc.p;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return SNC_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return SNC_EDEVICE; }
  float best = 0.f;
  for (int rep = 0; rep < 4; ++rep) {  // the first launch warms up; the best of the others counts
    (void)hipEventRecord(e0, s);
    if (kind == SNC_MB_MONTGOMERY)
      hipLaunchKernelGGL(k_microbench<SNC_MB_MONTGOMERY>, dim3(blocks), dim3(MB_THREADS), 0, s, (uint32_t*)d_buf, iters, y, pc);
    else if (kind == SNC_MB_MUL_LO)
      hipLaunchKernelGGL(k_microbench<SNC_MB_MUL_LO>, dim3(blocks), dim3(MB_THREADS), 0, s, (uint32_t*)d_buf, iters, y, pc);
    else
      hipLaunchKernelGGL(k_microbench<SNC_MB_MAD_U64>, dim3(blocks), dim3(MB_THREADS), 0, s, (uint32_t*)d_buf, iters, y, pc);
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) {
      c->err = "microbench launch failed";
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return SNC_EDEVICE;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (rep > 0 && (best == 0.f || ms < best)) best = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const double ops = (double)blocks * MB_THREADS * MB_CHAINS * (double)iters;
  *ops_per_s = best > 0.f ? ops / (best * 1e-3) : 0.0;
  return SNC_OK;
}
