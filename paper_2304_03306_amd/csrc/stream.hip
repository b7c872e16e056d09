// Streaming-bandwidth probe of the device: R input arrays are read and W
// output arrays written, element by element, 16 bytes per lane and access, so
// that the achievable HBM rate for a given read:write mix can be set beside
// the step kernels' rates.  Each workgroup walks a contiguous range of the
// arrays (consecutive lanes on consecutive 16-byte words, kUnroll accesses per
// lane in flight) and then strides over the grid.
#include <hip/hip_runtime.h>

#include "../../include/ttsh.h"
#include "launch.hpp"

namespace ttsh {
namespace {

constexpr int kStreamBS = 256;
constexpr int kUnroll = 4;

template <int R, int W>
__global__ void __launch_bounds__(kStreamBS) k_stream(const float4* __restrict__ in, float4* __restrict__ out,
                                                      size_t n) {
  // array a of the inputs starts at in + a n, output b at out + b n
  const size_t per_block = (size_t)kStreamBS * kUnroll;
  for (size_t base = (size_t)blockIdx.x * per_block; base < n; base += (size_t)gridDim.x * per_block) {
    float4 acc[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) acc[u] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int a = 0; a < R; ++a) {
      float4 v[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const size_t i = base + (size_t)u * kStreamBS + threadIdx.x;
        v[u] = i < n ? in[(size_t)a * n + i] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        acc[u].x += v[u].x;
        acc[u].y += v[u].y;
        acc[u].z += v[u].z;
        acc[u].w += v[u].w;
      }
    }
#pragma unroll
    for (int b = 0; b < W; ++b)
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const size_t i = base + (size_t)u * kStreamBS + threadIdx.x;
        if (i < n) out[(size_t)b * n + i] = acc[u];
      }
    if constexpr (W == 0) {
      // read only: a store that a zero-filled buffer never triggers keeps the
      // loads alive
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const size_t i = base + (size_t)u * kStreamBS + threadIdx.x;
        if (i < n && acc[u].x == 1.0e30f) out[i] = acc[u];
      }
    }
  }
}

template <int R, int W>
hipError_t launch(const float4* in, float4* out, size_t n, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((k_stream<R, W>), dim3(blocks), dim3(kStreamBS), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_rw(int r, int w, const float4* in, float4* out, size_t n, int blocks, hipStream_t s) {
  switch (r * 10 + w) {
    case 11: return launch<1, 1>(in, out, n, blocks, s);
    case 21: return launch<2, 1>(in, out, n, blocks, s);
    case 31: return launch<3, 1>(in, out, n, blocks, s);
    case 52: return launch<5, 2>(in, out, n, blocks, s);
    case 10: return launch<1, 0>(in, out, n, blocks, s);
    case 1: return launch<0, 1>(in, out, n, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace
}  // namespace ttsh

extern "C" int ttsh_stream_bench(int reads, int writes, int64_t elems, int blocks, int reps, void* buf,
                                 double* us_out) {
  using namespace ttsh;
  if (!buf || !us_out) return record_error(TTSH_EINVAL, "null argument");
  if (elems < 1 || reps < 1 || reps > 100000 || blocks < 1 || blocks > (1 << 20))
    return record_error(TTSH_EINVAL, "elems, reps or blocks out of range");
  if ((reinterpret_cast<uintptr_t>(buf) & 15) != 0) return record_error(TTSH_EINVAL, "buffer must be 16-byte aligned");
  const size_t n = (size_t)elems;
  const float4* in = (const float4*)buf;
  // a read-only run keeps one output array for its never-taken store
  float4* out = (float4*)buf + (size_t)reads * n;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return record_error(TTSH_EHIP, "event creation failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return record_error(TTSH_EHIP, "event creation failed");
  }
  int rc = TTSH_OK;
  // one untimed launch, then reps timed back to back on the null stream
  if (launch_rw(reads, writes, in, out, n, blocks, 0) != hipSuccess)
    rc = record_error(TTSH_EINVAL, "unsupported read/write mix (11, 21, 31, 52, 10, 01)");
  if (rc == TTSH_OK) {
    hipEventRecord(e0, 0);
    for (int q = 0; q < reps && rc == TTSH_OK; ++q)
      if (launch_rw(reads, writes, in, out, n, blocks, 0) != hipSuccess) rc = record_error(TTSH_EHIP, "launch failed");
    hipEventRecord(e1, 0);
    if (rc == TTSH_OK && hipEventSynchronize(e1) != hipSuccess) rc = record_error(TTSH_EHIP, "sync failed");
    float ms = 0.f;
    if (rc == TTSH_OK) hipEventElapsedTime(&ms, e0, e1);
    *us_out = 1000.0 * ms / reps;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return rc;
}
