// Streaming reference kernels: what the memory system sustains for pure 16-byte streaming on
// this device, measured with the access pattern the pass kernels use (consecutive lanes on
// consecutive 16-byte elements, non-temporal loads and stores, several loads in flight per
// thread).  The pass kernels' bandwidth is reported beside this ceiling.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "api_internal.h"

namespace ucc {
namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 4;  // 16-byte loads in flight per thread

typedef double dv2 __attribute__((ext_vector_type(2)));

// COPY: dst = src.  Otherwise: every workgroup writes the sum of the components it read to
// part[blockIdx.x] (the data dependence keeps the loads).
template <bool COPY>
__global__ __launch_bounds__(kThreads) void k_stream(const dv2* __restrict__ src, dv2* __restrict__ dst,
                                                     size_t n, double* __restrict__ part) {
  const size_t chunk = size_t(kThreads) * kUnroll;
  const size_t stride = size_t(gridDim.x) * chunk;
  double acc = 0.0;
  size_t i = size_t(blockIdx.x) * chunk + threadIdx.x;
  for (; i + (kUnroll - 1) * kThreads < n; i += stride) {
    dv2 v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) v[u] = __builtin_nontemporal_load(src + i + u * kThreads);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (COPY)
        __builtin_nontemporal_store(v[u], dst + i + u * kThreads);
      else
        acc += v[u].x + v[u].y;
    }
  }
  for (int u = 0; u < kUnroll; ++u, i += kThreads)  // the ragged end of the last chunk
    if (i < n) {
      const dv2 v = __builtin_nontemporal_load(src + i);
      if (COPY)
        __builtin_nontemporal_store(v, dst + i);
      else
        acc += v.x + v.y;
    }
  if (!COPY) {
    __shared__ double red[kThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
  }
}

}  // namespace
}  // namespace ucc

using namespace ucc;

extern "C" ucc_status ucc_stream_probe(const void* src, void* dst, size_t bytes, int32_t mode,
                                       void* stream) {
  g_last_error.clear();
  if (!src || !dst) return fail(UCC_EINVAL, "NULL buffer");
  if (bytes == 0 || bytes % 16 != 0) return fail(UCC_EINVAL, "bytes must be a positive multiple of 16");
  if (mode != 0 && mode != 1) return fail(UCC_EINVAL, "mode must be 0 (copy) or 1 (read)");
  if (!is_device_ptr(src) || !is_device_ptr(dst)) return fail(UCC_EINVAL, "device pointers expected");
  const size_t n = bytes / 16;
  // eight resident workgroups per compute unit, never more than the chunks there are
  const size_t chunks = (n + kThreads * kUnroll - 1) / (kThreads * kUnroll);
  const int grid = (int)std::min<size_t>(chunks, size_t(device_cus()) * 8);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (mode == 0)
    hipLaunchKernelGGL(k_stream<true>, dim3(grid), dim3(kThreads), 0, st,
                       static_cast<const dv2*>(src), static_cast<dv2*>(dst), n, nullptr);
  else
    hipLaunchKernelGGL(k_stream<false>, dim3(grid), dim3(kThreads), 0, st,
                       static_cast<const dv2*>(src), nullptr, n, static_cast<double*>(dst));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "launch k_stream");
  return UCC_OK;
}
