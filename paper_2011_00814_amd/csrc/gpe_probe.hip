// gpe_probe.hip -- HBM streaming probe: the bandwidth a plain streaming
// kernel reaches on this device (read-only, write-only and copy, 16-byte
// accesses), the practical ceiling the stencil kernels are compared with.
// A measurement aid, not part of the method.
#include <hip/hip_runtime.h>

#include "gpe.h"

namespace {

constexpr int kBlock = 256;
constexpr int kUnroll = 4;  // independent 16-byte accesses in flight per thread and iteration

// Grid-strided over n float4 elements; each iteration issues kUnroll loads
// before it uses any of them.  The sum is stored only if it equals a value
// it never takes, which keeps the loads without writing anything.
__global__ __launch_bounds__(kBlock) void stream_read_kernel(const float4* __restrict__ src, size_t n,
                                                             float* __restrict__ sink) {
  const size_t stride = (size_t)gridDim.x * kBlock;
  size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  float acc = 0.f;
  for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
    float4 v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) v[u] = src[i + u * stride];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  for (; i < n; i += stride) {
    const float4 v = src[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  if (acc == -1.2345e38f) sink[0] = acc;
}

__global__ __launch_bounds__(kBlock) void stream_write_kernel(float4* __restrict__ dst, size_t n, float val) {
  const size_t stride = (size_t)gridDim.x * kBlock;
  const float4 v = make_float4(val, val, val, val);
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) dst[i] = v;
}

__global__ __launch_bounds__(kBlock) void stream_copy_kernel(float4* __restrict__ dst, const float4* __restrict__ src,
                                                             size_t n) {
  const size_t stride = (size_t)gridDim.x * kBlock;
  size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
    float4 v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) v[u] = src[i + u * stride];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) dst[i + u * stride] = v[u];
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" int gpe_hbm_stream(int32_t mode, void* d_dst, const void* d_src, size_t bytes, int32_t workgroups,
                              void* stream) {
  if (bytes == 0 || bytes % 16 != 0 || workgroups < 0) return GPE_EINVAL;
  if ((mode == GPE_STREAM_READ || mode == GPE_STREAM_COPY) && !d_src) return GPE_EINVAL;
  if (!d_dst) return GPE_EINVAL;
  if ((uintptr_t)d_dst % 16 != 0 || (uintptr_t)d_src % 16 != 0) return GPE_EINVAL;
  int wg = workgroups;
  if (wg == 0) {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
      ncu = 256;
    wg = 8 * ncu;  // 8 work-groups of 4 waves per CU: 32 waves, the CU's limit
  }
  const size_t n = bytes / 16;
  hipStream_t s = (hipStream_t)stream;
  switch (mode) {
    case GPE_STREAM_READ:
      hipLaunchKernelGGL(stream_read_kernel, dim3(wg), dim3(kBlock), 0, s, (const float4*)d_src, n, (float*)d_dst);
      break;
    case GPE_STREAM_WRITE:
      hipLaunchKernelGGL(stream_write_kernel, dim3(wg), dim3(kBlock), 0, s, (float4*)d_dst, n, 1.0f);
      break;
    case GPE_STREAM_COPY:
      hipLaunchKernelGGL(stream_copy_kernel, dim3(wg), dim3(kBlock), 0, s, (float4*)d_dst, (const float4*)d_src, n);
      break;
    default:
      return GPE_EINVAL;
  }
  return hipGetLastError() == hipSuccess ? GPE_OK : GPE_EHIP;
}
