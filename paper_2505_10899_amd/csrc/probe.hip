// Achievable-bandwidth probe: plain grid-stride kernels over 16-byte vectors that copy,
// read or write one buffer.  The step kernels are bounded by HBM bandwidth; what this
// measures on the same device is the practical ceiling their rates are compared with.
#include <hip/hip_runtime.h>

#include "probe.hpp"

namespace vclb {

__global__ void __launch_bounds__(256) k_probe_copy(const float4* __restrict__ src, float4* __restrict__ dst, long n) {
  for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < n; i += long(gridDim.x) * blockDim.x) dst[i] = src[i];
}

// sums what it reads and stores the sum only when it equals an arbitrary constant: the
// loads cannot be dropped, and in practice no store is issued
__global__ void __launch_bounds__(256) k_probe_read(const float4* __restrict__ src, float* __restrict__ sink, long n) {
  float s = 0.0f;
  for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < n; i += long(gridDim.x) * blockDim.x) {
    const float4 v = src[i];
    s += (v.x + v.y) + (v.z + v.w);
  }
  if (s == -1.2345e-30f) sink[0] = s;
}

__global__ void __launch_bounds__(256) k_probe_write(float4* __restrict__ dst, long n) {
  for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < n; i += long(gridDim.x) * blockDim.x)
    dst[i] = make_float4(1.0f, 2.0f, 3.0f, 4.0f);
}

int launch_probe(int mode, void* dst, const void* src, long n16, int blocks, hipStream_t s) {
  const dim3 grid(blocks), block(256);
  if (mode == 0)
    hipLaunchKernelGGL(k_probe_copy, grid, block, 0, s, static_cast<const float4*>(src), static_cast<float4*>(dst), n16);
  else if (mode == 1)
    hipLaunchKernelGGL(k_probe_read, grid, block, 0, s, static_cast<const float4*>(src), static_cast<float*>(dst), n16);
  else
    hipLaunchKernelGGL(k_probe_write, grid, block, 0, s, static_cast<float4*>(dst), n16);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace vclb
