// Achievable-bandwidth probe: grid-stride kernels over 16-byte vectors that copy, read or
// write one buffer.  The step kernels are bounded by HBM bandwidth; what this measures on
// the same device is the practical ceiling their rates are compared with.  Each lane
// keeps U vectors in flight (U loads issued before the first store or use), with plain or
// non-temporal accesses; the host sweeps U, the non-temporal choice and the number of
// resident workgroups, and keeps the fastest.
#include <hip/hip_runtime.h>

#include "probe.hpp"

namespace vclb {

typedef float v4f __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ v4f ld4(const v4f* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT>
__device__ __forceinline__ void st4(v4f* p, v4f v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// a workgroup's tile is U * blockDim consecutive vectors; lane l takes vectors l,
// l + blockDim, ..., so every load instruction of a wave reads 1 KiB of consecutive memory
template <int U, bool NT>
__global__ void __launch_bounds__(256) k_probe_copy(const v4f* __restrict__ src, v4f* __restrict__ dst, long n) {
  const long tile = long(blockDim.x) * U;
  for (long base = blockIdx.x * tile; base < n; base += long(gridDim.x) * tile) {
    v4f v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long i = base + long(u) * blockDim.x + threadIdx.x;
      if (i < n) v[u] = ld4<NT>(src + i);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long i = base + long(u) * blockDim.x + threadIdx.x;
      if (i < n) st4<NT>(dst + i, v[u]);
    }
  }
}

// sums what it reads and stores the sum only when it equals an arbitrary constant: the
// loads cannot be dropped, and in practice no store is issued
template <int U, bool NT>
__global__ void __launch_bounds__(256) k_probe_read(const v4f* __restrict__ src, float* __restrict__ sink, long n) {
  const long tile = long(blockDim.x) * U;
  float s = 0.0f;
  for (long base = blockIdx.x * tile; base < n; base += long(gridDim.x) * tile) {
    v4f v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long i = base + long(u) * blockDim.x + threadIdx.x;
      v[u] = i < n ? ld4<NT>(src + i) : v4f{0.0f, 0.0f, 0.0f, 0.0f};
    }
#pragma unroll
    for (int u = 0; u < U; ++u) s += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  if (s == -1.2345e-30f) sink[0] = s;
}

template <int U, bool NT>
__global__ void __launch_bounds__(256) k_probe_write(v4f* __restrict__ dst, long n) {
  const long tile = long(blockDim.x) * U;
  const v4f val = {1.0f, 2.0f, 3.0f, 4.0f};
  for (long base = blockIdx.x * tile; base < n; base += long(gridDim.x) * tile) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long i = base + long(u) * blockDim.x + threadIdx.x;
      if (i < n) st4<NT>(dst + i, val);
    }
  }
}

template <int U, bool NT>
static void launch_probe_t(int mode, void* dst, const void* src, long n16, int blocks, hipStream_t s) {
  const dim3 grid(blocks), block(256);
  if (mode == 0)
    hipLaunchKernelGGL((k_probe_copy<U, NT>), grid, block, 0, s, static_cast<const v4f*>(src), static_cast<v4f*>(dst), n16);
  else if (mode == 1)
    hipLaunchKernelGGL((k_probe_read<U, NT>), grid, block, 0, s, static_cast<const v4f*>(src), static_cast<float*>(dst), n16);
  else
    hipLaunchKernelGGL((k_probe_write<U, NT>), grid, block, 0, s, static_cast<v4f*>(dst), n16);
}

int launch_probe(int mode, int unroll, int nontemporal, void* dst, const void* src, long n16, int blocks,
                 hipStream_t s) {
  auto go = [&](auto nt) {
    constexpr bool NT = decltype(nt)::value;
    switch (unroll) {
      case 1: launch_probe_t<1, NT>(mode, dst, src, n16, blocks, s); return 0;
      case 2: launch_probe_t<2, NT>(mode, dst, src, n16, blocks, s); return 0;
      case 4: launch_probe_t<4, NT>(mode, dst, src, n16, blocks, s); return 0;
      case 8: launch_probe_t<8, NT>(mode, dst, src, n16, blocks, s); return 0;
      default: return -1;
    }
  };
  const int rc = nontemporal ? go(std::true_type{}) : go(std::false_type{});
  if (rc) return rc;
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace vclb
