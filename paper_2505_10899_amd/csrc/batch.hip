// Many independent D2Q9 cases of uneven sizes advanced by one work-list kernel per step.
//
// A fixed number of resident workgroups strides over the work items (case, x strip,
// band of rows) of all cases; each item is the same tile march as the single-case
// fused step (step2d_tile).  The n launches of a call are captured in one hipGraph and
// replayed as one launch.  Per-case volume reductions: every item writes its partial
// sums; the next launch (or a fold-only launch at the end of a call) sums each case's
// items in a fixed order into that case's observation history.
#include <hip/hip_runtime.h>

#include "devcase.hpp"
#include "launch.hpp"
#include "step2d.hpp"

namespace vclb {

// sum case cs's item partials in item order into its history slot
template <class St>
__device__ __forceinline__ void fold_case(const DevCase<D2Q9, St>& c, const BatchArgs& a, int cs) {
  __shared__ double red[16 * 12];
  const int2 r = a.case_items[cs];
  double v[12];
#pragma unroll
  for (int f = 0; f < 12; ++f) v[f] = 0.0;
  for (int i = threadIdx.x; i < r.y; i += blockDim.x) {
#pragma unroll
    for (int f = 0; f < 12; ++f) v[f] += a.part_r[long(f) * a.nitems + r.x + i];
  }
  const double s = block_sum_fields<12>(v, 12, red);
  if (threadIdx.x < 12) {
    double* dest = c.hist + (a.pend_step % kHistory) * kObsFields;
    dest[threadIdx.x] = s;
    if (threadIdx.x == 0) dest[12] = double(a.pend_step);
  }
  __syncthreads();
}

template <class St>
__global__ void __launch_bounds__(256, sizeof(typename St::R) == 8 ? 2 : 4)
    k_batch_step2d(const DevCase<D2Q9, St>* __restrict__ cases, BatchArgs a) {
  extern __shared__ unsigned char smem_raw[];
  if (a.pend)
    for (int cs = blockIdx.x; cs < a.ncases; cs += gridDim.x) fold_case<St>(cases[cs], a, cs);
  // rounds of gridDim.x consecutive items; within a round, consecutive items go to one
  // XCD (neighbouring tiles of a case share halo lines in its L2)
  const int slot = xcd_tile(blockIdx.x, gridDim.x);
  for (int base = 0; base < a.nitems; base += gridDim.x) {
    const int it = base + slot;
    if (it >= a.nitems) break;
    const int4 w = a.items[it];
    step2d_tile<St, true>(cases[w.x], a.t, w.y, w.z, w.w, a.reduce != 0, a.part_w, a.nitems, it, smem_raw);
    __syncthreads();
  }
}

template <class St>
__global__ void __launch_bounds__(256) k_batch_fold(const DevCase<D2Q9, St>* __restrict__ cases, BatchArgs a) {
  for (int cs = blockIdx.x; cs < a.ncases; cs += gridDim.x) fold_case<St>(cases[cs], a, cs);
}

template <class St>
int launch_batch_step(const void* cases, const BatchArgs& a, int blocks, int bx, hipStream_t s) {
  const size_t lds = size_t(2) * 4 * (bx + 2) * sizeof(typename St::R);
  hipLaunchKernelGGL((k_batch_step2d<St>), dim3(blocks), dim3(bx), lds, s,
                     static_cast<const DevCase<D2Q9, St>*>(cases), a);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <class St>
int launch_batch_fold(const void* cases, const BatchArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_batch_fold<St>), dim3(a.ncases < 1024 ? a.ncases : 1024), dim3(256), 0, s,
                     static_cast<const DevCase<D2Q9, St>*>(cases), a);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <class St>
int batch_max_blocks_per_cu(int bx) {
  int nb = 0;
  const size_t lds = size_t(2) * 4 * (bx + 2) * sizeof(typename St::R);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_step2d<St>, bx, lds) != hipSuccess) return 0;
  return nb;
}

template int launch_batch_step<StoreF64>(const void*, const BatchArgs&, int, int, hipStream_t);
template int launch_batch_step<StoreF32>(const void*, const BatchArgs&, int, int, hipStream_t);
template int launch_batch_step<StoreF16S>(const void*, const BatchArgs&, int, int, hipStream_t);
template int launch_batch_fold<StoreF64>(const void*, const BatchArgs&, hipStream_t);
template int launch_batch_fold<StoreF32>(const void*, const BatchArgs&, hipStream_t);
template int launch_batch_fold<StoreF16S>(const void*, const BatchArgs&, hipStream_t);
template int batch_max_blocks_per_cu<StoreF64>(int);
template int batch_max_blocks_per_cu<StoreF32>(int);
template int batch_max_blocks_per_cu<StoreF16S>(int);

}  // namespace vclb
