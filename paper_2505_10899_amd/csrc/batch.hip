// Many independent D2Q9 cases of uneven sizes advanced by one work-list kernel per step.
//
// A fixed number of resident workgroups each take one run of consecutive work items,
// the runs cut on the host so that every workgroup has about the same number of
// iterations, or iterations in proportion to the speed its slot was measured at (items
// are split between rows where a run ends).  An item is either a strip of columns marched
// row by row (step2d_tile, one lane per column: best when the width is close to a
// multiple of the wave size) or a band of whole rows marched in the case's stored
// row-major order (step2d_flat: every lane busy for any width, every wave storing whole
// cache lines); the host picks per case.  The n launches of a call are captured in one
// hipGraph and replayed as one launch.  Per-case volume reductions: every item writes its partial
// sums; the next launch (or a fold-only launch at the end of a call) sums each case's
// items in a fixed order into that case's observation history.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "devcase.hpp"
#include "launch.hpp"
#include "flat2d.hpp"

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

// Workgroups per CU the register budget is sized for: FP32 arithmetic fits 4 waves per
// SIMD, except the lag-3 FIFO with general rates (a little more than 128 VGPRs: 3); FP64
// fits 2, or 3 for the short lag with unit rates (at most 168 VGPRs).  A 1024-lane
// workgroup alone puts 4 waves on each SIMD.
template <class St, int DL, int BS, bool UNIT>
constexpr int batch_min_blocks() {
  constexpr int waves = sizeof(typename St::R) == 8 ? (UNIT && DL == 1 ? 3 : 2) : (DL == 3 && !UNIT ? 3 : 4);
  constexpr int per_block = BS / 256;                                          // waves per SIMD
  return waves / per_block > 0 ? waves / per_block : 1;
}

// VISC: some case of the batch has unequal viscosities (per-node tau_f, Eq. 27); the
// others then take the same per-node form, which gives their constant tau_f
template <class St, int DL, int BS, bool UNIT, bool VISC>
__global__ void __launch_bounds__(BS, (batch_min_blocks<St, DL, BS, UNIT>()))
    k_batch_step2d(const DevCase<D2Q9, St>* __restrict__ cases, BatchArgs a) {
  extern __shared__ unsigned char smem_raw[];
  if (a.pend)
    for (int cs = blockIdx.x; cs < a.ncases; cs += gridDim.x) fold_case<St>(cases[cs], a, cs);
  // consecutive runs go to one XCD: the rows where one run ends and the next begins are
  // read by both, through that XCD's L2
  const int slot = xcd_tile(blockIdx.x, gridDim.x);
  const int2 run = a.runs[slot];
  const unsigned long long t_begin = a.ticks ? wall_clock64() : 0ull;
  for (int it = run.x; it < run.x + run.y; ++it) {
    const int4 w = a.items[it];
    if (w.y < 0)   // a band of whole rows, marched in stored row-major order
      step2d_flat<St, DL, UNIT, VISC>(cases[w.x], a.t, w.z, w.w, a.reduce != 0, a.cap, a.part_w, a.nitems, it,
                                      smem_raw);
    else           // a strip of columns [w.y, w.y + blockDim.x), one lane per column
      step2d_tile<St, true, unsigned, UNIT, VISC>(cases[w.x], a.t, w.y, w.z, w.w, a.reduce != 0, a.part_w, a.nitems,
                                                  it, smem_raw);
    __syncthreads();
  }
  // balancing launches record how long this slot took over its run (constant-rate clock)
  if (a.ticks && threadIdx.x == 0) a.ticks[slot] = unsigned(wall_clock64() - t_begin);
}

template <class St>
__global__ void __launch_bounds__(256) k_batch_fold(const DevCase<D2Q9, St>* __restrict__ cases, BatchArgs a) {
  for (int cs = blockIdx.x; cs < a.ncases; cs += gridDim.x) fold_case<St>(cases[cs], a, cs);
}

template <class St>
size_t batch_lds_bytes(int cap, int bx) {
  const size_t flat = size_t(2) * cap * sizeof(typename St::R);
  const size_t rows = size_t(2) * 4 * (bx + 2) * sizeof(typename St::R);
  return flat > rows ? flat : rows;
}

// the kernel instantiation for a launch shape (bx lanes, lag, unit rates, unequal
// viscosities); fn receives a pointer to it.  1024-lane workgroups (4 waves per SIMD in
// one workgroup per CU) exist for 4-byte arithmetic only: FP64 needs more than the 128
// registers they leave a lane.
template <class St, class Fn>
int with_batch_kernel(int bx, int lag, bool unit, bool visc, Fn&& fn) {
  if (lag != 1 && lag != 3) return -1;
  auto pick = [&](auto bs) -> int {
    constexpr int BS = decltype(bs)::value;
    auto by_rates = [&](auto v) -> int {
      constexpr bool V = decltype(v)::value;
      if (lag == 1) return unit ? fn(k_batch_step2d<St, 1, BS, true, V>) : fn(k_batch_step2d<St, 1, BS, false, V>);
      return unit ? fn(k_batch_step2d<St, 3, BS, true, V>) : fn(k_batch_step2d<St, 3, BS, false, V>);
    };
    return visc ? by_rates(std::true_type{}) : by_rates(std::false_type{});
  };
  if (bx > 512) {
    if constexpr (sizeof(typename St::R) == 4) return pick(std::integral_constant<int, 1024>{});
    else return -1;
  }
  return bx <= 256 ? pick(std::integral_constant<int, 256>{}) : pick(std::integral_constant<int, 512>{});
}

template <class St>
int launch_batch_step(const void* cases, const BatchArgs& a, int blocks, int bx, hipStream_t s) {
  const size_t lds = batch_lds_bytes<St>(a.cap, bx);
  const auto* cs = static_cast<const DevCase<D2Q9, St>*>(cases);
  const int rc = with_batch_kernel<St>(bx, a.lag, a.unit != 0, a.visc != 0, [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(bx), lds, s, cs, a);
    return 0;
  });
  if (rc) return rc;
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <class St>
int launch_batch_fold(const void* cases, const BatchArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_batch_fold<St>), dim3(a.ncases < 1024 ? a.ncases : 1024), dim3(256), 0, s,
                     static_cast<const DevCase<D2Q9, St>*>(cases), a);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <class St>
int batch_max_blocks_per_cu(int bx, int cap, int lag, bool unit, bool visc) {
  int nb = 0;
  const size_t lds = batch_lds_bytes<St>(cap, bx);
  const int rc = with_batch_kernel<St>(bx, lag, unit, visc, [&](auto kern) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, bx, lds) == hipSuccess ? 0 : -1;
  });
  return rc ? 0 : nb;
}

template int launch_batch_step<StoreF64>(const void*, const BatchArgs&, int, int, hipStream_t);
template int launch_batch_step<StoreF32>(const void*, const BatchArgs&, int, int, hipStream_t);
template int launch_batch_step<StoreF16S>(const void*, const BatchArgs&, int, int, hipStream_t);
template int launch_batch_fold<StoreF64>(const void*, const BatchArgs&, hipStream_t);
template int launch_batch_fold<StoreF32>(const void*, const BatchArgs&, hipStream_t);
template int launch_batch_fold<StoreF16S>(const void*, const BatchArgs&, hipStream_t);
template int batch_max_blocks_per_cu<StoreF64>(int, int, int, bool, bool);
template int batch_max_blocks_per_cu<StoreF32>(int, int, int, bool, bool);
template int batch_max_blocks_per_cu<StoreF16S>(int, int, int, bool, bool);
template size_t batch_lds_bytes<StoreF64>(int, int);
template size_t batch_lds_bytes<StoreF32>(int, int);
template size_t batch_lds_bytes<StoreF16S>(int, int);

}  // namespace vclb
