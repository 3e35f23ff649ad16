// Volume reductions of phi over caller-supplied labels (device code and launchers).
//
// The reductions are observables of the phase field (the paper's correction term,
// Eq. 32, is local and uses no global quantity): for every label l, over the nodes n
// with labels[n] == l, the FP64 sums of phi, of the count of phi >= 1/2, of phi x and
// of phi x x^T (x the node's position (i, j, k)), and the count of non-finite phi.
// Negative labels mark nodes that belong to no label; labels >= nlabels are counted as
// invalid and reported to the caller.
//
// Deterministic: workgroup b owns a fixed chunk of nodes and, for each distinct label
// present in its chunk (in increasing order), sums the chunk's contributions with a
// fixed-order tree into its own slot of partials[label][field][b]; a second kernel sums
// each (label, field) over the workgroups in order.  The result does not depend on
// timing, only on n.
#include <hip/hip_runtime.h>

#include <climits>
#include <mutex>

#include "devcase.hpp"
#include "reduce.hpp"

namespace vclb {

// 12 observable fields and the count of invalid labels
constexpr int kLabFields = 13;

__device__ __forceinline__ int block_min_int(int v, int* red) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  int m = INT_MAX;
  for (int w = 0; w < nw; ++w) m = min(m, red[w]);
  return m;
}

// Fixed-order sum of NF doubles over the workgroup; thread f < NF returns field f.
template <int NF>
__device__ __forceinline__ double block_sum_n(const double (&v)[NF], double* red) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    double s = v[f];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red[wave * NF + f] = s;
  }
  __syncthreads();
  double out = 0.0;
  if (int(threadIdx.x) < NF)
    for (int w = 0; w < nw; ++w) out += red[w * NF + threadIdx.x];
  return out;
}

// zero the partials (a fill kernel rather than a memset, so that the launches can be
// recorded into a graph)
__global__ void __launch_bounds__(256) k_label_clear(double* __restrict__ part, long count) {
  const long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (i < count) part[i] = 0.0;
}

template <class R>
__global__ void __launch_bounds__(256) k_label_partials(const R* __restrict__ phi, const int* __restrict__ labels,
                                                        long n, int nx, int ny, int nl, long chunk,
                                                        double* __restrict__ part) {
  __shared__ double red[4 * kLabFields];
  __shared__ int ired[4];
  const int nb = gridDim.x, b = blockIdx.x;
  const long lo = long(b) * chunk, hi = min(n, lo + chunk);
  // first label of the chunk, and its invalid labels (counted once, with the first label)
  int first = INT_MAX, invalid = 0;
  for (long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const int l = labels[i];
    if (l >= nl) ++invalid;
    else if (l >= 0) first = min(first, l);
  }
  int target = block_min_int(first, ired);
  {
    double v[1] = {double(invalid)};
    const double s = block_sum_n<1>(v, red);
    if (threadIdx.x == 0) part[(long(nl) * kLabFields) * nb + b] = s;   // the invalid-label slot
  }
  while (target != INT_MAX) {
    double v[kLabFields];
#pragma unroll
    for (int f = 0; f < kLabFields; ++f) v[f] = 0.0;
    int next = INT_MAX;
    for (long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      const int l = labels[i];
      if (l == target) {
        const double p = double(phi[i]);
        const double x = double(i % nx), y = double((i / nx) % ny), z = double(i / (long(nx) * ny));
        const bool fin = isfinite(p);
        v[0] += p;
        v[1] += p >= 0.5 ? 1.0 : 0.0;
        v[2] += p * x;
        v[3] += p * y;
        v[4] += p * z;
        v[5] += p * x * x;
        v[6] += p * y * y;
        v[7] += p * z * z;
        v[8] += p * x * y;
        v[9] += p * x * z;
        v[10] += p * y * z;
        v[11] += fin ? 0.0 : 1.0;
      } else if (l > target && l < nl) {
        next = min(next, l);
      }
    }
    const double s = block_sum_n<kLabFields>(v, red);
    if (int(threadIdx.x) < 12) part[(long(target) * kLabFields + threadIdx.x) * nb + b] = s;
    target = block_min_int(next, ired);
  }
}

// out[l]: vclb_obs-shaped record of label l; bad: total of invalid labels
__global__ void __launch_bounds__(256) k_label_fold(const double* __restrict__ part, int nb, int nl, long step,
                                                    LabelObs* __restrict__ out, double* __restrict__ bad) {
  const long j = blockIdx.x * long(blockDim.x) + threadIdx.x;
  const long nf = long(nl) * 12;
  if (j > nf) return;
  const long row = j < nf ? (j / 12) * kLabFields + (j % 12) : long(nl) * kLabFields;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[row * nb + b];
  if (j == nf) {
    *bad = s;
    return;
  }
  const int l = int(j / 12), f = int(j % 12);
  LabelObs& o = out[l];
  if (f == 0) {
    o.sum_phi = s;
    o.step = step;
    o.label = l;
  } else if (f == 1) {
    o.count_half = s;
  } else if (f < 5) {
    o.sum_phi_d[f - 2] = s;
  } else if (f < 11) {
    o.sum_phi_dd[f - 5] = s;
  } else {
    o.nonfinite = s > 0.0 ? 1 : 0;
  }
}

int label_blocks(long n) {
  const long nb = (n + kLabelChunkMin - 1) / kLabelChunkMin;
  return int(nb < kLabelMaxBlocks ? (nb < 1 ? 1 : nb) : kLabelMaxBlocks);
}

size_t label_scratch_bytes(long n, int nlabels) {
  return label_result_offset(n, nlabels) + size_t(nlabels) * sizeof(LabelObs) + sizeof(double);
}

template <class R>
int launch_label_reduce(const R* phi, const int* labels, long n, int nx, int ny, int nlabels, long step,
                        void* scratch, hipStream_t s) {
  const int nb = label_blocks(n);
  const long chunk = (n + nb - 1) / nb;
  double* part = static_cast<double*>(scratch);
  const long count = (long(nlabels) * kLabFields + 1) * nb;
  static_assert(kLabFields == 13, "label_result_offset assumes 13 fields");
  LabelObs* out = reinterpret_cast<LabelObs*>(static_cast<char*>(scratch) + label_result_offset(n, nlabels));
  double* bad = reinterpret_cast<double*>(out + nlabels);
  hipLaunchKernelGGL(k_label_clear, dim3(unsigned((count + 255) / 256)), dim3(256), 0, s, part, count);
  hipLaunchKernelGGL((k_label_partials<R>), dim3(nb), dim3(256), 0, s, phi, labels, n, nx, ny, nlabels, chunk, part);
  const long nf = long(nlabels) * 12 + 1;
  hipLaunchKernelGGL(k_label_fold, dim3(unsigned((nf + 255) / 256)), dim3(256), 0, s, part, nb, nlabels, step, out,
                     bad);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template int launch_label_reduce<double>(const double*, const int*, long, int, int, int, long, void*, hipStream_t);
template int launch_label_reduce<float>(const float*, const int*, long, int, int, int, long, void*, hipStream_t);

// ---------------------------------------------------------------- fixed device scratch
// Scratch of the label reductions for callers that cannot allocate (kStaticScratchBytes per
// device, held until the process ends).  Its host-side name is only a handle: the device
// address comes from hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

int static_scratch(void** ptr) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -3;
  if (dev < 0 || dev >= kMaxDevices) return -1;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -3;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return 0;
}

}  // namespace vclb
