// Device-side description of one case and the helpers every kernel shares:
// pull streaming with bounce-back walls and storage decoding, fixed-order block
// reductions, and the end-of-step "last block" that finishes the volume reductions
// and advances the step counter.
#pragma once
#include <hip/hip_runtime.h>

#include "node.hpp"

namespace vclb {

constexpr int kMaxLabels = 2;
constexpr int kObsFields = 13;   // sum, count, d[3], dd[6], nonfinite, step
constexpr int kHistory = 4096;

template <class L, class St>
struct DevCase {
  using S = typename St::S;
  using R = typename St::R;
  int nx, ny, nz;
  long n;                       // nx * ny * nz
  long ns;                      // entries per plane of the populations and of J: n rounded up
                                // to a multiple of 64, so that every plane starts on a cache line
  int wall;                     // bounce-back walls bound y
  int nl;                       // labels (1..kMaxLabels)
  int unit_rates;               // every rate outside the g flux and f stress rows is 1
  int visc;                     // the phases have different viscosities (per-node tau_f)
  double cen[kMaxLabels][3];    // label centres
  S* pop[2][2];                 // [g = 0, f = 1][buffer]; f is null in vortex mode
  R* J;                         // previous phi u, D planes of ns entries
  float* phis[2];               // FP16S: phi of the node that wrote each buffer entry
  long t;                       // step index of the state this launch reads
  double* part_w;               // this launch's workgroup partials, [label * 12 + field][workgroup]
  const double* part_r;         // partials of an earlier launch still to be summed (pend_nb > 0)
  int pend_nb;                  // workgroups of that launch, 0 if none pending
  double* pend_dest;            // where its sums go: [label][kObsFields]
  long pend_step;               // the step it belongs to
  double* hist;                 // [kHistory][label][kObsFields]
  double* cur;                  // [label][kObsFields] reductions of the current state
  R* tmp_phi;                   // scratch N: phi (plain path and observe)
  R* tmp_psi;                   // scratch N: psi
  int mfix;                     // the global volume correction is on (rate np.mass_fix)
  double* mass;                 // [V_ref, kappa, V, sum delta] of the global correction
  double* mass_part;            // its workgroup partials, [2][workgroup]
  NodeParams<L, R> np;
};

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Displacement wrapped to [-n/2, n/2) along a periodic axis; valid for node and centre
// both in [0, n) (the host moves label centres there), so no division is needed.
__device__ __forceinline__ double min_image(double d, int n, bool periodic) {
  if (!periodic) return d;
  const double h = 0.5 * double(n);
  return d < -h ? d + double(n) : (d >= h ? d - double(n) : d);
}

// Shifted storage keeps each stored g as a deviation from the rest state of the node that
// will read it: d_i = g*_i - r_i phi_r, with phi_r the reader's phi at the writer's time
// level, which the reader finds in its own entry of phis.  A node then decodes all its
// pulls with one load of its own phis entry.  The writer knows phi_r: it is the stencil
// value of phi at x + c_i, or its own phi when c_i leaves through a wall (the value
// bounces back to the writer).  With e*_i = g*_i - r_i phi (the collision's deviation from
// the writer's own rest state) the stored value is e*_i + r_i (phi - phi_r).
template <class R>
__device__ __forceinline__ R encode_dev(R e, R rest_i, R phi_self, R phi_reader) {
  return e + rest_i * (phi_self - phi_reader);
}
// whether direction i of a node in row y leaves through a wall (and comes back to it)
template <class L>
__device__ __forceinline__ bool leaves_through_wall(int i, int y, int ny, bool wall) {
  return wall && ((y == 0 && L::cy[i] < 0) || (y == ny - 1 && L::cy[i] > 0));
}

// Pull the Q populations of one set arriving at node (x, y, z):
// pop_i(x) = post_i(x - c_i), or the node's own opposite post-collision value when
// x - c_i lies behind a wall.  For shifted storage (g set) `out` receives the stored
// deviations d_i and `ps` the phi they are relative to: the node's own phis entry.
template <class L, class St, class Case>
__device__ __forceinline__ void pull(const Case& c, const typename St::S* __restrict__ src,
                                     const float* __restrict__ phis, int x, int y, int z,
                                     typename St::R (&out)[L::Q], typename St::R* ps) {
  using R = typename St::R;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    int xs = x - L::cx[i], ys = y - L::cy[i], zs = z - L::cz[i];
    int pi = i;
    if (L::cy[i] != 0 && (ys < 0 || ys >= c.ny)) {
      if (c.wall) {
        xs = x;
        ys = y;
        zs = z;
        pi = L::opp[i];
      } else {
        ys = wrapi(ys, c.ny);
      }
    }
    if (L::cx[i] != 0) xs = wrapi(xs, c.nx);
    if (L::cz[i] != 0) zs = wrapi(zs, c.nz);
    const long s = xs + long(c.nx) * (ys + long(c.ny) * zs);
    out[i] = St::load(src, long(pi) * c.ns + s);
  }
  if constexpr (St::shifted) {
    if (ps) {
      const R own = R(ldg(phis, x + long(c.nx) * (y + long(c.ny) * z)));
#pragma unroll
      for (int i = 0; i < L::Q; ++i) ps[i] = own;
    }
  }
}

// phi of a stencil ghost row behind a wall, from the edge row's phi_e: the one-sided
// difference across the half-way wall equals the wetting flux (4 / W) cos(theta)
// phi_e (1 - phi_e), c = (4 / W) cos(theta); c = 0 gives the mirror phi_e itself
template <class R>
__device__ __forceinline__ R wet_ghost(R phi_e, R c) {
  return phi_e + c * (phi_e * (R(1) - phi_e));
}

// phi = sum_i g_i (Eq. 35) of a pulled g set.  For shifted storage g_i = d_i + r_i phi_s
// (phi_s: the phi the stored deviations refer to), and on return v holds
// e_i = g_i - r_i phi = d_i + r_i (phi_s - phi): the deviation from this node's own rest
// state, formed without rounding at the magnitude of g.
template <class L, class St>
__device__ __forceinline__ typename St::R phi_of_pulled(typename St::R (&v)[L::Q], const typename St::R (&ps)[L::Q],
                                                        const typename St::R (&rest)[L::Q]) {
  using R = typename St::R;
  R phi = R(0);
  if constexpr (St::shifted) {
#pragma unroll
    for (int i = 0; i < L::Q; ++i) phi += v[i] + rest[i] * ps[i];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) v[i] = v[i] + rest[i] * (ps[i] - phi);
  } else {
#pragma unroll
    for (int i = 0; i < L::Q; ++i) phi += v[i];
  }
  return phi;
}

template <class R>
__device__ __forceinline__ R sum_pops(const R* g, int Q) {
  R s = R(0);
  for (int i = 0; i < Q; ++i) s += g[i];
  return s;
}

// ---------------------------------------------------------------- reductions
// Per-thread accumulators of the volume reductions (FP64), for up to kMaxLabels labels.
struct Acc {
  double v[kMaxLabels][12];
  __device__ void zero() {
#pragma unroll
    for (int k = 0; k < kMaxLabels; ++k)
#pragma unroll
      for (int f = 0; f < 12; ++f) v[k][f] = 0.0;
  }
};

template <class Case>
__device__ __forceinline__ void accumulate(const Case& c, Acc& a, double phi, int x, int y, int z) {
  double d[kMaxLabels][3];
  const bool py = !c.wall;
#pragma unroll
  for (int k = 0; k < kMaxLabels; ++k) {
    d[k][0] = min_image(double(x) - c.cen[k][0], c.nx, true);
    d[k][1] = min_image(double(y) - c.cen[k][1], c.ny, py);
    d[k][2] = min_image(double(z) - c.cen[k][2], c.nz, true);
  }
  int lab = 0;
  if (c.nl > 1) {
    const double r0 = d[0][0] * d[0][0] + d[0][1] * d[0][1] + d[0][2] * d[0][2];
    const double r1 = d[1][0] * d[1][0] + d[1][1] * d[1][1] + d[1][2] * d[1][2];
    lab = (r1 < r0) ? 1 : 0;
  }
  const bool fin = isfinite(phi);
  // branch-free on the label so that the accumulators keep static register indices
#pragma unroll
  for (int k = 0; k < kMaxLabels; ++k) {
    const double w = (k == lab) ? phi : 0.0;
    const double dx = d[k][0], dy = d[k][1], dz = d[k][2];
    a.v[k][0] += w;
    a.v[k][1] += (k == lab && phi >= 0.5) ? 1.0 : 0.0;
    a.v[k][2] += w * dx;
    a.v[k][3] += w * dy;
    a.v[k][4] += w * dz;
    a.v[k][5] += w * dx * dx;
    a.v[k][6] += w * dy * dy;
    a.v[k][7] += w * dz * dz;
    a.v[k][8] += w * dx * dy;
    a.v[k][9] += w * dx * dz;
    a.v[k][10] += w * dy * dz;
    a.v[k][11] += (k == lab && !fin) ? 1.0 : 0.0;
  }
}

// Sum nf <= 24 values over the workgroup in a fixed order (deterministic): butterfly
// within each wave, then wave results in wave order.  Thread f < nf returns field f.
template <int NF>
__device__ __forceinline__ double block_sum_fields(const double (&v)[NF], int nf, double* red) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    if (f < nf) {
      double s = v[f];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0) red[wave * NF + f] = s;
    }
  }
  __syncthreads();
  double out = 0.0;
  if (int(threadIdx.x) < nf)
    for (int w = 0; w < nw; ++w) out += red[w * NF + threadIdx.x];
  return out;
}

// End of a step kernel: this workgroup's partial volume reductions, written to its own
// slot; k_finalize sums the slots in workgroup order after the kernel has finished
// (no device-scope fence inside the step: on gfx950 it would write back and invalidate
// the XCD's whole L2, which the neighbouring tiles are still reading).
// red: LDS scratch of at least (waves of the workgroup) x 24 doubles
__device__ __forceinline__ void write_partials(const Acc& a, int nl, double* part, long stride, long index,
                                               double* red) {
  constexpr int NF = kMaxLabels * 12;
  const int nf = nl * 12;
  double v[NF];
#pragma unroll
  for (int k = 0; k < kMaxLabels; ++k)
#pragma unroll
    for (int f = 0; f < 12; ++f) v[k * 12 + f] = a.v[k][f];
  const double s = block_sum_fields<NF>(v, nf, red);
  // field-major [field][workgroup]: the second pass reads each field coalesced
  if (int(threadIdx.x) < nf) part[long(threadIdx.x) * stride + index] = s;
}
__device__ __forceinline__ void write_partials(const Acc& a, int nl, double* part, long stride, long index) {
  __shared__ double red[16 * kMaxLabels * 12];
  write_partials(a, nl, part, stride, index, red);
}

template <class Case>
__device__ __forceinline__ void finish_block(const Case& c, const Acc& a, bool reduce) {
  if (reduce) write_partials(a, c.nl, c.part_w, gridDim.x, blockIdx.x);
}
template <class Case>
__device__ __forceinline__ void finish_block(const Case& c, const Acc& a, bool reduce, double* red) {
  if (reduce) write_partials(a, c.nl, c.part_w, gridDim.x, blockIdx.x, red);
}

// store one node's post-collision state (with the moving-wall term on f for the
// directions that leave through a wall, read back by the bounce-back pull)
// nphi: phi at x + c_i (the readers of the shifted g, see encode_dev)
template <class L, class St, bool COUPLED>
__device__ __forceinline__ void store_node(const DevCase<L, St>& c, int par, long n, int y,
                                           const typename St::R (&nphi)[L::Q], typename St::R rho,
                                           const typename St::R (&g)[L::Q], typename St::R (&f)[L::Q],
                                           const typename St::R (&J)[L::D]) {
  using R = typename St::R;
  const int dst = par ^ 1;
  const R phi = nphi[0];
  R res = R(0);   // rounding of the stored g deviations, taken off the stored phi
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    R d = g[i];
    if constexpr (St::shifted)
      d = encode_dev(g[i], c.np.rest[i], phi, leaves_through_wall<L>(i, y, c.ny, c.wall != 0) ? phi : nphi[i]);
    St::store(c.pop[0][dst], long(i) * c.ns + n, d);
    if constexpr (St::fold) res += St::rounding(d);
  }
  if constexpr (COUPLED) {
    if (c.wall) {
      if (y == 0) {
#pragma unroll
        for (int i = 0; i < L::Q; ++i)
          if (L::cy[i] < 0) f[i] += c.np.wb[i] * rho;
      }
      if (y == c.ny - 1) {
#pragma unroll
        for (int i = 0; i < L::Q; ++i)
          if (L::cy[i] > 0) f[i] += c.np.wt[i] * rho;
      }
    }
#pragma unroll
    for (int i = 0; i < L::Q; ++i) St::store(c.pop[1][dst], long(i) * c.ns + n, f[i]);
  }
#pragma unroll
  for (int d = 0; d < L::D; ++d) stg(c.J, d * c.ns + n, J[d]);
  if constexpr (St::shifted) stg(c.phis[dst], n, float(phi - res));
}

template <class L, class St, bool COUPLED>
__device__ __forceinline__ void prescribed(const DevCase<L, St>& c, int x, int y, long t,
                                           NodeIn<L, typename St::R>& in) {
  if constexpr (!COUPLED) {
    typename St::R ux, uy;
    vortex_u<typename St::R>(c.np.U0, c.np.T, x, y, c.nx, c.ny, t, ux, uy);
    in.u[0] = ux;
    in.u[1] = uy;
  }
}

// Second pass of the volume reductions: sum the pending partials of an earlier launch
// in a fixed order (deterministic) into c.pend_dest.  Run by one whole workgroup.
template <class Case>
__device__ __forceinline__ void fold_pending(const Case& c, double* red) {
  constexpr int NF = kMaxLabels * 12;
  const int nf = c.nl * 12;
  const int nb = c.pend_nb;
  double v[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) v[f] = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
#pragma unroll
    for (int f = 0; f < NF; ++f)
      if (f < nf) v[f] += c.part_r[long(f) * nb + b];
  }
  const double s = block_sum_fields<NF>(v, nf, red);
  if (int(threadIdx.x) < nf) {
    const int k = threadIdx.x / 12, f = threadIdx.x % 12;
    c.pend_dest[k * kObsFields + f] = s;
    if (f == 0) c.pend_dest[k * kObsFields + 12] = double(c.pend_step);
  }
  __syncthreads();
}
template <class Case>
__device__ __forceinline__ void fold_pending(const Case& c) {
  __shared__ double red[16 * kMaxLabels * 12];
  fold_pending(c, red);
}

// XCD-aware tile order: workgroups are dispatched round-robin over the 8 XCDs, so
// block b runs on XCD b % 8.  Give each XCD a contiguous range of tiles so that
// neighbouring tiles (which re-read each other's halo rows) share one L2.
__device__ __forceinline__ int xcd_tile(int b, int B) {
  const int q = B >> 3, r = B & 7, x = b & 7, i = b >> 3;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

}  // namespace vclb
