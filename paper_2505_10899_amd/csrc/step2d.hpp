// The 2D fused tile march (device code shared by the single-case and batched steps).
#pragma once
#include <hip/hip_runtime.h>

#include "devcase.hpp"

namespace vclb {

// Source offsets of the nine pulls at one node, 32-bit (cases have < 2^31 nodes).
// Columns: x, x-1, x+1 (periodic); rows: y, y-1, y+1 as row offsets (periodic, or
// flags lo / hi on the first / last row when walls bound y: the populations whose
// source lies behind the wall come from the node's own opposite direction).
struct Col3 { int c, m, p; };
struct Row3 { int c, m, p; bool lo, hi; };

// IX: index type of the accesses; unsigned when every node index times the element size
// fits 32 bits (32-bit byte offsets from uniform bases), else long.  NT: population loads
// with the non-temporal hint.
template <class St, class IX, bool NT = false>
__device__ __forceinline__ void pull9(const typename St::S* const (&src)[9], const float* __restrict__ phis,
                                      const Col3& x, const Row3& y, typename St::R (&v)[9],
                                      typename St::R* ps) {
  using R = typename St::R;
  const int s0 = y.c + x.c;
  int off[9] = {s0, y.c + x.m, y.m + x.c, y.c + x.p, y.p + x.c, y.m + x.m, y.m + x.p, y.p + x.p, y.p + x.m};
  const typename St::S* base[9] = {src[0], src[1], src[2], src[3], src[4], src[5], src[6], src[7], src[8]};
  if (y.lo) {   // c_y = +1 directions 2, 5, 6 bounce back from 4, 7, 8
    off[2] = s0; base[2] = src[4];
    off[5] = s0; base[5] = src[7];
    off[6] = s0; base[6] = src[8];
  }
  if (y.hi) {   // c_y = -1 directions 4, 7, 8 bounce back from 2, 5, 6
    off[4] = s0; base[4] = src[2];
    off[7] = s0; base[7] = src[5];
    off[8] = s0; base[8] = src[6];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) v[i] = NT ? St::load_nt(base[i], IX(off[i])) : St::load(base[i], IX(off[i]));
  if constexpr (St::shifted) {   // every deviation refers to this node's own phis entry
    if (ps) {
      const R own = R(ldg(phis, IX(s0)));
#pragma unroll
      for (int i = 0; i < 9; ++i) ps[i] = own;
    }
  }
}

// Per-thread volume reductions of the fused 2D step: the lane's column is fixed, so
// for each label only sum phi, sum phi dy, sum phi dy^2, #(phi >= 1/2) and the
// non-finite count are accumulated; the x moments follow from the fixed dx at the end.
struct Acc2 {
  double s0[kMaxLabels], s1[kMaxLabels], s2[kMaxLabels];
  int cnt[kMaxLabels], bad[kMaxLabels];
};

// One workgroup owns bx consecutive x columns (one per lane) and marches up ty rows.
// For each row it pulls the next row's g, forms phi and psi into a 4-row LDS ring
// (plus one halo column on each side, computed by lanes 0 and 1), then applies the
// stencils from LDS and updates the current row: every population is read from HBM
// once, except the two halo columns and the two halo rows of the tile.
// UNIT: the case's rates outside the g flux and f stress rows are all 1.  NT: population
// loads and stores with the non-temporal hint (measured faster for the single-case
// strips of 4-byte and 8-byte storage, slower in the batched march).
template <class St, bool COUPLED, class IX, bool UNIT, bool VISC = false, bool NT = false>
__device__ __forceinline__ void step2d_tile(const DevCase<D2Q9, St>& c, long t, int x0, int y0, int y1, bool reduce,
                                            double* __restrict__ part, long part_stride, long part_index,
                                            unsigned char* smem_raw) {
  using L = D2Q9;
  using R = typename St::R;
  using S = typename St::S;
  constexpr int Q = 9;
  const int BX = blockDim.x;
  const int W = BX + 2;
  // phi and psi of a node side by side: one 2-word LDS access per stencil point
  struct alignas(2 * sizeof(R)) PhiPsi {
    R phi, psi;
  };
  PhiPsi* sring = reinterpret_cast<PhiPsi*>(smem_raw);
  const int nx = c.nx, ny = c.ny, ns = int(c.ns);   // ns: entries per plane
  const int lane = threadIdx.x;
  const int xg = x0 + lane;
  const bool active_x = xg < nx;
  const int xw = xg % nx;
  const Col3 col{xw, xw == 0 ? nx - 1 : xw - 1, xw == nx - 1 ? 0 : xw + 1};
  const bool halo_lane = lane < 2;
  const int xh = (lane == 0) ? wrapi(x0 - 1, nx) : (x0 + BX) % nx;
  const Col3 hcol{xh, xh == 0 ? nx - 1 : xh - 1, xh == nx - 1 ? 0 : xh + 1};
  const int hidx = (lane == 0) ? 0 : W - 1;
  const int par = int(t & 1);
  const int dst = par ^ 1;
  const S* gsrc[9];
  const S* fsrc[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    gsrc[i] = c.pop[0][par] + long(i) * ns;
    fsrc[i] = COUPLED ? c.pop[1][par] + long(i) * ns : nullptr;
  }
  const float* phis = c.phis[par];
  const bool wall = c.wall != 0;
  auto row3 = [&](int r) -> Row3 {
    // r in [-1, ny]: rows outside [0, ny) wrap (periodic) or mirror the edge row (walls)
    int yr = r;
    if (r < 0) yr = wall ? 0 : r + ny;
    if (r >= ny) yr = wall ? ny - 1 : r - ny;
    Row3 o;
    o.c = yr * nx;
    o.m = (yr == 0 ? ny - 1 : yr - 1) * nx;
    o.p = (yr == ny - 1 ? 0 : yr + 1) * nx;
    o.lo = wall && yr == 0;
    o.hi = wall && yr == ny - 1;
    return o;
  };
  auto slot = [](int r) -> int { return (r + 4) & 3; };
  // the ring holds, for a ghost row behind a wall, the wetting ghost of the edge row
  auto ghost = [&](int r, R ph) -> R {
    if (wall && r < 0) return wet_ghost<R>(ph, c.np.wet_lo);
    if (wall && r >= ny) return wet_ghost<R>(ph, c.np.wet_hi);
    return ph;
  };
  auto phi_row = [&](int r, R (&g)[Q]) {
    const Row3 rw = row3(r);
    R ps[Q];
    pull9<St, IX, NT>(gsrc, phis, col, rw, g, ps);
    const R ph = ghost(r, phi_of_pulled<L, St>(g, ps, c.np.rest));
    sring[slot(r) * W + lane + 1] = PhiPsi{ph, psi_of<R>(ph, c.np.W4, c.np.xi)};
    if (halo_lane) {
      R gh[Q], hps[Q];
      pull9<St, IX, NT>(gsrc, phis, hcol, rw, gh, hps);
      const R hp = ghost(r, phi_of_pulled<L, St>(gh, hps, c.np.rest));
      sring[slot(r) * W + hidx] = PhiPsi{hp, psi_of<R>(hp, c.np.W4, c.np.xi)};
    }
  };
  // reductions: label displacement along x is fixed for the lane
  double dxl[kMaxLabels];
#pragma unroll
  for (int k = 0; k < kMaxLabels; ++k) dxl[k] = min_image(double(xw) - c.cen[k][0], nx, true);
  Acc2 acc;
#pragma unroll
  for (int k = 0; k < kMaxLabels; ++k) {
    acc.s0[k] = acc.s1[k] = acc.s2[k] = 0.0;
    acc.cnt[k] = acc.bad[k] = 0;
  }
  R gcur[Q], gnext[Q];
  phi_row(y0 - 1, gnext);
  phi_row(y0, gcur);
  for (int y = y0; y < y1; ++y) {
    // this row's f and previous phi u are requested together with the next row's g,
    // so that one memory round trip per row covers both
    const int nn = xw + nx * y;
    R f[Q], J[2];
    if constexpr (COUPLED) pull9<St, IX, NT>(fsrc, phis, col, row3(y), f, nullptr);
    J[0] = ldg(c.J, IX(nn));
    J[1] = ldg(c.J + ns, IX(nn));
    phi_row(y + 1, gnext);
    __syncthreads();
    if (active_x) {
      NodeIn<L, R> in;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int si = slot(y + L::cy[i]) * W + lane + 1 + L::cx[i];
        const PhiPsi v = sring[si];
        in.nphi[i] = v.phi;
        in.npsi[i] = v.psi;
      }
      if constexpr (!COUPLED) {
        R ux, uy;
        vortex_u<R>(c.np.U0, c.np.T, xw, y, nx, ny, t, ux, uy);
        in.u[0] = ux;
        in.u[1] = uy;
      }
      NodeOut<L, R> out;
      node_update_d2q9<R, COUPLED, St::shifted, UNIT, VISC>(c.np, in, gcur, f, J, out);
      R res = R(0);   // rounding of the stored g deviations, taken off the stored phi
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        R d = gcur[i];
        if constexpr (St::shifted)   // relative to the reader's phi (encode_dev)
          d = encode_dev(gcur[i], c.np.rest[i], in.nphi[0],
                         leaves_through_wall<L>(i, y, ny, wall) ? in.nphi[0] : in.nphi[i]);
        if constexpr (NT) St::store_nt(c.pop[0][dst] + long(i) * ns, IX(nn), d);
        else St::store(c.pop[0][dst] + long(i) * ns, IX(nn), d);
        if constexpr (St::fold) res += St::rounding(d);
      }
      if constexpr (COUPLED) {
        if (wall && y == 0) {
#pragma unroll
          for (int i = 0; i < Q; ++i)
            if (L::cy[i] < 0) f[i] += c.np.wb[i] * out.rho;
        }
        if (wall && y == ny - 1) {
#pragma unroll
          for (int i = 0; i < Q; ++i)
            if (L::cy[i] > 0) f[i] += c.np.wt[i] * out.rho;
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          if constexpr (NT) St::store_nt(c.pop[1][dst] + long(i) * ns, IX(nn), f[i]);
          else St::store(c.pop[1][dst] + long(i) * ns, IX(nn), f[i]);
        }
      }
      stg(c.J, IX(nn), J[0]);
      stg(c.J + ns, IX(nn), J[1]);
      if constexpr (St::shifted) stg(c.phis[dst], IX(nn), float(in.nphi[0] - res));
      if (reduce) {
        const double ph = double(in.nphi[0]);
        double dy[kMaxLabels];
#pragma unroll
        for (int k = 0; k < kMaxLabels; ++k) dy[k] = min_image(double(y) - c.cen[k][1], ny, !wall);
        int lab = 0;
        if (c.nl > 1) lab = (dxl[1] * dxl[1] + dy[1] * dy[1] < dxl[0] * dxl[0] + dy[0] * dy[0]) ? 1 : 0;
        const bool fin = isfinite(ph);
#pragma unroll
        for (int k = 0; k < kMaxLabels; ++k) {
          const double w = (k == lab) ? ph : 0.0;
          acc.s0[k] += w;
          acc.s1[k] += w * dy[k];
          acc.s2[k] += w * dy[k] * dy[k];
          acc.cnt[k] += (k == lab && ph >= 0.5) ? 1 : 0;
          acc.bad[k] += (k == lab && !fin) ? 1 : 0;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) gcur[i] = gnext[i];
  }
  Acc full;
#pragma unroll
  for (int k = 0; k < kMaxLabels; ++k) {
    const double dx = dxl[k];
    full.v[k][0] = acc.s0[k];
    full.v[k][1] = double(acc.cnt[k]);
    full.v[k][2] = dx * acc.s0[k];
    full.v[k][3] = acc.s1[k];
    full.v[k][4] = 0.0;
    full.v[k][5] = dx * dx * acc.s0[k];
    full.v[k][6] = acc.s2[k];
    full.v[k][7] = 0.0;
    full.v[k][8] = dx * acc.s1[k];
    full.v[k][9] = 0.0;
    full.v[k][10] = 0.0;
    full.v[k][11] = double(acc.bad[k]);
  }
  if (reduce) write_partials(full, c.nl, part, part_stride, part_index);
}


}  // namespace vclb
