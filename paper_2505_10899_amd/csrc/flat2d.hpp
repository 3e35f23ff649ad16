// One work item of the batched D2Q9 step: a band of rows [y0, y1) of one case, marched
// in the case's stored (row-major) order.
//
// Lanes walk consecutive stored nodes, so a row of any width keeps every lane busy and
// successive rows run back to back.  Chunks of B lanes start on multiples of 64 nodes;
// with every plane starting on a cache line (planes of ns entries, a multiple of 64),
// each wave then stores whole cache lines.  The band's window is the rows y0 - 1 .. y1 in
// extended stored order e = r nx + x (r in [y0 - 1, y1]); its first and last rows are
// halo rows, pulled for phi and not updated.  Row r = -1 or ny holds the periodic
// neighbour row or, behind a wall, the wetting ghost of the edge row (the edge row itself
// for a neutral wall).
//
// phi and psi go into an LDS ring of `cap` entries (a power of two) at the padded
// position v = (r + 1) P + x + 1, P = nx + 2, so that the stencil neighbours of v are
// v + cx + P cy.  Column -1 of a row holds the periodic image of its column nx - 1,
// formed with a second pull in the iteration whose chunk holds the row's first node, so
// that it is ready as early as that node (by the chunk's first threads, one row each, or
// by the lane of column 0).  A neighbour past column nx - 1 is read from column 0 of its
// row.
//
// Iteration i pulls the populations of chunk i, forms phi and psi into the ring, and
// keeps the pulled populations in a register FIFO of DL + 1 slots; it then updates chunk
// i - DL from the FIFO, in the same lanes that pulled it, once the ring holds every
// stencil input of that chunk.  Node e needs the ring up to stored node e + nx + 1, so
// DL B >= nx + 1.  Each population is read from memory once, as in the row march.  One
// barrier per iteration suffices when the ring spans the reads of iteration i together
// with the writes of iteration i + 1 (flat_ring_cap).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "devcase.hpp"
#include "launch.hpp"
#include "step2d.hpp"

namespace vclb {

// Pull of the 9 populations arriving at node (x, y) of an nx x ny case from the stored
// direction planes src[i] (uniform over the wave): periodic wrap and, behind a wall, the
// node's own opposite population.  Every offset is a non-negative 32-bit index from a
// uniform base, so each address is one shift-add with no sign extension: directions
// 2, 5, 6 index from their own planes (a bounce from the bottom wall reads plane
// opp(i) = i + 2 at s0 + 2n), directions 4, 7, 8 from the plane of opp(i) = i - 2 (their
// own entry lies 2 ns further on; a bounce from the top wall reads s0 there).  ps
// (shifted storage): the phi the stored deviations refer to, this node's own phis entry.
template <class St>
__device__ __forceinline__ void pull9_flat(const typename St::S* const (&src)[9], const float* __restrict__ phis,
                                           int x, int y, int nx, int ny, int ns, bool wall,
                                           typename St::R (&v)[9], typename St::R* ps) {
  using R = typename St::R;
  const unsigned s0 = unsigned(x + nx * y);
  const int xm = x == 0 ? nx - 1 : -1;                 // to column x - 1 (wrapped)
  const int xp = x == nx - 1 ? 1 - nx : 1;             // to column x + 1
  const int ym = y == 0 ? (ny - 1) * nx : -nx;         // to row y - 1 (periodic)
  const int yp = y == ny - 1 ? (1 - ny) * nx : nx;     // to row y + 1
  // writer of direction i sits at (x - cx_i, y - cy_i)
  unsigned nd[9] = {s0, s0 + xm, s0 + ym, s0 + xp, s0 + yp, s0 + xm + ym, s0 + xp + ym, s0 + xp + yp, s0 + xm + yp};
  const unsigned n2 = 2u * unsigned(ns);
  unsigned off[9] = {nd[0], nd[1], nd[2], nd[3], nd[4] + n2, nd[5], nd[6], nd[7] + n2, nd[8] + n2};
  if (wall && y == 0) {        // c_y = +1 directions 2, 5, 6 come back from 4, 7, 8 of this node
    nd[2] = nd[5] = nd[6] = s0;
    off[2] = off[5] = off[6] = s0 + n2;
  }
  if (wall && y == ny - 1) {   // c_y = -1 directions 4, 7, 8 come back from 2, 5, 6
    nd[4] = nd[7] = nd[8] = s0;
    off[4] = off[7] = off[8] = s0;
  }
  const typename St::S* base[9] = {src[0], src[1], src[2], src[3], src[2], src[5], src[6], src[5], src[6]};
#pragma unroll
  for (int i = 0; i < 9; ++i) v[i] = St::load(base[i], off[i]);
  if constexpr (St::shifted) {   // every deviation refers to this node's own phis entry
    if (ps) {
      const R own = R(ldg(phis, s0));
#pragma unroll
      for (int i = 0; i < 9; ++i) ps[i] = own;
    }
  }
}

// UNIT: the case's rates outside the g flux and f stress rows are all 1; VISC: the f
// stress rows relax at the node's own rate (unequal viscosities, Eq. 27)
template <class St, int DL, bool UNIT, bool VISC = false>
__device__ __forceinline__ void step2d_flat(const DevCase<D2Q9, St>& c, long t, int y0, int y1, bool reduce,
                                            int cap, double* __restrict__ part, long part_stride, long part_index,
                                            unsigned char* smem_raw) {
  using L = D2Q9;
  using R = typename St::R;
  using S = typename St::S;
  constexpr int Q = 9;
  constexpr int DEPTH = DL + 1;
  static_assert((DEPTH & (DEPTH - 1)) == 0, "FIFO depth must be a power of two");
  // Column -1 of a row (the periodic image of its column nx - 1) needs a second pull in
  // the iteration whose chunk holds the row's first node.  COMPACT_COL: the chunk's first
  // threads take one such row each, so that the fewest waves run these pulls with their
  // lanes busy (FP16S and FP64, 4% and 3% faster); else the lane of column 0 pulls it
  // (FP32, memory-bound: 1% faster than either compact or one row per wave)
  constexpr bool COMPACT_COL = !std::is_same<St, StoreF32>::value;
  // population stores (whole cache lines) with the non-temporal hint for 4-byte arithmetic
  // (FP32 and FP16S storage: measured 2% faster there, and no faster in FP64); the pulls,
  // which straddle cache lines, stay plain (with the hint on them too the step was 3-5%
  // slower than with no hint at all)
  constexpr bool NT_STORE = sizeof(R) == 4;
  const int B = blockDim.x;
  const int lane = threadIdx.x;
  const int nx = c.nx, ny = c.ny, ns = int(c.ns);
  const int P = nx + 2;
  const int mask = cap - 1;
  // phi and psi of a node side by side: one 2-word LDS access per stencil point
  struct alignas(2 * sizeof(R)) PhiPsi {
    R phi, psi;
  };
  PhiPsi* sring = reinterpret_cast<PhiPsi*>(smem_raw);
  const int par = int(t & 1);
  const int dst = par ^ 1;
  const S* gsrc[9];
  const S* fsrc[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    gsrc[i] = c.pop[0][par] + long(i) * ns;
    fsrc[i] = c.pop[1][par] + long(i) * ns;
  }
  const float* phis = c.phis[par];
  const bool wall = c.wall != 0;
  // the window's extended stored range [e_begin, e_end) and the first chunk's start, the
  // multiple of 64 at or below e_begin
  const int e_begin = (y0 - 1) * nx, e_end = (y1 + 1) * nx;
  const int e_first = e_begin - (((e_begin % 64) + 64) % 64);
  const int nchunk = (e_end - e_first + B - 1) / B;
  const int niter = nchunk + DL;
  R e[DEPTH][Q];          // pulled populations of the last DEPTH chunks (static indices only)
  int ex[DEPTH], ey[DEPTH];   // their nodes' column and row (row -2: the lane has no node)
#pragma unroll
  for (int k = 0; k < DEPTH; ++k) {
    ex[k] = 0;
    ey[k] = -2;
  }
  double a0 = 0.0, ax = 0.0, ay = 0.0, axx = 0.0, ayy = 0.0, axy = 0.0;   // one label per case
  int acnt = 0, abad = 0;
  // row and column of stored node e (floor division: e < 0 lies in the rows above row 0)
  auto node_of = [&](int e, int& r, int& x) {
    r = e / nx;
    x = e - r * nx;
    if (x < 0) {
      x += nx;
      --r;
    }
  };
  // this lane's front node, and the first and last nodes of the front chunk (the same for
  // every lane), each advanced by B nodes per iteration
  int rf, xf, ra, xa, rb, xb;
  node_of(e_first + lane, rf, xf);
  node_of(e_first, ra, xa);
  node_of(e_first + B - 1, rb, xb);
  const int dq = B / nx, dr = B - dq * nx;
  auto advance = [&](int& r, int& x) {
    x += dr;
    r += dq;
    if (x >= nx) {
      x -= nx;
      ++r;
    }
  };
  // phi and psi of a pulled node of ring row r (stored row yr) into ring position v
  auto form = [&](R (&g)[Q], const R (&ps)[Q], int r, int v) {
    R ph = phi_of_pulled<L, St>(g, ps, c.np.rest);
    if (wall && r < 0) ph = wet_ghost<R>(ph, c.np.wet_lo);          // ghost row y = -1
    else if (wall && r >= ny) ph = wet_ghost<R>(ph, c.np.wet_hi);   // ghost row y = ny
    sring[v & mask] = PhiPsi{ph, psi_of<R>(ph, c.np.W4, c.np.xi)};
  };

  auto iteration = [&](int i, auto front_slot) {
    constexpr int SF = decltype(front_slot)::value;
    constexpr int SU = (SF + DEPTH - DL) % DEPTH;
    // the chunk updated in this iteration (pulled DL iterations ago by this same lane):
    // its f and previous phi u are requested first, so that they are in flight while the
    // front's phi is formed
    const int x = ex[SU], y = ey[SU];
    const bool act = i >= DL && y >= y0 && y < y1;
    R f[Q], J[2];
    const unsigned nn = unsigned(x + nx * y);
    if (act) {
      pull9_flat<St>(fsrc, phis, x, y, nx, ny, ns, wall, f, nullptr);
      J[0] = ldg(c.J, nn);
      J[1] = ldg(c.J + ns, nn);
    }
    // front: chunk i
    {
      const int ef = e_first + i * B + lane;
      const bool valid = i < nchunk && ef >= e_begin && ef < e_end;
      ex[SF] = xf;
      ey[SF] = valid ? rf : -2;
      if (valid) {
        int yr = rf;
        if (yr < 0) yr = wall ? 0 : ny - 1;
        else if (yr >= ny) yr = wall ? ny - 1 : 0;
        const int vf = (rf + 1) * P + xf + 1;
        R ps[Q];
        pull9_flat<St>(gsrc, phis, xf, yr, nx, ny, ns, wall, e[SF], ps);
        form(e[SF], ps, rf, vf);
        if (!COMPACT_COL && xf == 0) {   // column -1 of this row, in the lane of column 0
          R gh[Q], hps[Q];
          pull9_flat<St>(gsrc, phis, nx - 1, yr, nx, ny, ns, wall, gh, hps);
          form(gh, hps, rf, vf - 1);
        }
      }
      if constexpr (COMPACT_COL) {
        // column -1 of every window row that starts in this chunk, one row per thread
        // from thread 0
        const int rh = ra + (xa != 0 ? 1 : 0) + lane;
        if (i < nchunk && rh <= rb && rh >= y0 - 1 && rh <= y1) {
          int yh = rh;
          if (yh < 0) yh = wall ? 0 : ny - 1;
          else if (yh >= ny) yh = wall ? ny - 1 : 0;
          R gh[Q], hps[Q];
          pull9_flat<St>(gsrc, phis, nx - 1, yh, nx, ny, ns, wall, gh, hps);
          form(gh, hps, rh, (rh + 1) * P);
        }
        advance(ra, xa);
        advance(rb, xb);
      }
      advance(rf, xf);
    }
    __syncthreads();
    if (act) {
      const int vu = (y + 1) * P + x + 1;
      NodeIn<L, R> in;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        int s = vu + L::cx[j] + P * L::cy[j];
        if (L::cx[j] > 0 && x == nx - 1) s -= nx;   // past the last column: column 0
        const PhiPsi v = sring[s & mask];
        in.nphi[j] = v.phi;
        in.npsi[j] = v.psi;
      }
      NodeOut<L, R> out;
      node_update_d2q9<R, true, St::shifted, UNIT, VISC>(c.np, in, e[SU], f, J, out);
      R res = R(0);   // rounding of the stored g deviations, taken off the stored phi
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        R d = e[SU][j];
        if constexpr (St::shifted)   // relative to the reader's phi (encode_dev)
          d = encode_dev(e[SU][j], c.np.rest[j], in.nphi[0],
                         leaves_through_wall<L>(j, y, ny, wall) ? in.nphi[0] : in.nphi[j]);
        if constexpr (NT_STORE) St::store_nt(c.pop[0][dst] + long(j) * ns, nn, d);
        else St::store(c.pop[0][dst] + long(j) * ns, nn, d);
        if constexpr (St::fold) res += St::rounding(d);
      }
      if (wall && y == 0) {
#pragma unroll
        for (int j = 0; j < Q; ++j)
          if (L::cy[j] < 0) f[j] += c.np.wb[j] * out.rho;
      }
      if (wall && y == ny - 1) {
#pragma unroll
        for (int j = 0; j < Q; ++j)
          if (L::cy[j] > 0) f[j] += c.np.wt[j] * out.rho;
      }
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        if constexpr (NT_STORE) St::store_nt(c.pop[1][dst] + long(j) * ns, nn, f[j]);
        else St::store(c.pop[1][dst] + long(j) * ns, nn, f[j]);
      }
      stg(c.J, nn, J[0]);
      stg(c.J + ns, nn, J[1]);
      if constexpr (St::shifted) stg(c.phis[dst], nn, float(in.nphi[0] - res));
      if (reduce) {
        const double ph = double(in.nphi[0]);
        const double dx = min_image(double(x) - c.cen[0][0], nx, true);
        const double dy = min_image(double(y) - c.cen[0][1], ny, !wall);
        a0 += ph;
        ax += ph * dx;
        ay += ph * dy;
        axx += ph * dx * dx;
        ayy += ph * dy * dy;
        axy += ph * dx * dy;
        acnt += ph >= 0.5 ? 1 : 0;
        abad += isfinite(ph) ? 0 : 1;
      }
    }
  };
  // unrolled by the FIFO depth so that every slot index is a compile-time constant;
  // i is uniform over the workgroup, so the barriers inside stay uniform
  for (int i0 = 0; i0 < niter; i0 += DEPTH) {
    iteration(i0, std::integral_constant<int, 0>{});
    if (i0 + 1 < niter) iteration(i0 + 1, std::integral_constant<int, 1 % DEPTH>{});
    if constexpr (DEPTH > 2) {
      if (i0 + 2 < niter) iteration(i0 + 2, std::integral_constant<int, 2 % DEPTH>{});
      if (i0 + 3 < niter) iteration(i0 + 3, std::integral_constant<int, 3 % DEPTH>{});
    }
  }
  if (reduce) {
    Acc full;
    full.zero();
    full.v[0][0] = a0;
    full.v[0][1] = double(acnt);
    full.v[0][2] = ax;
    full.v[0][3] = ay;
    full.v[0][5] = axx;
    full.v[0][6] = ayy;
    full.v[0][8] = axy;
    full.v[0][11] = double(abad);
    write_partials(full, 1, part, part_stride, part_index);
  }
}

}  // namespace vclb
