// Fused D3Q19 step for gfx950 (3D workloads: x and z periodic, y periodic or bounded by
// half-way walls).
//
// A workgroup of bx * by threads owns a bx x by column tile of the (x, y) plane and
// marches over tz planes of z.  For each plane it pulls the next plane's g, forms
// phi and psi into a 4-plane LDS ring padded by one halo node on every side (the
// ring of halo nodes is shared out evenly over the waves), then applies the
// 18-neighbour stencils from LDS and updates the current plane with the moment-space
// node update.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "devcase.hpp"
#include "launch.hpp"

namespace vclb {

// Node offsets of one 3D pull: the writer of direction i sits at x - c_i, reached from
// the node's own index s0 by one of xm / xp, ym / yp, zm / zp per axis (the wrapped steps
// to x - 1 / x + 1 and so on; x and z are periodic).  With walls bounding y, lo / hi mark
// the first / last row, where the directions coming from behind the wall are the node's
// own opposite populations (half-way bounce-back).
struct Nbr3 {
  int s0, xm, xp, ym, yp, zm, zp;
  bool lo, hi;
};

__device__ __forceinline__ Nbr3 nbr3(int x, int y, int z, int nx, int ny, int nz, int nxy, bool wall) {
  Nbr3 o;
  o.s0 = x + nx * y + nxy * z;
  o.lo = wall && y == 0;
  o.hi = wall && y == ny - 1;
  o.xm = x == 0 ? nx - 1 : -1;
  o.xp = x == nx - 1 ? 1 - nx : 1;
  o.ym = y == 0 ? (ny - 1) * nx : -nx;
  o.yp = y == ny - 1 ? (1 - ny) * nx : nx;
  o.zm = z == 0 ? (nz - 1) * nxy : -nxy;
  o.zp = z == nz - 1 ? (1 - nz) * nxy : nxy;
  return o;
}

// Offset of the writer of direction i from the uniform base of its plane: the node's own
// index s0 moved by one of xm / xp, ym / yp, zm / zp per axis.
template <int i>
__device__ __forceinline__ int pull_index(const Nbr3& o) {
  using L = D3Q19;
  int s = o.s0;
  if constexpr (L::cx[i] > 0) s += o.xm;
  if constexpr (L::cx[i] < 0) s += o.xp;
  if constexpr (L::cy[i] > 0) s += o.ym;
  if constexpr (L::cy[i] < 0) s += o.yp;
  if constexpr (L::cz[i] > 0) s += o.zm;
  if constexpr (L::cz[i] < 0) s += o.zp;
  return s;
}

// Buffer-resource access, for periodic cases whose arrays each span less than 2 GiB: one
// resource per array (uniform), the plane's byte offset as the scalar offset (the same
// scalar for every array of equal plane stride) and the node's byte offset as the vector
// offset, so that an access needs one 32-bit offset per lane and no 64-bit address.
struct Bufs3 {
  __amdgpu_buffer_rsrc_t g, f, phis, gd, fd, phisd, J;   // read: g, f, phis; written: gd, fd, phisd; J both
  int pb;   // bytes per population plane (ns entries of the stored type)
  int jb;   // bytes per plane of J
};
// fourth word of a raw (unswizzled, unstrided) buffer resource on gfx9-family GPUs:
// 32-bit data format, every destination selector zero
constexpr int kRawBufferWord3 = 0x00020000;

template <class T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const T* p, long entries) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p), short(0), int(entries * long(sizeof(T))),
                                           kRawBufferWord3);
}
template <class T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff) {
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <class T>
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff, T v) {
  if constexpr (sizeof(T) == 4) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
  else {
    using U2 = unsigned __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, voff, soff, 0);
  }
}
// a population in the storage's form: decoded to / encoded from the arithmetic type
template <class St>
__device__ __forceinline__ typename St::R buf_load_pop(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff) {
  if constexpr (sizeof(typename St::S) == 2)
    return __half2float(__ushort_as_half(__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0)));
  else return buf_ld<typename St::S>(r, voff, soff);
}
template <class St>
__device__ __forceinline__ void buf_store_pop(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff,
                                              typename St::R v) {
  if constexpr (sizeof(typename St::S) == 2)
    __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(__float2half_rn(v)), r, voff, soff, 0);
  else buf_st<typename St::S>(r, voff, soff, typename St::S(v));
}

// The 19 pulls at one node: 32-bit node offsets from the uniform base of each
// direction's plane (planes of ns entries; the case has fewer than 2^31 nodes), accessed with index type IX
// (unsigned: 32-bit byte offsets, when n times the element size fits them).  ps (shifted
// storage): the phi the stored deviations refer to, this node's own phis entry.
// BUF: through the buffer resources rs (the set) and rph (phis), planes pb bytes apart;
// periodic cases only (no pull is redirected at a wall).
template <class St, class IX, bool BUF>
__device__ __forceinline__ void pull19(const typename St::S* __restrict__ src, const float* __restrict__ phis,
                                       long ns, __amdgpu_buffer_rsrc_t rs, __amdgpu_buffer_rsrc_t rph, int pb,
                                       const Nbr3& o, typename St::R (&out)[19], typename St::R* ps) {
  using L = D3Q19;
  using R = typename St::R;
  if constexpr (BUF) {
    static_for<0, L::Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      out[i] = buf_load_pop<St>(rs, unsigned(pull_index<i>(o)) * unsigned(sizeof(typename St::S)), i * pb);
    });
    if constexpr (St::shifted) {
      if (ps) {
        const R own = R(buf_ld<float>(rph, unsigned(o.s0) * 4u, 0));
#pragma unroll
        for (int i = 0; i < L::Q; ++i) ps[i] = own;
      }
    }
    return;
  }
  static_for<0, L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    int s = pull_index<i>(o);
    const typename St::S* base = src + i * ns;
    if constexpr (L::cy[i] > 0) {   // from the row below: behind the bottom wall at y = 0
      if (o.lo) {
        s = o.s0;
        base = src + L::opp[i] * ns;
      }
    }
    if constexpr (L::cy[i] < 0) {   // from the row above: behind the top wall at y = ny - 1
      if (o.hi) {
        s = o.s0;
        base = src + L::opp[i] * ns;
      }
    }
    out[i] = St::load(base, IX(s));
  });
  if constexpr (St::shifted) {   // every deviation refers to this node's own phis entry
    if (ps) {
      const R own = R(ldg(phis, IX(o.s0)));
#pragma unroll
      for (int i = 0; i < L::Q; ++i) ps[i] = own;
    }
  }
}

// Workgroups per CU the register budget is sized for (256 lanes each): with 4-byte
// arithmetic the next plane's pulled g waits in LDS instead of registers, so three fit
// (at most 168 VGPRs); FP64 keeps it in registers at two.
template <class St>
constexpr bool stage3d() {
  return sizeof(typename St::R) == 4;
}
// Sections of up to BS lanes: 256, or 768 with 4-byte arithmetic (one workgroup putting
// 3 waves on each SIMD, the same register budget as three of 256).
template <class St, int BS>
constexpr int step3d_min_blocks() {
  return BS > 256 ? 1 : (stage3d<St>() ? 3 : 2);
}
// Periodic cases get kernels of their own, with no wall tests in the pulls, in FP16S and
// FP64: 6% faster on the 96 x 96 x 384 column (fewer registers, no spills).  In FP32 the
// kernel that tests c.wall was 0.6% faster on the same column, so it serves every case.
template <class St>
constexpr bool periodic3d_kernel() {
  return !std::is_same<St, StoreF32>::value;
}
// Periodic kernels with buffer-resource access (32-bit offsets, scalar plane offsets)
template <class St>
constexpr bool buf3d_kernel() {
  return std::is_same<St, StoreF16S>::value;
}
// every array of the case spans less than 2 GiB (the byte offsets and sizes of a buffer
// resource are 32-bit)
template <class St>
bool buf3d_fits(const DevCase<D3Q19, St>& c) {
  const long lim = (1L << 31) - 1;
  return long(D3Q19::Q) * c.ns * long(sizeof(typename St::S)) <= lim &&
         long(D3Q19::D) * c.ns * long(sizeof(typename St::R)) <= lim && c.ns * 4 <= lim;
}

// phi and psi of a node side by side: one 2-word LDS access per stencil point
template <class R>
struct alignas(2 * sizeof(R)) PhiPsi3 {
  R phi, psi;
};

// slot of plane z in the 4-plane ring (z >= -1)
__device__ __forceinline__ int ring_slot3d(int z) { return (z + 4) & 3; }

// Update of the node (xw, yw, z) held by lane (tx, ty) of its section: g (pulled, as
// deviations from the node's own rest state for shifted storage), f and the previous
// phi u in registers, phi and psi of the 18 neighbours in the ring of PS = PW x (BY + 2)
// nodes per plane.  Stores the post-collision state and accumulates the reductions.
template <class St, int NL, bool UNIT, bool VISC, bool WALL, class IX, bool BUF>
__device__ __forceinline__ void update_node3d(const DevCase<D3Q19, St>& c, const Bufs3& bf,
                                              const PhiPsi3<typename St::R>* sring,
                                              int PS, int PW, int tx, int ty, int xw, int yw, int z, int nn, int par,
                                              typename St::R (&gcur)[19], typename St::R (&f)[19],
                                              typename St::R (&J)[3], bool reduce, double (&s0)[NL], double (&s1)[NL],
                                              double (&s2)[NL], int (&cnt)[NL], int (&bad)[NL]) {
  using L = D3Q19;
  using R = typename St::R;
  constexpr int Q = L::Q;
  // stencils of Eqs. 39-40 accumulated straight from the LDS ring
  StencilOut<L, R> st;
  const int s0i = ring_slot3d(z) * PS + (ty + 1) * PW + tx + 1;
  st.phi = sring[s0i].phi;
  st.lap = R(0);
#pragma unroll
  for (int d = 0; d < 3; ++d) st.gphi[d] = st.gpsi[d] = R(0);
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const int s = ring_slot3d(z + L::cz[i]) * PS + (ty + 1 + L::cy[i]) * PW + tx + 1 + L::cx[i];
    const PhiPsi3<R> v = sring[s];
    const R ph = v.phi, ps = v.psi;
    st.lap += R(6.0 * L::w[i]) * (ph - st.phi);
    if (L::cx[i] != 0) { st.gphi[0] += R(3.0 * L::w[i] * L::cx[i]) * ph; st.gpsi[0] += R(3.0 * L::w[i] * L::cx[i]) * ps; }
    if (L::cy[i] != 0) { st.gphi[1] += R(3.0 * L::w[i] * L::cy[i]) * ph; st.gpsi[1] += R(3.0 * L::w[i] * L::cy[i]) * ps; }
    if (L::cz[i] != 0) { st.gphi[2] += R(3.0 * L::w[i] * L::cz[i]) * ph; st.gpsi[2] += R(3.0 * L::w[i] * L::cz[i]) * ps; }
  }
  NodeOut<L, R> out;
  node_update_mom_s<L, R, true, St::shifted, UNIT, VISC>(c.np, st, gcur, f, J, out);
  const int dst = par ^ 1;
  const bool wall = WALL && c.wall != 0;
  R res = R(0);   // rounding of the stored g deviations, taken off the stored phi
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    R d = gcur[i];
    if constexpr (St::shifted) {   // relative to the reader's phi, read back from the ring
      const int sr = ring_slot3d(z + L::cz[i]) * PS + (ty + 1 + L::cy[i]) * PW + tx + 1 + L::cx[i];
      d = encode_dev(gcur[i], c.np.rest[i], st.phi,
                     leaves_through_wall<L>(i, yw, c.ny, wall) ? st.phi : sring[sr].phi);
    }
    if constexpr (BUF) buf_store_pop<St>(bf.gd, unsigned(nn) * unsigned(sizeof(typename St::S)), i * bf.pb, d);
    else St::store(c.pop[0][dst] + i * c.ns, IX(nn), d);
    if constexpr (St::fold) res += St::rounding(d);
  }
  if (wall && yw == 0) {   // moving-wall term of the populations the bottom wall returns
#pragma unroll
    for (int i = 0; i < Q; ++i)
      if (L::cy[i] < 0) f[i] += c.np.wb[i] * out.rho;
  }
  if (wall && yw == c.ny - 1) {
#pragma unroll
    for (int i = 0; i < Q; ++i)
      if (L::cy[i] > 0) f[i] += c.np.wt[i] * out.rho;
  }
  if constexpr (BUF) {
    const unsigned vo = unsigned(nn) * unsigned(sizeof(typename St::S));
#pragma unroll
    for (int i = 0; i < Q; ++i) buf_store_pop<St>(bf.fd, vo, i * bf.pb, f[i]);
#pragma unroll
    for (int d = 0; d < L::D; ++d) buf_st<R>(bf.J, unsigned(nn) * unsigned(sizeof(R)), d * bf.jb, J[d]);
    if constexpr (St::shifted) buf_st<float>(bf.phisd, unsigned(nn) * 4u, 0, float(st.phi - res));
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) St::store(c.pop[1][dst] + i * c.ns, IX(nn), f[i]);
#pragma unroll
    for (int d = 0; d < L::D; ++d) stg(c.J + d * c.ns, IX(nn), J[d]);
    if constexpr (St::shifted) stg(c.phis[dst], IX(nn), float(st.phi - res));
  }
  if (reduce) {
    const double ph = double(st.phi);
    int lab = 0;
    if constexpr (NL > 1) {
      double r[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const double dx = min_image(double(xw) - c.cen[k][0], c.nx, true);
        const double dy = min_image(double(yw) - c.cen[k][1], c.ny, !wall);
        const double dz = min_image(double(z) - c.cen[k][2], c.nz, true);
        r[k] = dx * dx + dy * dy + dz * dz;
      }
      lab = (r[1] < r[0]) ? 1 : 0;
    }
    const bool fin = isfinite(ph);
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const double dz = min_image(double(z) - c.cen[k][2], c.nz, true);
      const double w = (k == lab) ? ph : 0.0;
      s0[k] += w;
      s1[k] += w * dz;
      s2[k] += w * dz * dz;
      cnt[k] += (k == lab && ph >= 0.5) ? 1 : 0;
      bad[k] += (k == lab && !fin) ? 1 : 0;
    }
  }
}

// End of a section's march: its partial reductions (the lane's x and y are fixed, so
// only the z moments were accumulated per plane) into the workgroup's slot.
template <class St, int NL>
__device__ __forceinline__ void finish_section3d(const DevCase<D3Q19, St>& c, int xw, int yw, const double (&s0)[NL],
                                                 const double (&s1)[NL], const double (&s2)[NL], const int (&cnt)[NL],
                                                 const int (&bad)[NL], int reduce, double* red) {
  Acc acc;
  acc.zero();
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const double dx = min_image(double(xw) - c.cen[k][0], c.nx, true);
    const double dy = min_image(double(yw) - c.cen[k][1], c.ny, !c.wall);
    acc.v[k][0] = s0[k];
    acc.v[k][1] = double(cnt[k]);
    acc.v[k][2] = dx * s0[k];
    acc.v[k][3] = dy * s0[k];
    acc.v[k][4] = s1[k];
    acc.v[k][5] = dx * dx * s0[k];
    acc.v[k][6] = dy * dy * s0[k];
    acc.v[k][7] = s2[k];
    acc.v[k][8] = dx * dy * s0[k];
    acc.v[k][9] = dx * s1[k];
    acc.v[k][10] = dy * s1[k];
    acc.v[k][11] = double(bad[k]);
  }
  __syncthreads();
  finish_block(c, acc, reduce != 0, red);
}

// NL: labels of the volume reductions (1 or 2), fixed per case; UNIT: the case's rates
// outside the g flux and f stress rows are all 1
// VISC: the phases have different viscosities (per-node tau_f of the stress rows)
// WALL: the case may have walls bounding y (c.wall decides); without it every axis is
// periodic and no pull is redirected
// BUF: arrays accessed through buffer resources (periodic cases whose arrays each span
// less than 2 GiB)
template <class St, int NL, bool UNIT, class IX, int BS, bool VISC, bool WALL, bool BUF>
__global__ void __launch_bounds__(BS, (step3d_min_blocks<St, BS>())) k_step3d(DevCase<D3Q19, St> c, int BX, int BY,
                                                                            int nby, int nbz, int reduce) {
  static_assert(!(BUF && WALL), "buffer access serves periodic cases only");
  using L = D3Q19;
  using R = typename St::R;
  constexpr int Q = L::Q;
  constexpr bool STAGE = stage3d<St>();
  extern __shared__ unsigned char smem_raw[];
  const int PW = BX + 2, PH = BY + 2, PS = PW * PH;
  using PhiPsi = PhiPsi3<R>;
  PhiPsi* sring = reinterpret_cast<PhiPsi*>(smem_raw);
  R* sg = reinterpret_cast<R*>(sring + 4 * PS);   // STAGE: [2][Q][nthr], the pulled g of planes z and z + 1, per lane
  const int nthr = BX * BY;
  const int tid = threadIdx.x;
  const int tx = tid % BX, ty = tid / BX;
  // x sections fastest, then y, then z segments: the sections of one z segment march
  // together on one XCD, so the lines a section shares with its neighbours (the pulls
  // across its edges and its halo ring) are found in that XCD's L2
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int nbx = int(gridDim.x) / (nby * nbz);
  const int bxi = tile % nbx;
  const int rest = tile / nbx;
  const int byi = rest % nby, bz = rest / nby;
  // the nbz workgroups of a column share its planes evenly (they differ by at most one)
  const int x0 = bxi * BX, y0 = byi * BY;
  const int z0 = int(long(bz) * c.nz / nbz), z1 = int(long(bz + 1) * c.nz / nbz);
  const int xg = x0 + tx, yg = y0 + ty;
  const bool active = xg < c.nx && yg < c.ny;
  const bool wall = WALL && c.wall != 0;
  // a lane past the last row pulls the last row (walls: the ring holds its wetting ghost
  // there) or the periodic image
  const int xw = xg % c.nx, yw = wall ? min(yg, c.ny - 1) : yg % c.ny;
  const int yside = wall && yg >= c.ny ? 1 : 0;
  const long t = c.t;
  const int par = int(t & 1);
  const typename St::S* gsrc = c.pop[0][par];
  const typename St::S* fsrc = c.pop[1][par];
  const float* phis = c.phis[par];
  const int nx = c.nx, ny = c.ny, nz = c.nz, nxy = nx * ny;
  Bufs3 bf;
  bf.pb = int(c.ns * long(sizeof(typename St::S)));
  bf.jb = int(c.ns * long(sizeof(R)));
  bf.g = raw_rsrc(gsrc, Q * c.ns);
  bf.f = raw_rsrc(fsrc, Q * c.ns);
  bf.gd = raw_rsrc(c.pop[0][par ^ 1], Q * c.ns);
  bf.fd = raw_rsrc(c.pop[1][par ^ 1], Q * c.ns);
  bf.phis = raw_rsrc(phis, St::shifted ? c.ns : 0);
  bf.phisd = raw_rsrc(c.phis[par ^ 1], St::shifted ? c.ns : 0);
  bf.J = raw_rsrc(c.J, L::D * c.ns);
  // a section spanning the whole (periodic) x extent holds its own x halo: the columns
  // beside it are the images of its last and first columns, so only the two halo rows
  // are pulled
  const bool own_x_halo = BX == nx;
  const int ring = own_x_halo ? 2 * PW : 2 * PW + 2 * BY;
  // pull plane z into g, form phi and psi into the ring (with the halo ring)
  auto plane = [&](int z, R (&g)[Q]) {
    const int zr = wrapi(z, c.nz);
    const int s = ring_slot3d(z) * PS;
    R ps[Q];
    pull19<St, IX, BUF>(gsrc, phis, c.ns, bf.g, bf.phis, bf.pb, nbr3(xw, yw, zr, nx, ny, nz, nxy, wall), g, ps);
    R ph = phi_of_pulled<L, St>(g, ps, c.np.rest);
    if (yside) ph = wet_ghost<R>(ph, c.np.wet_hi);   // a lane past a wall holds the ghost row
    const PhiPsi own = PhiPsi{ph, psi_of<R>(ph, c.np.W4, c.np.xi)};
    sring[s + (ty + 1) * PW + tx + 1] = own;
    if (own_x_halo) {
      if (tx == BX - 1) sring[s + (ty + 1) * PW] = own;
      if (tx == 0) sring[s + (ty + 1) * PW + PW - 1] = own;
    }
    // halo cells on consecutive threads (thread k takes cell k): the fewest waves run the
    // halo pulls, with every lane busy (measured 4.5% faster on C3 than spreading the
    // cells over all waves)
    for (int k = tid; k < ring; k += nthr) {
      int px, py;
      if (k < PW) { px = k; py = 0; }
      else if (k < 2 * PW) { px = k - PW; py = PH - 1; }
      else if (k < 2 * PW + BY) { px = 0; py = 1 + k - 2 * PW; }
      else { px = PW - 1; py = 1 + k - 2 * PW - BY; }
      const int hx = ((x0 - 1 + px) % nx + nx) % nx;
      // rows behind a wall: the edge row's wetting ghost (its mirror for a neutral wall)
      const int hyr = y0 - 1 + py;
      const int hside = wall ? (hyr < 0 ? -1 : (hyr >= ny ? 1 : 0)) : 0;
      const int hy = wall ? (hyr < 0 ? 0 : (hyr >= ny ? ny - 1 : hyr)) : ((hyr % ny) + ny) % ny;
      R gh[Q], hps[Q];
      pull19<St, IX, BUF>(gsrc, phis, c.ns, bf.g, bf.phis, bf.pb, nbr3(hx, hy, zr, nx, ny, nz, nxy, wall), gh,
                          hps);
      R hp = phi_of_pulled<L, St>(gh, hps, c.np.rest);
      if (hside) hp = wet_ghost<R>(hp, hside < 0 ? c.np.wet_lo : c.np.wet_hi);
      sring[s + py * PW + px] = PhiPsi{hp, psi_of<R>(hp, c.np.W4, c.np.xi)};
    }
  };
  // lane-private staging of a pulled plane (consecutive lanes, consecutive words)
  auto stage_put = [&](int z, const R (&g)[Q]) {
    R* d = sg + (z & 1) * Q * nthr + tid;
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i * nthr] = g[i];
  };
  auto stage_get = [&](int z, R (&g)[Q]) {
    const R* d = sg + (z & 1) * Q * nthr + tid;
#pragma unroll
    for (int i = 0; i < Q; ++i) g[i] = d[i * nthr];
  };
  // the ring's LDS serves as reduction scratch before the march and after it
  if (blockIdx.x == 0 && c.pend_nb > 0) fold_pending(c, reinterpret_cast<double*>(smem_raw));
  // reductions: the lane's (x, y) is fixed, so per label only sum phi, sum phi dz,
  // sum phi dz^2 and the counts are accumulated; the x and y moments follow at the end
  double s0[NL], s1[NL], s2[NL];
  int cnt[NL], bad[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    s0[k] = s1[k] = s2[k] = 0.0;
    cnt[k] = bad[k] = 0;
  }
  // Segments march up (even bz) and down (odd bz) in turn, so that the two segments on
  // either side of a cut reach it together, both first or both last: the planes each
  // pulls across the cut are the other's own planes of the same moment, found in L2.
  const int dir = (bz & 1) ? -1 : 1;
  const int zs = dir > 0 ? z0 : z1 - 1, ze = dir > 0 ? z1 : z0 - 1;   // first plane, one past the last
  R gcur[Q], gnext[Q];
  if constexpr (STAGE) {
    plane(zs - dir, gnext);
    stage_put(zs - dir, gnext);
    plane(zs, gnext);
    stage_put(zs, gnext);
  } else {
    plane(zs - dir, gnext);
    plane(zs, gcur);
  }
  for (int z = zs; z != ze; z += dir) {
    // this plane's f and previous phi u are requested together with the next plane's
    // g, so that one memory round trip per plane covers both
    const Nbr3 o = nbr3(xw, yw, z, nx, ny, nz, nxy, wall);
    const int nn = o.s0;
    R f[Q], J[L::D];
    if (active) {
      pull19<St, IX, BUF>(fsrc, phis, c.ns, bf.f, bf.phis, bf.pb, o, f, nullptr);
#pragma unroll
      for (int d = 0; d < L::D; ++d) {
        if constexpr (BUF) J[d] = buf_ld<R>(bf.J, unsigned(nn) * unsigned(sizeof(R)), d * bf.jb);
        else J[d] = ldg(c.J + d * c.ns, IX(nn));
      }
    }
    plane(z + dir, gnext);
    if constexpr (STAGE) stage_put(z + dir, gnext);
    __syncthreads();
    if (active) {
      if constexpr (STAGE) stage_get(z, gcur);
      update_node3d<St, NL, UNIT, VISC, WALL, IX, BUF>(c, bf, sring, PS, PW, tx, ty, xw, yw, z, nn, par, gcur, f,
                                                       J, reduce != 0, s0, s1, s2, cnt, bad);
    }
    if constexpr (!STAGE) {
#pragma unroll
      for (int i = 0; i < Q; ++i) gcur[i] = gnext[i];
    }
  }
  finish_section3d<St, NL>(c, xw, yw, s0, s1, s2, cnt, bad, reduce, reinterpret_cast<double*>(smem_raw));
}

template <class St>
int step3d_max_lanes() {
  return stage3d<St>() ? 768 : 256;
}

template <class St>
size_t step3d_lds_bytes(int bx, int by3) {
  const size_t ring = size_t(2) * 4 * (bx + 2) * (by3 + 2) * sizeof(typename St::R);
  const size_t stage = stage3d<St>() ? size_t(2) * D3Q19::Q * bx * by3 * sizeof(typename St::R) : 0;
  return ring + stage;
}

template <class St>
int launch_step3d(const DevCase<D3Q19, St>& c, const Tile& tile, int reduce, hipStream_t s) {
  const int nbx = (c.nx + tile.bx - 1) / tile.bx;
  const int nby = (c.ny + tile.by3 - 1) / tile.by3;
  const int nbz = (c.nz + tile.ty - 1) / tile.ty;
  const int lanes = tile.bx * tile.by3;
  if (lanes > step3d_max_lanes<St>()) return -1;
  const size_t lds = step3d_lds_bytes<St>(tile.bx, tile.by3);
  const dim3 grid(nbx * nby * nbz), block(lanes);
  int rc = 0;
  auto go = [&](auto nl, auto unit, auto ix, auto visc, auto wall, auto buf) {
    constexpr bool V = decltype(visc)::value;
    constexpr bool WL = decltype(wall)::value;
    constexpr bool BF = decltype(buf)::value;
    constexpr int NL = decltype(nl)::value;
    constexpr bool U = decltype(unit)::value;
    if (lanes <= 256) {
      hipLaunchKernelGGL((k_step3d<St, NL, U, decltype(ix), 256, V, WL, BF>), grid, block, lds, s, c, tile.bx, tile.by3,
                         nby, nbz, reduce);
    } else if constexpr (stage3d<St>()) {
      // wide sections stage more than the default 64 KiB of dynamic LDS: raise this
      // instantiation's limit to the device maximum once per device (the tile check has
      // compared the section with that maximum)
      auto kern = k_step3d<St, NL, U, decltype(ix), 768, V, WL, BF>;
      static int raised[64] = {};   // per instantiation and device; a repeated raise is harmless
      int dev = 0, max_lds = 0;
      if (hipGetDevice(&dev) != hipSuccess) {
        rc = -3;
        return;
      }
      if (dev >= 64 || !raised[dev]) {
        if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
            hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                max_lds) != hipSuccess) {
          rc = -3;
          return;
        }
        if (dev < 64) raised[dev] = 1;
      }
      hipLaunchKernelGGL(kern, grid, block, lds, s, c, tile.bx, tile.by3, nby, nbz, reduce);
    }
  };
  using One = std::integral_constant<int, 1>;
  using Two = std::integral_constant<int, 2>;
  // periodic cases in FP16S and FP64: the kernels with no wall tests (FP16S through buffer
  // resources while its arrays fit them)
  auto pick_wall = [&](auto nl, auto unit, auto ix, auto visc) {
    if constexpr (periodic3d_kernel<St>()) {
      if (!c.wall) {
        if constexpr (buf3d_kernel<St>()) {
          if (buf3d_fits(c)) {
            go(nl, unit, ix, visc, std::false_type{}, std::true_type{});
            return;
          }
        }
        go(nl, unit, ix, visc, std::false_type{}, std::false_type{});
        return;
      }
    }
    go(nl, unit, ix, visc, std::true_type{}, std::false_type{});
  };
  // 64-bit indexing (IX = long): the 32-bit byte-offset form (unsigned IX) measured 0.5%
  // slower in FP32 and 5.6% slower in FP16S on this kernel (and equal in FP64)
  auto pick_visc = [&](auto nl, auto unit) {
    if (c.visc) pick_wall(nl, unit, 0L, std::true_type{});
    else pick_wall(nl, unit, 0L, std::false_type{});
  };
  auto pick_unit = [&](auto nl) {
    if (c.unit_rates) pick_visc(nl, std::true_type{});
    else pick_visc(nl, std::false_type{});
  };
  if (c.nl > 1) pick_unit(Two{});
  else pick_unit(One{});
  if (rc) return rc;
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template size_t step3d_lds_bytes<StoreF64>(int, int);
template size_t step3d_lds_bytes<StoreF32>(int, int);
template size_t step3d_lds_bytes<StoreF16S>(int, int);
template int launch_step3d<StoreF64>(const DevCase<D3Q19, StoreF64>&, const Tile&, int, hipStream_t);
template int launch_step3d<StoreF32>(const DevCase<D3Q19, StoreF32>&, const Tile&, int, hipStream_t);
template int launch_step3d<StoreF16S>(const DevCase<D3Q19, StoreF16S>&, const Tile&, int, hipStream_t);

}  // namespace vclb
