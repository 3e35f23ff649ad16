// Step, init, observe and reduction kernels of the phase-field lattice Boltzmann model
// for gfx950, and their host-side launchers.
//
// Layout in HBM (per case, structure of arrays): population set s (g or f), buffer b
// (A/B, swapped every step) and direction i at node n: pop[s][b][i * N + n], with
// n = x + nx (y + ny z), x fastest.  Buffers hold post-collision values; a step pulls
// pop_i(x) = post_i(x - c_i) from the buffer the previous step wrote.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "devcase.hpp"
#include "launch.hpp"
#include "step2d.hpp"

namespace vclb {

// ---------------------------------------------------------------- init (A13)
// g = g_eq(phi0, mu0, u0), f = f_eq(p = 0, rho(phi0), u0), previous phi u = phi0 u0.
// Values are written where the first pull will look for them (inverse streaming).
template <class L, class St, bool COUPLED>
__global__ void __launch_bounds__(256) k_init(DevCase<L, St> c, const double* __restrict__ phi0,
                                              const double* __restrict__ u0) {
  using R = typename St::R;
  constexpr int Q = L::Q, D = L::D;
  const long n = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (n >= c.n) return;
  const int x = int(n % c.nx), y = int((n / c.nx) % c.ny), z = int(n / (long(c.nx) * c.ny));
  // Laplacian of phi0 (Eq. 40), wetting ghosts behind walls
  R nb[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int xn = wrapi(x + L::cx[i], c.nx), yn = y + L::cy[i], zn = wrapi(z + L::cz[i], c.nz);
    const int side = c.wall ? (yn < 0 ? -1 : (yn >= c.ny ? 1 : 0)) : 0;
    yn = c.wall ? (yn < 0 ? 0 : (yn >= c.ny ? c.ny - 1 : yn)) : wrapi(yn, c.ny);
    nb[i] = R(phi0[xn + long(c.nx) * (yn + long(c.ny) * zn)]);
    if (side) nb[i] = wet_ghost<R>(nb[i], side < 0 ? c.np.wet_lo : c.np.wet_hi);
  }
  const R phi = nb[0];
  const R lphi = stencil_lap<L, R>(nb);
  const R mu = c.np.beta4 * phi * (phi - R(1)) * (phi - R(0.5)) - c.np.kappa * lphi;
  R u[D];
  if constexpr (COUPLED) {
#pragma unroll
    for (int d = 0; d < D; ++d) u[d] = u0 ? R(u0[d * c.n + n]) : R(0);
  } else {
    R ux, uy;
    vortex_u<R>(c.np.U0, c.np.T, x, y, c.nx, c.ny, 0, ux, uy);
    u[0] = ux;
    u[1] = uy;
  }
  const R H = mu + c.np.lam * phi;
  const R rho = c.np.rho_l + phi * c.np.drho;
  R uu = R(0);
#pragma unroll
  for (int d = 0; d < D; ++d) uu += u[d] * u[d];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cc[3] = {L::cx[i], L::cy[i], L::cz[i]};
    R cJ = R(0), cu = R(0);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if (cc[d] == 1) { cJ += phi * u[d]; cu += u[d]; }
      else if (cc[d] == -1) { cJ -= phi * u[d]; cu -= u[d]; }
    }
    const R wi = R(L::w[i]);
    const R geq = (i == 0) ? phi + R(L::w[0] - 1.0) * H : wi * H + wi * (R(3) * cJ);
    const R si = wi * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu);
    const R feq = rho * si;   // p = 0
    // where the first pull of direction i at this node reads
    int xs = x - L::cx[i], ys = y - L::cy[i], zs = z - L::cz[i], pi = i;
    if (L::cy[i] != 0 && (ys < 0 || ys >= c.ny)) {
      if (c.wall) { xs = x; ys = y; zs = z; pi = L::opp[i]; }
      else ys = wrapi(ys, c.ny);
    }
    xs = wrapi(xs, c.nx);
    zs = wrapi(zs, c.nz);
    const long s = xs + long(c.nx) * (ys + long(c.ny) * zs);
    R gv = geq;
    // shifted storage: relative to the reader's phis entry, phi0 at this node n
    if constexpr (St::shifted) gv -= R(float(phi0[n])) * c.np.rest[pi];
    St::store(c.pop[0][0], long(pi) * c.ns + s, gv);
    if constexpr (COUPLED) St::store(c.pop[1][0], long(pi) * c.ns + s, feq);
  }
#pragma unroll
  for (int d = 0; d < D; ++d) c.J[d * c.ns + n] = phi * u[d];
  if constexpr (St::shifted) c.phis[0][n] = float(phi0[n]);
}

// ---------------------------------------------------------------- explicit state
// Store a given time-t state (post-streaming populations in FP64) where the next pull
// looks for it.  FP16S: the phi of node s that encodes entry s is sum_i g_i(s).
template <class L, class St, bool COUPLED>
__global__ void __launch_bounds__(256) k_set_state(DevCase<L, St> c, const double* __restrict__ g,
                                                   const double* __restrict__ f, const double* __restrict__ J,
                                                   int par) {
  using R = typename St::R;
  const long n = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (n >= c.n) return;
  const int x = int(n % c.nx), y = int((n / c.nx) % c.ny), z = int(n / (long(c.nx) * c.ny));
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    int xs = x - L::cx[i], ys = y - L::cy[i], zs = z - L::cz[i], pi = i;
    if (L::cy[i] != 0 && (ys < 0 || ys >= c.ny)) {
      if (c.wall) { xs = x; ys = y; zs = z; pi = L::opp[i]; }
      else ys = wrapi(ys, c.ny);
    }
    xs = wrapi(xs, c.nx);
    zs = wrapi(zs, c.nz);
    const long s = xs + long(c.nx) * (ys + long(c.ny) * zs);
    R gv = R(g[long(i) * c.n + n]);
    if constexpr (St::shifted) {   // relative to the reader's (this node n's) phis entry
      double ps = 0.0;
      for (int k = 0; k < L::Q; ++k) ps += g[long(k) * c.n + n];
      gv -= R(float(ps)) * c.np.rest[pi];
    }
    St::store(c.pop[0][par], long(pi) * c.ns + s, gv);
    if constexpr (COUPLED) St::store(c.pop[1][par], long(pi) * c.ns + s, R(f[long(i) * c.n + n]));
  }
#pragma unroll
  for (int d = 0; d < L::D; ++d) c.J[d * c.ns + n] = R(J[d * c.n + n]);
  if constexpr (St::shifted) {
    double ps = 0.0;
    for (int k = 0; k < L::Q; ++k) ps += g[long(k) * c.n + n];
    c.phis[par][n] = float(ps);
  }
}

// The time-t state (pulled, decoded populations and previous phi u) in FP64.
template <class L, class St, bool COUPLED>
__global__ void __launch_bounds__(256) k_get_state(DevCase<L, St> c, double* __restrict__ g,
                                                   double* __restrict__ f, double* __restrict__ J) {
  using R = typename St::R;
  const long n = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (n >= c.n) return;
  const int x = int(n % c.nx), y = int((n / c.nx) % c.ny), z = int(n / (long(c.nx) * c.ny));
  const int par = int(c.t & 1);
  R v[L::Q], ps[L::Q];
  pull<L, St>(c, c.pop[0][par], c.phis[par], x, y, z, v, ps);
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    R gi = v[i];
    if constexpr (St::shifted) gi += c.np.rest[i] * ps[i];
    g[long(i) * c.n + n] = double(gi);
  }
  if constexpr (COUPLED) {
    pull<L, St>(c, c.pop[1][par], c.phis[par], x, y, z, v, nullptr);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) f[long(i) * c.n + n] = double(v[i]);
  }
#pragma unroll
  for (int d = 0; d < L::D; ++d) J[d * c.n + n] = double(c.J[d * c.ns + n]);
}

// ---------------------------------------------------------------- plain path, pass 1
// phi = sum g (Eq. 35) and psi (Eq. 37) of every node into scratch arrays.
template <class L, class St>
__global__ void __launch_bounds__(256) k_phi_psi(DevCase<L, St> c) {
  using R = typename St::R;
  const long n = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (n >= c.n) return;
  const int x = int(n % c.nx), y = int((n / c.nx) % c.ny), z = int(n / (long(c.nx) * c.ny));
  const int par = int(c.t & 1);
  R g[L::Q], ps[L::Q];
  pull<L, St>(c, c.pop[0][par], c.phis[par], x, y, z, g, ps);
  const R phi = phi_of_pulled<L, St>(g, ps, c.np.rest);
  c.tmp_phi[n] = phi;
  c.tmp_psi[n] = psi_of<R>(phi, c.np.W4, c.np.xi);
}

// ---------------------------------------------------------------- global volume correction
// (an ablation of the kind of correction the paper argues against; off by default)
// Per workgroup: sum H(phi_c) and sum delta(phi_c) of the scratch phi, H(p) = p^2 (3 - 2p),
// delta(p) = 4 p (1 - p).
template <class L, class St>
__global__ void __launch_bounds__(256) k_mass_partials(DevCase<L, St> c) {
  __shared__ double red[4 * 2];
  const long n = blockIdx.x * long(blockDim.x) + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (n < c.n) {
    const double pc = double(clamp01(c.tmp_phi[n]));
    v[0] = pc * pc * (3.0 - 2.0 * pc);
    v[1] = 4.0 * pc * (1.0 - pc);
  }
  const double s = block_sum_fields<2>(v, 2, red);
  if (threadIdx.x < 2) c.mass_part[long(threadIdx.x) * gridDim.x + blockIdx.x] = s;
}

// Sum the partials in workgroup order.  set_ref: the volume becomes the reference V_ref
// (kappa 0); else kappa = r (V_ref - V) / sum delta.
template <class L, class St>
__global__ void __launch_bounds__(256) k_mass_fold(DevCase<L, St> c, int nb, int set_ref) {
  __shared__ double red[4 * 2];
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    v[0] += c.mass_part[b];
    v[1] += c.mass_part[nb + b];
  }
  const double s = block_sum_fields<2>(v, 2, red);
  __shared__ double tot[2];
  if (threadIdx.x < 2) tot[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double V = tot[0], sd = tot[1];
    if (set_ref) {
      c.mass[0] = V;
      c.mass[1] = 0.0;
    } else {
      c.mass[1] = sd > 0.0 ? c.np.mass_fix * (c.mass[0] - V) / sd : 0.0;
    }
    c.mass[2] = V;
    c.mass[3] = sd;
  }
}

template <class L, class St>
static void launch_mass(const DevCase<L, St>& c, int set_ref, hipStream_t s) {
  const unsigned nb = unsigned((c.n + 255) / 256);
  hipLaunchKernelGGL((k_mass_partials<L, St>), dim3(nb), dim3(256), 0, s, c);
  hipLaunchKernelGGL((k_mass_fold<L, St>), dim3(1), dim3(256), 0, s, c, int(nb), set_ref);
}

// gather phi and psi of the scratch fields at x + c_i with periodic wrap; behind a wall,
// the wetting ghost of the edge row's phi and psi (Eq. 37) of that ghost
template <class L, class St>
__device__ __forceinline__ void gather_phi_psi(const DevCase<L, St>& c, int x, int y, int z,
                                               typename St::R (&nphi)[L::Q], typename St::R (&npsi)[L::Q]) {
  using R = typename St::R;
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    int xn = wrapi(x + L::cx[i], c.nx), yn = y + L::cy[i], zn = wrapi(z + L::cz[i], c.nz);
    const int side = c.wall ? (yn < 0 ? -1 : (yn >= c.ny ? 1 : 0)) : 0;
    yn = c.wall ? (yn < 0 ? 0 : (yn >= c.ny ? c.ny - 1 : yn)) : wrapi(yn, c.ny);
    const long m = xn + long(c.nx) * (yn + long(c.ny) * zn);
    if (side) {
      nphi[i] = wet_ghost<R>(c.tmp_phi[m], side < 0 ? c.np.wet_lo : c.np.wet_hi);
      npsi[i] = psi_of<R>(nphi[i], c.np.W4, c.np.xi);
    } else {
      nphi[i] = c.tmp_phi[m];
      npsi[i] = c.tmp_psi[m];
    }
  }
}

// ---------------------------------------------------------------- plain path, pass 2
template <class L, class St, bool COUPLED>
__global__ void __launch_bounds__(256) k_collide_plain(DevCase<L, St> c, int reduce) {
  using R = typename St::R;
  const long n = blockIdx.x * long(blockDim.x) + threadIdx.x;
  const long t = c.t;
  const int par = int(t & 1);
  Acc acc;
  acc.zero();
  if (n < c.n) {
    const int x = int(n % c.nx), y = int((n / c.nx) % c.ny), z = int(n / (long(c.nx) * c.ny));
    NodeIn<L, R> in;
    gather_phi_psi<L, St>(c, x, y, z, in.nphi, in.npsi);
    prescribed<L, St, COUPLED>(c, x, y, t, in);
    R g[L::Q], ps[L::Q], f[L::Q], J[L::D];
    pull<L, St>(c, c.pop[0][par], c.phis[par], x, y, z, g, ps);
    (void)phi_of_pulled<L, St>(g, ps, c.np.rest);
    if constexpr (COUPLED) pull<L, St>(c, c.pop[1][par], c.phis[par], x, y, z, f, nullptr);
#pragma unroll
    for (int d = 0; d < L::D; ++d) J[d] = c.J[d * c.ns + n];
    NodeOut<L, R> out;
    node_update_any<L, R, COUPLED, St::shifted>(c.np, c.visc != 0, in, g, f, J, out);
    if (c.mfix) {   // g_i += w_i kappa delta(phi_c): the global correction's source
      const R pc = clamp01(in.nphi[0]);
      const R src = R(c.mass[1]) * (R(4) * pc * (R(1) - pc));
#pragma unroll
      for (int i = 0; i < L::Q; ++i) g[i] += R(L::w[i]) * src;
    }
    store_node<L, St, COUPLED>(c, par, n, y, in.nphi, out.rho, g, f, J);
    if (reduce) accumulate(c, acc, double(in.nphi[0]), x, y, z);
  }
  finish_block(c, acc, reduce != 0);
}

// ---------------------------------------------------------------- observe
template <class L, class St, bool COUPLED>
__global__ void __launch_bounds__(256) k_fields(DevCase<L, St> c, unsigned mask, double* __restrict__ out) {
  using R = typename St::R;
  const long n = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (n >= c.n) return;
  const long t = c.t;
  const int par = int(t & 1);
  const int x = int(n % c.nx), y = int((n / c.nx) % c.ny), z = int(n / (long(c.nx) * c.ny));
  NodeIn<L, R> in;
  gather_phi_psi<L, St>(c, x, y, z, in.nphi, in.npsi);
  prescribed<L, St, COUPLED>(c, x, y, t, in);
  R g[L::Q], ps[L::Q], f[L::Q], J[L::D];
  pull<L, St>(c, c.pop[0][par], c.phis[par], x, y, z, g, ps);
  (void)phi_of_pulled<L, St>(g, ps, c.np.rest);
  if constexpr (COUPLED) pull<L, St>(c, c.pop[1][par], c.phis[par], x, y, z, f, nullptr);
#pragma unroll
  for (int d = 0; d < L::D; ++d) J[d] = c.J[d * c.ns + n];
  NodeOut<L, R> o;
  node_update_any<L, R, COUPLED, St::shifted>(c.np, c.visc != 0, in, g, f, J, o);
  long off = 0;
  if (mask & 0x01u) { out[off + n] = double(in.nphi[0]); off += c.n; }
  if (mask & 0x02u) { out[off + n] = double(o.rho); off += c.n; }
  if (mask & 0x04u) {
#pragma unroll
    for (int d = 0; d < L::D; ++d) out[off + d * c.n + n] = double(o.u[d]);
    off += L::D * c.n;
  }
  if (mask & 0x08u) { out[off + n] = double(o.press); off += c.n; }
  if (mask & 0x10u) { out[off + n] = double(o.mu); off += c.n; }
  if (mask & 0x20u) { out[off + n] = double(in.npsi[0]); off += c.n; }
}

// reductions of the current state (phi from scratch), into c.cur
template <class L, class St>
__global__ void __launch_bounds__(256) k_reduce_state(DevCase<L, St> c) {
  const long n = blockIdx.x * long(blockDim.x) + threadIdx.x;
  Acc acc;
  acc.zero();
  if (n < c.n) {
    const int x = int(n % c.nx), y = int((n / c.nx) % c.ny), z = int(n / (long(c.nx) * c.ny));
    accumulate(c, acc, double(c.tmp_phi[n]), x, y, z);
  }
  finish_block(c, acc, true);
}

// ---------------------------------------------------------------- fused 2D step (A1-A11)
// Workgroups per CU the register budget is sized for, for workgroups of up to BS lanes:
// FP32 arithmetic fits 4 waves per SIMD; FP64 2, or 3 with unit rates.  BS is 256, or 1024
// for the wide strips of 4-byte arithmetic (4 waves per SIMD in one workgroup).
template <class St, bool UNIT, int BS>
constexpr int step2d_min_blocks() {
  constexpr int waves = sizeof(typename St::R) == 8 ? (UNIT ? 3 : 2) : 4;
  return waves / (BS / 256) > 0 ? waves / (BS / 256) : 1;
}

template <class St, bool COUPLED, class IX, bool UNIT, int BS, bool VISC>
__global__ void __launch_bounds__(BS, (step2d_min_blocks<St, UNIT, BS>()))
    k_step2d(DevCase<D2Q9, St> c, int TY, int nseg, int reduce) {
  extern __shared__ unsigned char smem_raw[];
  if (blockIdx.x == 0 && c.pend_nb > 0) fold_pending(c);
  // tiles of one row band (all strips) are consecutive, so that an XCD runs the strips
  // whose halo columns it shares (and the next band, whose halo rows it shares)
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int nstrips = gridDim.x / nseg;
  const int seg = tile / nstrips, strip = tile - seg * nstrips;
  const int y0 = seg * TY;
  // non-temporal population accesses for 4- and 8-byte storage (2-byte storage measured
  // no faster with them)
  constexpr bool NT = sizeof(typename St::S) >= 4;
  step2d_tile<St, COUPLED, IX, UNIT, VISC, NT>(c, c.t, strip * int(blockDim.x), y0, min(y0 + TY, c.ny),
                                               reduce != 0, c.part_w, gridDim.x, blockIdx.x, smem_raw);
}

// ---------------------------------------------------------------- second reduction pass
// Stand-alone second pass (the fused steps instead fold the previous launch's partials
// in their first workgroup).
template <class L, class St>
__global__ void __launch_bounds__(256) k_finalize(DevCase<L, St> c) {
  fold_pending(c);
}

template <class L, class St>
int launch_finalize(const DevCase<L, St>& c, hipStream_t s) {
  hipLaunchKernelGGL((k_finalize<L, St>), dim3(1), dim3(256), 0, s, c);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

// the pending pass that reads this launch's own partials
template <class L, class St>
static DevCase<L, St> self_pending(DevCase<L, St> c, int nblocks, double* dest) {
  c.part_r = c.part_w;
  c.pend_nb = nblocks;
  c.pend_dest = dest;
  c.pend_step = c.t;
  return c;
}

// ---------------------------------------------------------------- launchers
template <class L, class St, bool COUPLED>
int launch_init(const DevCase<L, St>& c, const double* phi0, const double* u0, hipStream_t s) {
  const unsigned nb = unsigned((c.n + 255) / 256);
  hipLaunchKernelGGL((k_init<L, St, COUPLED>), dim3(nb), dim3(256), 0, s, c, phi0, u0);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <class L, class St, bool COUPLED>
int launch_step_plain(const DevCase<L, St>& c, int reduce, hipStream_t s) {
  const unsigned nb = unsigned((c.n + 255) / 256);
  hipLaunchKernelGGL((k_phi_psi<L, St>), dim3(nb), dim3(256), 0, s, c);
  if (c.mfix) launch_mass(c, 0, s);
  hipLaunchKernelGGL((k_collide_plain<L, St, COUPLED>), dim3(nb), dim3(256), 0, s, c, reduce);
  if (reduce) launch_finalize(self_pending(c, int(nb), c.hist + (c.t % kHistory) * c.nl * kObsFields), s);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <class L, class St, bool COUPLED>
int launch_step_fused(const DevCase<L, St>& c, const Tile& tile, int reduce, hipStream_t s) {
  if constexpr (L::D == 2) {
    const int nstrips = (c.nx + tile.bx - 1) / tile.bx;
    const int nseg = (c.ny + tile.ty - 1) / tile.ty;
    const size_t lds = size_t(2) * 4 * (tile.bx + 2) * sizeof(typename St::R);
    // 32-bit byte offsets for the FP16S march, which is instruction-bound, when every
    // per-plane offset fits them (8-byte elements at most); the FP32 and FP64 marches
    // measured 0.6% and 2.6% faster with 64-bit indexing.  The unit-rate update when the
    // case's rates allow it.
    const dim3 grid(nstrips * nseg), block(tile.bx);
    // strips wider than 256 lanes (512 or 1024) take the 1024-lane instantiation, which
    // exists for 4-byte arithmetic only
    bool bad_shape = false;
    auto go = [&](auto ix, auto unit, auto visc) {
      constexpr bool U = decltype(unit)::value, V = decltype(visc)::value;
      if (tile.bx <= 256) {
        hipLaunchKernelGGL((k_step2d<St, COUPLED, decltype(ix), U, 256, V>), grid, block, lds, s, c, tile.ty, nseg,
                           reduce);
      } else if constexpr (sizeof(typename St::R) == 4) {
        hipLaunchKernelGGL((k_step2d<St, COUPLED, decltype(ix), U, 1024, V>), grid, block, lds, s, c, tile.ty, nseg,
                           reduce);
      } else {
        bad_shape = true;
      }
    };
    // per-node tau_f only where the phases' viscosities differ (coupled cases)
    auto pick_visc = [&](auto ix, auto unit) {
      if constexpr (COUPLED) {
        if (c.visc) {
          go(ix, unit, std::true_type{});
          return;
        }
      }
      go(ix, unit, std::false_type{});
    };
    auto pick = [&](auto ix) {
      if (c.unit_rates) pick_visc(ix, std::true_type{});
      else pick_visc(ix, std::false_type{});
    };
    if constexpr (std::is_same<St, StoreF16S>::value) {
      if (c.n < (1L << 29)) pick(0u);
      else pick(0L);
    } else {
      pick(0L);
    }
    if (bad_shape) return -1;
    return hipGetLastError() == hipSuccess ? 0 : -3;
  } else {
    return launch_step3d<St>(c, tile, reduce, s);
  }
}

template <class L, class St, bool COUPLED>
int launch_observe(const DevCase<L, St>& c, unsigned mask, double* out, hipStream_t s) {
  const unsigned nb = unsigned((c.n + 255) / 256);
  hipLaunchKernelGGL((k_phi_psi<L, St>), dim3(nb), dim3(256), 0, s, c);
  hipLaunchKernelGGL((k_fields<L, St, COUPLED>), dim3(nb), dim3(256), 0, s, c, mask, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <class L, class St>
int launch_phi_psi(const DevCase<L, St>& c, hipStream_t s) {
  const unsigned nb = unsigned((c.n + 255) / 256);
  hipLaunchKernelGGL((k_phi_psi<L, St>), dim3(nb), dim3(256), 0, s, c);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <class L, class St>
int launch_mass_ref(const DevCase<L, St>& c, hipStream_t s) {
  const unsigned nb = unsigned((c.n + 255) / 256);
  hipLaunchKernelGGL((k_phi_psi<L, St>), dim3(nb), dim3(256), 0, s, c);
  launch_mass(c, 1, s);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <class L, class St>
int launch_reduce_state(const DevCase<L, St>& c, hipStream_t s) {
  const unsigned nb = unsigned((c.n + 255) / 256);
  hipLaunchKernelGGL((k_phi_psi<L, St>), dim3(nb), dim3(256), 0, s, c);
  hipLaunchKernelGGL((k_reduce_state<L, St>), dim3(nb), dim3(256), 0, s, c);
  launch_finalize(self_pending(c, int(nb), c.cur), s);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <class L, class St, bool COUPLED>
int launch_set_state(const DevCase<L, St>& c, const double* g, const double* f, const double* J, long t,
                     hipStream_t s) {
  const unsigned nb = unsigned((c.n + 255) / 256);
  hipLaunchKernelGGL((k_set_state<L, St, COUPLED>), dim3(nb), dim3(256), 0, s, c, g, f, J, int(t & 1));
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <class L, class St, bool COUPLED>
int launch_get_state(const DevCase<L, St>& c, double* g, double* f, double* J, hipStream_t s) {
  const unsigned nb = unsigned((c.n + 255) / 256);
  hipLaunchKernelGGL((k_get_state<L, St, COUPLED>), dim3(nb), dim3(256), 0, s, c, g, f, J);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

#define VCLB_INSTANTIATE(L, St, C)                                                              \
  template int launch_set_state<L, St, C>(const DevCase<L, St>&, const double*, const double*, \
                                          const double*, long, hipStream_t);                   \
  template int launch_get_state<L, St, C>(const DevCase<L, St>&, double*, double*, double*,    \
                                          hipStream_t);                                        \
  template int launch_init<L, St, C>(const DevCase<L, St>&, const double*, const double*,      \
                                     hipStream_t);                                             \
  template int launch_step_plain<L, St, C>(const DevCase<L, St>&, int, hipStream_t);           \
  template int launch_step_fused<L, St, C>(const DevCase<L, St>&, const Tile&, int, hipStream_t); \
  template int launch_observe<L, St, C>(const DevCase<L, St>&, unsigned, double*, hipStream_t);

VCLB_INSTANTIATE(D2Q9, StoreF64, true)
VCLB_INSTANTIATE(D2Q9, StoreF64, false)
VCLB_INSTANTIATE(D2Q9, StoreF32, true)
VCLB_INSTANTIATE(D2Q9, StoreF32, false)
VCLB_INSTANTIATE(D2Q9, StoreF16S, true)
VCLB_INSTANTIATE(D2Q9, StoreF16S, false)
VCLB_INSTANTIATE(D3Q19, StoreF64, true)
VCLB_INSTANTIATE(D3Q19, StoreF32, true)
VCLB_INSTANTIATE(D3Q19, StoreF16S, true)
template int launch_reduce_state<D2Q9, StoreF64>(const DevCase<D2Q9, StoreF64>&, hipStream_t);
template int launch_mass_ref<D2Q9, StoreF64>(const DevCase<D2Q9, StoreF64>&, hipStream_t);
template int launch_mass_ref<D2Q9, StoreF32>(const DevCase<D2Q9, StoreF32>&, hipStream_t);
template int launch_mass_ref<D2Q9, StoreF16S>(const DevCase<D2Q9, StoreF16S>&, hipStream_t);
template int launch_mass_ref<D3Q19, StoreF64>(const DevCase<D3Q19, StoreF64>&, hipStream_t);
template int launch_mass_ref<D3Q19, StoreF32>(const DevCase<D3Q19, StoreF32>&, hipStream_t);
template int launch_mass_ref<D3Q19, StoreF16S>(const DevCase<D3Q19, StoreF16S>&, hipStream_t);
template int launch_phi_psi<D2Q9, StoreF64>(const DevCase<D2Q9, StoreF64>&, hipStream_t);
template int launch_phi_psi<D2Q9, StoreF32>(const DevCase<D2Q9, StoreF32>&, hipStream_t);
template int launch_phi_psi<D2Q9, StoreF16S>(const DevCase<D2Q9, StoreF16S>&, hipStream_t);
template int launch_phi_psi<D3Q19, StoreF64>(const DevCase<D3Q19, StoreF64>&, hipStream_t);
template int launch_phi_psi<D3Q19, StoreF32>(const DevCase<D3Q19, StoreF32>&, hipStream_t);
template int launch_phi_psi<D3Q19, StoreF16S>(const DevCase<D3Q19, StoreF16S>&, hipStream_t);
template int launch_finalize<D2Q9, StoreF64>(const DevCase<D2Q9, StoreF64>&, hipStream_t);
template int launch_finalize<D2Q9, StoreF32>(const DevCase<D2Q9, StoreF32>&, hipStream_t);
template int launch_finalize<D2Q9, StoreF16S>(const DevCase<D2Q9, StoreF16S>&, hipStream_t);
template int launch_finalize<D3Q19, StoreF64>(const DevCase<D3Q19, StoreF64>&, hipStream_t);
template int launch_finalize<D3Q19, StoreF32>(const DevCase<D3Q19, StoreF32>&, hipStream_t);
template int launch_finalize<D3Q19, StoreF16S>(const DevCase<D3Q19, StoreF16S>&, hipStream_t);
template int launch_reduce_state<D2Q9, StoreF32>(const DevCase<D2Q9, StoreF32>&, hipStream_t);
template int launch_reduce_state<D2Q9, StoreF16S>(const DevCase<D2Q9, StoreF16S>&, hipStream_t);
template int launch_reduce_state<D3Q19, StoreF64>(const DevCase<D3Q19, StoreF64>&, hipStream_t);
template int launch_reduce_state<D3Q19, StoreF32>(const DevCase<D3Q19, StoreF32>&, hipStream_t);
template int launch_reduce_state<D3Q19, StoreF16S>(const DevCase<D3Q19, StoreF16S>&, hipStream_t);

}  // namespace vclb
