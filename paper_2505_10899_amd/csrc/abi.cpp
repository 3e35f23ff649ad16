// Host side of the C ABI declared in include/vclb.h: parameter validation (no HIP call),
// workspace layout, per-case constants, launch dispatch over (lattice, storage, mode),
// observation history and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/vclb.h"
#include "adjoint.hpp"
#include "launch.hpp"
#include "probe.hpp"
#include "reduce.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(VCLB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call)                                  \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #call);  \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool finite(double v) { return std::isfinite(v); }

int lattice_q(int lattice) { return lattice == VCLB_D2Q9 ? 9 : 19; }
int lattice_d(int lattice) { return lattice == VCLB_D2Q9 ? 2 : 3; }
size_t storage_bytes(int storage) { return storage == VCLB_FP64 ? 8 : (storage == VCLB_FP32 ? 4 : 2); }
size_t arith_bytes(int storage) { return storage == VCLB_FP64 ? 8 : 4; }

bool wall_y(const vclb_params& p) { return p.bc[1][0] == VCLB_WALL; }
// unequal viscosities of the two phases: tau_f differs from node to node (Eq. 27)
bool visc_ratio(const vclb_params& p) { return p.nu_heavy != p.nu_light; }

// relaxation rates with defaults filled in (see lattice.hpp).  With unequal viscosities
// the f stress rows get the heavy phase's rate here; the kernels replace it per node.
void fill_rates(const vclb_params& p, double* sg, double* sf) {
  const int Q = lattice_q(p.lattice);
  const double tau_g = 0.5 + p.mobility * 3.0;   // Eq. 34, c_s^2 = 1/3
  const double tau_f = 0.5 + p.nu_heavy * 3.0;   // Eq. 27 with mu = rho nu
  for (int k = 0; k < Q; ++k) {
    bool gflux, fstress;
    if (p.lattice == VCLB_D2Q9) {
      gflux = vclb::D2Q9::g_flux_row[k];
      fstress = vclb::D2Q9::f_stress_row[k];
    } else {
      gflux = vclb::D3Q19::g_flux_row[k];
      fstress = vclb::D3Q19::f_stress_row[k];
    }
    sg[k] = p.s_g[k] != 0.0 ? p.s_g[k] : (gflux ? 1.0 / tau_g : 1.0);
    sf[k] = p.s_f[k] != 0.0 ? p.s_f[k] : (fstress ? 1.0 / tau_f : 1.0);
  }
}

int validate(const vclb_params* p) {
  if (!p) return fail(VCLB_EINVAL, "params is NULL");
  if (p->lattice != VCLB_D2Q9 && p->lattice != VCLB_D3Q19) return fail(VCLB_EINVAL, "unknown lattice");
  if (p->storage < VCLB_FP64 || p->storage > VCLB_FP16S) return fail(VCLB_EINVAL, "unknown storage");
  if (p->mode != VCLB_COUPLED && p->mode != VCLB_PRESCRIBED_VORTEX) return fail(VCLB_EINVAL, "unknown mode");
  if (p->mode == VCLB_PRESCRIBED_VORTEX && p->lattice != VCLB_D2Q9)
    return fail(VCLB_EINVAL, "the prescribed vortex is two-dimensional");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(VCLB_EINVAL, "grid sides must be >= 1");
  if (p->lattice == VCLB_D2Q9 && p->nz != 1) return fail(VCLB_EINVAL, "D2Q9 needs nz = 1");
  const double nn = double(p->nx) * p->ny * p->nz;
  if (nn > double(INT32_MAX)) return fail(VCLB_EINVAL, "more than 2^31 - 1 nodes");
  for (int a = 0; a < 3; ++a) {
    for (int sd = 0; sd < 2; ++sd)
      if (p->bc[a][sd] != VCLB_PERIODIC && p->bc[a][sd] != VCLB_WALL) return fail(VCLB_EINVAL, "unknown boundary type");
    if (p->bc[a][0] != p->bc[a][1]) return fail(VCLB_EINVAL, "both faces of an axis must have the same boundary type");
  }
  if (p->bc[0][0] == VCLB_WALL) return fail(VCLB_EINVAL, "walls on the x faces are not supported (x is periodic)");
  if (p->bc[2][0] == VCLB_WALL) return fail(VCLB_EINVAL, "walls on the z faces are not supported (z is periodic)");
  if (p->bc[1][0] == VCLB_WALL && p->ny < 2) return fail(VCLB_EINVAL, "walls need ny >= 2");
  if (p->nlabels < 0 || p->nlabels > VCLB_MAX_LABELS) return fail(VCLB_EINVAL, "nlabels out of range");
  if (!(finite(p->W) && p->W > 0)) return fail(VCLB_EINVAL, "W must be > 0");
  if (!(finite(p->sigma) && p->sigma >= 0)) return fail(VCLB_EINVAL, "sigma must be >= 0");
  if (!(finite(p->mobility) && p->mobility > 0)) return fail(VCLB_EINVAL, "mobility must be > 0");
  if (!(finite(p->lambda) && p->lambda >= 0)) return fail(VCLB_EINVAL, "lambda must be >= 0");
  if (!(finite(p->mass_fix) && p->mass_fix >= 0 && p->mass_fix <= 1))
    return fail(VCLB_EINVAL, "mass_fix must lie in [0, 1]");
  if (!(finite(p->xi) && p->xi > 0)) return fail(VCLB_EINVAL, "xi must be > 0");
  if (!(finite(p->eps_n) && p->eps_n >= 0)) return fail(VCLB_EINVAL, "eps_n must be >= 0");
  if (!(finite(p->rho_heavy) && p->rho_heavy > 0)) return fail(VCLB_EINVAL, "rho_heavy must be > 0");
  if (!(finite(p->rho_light) && p->rho_light > 0)) return fail(VCLB_EINVAL, "rho_light must be > 0");
  if (!(finite(p->nu_heavy) && p->nu_heavy > 0)) return fail(VCLB_EINVAL, "nu_heavy must be > 0");
  if (!(finite(p->nu_light) && p->nu_light > 0)) return fail(VCLB_EINVAL, "nu_light must be > 0");
  const int Q = lattice_q(p->lattice);
  for (int k = 0; k < 19; ++k) {
    const bool used = k < Q;
    for (double s : {p->s_g[k], p->s_f[k]}) {
      if (!finite(s)) return fail(VCLB_EINVAL, "relaxation rate not finite");
      if (s != 0.0 && (!used || !(s > 0.0 && s < 2.0)))
        return fail(VCLB_EINVAL, "relaxation rates must lie in (0, 2)");
    }
  }
  if (visc_ratio(*p)) {
    if (p->mode != VCLB_COUPLED) return fail(VCLB_EINVAL, "a viscosity ratio needs the coupled mode");
    for (int k = 0; k < Q; ++k) {
      const bool stress = p->lattice == VCLB_D2Q9 ? vclb::D2Q9::f_stress_row[k] : vclb::D3Q19::f_stress_row[k];
      if (stress && p->s_f[k] != 0.0)
        return fail(VCLB_EINVAL, "with unequal viscosities the stress rates of f follow Eq. 27 per node: leave them 0");
    }
  }
  double sg[19], sf[19];
  fill_rates(*p, sg, sf);
  for (int k = 0; k < Q; ++k)
    if (!(sg[k] > 0 && sg[k] < 2 && sf[k] > 0 && sf[k] < 2))
      return fail(VCLB_EINVAL, "derived relaxation rate outside (0, 2)");
  for (int a = 0; a < 3; ++a)
    for (int sd = 0; sd < 2; ++sd)
      for (int d = 0; d < 3; ++d) {
        if (!finite(p->wall_u[a][sd][d])) return fail(VCLB_EINVAL, "wall velocity not finite");
        if (p->bc[a][sd] == VCLB_WALL && d == a && p->wall_u[a][sd][d] != 0.0)
          return fail(VCLB_EINVAL, "a wall's velocity must be tangential (zero normal component)");
      }
  for (int a = 0; a < 3; ++a)
    for (int sd = 0; sd < 2; ++sd) {
      const double cw = p->wall_cos[a][sd];
      if (!finite(cw) || cw < -1.0 || cw > 1.0) return fail(VCLB_EINVAL, "wall_cos must lie in [-1, 1]");
      if (cw != 0.0 && p->bc[a][sd] != VCLB_WALL) return fail(VCLB_EINVAL, "wall_cos is for wall faces only");
    }
  if (p->mode == VCLB_PRESCRIBED_VORTEX && !(finite(p->T) && p->T > 0 && finite(p->U0)))
    return fail(VCLB_EINVAL, "vortex needs T > 0 and a finite U0");
  for (int k = 0; k < p->nlabels; ++k)
    for (int a = 0; a < 3; ++a)
      if (!finite(p->label_centre[k][a])) return fail(VCLB_EINVAL, "label centre");
  return VCLB_OK;
}

struct Layout {
  size_t pop[2][2], J, phis[2], partials[2], hist, cur, tmp_phi, tmp_psi, mass, mass_part, total;
  long partial_blocks;
};

Layout layout_for(const vclb_params& p) {
  Layout L{};
  const size_t n = size_t(p.nx) * p.ny * p.nz;
  const int Q = lattice_q(p.lattice), D = lattice_d(p.lattice);
  const size_t sb = storage_bytes(p.storage), rb = arith_bytes(p.storage);
  const int nl = std::max(1, p.nlabels);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  // planes of the populations and of J hold ns entries, so that each starts on a cache line
  const size_t ns = size_t(vclb::plane_stride(long(n)));
  for (int s = 0; s < 2; ++s)
    for (int b = 0; b < 2; ++b) {
      const bool need = s == 0 || p.mode == VCLB_COUPLED;
      L.pop[s][b] = need ? take(size_t(Q) * ns * sb) : SIZE_MAX;
    }
  L.J = take(size_t(D) * ns * rb);
  for (int b = 0; b < 2; ++b) L.phis[b] = p.storage != VCLB_FP64 ? take(n * 4) : SIZE_MAX;
  // every launch shape uses at least 64 nodes per workgroup, plus one partial row per
  // (y, z) line for tiles that are ragged in x
  L.partial_blocks = long(n / 64) + long(p.ny) * p.nz + 64;
  for (int b = 0; b < 2; ++b) L.partials[b] = take(size_t(L.partial_blocks) * nl * 12 * sizeof(double));
  L.hist = take(size_t(vclb::kHistory) * nl * vclb::kObsFields * sizeof(double));
  L.cur = take(size_t(nl) * vclb::kObsFields * sizeof(double));
  L.tmp_phi = take(n * rb);
  L.tmp_psi = take(n * rb);
  // the global volume correction: [V_ref, kappa, V, sum delta] and per-workgroup partials
  L.mass = take(4 * sizeof(double));
  L.mass_part = p.mass_fix > 0 ? take(2 * ((n + 255) / 256) * sizeof(double)) : SIZE_MAX;
  L.total = off;
  return L;
}

uint64_t fnv1a(const void* data, size_t bytes, uint64_t h = 1469598103934665603ULL) {
  const unsigned char* p = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < bytes; ++i) {
    h ^= p[i];
    h *= 1099511628211ULL;
  }
  return h;
}

}  // namespace

struct vclb_case {
  vclb_params p{};
  double sg[19]{}, sf[19]{};
  Layout lay{};
  char* ws = nullptr;
  bool own_ws = false;
  vclb::Tile tile{};
  int reduce_every = 1;
  int64_t t_host = 0;
  bool inited = false;
  std::vector<int64_t> recorded;   // step recorded in each history slot (-1: none)
  // reductions of a fused step whose second pass has not run yet: the next fused step
  // folds them in its first workgroup, anything that reads results flushes them first
  bool pending = false;
  int pend_nb = 0, pend_buf = 0;
  int64_t pend_step = 0;
  struct AdjStore* adj = nullptr;   // recorded forward pass of the adjoint (FP64 D2Q9 only)
  void* lab_scratch = nullptr;       // scratch of the caller-label reductions (grown on demand)
  size_t lab_scratch_bytes = 0;
};

namespace {
void adj_release(vclb_case* c);
}

namespace {

template <class L, class St>
vclb::DevCase<L, St> make_dev(const vclb_case& c) {
  using R = typename St::R;
  using S = typename St::S;
  vclb::DevCase<L, St> d{};
  const vclb_params& p = c.p;
  d.nx = p.nx;
  d.ny = p.ny;
  d.nz = p.nz;
  d.n = long(p.nx) * p.ny * p.nz;
  d.ns = vclb::plane_stride(d.n);
  d.wall = wall_y(p);
  d.visc = visc_ratio(p) ? 1 : 0;
  d.nl = std::max(1, p.nlabels);
  d.unit_rates = 1;
  for (int k = 0; k < L::Q; ++k)
    if ((!L::g_flux_row[k] && c.sg[k] != 1.0) || (!L::f_stress_row[k] && c.sf[k] != 1.0)) d.unit_rates = 0;
  for (int k = 0; k < vclb::kMaxLabels; ++k)
    for (int a = 0; a < 3; ++a) {
      double v;
      if (p.nlabels == 0) v = a == 0 ? (p.nx - 1) / 2.0 : (a == 1 ? (p.ny - 1) / 2.0 : (p.nz - 1) / 2.0);
      else v = p.label_centre[std::min(k, p.nlabels - 1)][a];
      // periodic axes: the minimum-image displacement is periodic in the centre, so the
      // centre is moved into [0, n) (the kernels rely on it to wrap without a division)
      const int na = a == 0 ? p.nx : (a == 1 ? p.ny : p.nz);
      const bool periodic = p.bc[a][0] == VCLB_PERIODIC;
      if (periodic) v = v - na * std::floor(v / na);
      d.cen[k][a] = v;
    }
  for (int s = 0; s < 2; ++s)
    for (int b = 0; b < 2; ++b)
      d.pop[s][b] = c.lay.pop[s][b] == SIZE_MAX ? nullptr : reinterpret_cast<S*>(c.ws + c.lay.pop[s][b]);
  d.J = reinterpret_cast<R*>(c.ws + c.lay.J);
  for (int b = 0; b < 2; ++b)
    d.phis[b] = c.lay.phis[b] == SIZE_MAX ? nullptr : reinterpret_cast<float*>(c.ws + c.lay.phis[b]);
  d.t = long(c.t_host);
  d.part_w = reinterpret_cast<double*>(c.ws + c.lay.partials[c.t_host & 1]);
  d.part_r = nullptr;
  d.pend_nb = 0;
  d.pend_dest = nullptr;
  d.pend_step = 0;
  if (c.pending) {
    d.part_r = reinterpret_cast<const double*>(c.ws + c.lay.partials[c.pend_buf]);
    d.pend_nb = c.pend_nb;
    d.pend_dest = reinterpret_cast<double*>(c.ws + c.lay.hist) +
                  size_t(c.pend_step % vclb::kHistory) * std::max(1, p.nlabels) * vclb::kObsFields;
    d.pend_step = long(c.pend_step);
  }
  d.hist = reinterpret_cast<double*>(c.ws + c.lay.hist);
  d.cur = reinterpret_cast<double*>(c.ws + c.lay.cur);
  d.tmp_phi = reinterpret_cast<R*>(c.ws + c.lay.tmp_phi);
  d.tmp_psi = reinterpret_cast<R*>(c.ws + c.lay.tmp_psi);
  d.mfix = p.mass_fix > 0 ? 1 : 0;
  d.mass = reinterpret_cast<double*>(c.ws + c.lay.mass);
  d.mass_part = c.lay.mass_part == SIZE_MAX ? nullptr : reinterpret_cast<double*>(c.ws + c.lay.mass_part);
  auto& np = d.np;
  const double sigma = p.sigma, W = p.W;
  np.W4 = R(W / 4.0);
  np.xi = R(p.xi);
  np.lamW = R(p.lambda / W);
  np.An4 = R(4.0 * (p.lambda / W) / ((1.0 + 2.0 * p.xi) * (1.0 + 2.0 * p.xi)));
  np.lam = R(p.lambda);
  np.beta4 = R(4.0 * (12.0 * sigma / W));
  np.kappa = R(1.5 * sigma * W);
  np.eps2 = R(p.eps_n * p.eps_n);
  np.rho_l = R(p.rho_light);
  np.drho = R(p.rho_heavy - p.rho_light);
  np.mu_l = R(p.rho_light * p.nu_light);
  np.dmu = R(p.rho_heavy * p.nu_heavy - p.rho_light * p.nu_light);
  for (int k = 0; k < L::Q; ++k) {
    np.sg[k] = R(c.sg[k] / vclb::row_norm<L>(k));
    np.sf[k] = R(c.sf[k] / vclb::row_norm<L>(k));
    np.sgr[k] = R(c.sg[k]);
    np.sfr[k] = R(c.sf[k]);
    np.rest[k] = R(k == 0 ? 1.0 + (L::w[0] - 1.0) * p.lambda : L::w[k] * p.lambda);
    // moving-wall term 2 w_i rho (c_i . u_wall) / cs^2 of the incoming direction i = opp(k),
    // stored on the outgoing direction k at the first (bottom) / last (top) y row
    const int i = L::opp[k];
    const double* ub = p.wall_u[1][0];
    const double* ut = p.wall_u[1][1];
    const double cub = L::cx[i] * ub[0] + L::cy[i] * ub[1] + L::cz[i] * ub[2];
    const double cut = L::cx[i] * ut[0] + L::cy[i] * ut[1] + L::cz[i] * ut[2];
    np.wb[k] = R(L::cy[k] < 0 ? 2.0 * L::w[i] * cub * 3.0 : 0.0);
    np.wt[k] = R(L::cy[k] > 0 ? 2.0 * L::w[i] * cut * 3.0 : 0.0);
  }
  // wetting ghosts behind the bottom / top wall: phi_g = phi_e + c phi_e (1 - phi_e)
  np.wet_lo = R(4.0 / W * (wall_y(p) ? p.wall_cos[1][0] : 0.0));
  np.wet_hi = R(4.0 / W * (wall_y(p) ? p.wall_cos[1][1] : 0.0));
  np.U0 = R(p.U0);
  np.mass_fix = p.mass_fix;
  np.T = p.T;
  return d;
}

// Call fn with a DevCase of the right template instance.
template <class Fn>
int dispatch(const vclb_case& c, Fn&& fn) {
  const bool coupled = c.p.mode == VCLB_COUPLED;
  if (c.p.lattice == VCLB_D2Q9) {
    switch (c.p.storage) {
      case VCLB_FP64: return coupled ? fn(make_dev<vclb::D2Q9, vclb::StoreF64>(c), std::true_type{})
                                     : fn(make_dev<vclb::D2Q9, vclb::StoreF64>(c), std::false_type{});
      case VCLB_FP32: return coupled ? fn(make_dev<vclb::D2Q9, vclb::StoreF32>(c), std::true_type{})
                                     : fn(make_dev<vclb::D2Q9, vclb::StoreF32>(c), std::false_type{});
      default: return coupled ? fn(make_dev<vclb::D2Q9, vclb::StoreF16S>(c), std::true_type{})
                              : fn(make_dev<vclb::D2Q9, vclb::StoreF16S>(c), std::false_type{});
    }
  }
  switch (c.p.storage) {
    case VCLB_FP64: return fn(make_dev<vclb::D3Q19, vclb::StoreF64>(c), std::true_type{});
    case VCLB_FP32: return fn(make_dev<vclb::D3Q19, vclb::StoreF32>(c), std::true_type{});
    default: return fn(make_dev<vclb::D3Q19, vclb::StoreF16S>(c), std::true_type{});
  }
}

template <class DC>
struct DevTraits;
template <class L_, class St_>
struct DevTraits<vclb::DevCase<L_, St_>> {
  using L = L_;
  using St = St_;
};

// run the second reduction pass of a pending fused step now
int flush_pending(vclb_case* c, hipStream_t s) {
  if (!c->pending) return VCLB_OK;
  int rc = dispatch(*c, [&](auto dc, auto) {
    using DC = decltype(dc);
    return vclb::launch_finalize<typename DevTraits<DC>::L, typename DevTraits<DC>::St>(dc, s);
  });
  c->pending = false;
  return rc ? fail(VCLB_EHIP, "finalize launch failed") : VCLB_OK;
}

vclb::Tile default_tile(const vclb_params& p, int ncu, bool wide_ok = true) {
  vclb::Tile t;
  if (p.lattice == VCLB_D2Q9) {
    // one lane per x column, rounded up to whole waves, at most 256 lanes, or 512 with
    // 4-byte arithmetic (measured 2.6% faster in FP32 and 7% in FP16S on 4096 columns)
    int bx = std::min(p.storage == VCLB_FP64 ? 256 : 512, (p.nx + 63) / 64 * 64);
    // a small case: narrower strips (down to one wave) until the marches of 8 rows give
    // every CU a workgroup
    while (bx > 64 && long((p.nx + bx - 1) / bx) * ((p.ny + 7) / 8) < ncu) bx /= 2;
    bx = (bx + 63) / 64 * 64;
    t.bx = bx;
    const long strips = (p.nx + bx - 1) / bx;
    // long marches amortise the two halo rows; keep 4 waves per SIMD resident when the
    // grid allows (1024 workgroups of up to 256 lanes, 512 of 512), with 8..64 rows each
    long ty = (long(p.ny) * strips) / (bx > 256 ? 512 : 1024);
    t.ty = int(std::max(8L, std::min(64L, ty)));
    t.by3 = 1;
  } else {
    // 32 x 8 columns per workgroup (a halo ring of a third of the tile, one wave per two
    // rows of 32): the fastest section measured on a 96 x 96 x 384 case.  Each workgroup
    // is bound by its own memory round trips, so the columns are cut along z into as many
    // segments as fill 2 (FP64, FP32) or 3 (FP16S) workgroups per CU once, with 8 to 64
    // planes each.  Three fit the registers with 4-byte arithmetic, but in FP32 the
    // longer segments of two per CU measured faster (fewer halo planes per segment).
    // With 4-byte arithmetic and at least 96 columns in x, one 96 x 8 section of 768
    // lanes per CU instead (measured 4.6% faster in FP32 and 15% in FP16S on 96 x 96 x 384).
    const bool wide = wide_ok && p.storage != VCLB_FP64 && p.nx >= 96;
    t.bx = wide ? 96 : 32;
    t.by3 = 8;
    const long cols = long((p.nx + t.bx - 1) / t.bx) * ((p.ny + 7) / 8);
    const long per_cu = wide ? 1 : (p.storage == VCLB_FP16S ? 3 : 2);
    const long segs = std::max(1L, per_cu * ncu / cols);
    t.ty = int(std::max(8L, std::min(64L, (p.nz + segs - 1) / segs)));
  }
  return t;
}

int check_tile(const vclb_params& p, const vclb::Tile& t) {
  if (p.lattice == VCLB_D2Q9) {
    const bool wide = (t.bx == 512 || t.bx == 1024) && p.storage != VCLB_FP64;
    if (!((t.bx >= 64 && t.bx <= 256 && t.bx % 64 == 0) || wide) || t.ty < 1)
      return fail(VCLB_EINVAL, "bad 2D tile (bx in {64, 128, 192, 256}, or 512 and 1024 with 4-byte storage)");
  } else {
    // sections of up to 256 lanes, or 768 with 4-byte arithmetic (one workgroup per CU,
    // whose staged planes may use up to the CU's 160 KiB of LDS)
    const int max_lanes = p.storage == VCLB_FP64 ? 256 : 768;
    if (t.bx < 1 || t.by3 < 1 || t.bx * t.by3 > max_lanes || (t.bx * t.by3) % 64 != 0 || t.ty < 1)
      return fail(VCLB_EINVAL, "bad 3D tile (bx * by3 a multiple of 64, at most 256, or 768 with 4-byte storage)");
    const size_t lds = p.storage == VCLB_FP64   ? vclb::step3d_lds_bytes<vclb::StoreF64>(t.bx, t.by3)
                       : p.storage == VCLB_FP32 ? vclb::step3d_lds_bytes<vclb::StoreF32>(t.bx, t.by3)
                                                : vclb::step3d_lds_bytes<vclb::StoreF16S>(t.bx, t.by3);
    if (t.bx * t.by3 <= 256) {
      if (lds > 65536) return fail(VCLB_EINVAL, "3D tile needs more than 64 KiB of LDS");
    } else {
      // the device's own limit on one workgroup's LDS (the only HIP query of a tile check)
      int dev = 0, max_lds = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
          lds > size_t(max_lds))
        return fail(VCLB_EINVAL, "wide 3D tile needs more LDS than a workgroup may have on this device");
    }
  }
  return VCLB_OK;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

extern "C" {

const char* vclb_strerror(int code) {
  switch (code) {
    case VCLB_OK: return "ok";
    case VCLB_EINVAL: return "invalid argument";
    case VCLB_ENOMEM: return "out of device memory";
    case VCLB_EHIP: return "HIP runtime error";
    case VCLB_ENONFINITE: return "non-finite phi";
    case VCLB_ESTATE: return "invalid state";
    default: return "unknown error";
  }
}

const char* vclb_last_error(void) { return g_last_error.c_str(); }

int vclb_version(void) { return VCLB_VERSION; }

int vclb_bandwidth_probe(int32_t mode, void* dst, const void* src, size_t bytes, int32_t reps, int32_t blocks,
                         double* gbs, void* stream) {
  return vclb_bandwidth_probe_ex(mode, 1, 0, dst, src, bytes, reps, blocks, gbs, stream);
}

int vclb_bandwidth_probe_ex(int32_t mode, int32_t unroll, int32_t nontemporal, void* dst, const void* src,
                            size_t bytes, int32_t reps, int32_t blocks, double* gbs, void* stream) {
  if (mode < 0 || mode > 2) return fail(VCLB_EINVAL, "mode is 0 (copy), 1 (read) or 2 (write)");
  if (unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8) return fail(VCLB_EINVAL, "unroll is 1, 2, 4 or 8");
  if (nontemporal != 0 && nontemporal != 1) return fail(VCLB_EINVAL, "nontemporal is 0 or 1");
  if (!gbs || reps < 1 || reps > 1000 || blocks < 0) return fail(VCLB_EINVAL, "bad probe arguments");
  if (bytes == 0 || bytes % 16 != 0) return fail(VCLB_EINVAL, "bytes must be a positive multiple of 16");
  if (!dst || (mode != 2 && !src)) return fail(VCLB_EINVAL, "NULL buffer");
  if (reinterpret_cast<uintptr_t>(dst) % 16 != 0 || reinterpret_cast<uintptr_t>(src) % 16 != 0)
    return fail(VCLB_EINVAL, "buffers must be 16-byte aligned");
  hipStream_t s = as_stream(stream);
  if (blocks == 0) {
    int dev = 0, ncu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    blocks = 4 * ncu;
  }
  const long n16 = long(bytes / 16);
  if (vclb::launch_probe(mode, unroll, nontemporal, dst, src, n16, blocks, s))
    return fail(VCLB_EHIP, "probe launch failed");   // warm-up
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int rc = VCLB_OK;
  hipError_t e = hipEventRecord(e0, s);
  for (int r = 0; e == hipSuccess && rc == VCLB_OK && r < reps; ++r)
    rc = vclb::launch_probe(mode, unroll, nontemporal, dst, src, n16, blocks, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return fail(VCLB_EHIP, "probe launch failed");
  if (e != hipSuccess) return hip_fail(e, "probe timing");
  const double moved = double(bytes) * (mode == 0 ? 2.0 : 1.0) * reps;
  *gbs = ms > 0.0f ? moved / (double(ms) * 1e-3) / 1e9 : 0.0;
  return VCLB_OK;
}

int vclb_params_validate(const vclb_params* p) { return validate(p); }

int vclb_case_workspace_bytes(const vclb_params* p, size_t* bytes) {
  int rc = validate(p);
  if (rc) return rc;
  if (!bytes) return fail(VCLB_EINVAL, "bytes is NULL");
  *bytes = layout_for(*p).total;
  return VCLB_OK;
}

int vclb_case_create(const vclb_params* p, void* workspace, size_t workspace_bytes, vclb_case** out) {
  int rc = validate(p);
  if (rc) return rc;
  if (!out) return fail(VCLB_EINVAL, "out is NULL");
  *out = nullptr;
  const Layout lay = layout_for(*p);
  if (workspace && workspace_bytes < lay.total) return fail(VCLB_ENOMEM, "workspace too small");
  if (workspace && (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
    return fail(VCLB_EINVAL, "workspace must be 256-byte aligned");
  vclb_case* c = new (std::nothrow) vclb_case();
  if (!c) return fail(VCLB_ENOMEM, "host allocation");
  c->p = *p;
  fill_rates(c->p, c->sg, c->sf);
  c->lay = lay;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      ncu < 1)
    ncu = 256;
  c->tile = default_tile(c->p, ncu);
  if (check_tile(c->p, c->tile) != VCLB_OK) c->tile = default_tile(c->p, ncu, false);   // no wide 3D section here
  c->recorded.assign(vclb::kHistory, -1);
  if (workspace) {
    c->ws = static_cast<char*>(workspace);
  } else {
    void* m = nullptr;
    hipError_t e = hipMalloc(&m, lay.total);
    if (e != hipSuccess) {
      delete c;
      return fail(e == hipErrorOutOfMemory ? VCLB_ENOMEM : VCLB_EHIP, "hipMalloc of the case workspace failed");
    }
    c->ws = static_cast<char*>(m);
    c->own_ws = true;
  }
  *out = c;
  return VCLB_OK;
}

void vclb_case_destroy(vclb_case* c) {
  if (!c) return;
  adj_release(c);
  if (c->lab_scratch) (void)hipFree(c->lab_scratch);
  if (c->own_ws && c->ws) (void)hipFree(c->ws);
  delete c;
}

int vclb_case_set_tile(vclb_case* c, int32_t bx, int32_t ty, int32_t by3) {
  if (!c) return fail(VCLB_EINVAL, "case is NULL");
  vclb::Tile t;
  t.bx = bx;
  t.ty = ty;
  t.by3 = c->p.lattice == VCLB_D2Q9 ? 1 : by3;
  int rc = check_tile(c->p, t);
  if (rc) return rc;
  const long blocks = vclb::fused_blocks(lattice_d(c->p.lattice), c->p.nx, c->p.ny, c->p.nz, t);
  if (blocks > c->lay.partial_blocks) return fail(VCLB_EINVAL, "tile gives too many workgroups");
  c->tile = t;
  return VCLB_OK;
}

int vclb_case_get_tile(const vclb_case* c, int32_t* bx, int32_t* ty, int32_t* by3) {
  if (!c || !bx || !ty || !by3) return fail(VCLB_EINVAL, "NULL argument");
  *bx = c->tile.bx;
  *ty = c->tile.ty;
  *by3 = c->tile.by3;
  return VCLB_OK;
}

int vclb_case_set_reduce_every(vclb_case* c, int32_t every) {
  if (!c || every < 0) return fail(VCLB_EINVAL, "bad reduce_every");
  c->reduce_every = every;
  return VCLB_OK;
}

}  // extern "C"

namespace {
// the global volume correction's reference volume V_ref from the case's current state
int mass_reference(vclb_case* c, hipStream_t s) {
  if (!(c->p.mass_fix > 0)) return VCLB_OK;
  int rc = dispatch(*c, [&](auto dc, auto) {
    using DC = decltype(dc);
    return vclb::launch_mass_ref<typename DevTraits<DC>::L, typename DevTraits<DC>::St>(dc, s);
  });
  return rc ? fail(VCLB_EHIP, "reference volume launch failed") : VCLB_OK;
}
}  // namespace

extern "C" {

int vclb_case_init(vclb_case* c, const double* phi0, const double* u0, int ptr_kind, void* stream) {
  if (!c || !phi0) return fail(VCLB_EINVAL, "case or phi0 is NULL");
  if (ptr_kind != VCLB_HOST && ptr_kind != VCLB_DEVICE) return fail(VCLB_EINVAL, "bad ptr_kind");
  hipStream_t s = as_stream(stream);
  const size_t n = size_t(c->p.nx) * c->p.ny * c->p.nz;
  const int D = lattice_d(c->p.lattice);
  const double* dphi = phi0;
  const double* du = u0;
  void* staging = nullptr;
  if (ptr_kind == VCLB_HOST) {
    for (size_t i = 0; i < n; ++i)
      if (!std::isfinite(phi0[i])) return fail(VCLB_ENONFINITE, "phi0 has a NaN/Inf");
    const size_t bytes = n * sizeof(double) * (1 + (u0 ? D : 0));
    HIP_TRY(hipMalloc(&staging, bytes));
    double* st = static_cast<double*>(staging);
    hipError_t e = hipMemcpyAsync(st, phi0, n * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && u0) e = hipMemcpyAsync(st + n, u0, n * D * sizeof(double), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
      (void)hipFree(staging);
      return hip_fail(e, "hipMemcpyAsync of the initial fields");
    }
    dphi = st;
    du = u0 ? st + n : nullptr;
  }
  int rc = dispatch(*c, [&](auto dc, auto coupled) {
    using DC = decltype(dc);
    using L = typename DevTraits<DC>::L;
    using St = typename DevTraits<DC>::St;
    return vclb::launch_init<L, St, decltype(coupled)::value>(dc, dphi, du, s);
  });
  if (staging) {
    hipError_t e = hipStreamSynchronize(s);
    (void)hipFree(staging);
    if (e != hipSuccess) return hip_fail(e, "init");
  }
  if (rc) return fail(VCLB_EHIP, "init kernel launch failed");
  if (int rm = mass_reference(c, s)) return rm;
  c->t_host = 0;
  std::fill(c->recorded.begin(), c->recorded.end(), -1);
  c->pending = false;
  c->inited = true;
  return VCLB_OK;
}

int vclb_case_set_state(vclb_case* c, const double* g, const double* f, const double* J, int64_t t,
                        int ptr_kind, void* stream) {
  if (!c || !g || !J || t < 0) return fail(VCLB_EINVAL, "bad argument");
  if (c->p.mode == VCLB_COUPLED && !f) return fail(VCLB_EINVAL, "f is NULL in coupled mode");
  if (ptr_kind != VCLB_HOST && ptr_kind != VCLB_DEVICE) return fail(VCLB_EINVAL, "bad ptr_kind");
  hipStream_t s = as_stream(stream);
  const size_t n = size_t(c->p.nx) * c->p.ny * c->p.nz;
  const int Q = lattice_q(c->p.lattice), D = lattice_d(c->p.lattice);
  const bool coupled = c->p.mode == VCLB_COUPLED;
  const double *dg = g, *df = f, *dJ = J;
  void* staging = nullptr;
  if (ptr_kind == VCLB_HOST) {
    const size_t cnt = n * (size_t(Q) * (coupled ? 2 : 1) + D);
    HIP_TRY(hipMalloc(&staging, cnt * sizeof(double)));
    double* st = static_cast<double*>(staging);
    hipError_t e = hipMemcpyAsync(st, g, n * Q * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && coupled) e = hipMemcpyAsync(st + n * Q, f, n * Q * sizeof(double), hipMemcpyHostToDevice, s);
    const size_t jo = n * Q * (coupled ? 2 : 1);
    if (e == hipSuccess) e = hipMemcpyAsync(st + jo, J, n * D * sizeof(double), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
      (void)hipFree(staging);
      return hip_fail(e, "hipMemcpyAsync of the state");
    }
    dg = st;
    df = coupled ? st + n * Q : nullptr;
    dJ = st + jo;
  }
  int rc = dispatch(*c, [&](auto dc, auto cp) {
    using DC = decltype(dc);
    return vclb::launch_set_state<typename DevTraits<DC>::L, typename DevTraits<DC>::St, decltype(cp)::value>(
        dc, dg, df, dJ, long(t), s);
  });
  hipError_t e = hipStreamSynchronize(s);
  if (staging) (void)hipFree(staging);
  if (rc) return fail(VCLB_EHIP, "set_state launch failed");
  if (e != hipSuccess) return hip_fail(e, "set_state");
  c->t_host = t;
  if (int rm = mass_reference(c, s)) return rm;
  std::fill(c->recorded.begin(), c->recorded.end(), -1);
  c->pending = false;
  c->inited = true;
  return VCLB_OK;
}

int vclb_case_get_state(vclb_case* c, double* g, double* f, double* J, int ptr_kind, void* stream) {
  if (!c || !g || !J) return fail(VCLB_EINVAL, "bad argument");
  if (!c->inited) return fail(VCLB_ESTATE, "get_state before init");
  const bool coupled = c->p.mode == VCLB_COUPLED;
  if (coupled && !f) return fail(VCLB_EINVAL, "f is NULL in coupled mode");
  if (ptr_kind != VCLB_HOST && ptr_kind != VCLB_DEVICE) return fail(VCLB_EINVAL, "bad ptr_kind");
  hipStream_t s = as_stream(stream);
  const size_t n = size_t(c->p.nx) * c->p.ny * c->p.nz;
  const int Q = lattice_q(c->p.lattice), D = lattice_d(c->p.lattice);
  double *dg = g, *df = f, *dJ = J;
  void* staging = nullptr;
  const size_t jo = n * Q * (coupled ? 2 : 1);
  if (ptr_kind == VCLB_HOST) {
    HIP_TRY(hipMalloc(&staging, (jo + n * D) * sizeof(double)));
    double* st = static_cast<double*>(staging);
    dg = st;
    df = coupled ? st + n * Q : nullptr;
    dJ = st + jo;
  }
  int rc = dispatch(*c, [&](auto dc, auto cp) {
    using DC = decltype(dc);
    return vclb::launch_get_state<typename DevTraits<DC>::L, typename DevTraits<DC>::St, decltype(cp)::value>(
        dc, dg, df, dJ, s);
  });
  hipError_t e = hipSuccess;
  if (!rc && staging) {
    e = hipMemcpyAsync(g, dg, n * Q * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && coupled) e = hipMemcpyAsync(f, df, n * Q * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(J, dJ, n * D * sizeof(double), hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (staging) (void)hipFree(staging);
  if (rc) return fail(VCLB_EHIP, "get_state launch failed");
  if (e != hipSuccess) return hip_fail(e, "get_state");
  return VCLB_OK;
}

static int do_steps(vclb_case* c, int64_t nsteps, void* stream, bool fused) {
  if (!c) return fail(VCLB_EINVAL, "case is NULL");
  if (c->p.mass_fix > 0) fused = false;   // the global correction runs on the plain path
  if (nsteps < 0) return fail(VCLB_EINVAL, "nsteps < 0");
  if (!c->inited) return fail(VCLB_ESTATE, "step before init");
  const long blocks = fused ? vclb::fused_blocks(lattice_d(c->p.lattice), c->p.nx, c->p.ny, c->p.nz, c->tile)
                            : long((size_t(c->p.nx) * c->p.ny * c->p.nz + 255) / 256);
  if (blocks > c->lay.partial_blocks) return fail(VCLB_EINVAL, "launch shape exceeds the reduction buffer");
  hipStream_t s = as_stream(stream);
  if (!fused) {
    int rc = flush_pending(c, s);
    if (rc) return rc;
  }
  for (int64_t k = 0; k < nsteps; ++k) {
    const int64_t t = c->t_host;
    const int reduce = (c->reduce_every > 0 && t % c->reduce_every == 0) ? 1 : 0;
    int rc = dispatch(*c, [&](auto dc, auto coupled) {
      using DC = decltype(dc);
      using L = typename DevTraits<DC>::L;
      using St = typename DevTraits<DC>::St;
      constexpr bool C = decltype(coupled)::value;
      return fused ? vclb::launch_step_fused<L, St, C>(dc, c->tile, reduce, s)
                   : vclb::launch_step_plain<L, St, C>(dc, reduce, s);
    });
    if (rc) return fail(VCLB_EHIP, std::string("step kernel launch failed: ") + hipGetErrorString(hipGetLastError()));
    // the fused kernel has folded the previous pending reductions; its own are pending
    c->pending = fused && reduce;
    c->pend_nb = int(blocks);
    c->pend_buf = int(t & 1);
    c->pend_step = t;
    if (reduce) c->recorded[size_t(t % vclb::kHistory)] = t;
    c->t_host = t + 1;
  }
  return VCLB_OK;
}

int vclb_step(vclb_case* c, int64_t nsteps, void* stream) { return do_steps(c, nsteps, stream, true); }

int vclb_case_autotune(vclb_case* c, const char* cache_path, int32_t steps, void* stream) {
  if (!c || steps < 1) return fail(VCLB_EINVAL, "bad autotune arguments");
  if (!c->inited) return fail(VCLB_ESTATE, "autotune needs an initialised case (its state is restored)");
  const vclb_params& p = c->p;
  const std::string desc = "case:" + std::to_string(p.lattice) + ":" + std::to_string(p.storage) + ":" +
                           std::to_string(p.mode) + ":" + std::to_string(p.nx) + "x" + std::to_string(p.ny) + "x" +
                           std::to_string(p.nz) + (wall_y(p) ? "w" : "p") + std::to_string(std::max(1, p.nlabels));
  char key[32];
  std::snprintf(key, sizeof(key), "%016llx", static_cast<unsigned long long>(fnv1a(desc.data(), desc.size())));
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char line[4096];
      int bx = 0, ty = 0, by3 = 0;
      while (std::fgets(line, sizeof(line), f)) {
        if (!std::strstr(line, key)) continue;
        const char* pb = std::strstr(line, "\"bx\": ");
        const char* pt = std::strstr(line, "\"ty\": ");
        const char* py = std::strstr(line, "\"by3\": ");
        if (pb && pt && py) {
          bx = std::atoi(pb + 6);
          ty = std::atoi(pt + 6);
          by3 = std::atoi(py + 7);
        }
      }
      std::fclose(f);
      if (bx > 0 && ty > 0 && by3 > 0) return vclb_case_set_tile(c, bx, ty, by3);
    }
  }
  // candidates: 2D strips of bx lanes by ty rows; 3D sections of bx x by3 columns with
  // their z extent cut into as many segments as fill 1..4 workgroups per CU once
  std::vector<vclb::Tile> cands;
  if (p.lattice == VCLB_D2Q9) {
    for (int bx : {64, 128, 256, 512, 1024}) {
      if (bx > 256 && c->p.storage == VCLB_FP64) continue;
      for (int ty : {8, 16, 32, 64, 128}) cands.push_back(vclb::Tile{bx, ty, 1});
    }
  } else {
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      ncu = 256;
    const int shapes[][2] = {{32, 8}, {64, 4}, {16, 16}, {32, 4}, {64, 2}, {16, 8}, {96, 8}, {48, 16}, {64, 12}};
    for (const auto& sh : shapes)
      for (int per_cu : {1, 2, 3, 4}) {
        if (sh[0] * sh[1] > 256 && (p.storage == VCLB_FP64 || per_cu > 1)) continue;   // wide: one per CU
        const long cols = long((p.nx + sh[0] - 1) / sh[0]) * ((p.ny + sh[1] - 1) / sh[1]);
        const long segs = std::max(1L, per_cu * long(ncu) / cols);
        const int ty = int(std::max(1L, (p.nz + segs - 1) / segs));
        vclb::Tile t{sh[0], ty, sh[1]};
        bool dup = false;
        for (const vclb::Tile& u : cands) dup = dup || (u.bx == t.bx && u.ty == t.ty && u.by3 == t.by3);
        if (!dup) cands.push_back(t);
      }
  }
  hipStream_t s = as_stream(stream);
  if (int rc0 = flush_pending(c, s)) return rc0;
  HIP_TRY(hipStreamSynchronize(s));
  // the timing steps run on the live state, which is saved and restored afterwards
  void* save = nullptr;
  HIP_TRY(hipMalloc(&save, c->lay.total));
  HIP_TRY(hipMemcpyAsync(save, c->ws, c->lay.total, hipMemcpyDeviceToDevice, s));
  const vclb::Tile tile0 = c->tile;
  const int64_t t0 = c->t_host;
  const std::vector<int64_t> rec0 = c->recorded;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  std::vector<float> ms(cands.size(), -1.0f);
  int rc = VCLB_OK;
  for (size_t i = 0; i < cands.size() && e == hipSuccess && rc == VCLB_OK; ++i) {
    const vclb::Tile& t = cands[i];
    if (check_tile(p, t) != VCLB_OK) continue;   // outside the launch limits
    if (vclb::fused_blocks(lattice_d(p.lattice), p.nx, p.ny, p.nz, t) > c->lay.partial_blocks) continue;
    c->tile = t;
    if ((rc = do_steps(c, 1, stream, true))) break;
    if ((e = hipEventRecord(e0, s)) != hipSuccess) break;
    if ((rc = do_steps(c, steps, stream, true))) break;
    if ((e = hipEventRecord(e1, s)) != hipSuccess) break;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
    float m = 0;
    if ((e = hipEventElapsedTime(&m, e0, e1)) != hipSuccess) break;
    ms[i] = m / float(steps);
  }
  (void)hipStreamSynchronize(s);
  (void)hipMemcpyAsync(c->ws, save, c->lay.total, hipMemcpyDeviceToDevice, s);
  (void)hipStreamSynchronize(s);
  (void)hipFree(save);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  c->t_host = t0;
  c->recorded = rec0;
  c->pending = false;
  c->tile = tile0;
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e, "autotune timing");
  int best = -1;
  for (size_t i = 0; i < cands.size(); ++i)
    if (ms[i] > 0 && (best < 0 || ms[i] < ms[size_t(best)])) best = int(i);
  if (best < 0) return fail(VCLB_EINVAL, "no launch shape fits this case");
  c->tile = cands[size_t(best)];
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "a")) {
      const vclb::Tile& b = c->tile;
      std::fprintf(f, "{\"key\": \"%s\", \"shape\": \"%s\", \"bx\": %d, \"ty\": %d, \"by3\": %d, \"ms_per_step\": %.6f, \"candidates\": [",
                   key, desc.c_str(), b.bx, b.ty, b.by3, double(ms[size_t(best)]));
      for (size_t i = 0; i < cands.size(); ++i)
        std::fprintf(f, "%s[%d, %d, %d, %.6f]", i ? ", " : "", cands[i].bx, cands[i].ty, cands[i].by3, double(ms[i]));
      std::fprintf(f, "]}\n");
      std::fclose(f);
    }
  }
  return VCLB_OK;
}
int vclb_step_plain(vclb_case* c, int64_t nsteps, void* stream) { return do_steps(c, nsteps, stream, false); }

int vclb_case_time(vclb_case* c, int64_t* t, void* stream) {
  if (!c || !t) return fail(VCLB_EINVAL, "NULL argument");
  HIP_TRY(hipStreamSynchronize(as_stream(stream)));
  *t = c->t_host;
  return VCLB_OK;
}

int vclb_observe(vclb_case* c, uint32_t mask, double* out, int ptr_kind, void* stream) {
  if (!c || !out) return fail(VCLB_EINVAL, "NULL argument");
  if (!c->inited) return fail(VCLB_ESTATE, "observe before init");
  if (mask == 0 || (mask & ~0x3Fu)) return fail(VCLB_EINVAL, "bad field mask");
  if (ptr_kind != VCLB_HOST && ptr_kind != VCLB_DEVICE) return fail(VCLB_EINVAL, "bad ptr_kind");
  hipStream_t s = as_stream(stream);
  if (int rc0 = flush_pending(c, s)) return rc0;
  const size_t n = size_t(c->p.nx) * c->p.ny * c->p.nz;
  const int D = lattice_d(c->p.lattice);
  size_t count = 0;
  for (int b = 0; b < 6; ++b)
    if (mask & (1u << b)) count += (b == 2 ? D : 1) * n;
  double* dout = out;
  void* staging = nullptr;
  if (ptr_kind == VCLB_HOST) {
    HIP_TRY(hipMalloc(&staging, count * sizeof(double)));
    dout = static_cast<double*>(staging);
  }
  int rc = dispatch(*c, [&](auto dc, auto coupled) {
    using DC = decltype(dc);
    using L = typename DevTraits<DC>::L;
    using St = typename DevTraits<DC>::St;
    return vclb::launch_observe<L, St, decltype(coupled)::value>(dc, mask, dout, s);
  });
  hipError_t e = hipSuccess;
  if (!rc && staging) e = hipMemcpyAsync(out, dout, count * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (staging) (void)hipFree(staging);
  if (rc) return fail(VCLB_EHIP, "observe kernel launch failed");
  if (e != hipSuccess) return hip_fail(e, "observe");
  return VCLB_OK;
}

static void unpack_obs(const double* v, int nl, vclb_obs* out) {
  bool bad = false;
  for (int k = 0; k < nl; ++k) {
    const double* r = v + k * vclb::kObsFields;
    out[k].sum_phi = r[0];
    out[k].count_half = r[1];
    for (int a = 0; a < 3; ++a) out[k].sum_phi_d[a] = r[2 + a];
    for (int a = 0; a < 6; ++a) out[k].sum_phi_dd[a] = r[5 + a];
    out[k].nonfinite = r[11] > 0 ? 1 : 0;
    out[k].step = int64_t(r[12]);
    out[k].label = k;
    bad = bad || out[k].nonfinite;
  }
  (void)bad;
}

}  // extern "C"

namespace {
constexpr int32_t kMaxCallerLabels = 1 << 20;

// checks shared by the caller-label reductions
int label_args(vclb_case* c, const int32_t* labels, int32_t nlabels, vclb_obs* out) {
  if (!c || !out || !labels) return fail(VCLB_EINVAL, "NULL argument");
  if (nlabels < 1 || nlabels > kMaxCallerLabels) return fail(VCLB_EINVAL, "nlabels must lie in 1..2^20");
  if (!c->inited) return fail(VCLB_ESTATE, "reduce before init");
  return VCLB_OK;
}

// phi of the current state into the case's scratch, then the label reductions into
// `scratch` (label_scratch_bytes), results copied to out; synchronises the stream
int label_reduce_into(vclb_case* c, const int32_t* labels, int32_t nlabels, vclb_obs* out, void* scratch,
                      hipStream_t s) {
  if (int rc0 = flush_pending(c, s)) return rc0;
  const long n = long(c->p.nx) * c->p.ny * c->p.nz;
  int rc = dispatch(*c, [&](auto dc, auto) {
    using DC = decltype(dc);
    using L = typename DevTraits<DC>::L;
    using St = typename DevTraits<DC>::St;
    int r = vclb::launch_phi_psi<L, St>(dc, s);
    if (r) return r;
    return vclb::launch_label_reduce(dc.tmp_phi, labels, n, c->p.nx, c->p.ny, nlabels, long(c->t_host), scratch, s);
  });
  if (rc) return fail(VCLB_EHIP, "label reduction launch failed");
  const char* res = static_cast<const char*>(scratch) + vclb::label_result_offset(n, nlabels);
  double bad = 0.0;
  HIP_TRY(hipMemcpyAsync(out, res, size_t(nlabels) * sizeof(vclb_obs), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&bad, res + size_t(nlabels) * sizeof(vclb_obs), sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (bad > 0.0) return fail(VCLB_EINVAL, std::to_string(int64_t(bad)) + " node label(s) >= nlabels");
  for (int k = 0; k < nlabels; ++k)
    if (out[k].nonfinite) return fail(VCLB_ENONFINITE, "phi has a NaN/Inf");
  return VCLB_OK;
}
}  // namespace

extern "C" {

int vclb_reduce(vclb_case* c, const int32_t* labels, int32_t nlabels, vclb_obs* out, void* stream) {
  if (labels) {
    if (int rc = label_args(c, labels, nlabels, out)) return rc;
    const long n = long(c->p.nx) * c->p.ny * c->p.nz;
    const size_t need = vclb::label_scratch_bytes(n, nlabels);
    hipStream_t s = as_stream(stream);
    if (c->lab_scratch_bytes < need) {
      HIP_TRY(hipStreamSynchronize(s));
      if (c->lab_scratch) (void)hipFree(c->lab_scratch);
      c->lab_scratch = nullptr;
      c->lab_scratch_bytes = 0;
      if (hipMalloc(&c->lab_scratch, need) != hipSuccess) {
        c->lab_scratch = nullptr;
        return fail(VCLB_ENOMEM, "label reduction scratch");
      }
      c->lab_scratch_bytes = need;
    }
    return label_reduce_into(c, labels, nlabels, out, c->lab_scratch, s);
  }
  if (!c || !out) return fail(VCLB_EINVAL, "NULL argument");
  if (nlabels != 0 && nlabels != std::max(1, c->p.nlabels))
    return fail(VCLB_EINVAL, "with the built-in labels nlabels is 0 or the case's label count");
  if (!c->inited) return fail(VCLB_ESTATE, "reduce before init");
  hipStream_t s = as_stream(stream);
  if (int rc0 = flush_pending(c, s)) return rc0;
  int rc = dispatch(*c, [&](auto dc, auto) {
    using DC = decltype(dc);
    using L = typename DevTraits<DC>::L;
    using St = typename DevTraits<DC>::St;
    return vclb::launch_reduce_state<L, St>(dc, s);
  });
  if (rc) return fail(VCLB_EHIP, "reduce kernel launch failed");
  const int nl = std::max(1, c->p.nlabels);
  std::vector<double> v(size_t(nl) * vclb::kObsFields);
  HIP_TRY(hipMemcpyAsync(v.data(), c->ws + c->lay.cur, v.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  unpack_obs(v.data(), nl, out);
  for (int k = 0; k < nl; ++k) out[k].step = c->t_host;
  for (int k = 0; k < nl; ++k)
    if (out[k].nonfinite) return fail(VCLB_ENONFINITE, "phi has a NaN/Inf");
  return VCLB_OK;
}

int vclb_reduce_static(vclb_case* c, const int32_t* labels, int32_t nlabels, vclb_obs* out, void* stream) {
  if (int rc = label_args(c, labels, nlabels, out)) return rc;
  const long n = long(c->p.nx) * c->p.ny * c->p.nz;
  const size_t need = vclb::label_scratch_bytes(n, nlabels);
  if (need > vclb::kStaticScratchBytes)
    return fail(VCLB_EINVAL, "the label reduction needs " + std::to_string(need) + " bytes of scratch; the fixed scratch holds " +
                                 std::to_string(vclb::kStaticScratchBytes) + " (use fewer labels or vclb_reduce)");
  void* scratch = nullptr;
  const int rs = vclb::static_scratch(&scratch);
  if (rs == -1) return fail(VCLB_EINVAL, "device index beyond the fixed scratch table");
  if (rs) return fail(VCLB_EHIP, "hipGetSymbolAddress of the fixed scratch failed");
  return label_reduce_into(c, labels, nlabels, out, scratch, as_stream(stream));
}

int vclb_history(vclb_case* c, int64_t t_first, int32_t count, vclb_obs* out, void* stream) {
  if (!c || !out || count < 0 || t_first < 0) return fail(VCLB_EINVAL, "bad argument");
  if (count == 0) return VCLB_OK;
  for (int64_t t = t_first; t < t_first + count; ++t)
    if (c->recorded[size_t(t % vclb::kHistory)] != t) return fail(VCLB_ESTATE, "step not in the history");
  hipStream_t s = as_stream(stream);
  if (int rc0 = flush_pending(c, s)) return rc0;
  const int nl = std::max(1, c->p.nlabels);
  const size_t row = size_t(nl) * vclb::kObsFields;
  std::vector<double> all(size_t(vclb::kHistory) * row);
  HIP_TRY(hipMemcpyAsync(all.data(), c->ws + c->lay.hist, all.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  bool bad = false;
  for (int32_t k = 0; k < count; ++k) {
    const int64_t t = t_first + k;
    unpack_obs(all.data() + size_t(t % vclb::kHistory) * row, nl, out + size_t(k) * nl);
    for (int l = 0; l < nl; ++l) {
      if (out[size_t(k) * nl + l].step != t) return fail(VCLB_ESTATE, "history slot overwritten");
      bad = bad || out[size_t(k) * nl + l].nonfinite;
    }
  }
  if (bad) return fail(VCLB_ENONFINITE, "phi had a NaN/Inf");
  return VCLB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- checkpoints
namespace {
struct CkptHeader {
  char magic[8];
  uint32_t version, storage;
  uint64_t param_hash;
  int64_t step;
  uint64_t payload_bytes;
  uint64_t checksum;
};

struct Span { size_t off, bytes; };

std::vector<Span> state_spans(const vclb_case* c, int par) {
  const size_t n = size_t(c->p.nx) * c->p.ny * c->p.nz;
  const size_t ns = size_t(vclb::plane_stride(long(n)));   // entries per population and J plane
  const int Q = lattice_q(c->p.lattice), D = lattice_d(c->p.lattice);
  std::vector<Span> v;
  v.push_back({c->lay.pop[0][par], size_t(Q) * ns * storage_bytes(c->p.storage)});
  if (c->p.mode == VCLB_COUPLED) v.push_back({c->lay.pop[1][par], size_t(Q) * ns * storage_bytes(c->p.storage)});
  v.push_back({c->lay.J, size_t(D) * ns * arith_bytes(c->p.storage)});
  if (c->p.storage != VCLB_FP64) v.push_back({c->lay.phis[par], n * 4});
  v.push_back({c->lay.mass, sizeof(double)});   // V_ref of the global volume correction
  return v;
}

// fingerprint of the parameter values: the bytes of the struct up to nlabels and from
// wall_u on, skipping the alignment padding between them (whatever a caller left there)
uint64_t params_hash(const vclb_params& p) {
  const size_t head = offsetof(vclb_params, nlabels) + sizeof(p.nlabels);
  const size_t tail = offsetof(vclb_params, wall_u);
  static_assert(offsetof(vclb_params, wall_u) % alignof(double) == 0, "layout");
  return fnv1a(reinterpret_cast<const char*>(&p) + tail, sizeof(p) - tail, fnv1a(&p, head));
}
}  // namespace

extern "C" {

int vclb_state_bytes(const vclb_case* c, size_t* bytes) {
  if (!c || !bytes) return fail(VCLB_EINVAL, "NULL argument");
  size_t b = sizeof(CkptHeader);
  for (auto& s : state_spans(c, 0)) b += s.bytes;
  *bytes = b;
  return VCLB_OK;
}

int vclb_state_save(vclb_case* c, void* host_buf, size_t bytes, void* stream) {
  if (!c || !host_buf) return fail(VCLB_EINVAL, "NULL argument");
  if (!c->inited) return fail(VCLB_ESTATE, "save before init");
  size_t need = 0;
  vclb_state_bytes(c, &need);
  if (bytes < need) return fail(VCLB_EINVAL, "checkpoint buffer too small");
  hipStream_t s = as_stream(stream);
  const int par = int(c->t_host & 1);
  char* dst = static_cast<char*>(host_buf) + sizeof(CkptHeader);
  size_t off = 0;
  for (auto& sp : state_spans(c, par)) {
    HIP_TRY(hipMemcpyAsync(dst + off, c->ws + sp.off, sp.bytes, hipMemcpyDeviceToHost, s));
    off += sp.bytes;
  }
  HIP_TRY(hipStreamSynchronize(s));
  CkptHeader h{};
  std::memcpy(h.magic, "VCLBCKP1", 8);
  h.version = 2;   // 2: population and J planes padded to a multiple of 64 entries
  h.storage = uint32_t(c->p.storage);
  h.param_hash = params_hash(c->p);
  h.step = c->t_host;
  h.payload_bytes = off;
  h.checksum = fnv1a(dst, off);
  std::memcpy(host_buf, &h, sizeof(h));
  return VCLB_OK;
}

int vclb_state_load(vclb_case* c, const void* host_buf, size_t bytes, void* stream) {
  if (!c || !host_buf) return fail(VCLB_EINVAL, "NULL argument");
  size_t need = 0;
  vclb_state_bytes(c, &need);
  if (bytes < need) return fail(VCLB_EINVAL, "checkpoint truncated");
  CkptHeader h;
  std::memcpy(&h, host_buf, sizeof(h));
  if (std::memcmp(h.magic, "VCLBCKP1", 8) != 0 || h.version != 2) return fail(VCLB_EINVAL, "not a checkpoint of this layout");
  if (h.param_hash != params_hash(c->p)) return fail(VCLB_EINVAL, "checkpoint of a different case");
  if (h.payload_bytes != need - sizeof(CkptHeader) || h.step < 0) return fail(VCLB_EINVAL, "corrupt checkpoint header");
  const char* src = static_cast<const char*>(host_buf) + sizeof(CkptHeader);
  if (fnv1a(src, h.payload_bytes) != h.checksum) return fail(VCLB_EINVAL, "checkpoint checksum mismatch");
  hipStream_t s = as_stream(stream);
  const int par = int(h.step & 1);
  size_t off = 0;
  for (auto& sp : state_spans(c, par)) {
    HIP_TRY(hipMemcpyAsync(c->ws + sp.off, src + off, sp.bytes, hipMemcpyHostToDevice, s));
    off += sp.bytes;
  }
  HIP_TRY(hipStreamSynchronize(s));
  c->t_host = h.step;
  std::fill(c->recorded.begin(), c->recorded.end(), -1);
  c->pending = false;
  c->inited = true;
  return VCLB_OK;
}

}  // extern "C"

// ================================================================ batches
struct vclb_batch {
  int n = 0;
  int storage = 0;
  std::vector<vclb_case*> cases;
  char* ws = nullptr;
  size_t dcase_stride = 0;            // bytes per DevCase in the device table
  void* d_cases = nullptr;
  int4* d_items = nullptr;
  int2* d_case_items = nullptr;
  int2* d_runs = nullptr;             // (first item, count) per resident workgroup slot
  unsigned* d_ticks = nullptr;        // per slot: clock ticks of its run (balancing launches)
  size_t runs_cap = 0;
  double* part[2] = {nullptr, nullptr};
  size_t items_cap = 0;
  std::vector<int4> items;
  std::vector<int2> case_items;
  std::vector<int2> runs;
  int bx = 512, ty = 1024, blocks = 0, cap = 0, lag = 1, flat_pct = 100;
  // relative speed of each run slot (mean 1; empty: all equal) and the launch shape it
  // was measured with
  std::vector<double> weight;
  int wbx = 0, wty = 0, wfp = -1;
  bool ticking = false;               // launches record per-slot ticks
  int reduce_every = 1;
  bool unit = true;                   // every case has unit rates outside the g flux / f stress rows
  bool visc = false;                  // some case has unequal viscosities (per-node tau_f)
  int64_t nodes = 0;
  bool pend = false;
  int pend_buf = 0;
  int64_t pend_step = 0;
  hipStream_t own = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
};

namespace {

template <class Fn>
int dispatch_storage(int storage, Fn&& fn) {
  switch (storage) {
    case VCLB_FP64: return fn(vclb::StoreF64{});
    case VCLB_FP32: return fn(vclb::StoreF32{});
    default: return fn(vclb::StoreF16S{});
  }
}

// whether the flattened march's LDS ring for rows of nx nodes fits 64 KiB at this lag
bool flat_ring_fits(const vclb_params& p, int bx, int lag) {
  return size_t(vclb::flat_ring_cap(p.nx, bx, lag)) * 2 * arith_bytes(p.storage) <= 64 * 1024;
}

// Whether case p may run as flattened bands: when one lane per column would leave more
// than (100 - flat_pct)% of the lanes of its strips idle (strips of bx columns, each on
// a bx-lane workgroup) and its rows fit the flattened march with bx lanes (a lag of at
// most 3 chunks, and its LDS ring within 64 KiB).  Below 101 only cases that need the
// short lag (a row fits in one chunk) qualify: the long lag holds more populations in
// flight and costs the whole kernel a wave of occupancy.
bool batch_case_band_candidate(const vclb_params& p, int bx, int flat_pct) {
  const long lanes = long((p.nx + bx - 1) / bx) * bx;
  const int lag = vclb::flat_lag(p.nx, bx);
  if (lag == 0 || 100L * p.nx >= long(flat_pct) * lanes || !flat_ring_fits(p, bx, lag)) return false;
  return flat_pct > 100 || lag == 1;
}

// The lag of a batch's flattened march: the longest its band candidates need.
int batch_flat_lag(const vclb_batch* b, int bx, int flat_pct) {
  int lag = 1;
  for (const vclb_case* c : b->cases)
    if (batch_case_band_candidate(c->p, bx, flat_pct)) lag = std::max(lag, vclb::flat_lag(c->p.nx, bx));
  return lag;
}

// Whether case p runs as flattened bands in a march of this lag: a candidate whose ring
// still fits at the batch's lag (the ring of narrow rows grows with the lag).
bool batch_case_flat(const vclb_params& p, int bx, int flat_pct, int lag) {
  return batch_case_band_candidate(p, bx, flat_pct) && flat_ring_fits(p, bx, lag);
}

// Work items, case-major: flattened bands of whole rows holding about ty * 256 nodes, or
// strips of bx columns by bands of rows holding about as many nodes (strip-major, so that
// a run of items marches on down one strip).
void build_items(vclb_batch* b, int bx, int ty, int flat_pct, int lag, std::vector<int4>& items,
                 std::vector<int2>& ci) {
  items.clear();
  ci.assign(size_t(b->n), int2{0, 0});
  for (int k = 0; k < b->n; ++k) {
    const vclb_params& p = b->cases[size_t(k)]->p;
    const int first = int(items.size());
    if (batch_case_flat(p, bx, flat_pct, lag)) {
      const int P = p.nx + 2;
      const int rows = std::max(1, std::min(p.ny, (ty * 256 + P / 2) / P));
      for (int y0 = 0; y0 < p.ny; y0 += rows) items.push_back(int4{k, -1, y0, std::min(y0 + rows, p.ny)});
    } else {
      const int w = std::min(bx, (p.nx + 63) / 64 * 64);
      const int rows = std::max(4, std::min(p.ny, ty * 256 / w));
      for (int x0 = 0; x0 < p.nx; x0 += bx)
        for (int y0 = 0; y0 < p.ny; y0 += rows) items.push_back(int4{k, x0, y0, std::min(y0 + rows, p.ny)});
    }
    ci[size_t(k)] = int2{first, int(items.size()) - first};
  }
}

// Modelled cost of a work item in march iterations: a flattened band of r rows costs
// about ((r + 2) nx + 32) / bx + lag chunk iterations, a strip band r + 2 row iterations
// (both pull two halo rows); returned as a per-item overhead plus a cost per row.  A band
// row also carries one extra pull (its column -1), counted as one more node.
struct ItemCost {
  double over, row;
};
ItemCost item_cost(const vclb_batch* b, const int4& w, int bx, int lag) {
  if (w.y < 0) {
    const double nx = b->cases[size_t(w.x)]->p.nx;
    return {(2.0 * (nx + 1.0) + 32.0) / bx + lag + 0.5, (nx + 1.0) / bx};
  }
  return {2.0, 1.0};
}

// Cut the case-major item list into nb runs of consecutive items, one per resident
// workgroup slot, each with a modelled cost in proportion to its slot's weight (all
// equal when weight is empty).  An item that straddles the end of a run is split between
// rows.  The smallest budget scale that fits in nb runs is found by bisection.
void partition_runs(const vclb_batch* b, int bx, int lag, int nb, const std::vector<double>& weight,
                    std::vector<int4>& items, std::vector<int2>& ci, std::vector<int2>& runs) {
  auto wt = [&](int r) { return r < int(weight.size()) ? weight[size_t(r)] : 1.0; };
  // fn(piece, new_run) for each piece of the cut with budget scale T (run r holds at
  // most T wt(r)); returns the runs used
  auto cut = [&](double T, auto&& fn) -> int {
    int used = 0;
    bool open = false;
    double fill = 0.0, budget = 0.0;
    for (const int4& w : items) {
      const ItemCost c = item_cost(b, w, bx, lag);
      int y = w.z;
      while (y < w.w) {
        if (!open) {   // start the next run
          budget = T * wt(used);
          ++used;
          fill = 0.0;
          open = true;
        }
        const bool first = fill == 0.0;
        const int left = w.w - y;
        if (fill + c.over + left * c.row <= budget) {
          fn(int4{w.x, w.y, y, w.w}, first);
          fill += c.over + left * c.row;
          break;
        }
        int rr = int((budget - fill - c.over) / c.row);
        if (rr < 1 && !first) {   // no room left here: the next run starts with this item
          open = false;
          continue;
        }
        rr = std::max(1, std::min(rr, left));
        fn(int4{w.x, w.y, y, y + rr}, first);
        y += rr;
        open = false;   // the run is full
      }
    }
    return used;
  };
  double total = 0.0, wmin = 1.0;
  for (const int4& w : items) {
    const ItemCost c = item_cost(b, w, bx, lag);
    total += c.over + (w.w - w.z) * c.row;
  }
  for (int r = 0; r < nb; ++r) wmin = std::min(wmin, wt(r));
  double lo = 0.0, hi = (total + 1.0) / std::max(wmin, 1e-3);
  auto none = [](const int4&, bool) {};
  for (int k = 0; k < 64 && hi - lo > 1e-4 * hi; ++k) {
    const double mid = 0.5 * (lo + hi);
    if (cut(mid, none) <= nb) hi = mid;
    else lo = mid;
  }
  std::vector<int4> out;
  out.reserve(items.size() + size_t(nb));
  runs.clear();
  cut(hi, [&](const int4& w, bool fresh) {
    if (fresh) runs.push_back(int2{int(out.size()), 0});
    out.push_back(w);
    runs.back().y += 1;
  });
  runs.resize(size_t(nb), int2{int(out.size()), 0});   // spare slots take no items
  items.swap(out);
  ci.assign(size_t(b->n), int2{0, 0});
  for (size_t i = 0; i < items.size(); ++i) {
    int2& r = ci[size_t(items[i].x)];
    if (r.y == 0) r.x = int(i);
    r.y += 1;
  }
}

int batch_set_tile(vclb_batch* b, int bx, int ty, int flat_pct) {
  if (!(bx == 64 || bx == 128 || bx == 256 || bx == 512 || bx == 1024) || ty < 1 || ty > 1024 || flat_pct < 0 ||
      flat_pct > 101)
    return fail(VCLB_EINVAL, "bad batch launch shape (bx in {64, 128, 256, 512, 1024}; ty in 1..1024; flat_pct in 0..101)");
  if (bx == 1024 && b->storage == VCLB_FP64) return fail(VCLB_EINVAL, "1024-lane workgroups need FP32 or FP16S storage");
  const int lag = batch_flat_lag(b, bx, flat_pct);
  int cap = 1;
  for (const vclb_case* c : b->cases)
    if (batch_case_flat(c->p, bx, flat_pct, lag)) cap = std::max(cap, vclb::flat_ring_cap(c->p.nx, bx, lag));
  const size_t lds = dispatch_storage(b->storage, [&](auto st) { return int(vclb::batch_lds_bytes<decltype(st)>(cap, bx)); });
  if (lds > 64 * 1024) return fail(VCLB_EINVAL, "a case is too wide for the batched step with this tile");
  std::vector<int4> items;
  std::vector<int2> ci, runs;
  build_items(b, bx, ty, flat_pct, lag, items, ci);
  int per_cu = dispatch_storage(b->storage, [&](auto st) {
    return vclb::batch_max_blocks_per_cu<decltype(st)>(bx, cap, lag, b->unit, b->visc);
  });
  int dev = 0, ncu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  if (per_cu < 1) per_cu = 1;
  const int nb = int(std::min<long>(long(per_cu) * ncu, long(b->runs_cap)));
  // slot weights hold for the launch shape they were measured with
  if (b->weight.size() != size_t(nb) || b->wbx != bx || b->wty != ty || b->wfp != flat_pct) b->weight.clear();
  partition_runs(b, bx, lag, nb, b->weight, items, ci, runs);
  if (items.size() > b->items_cap) return fail(VCLB_EINVAL, "too many work items");
  HIP_TRY(hipMemcpy(b->d_items, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_case_items, ci.data(), ci.size() * sizeof(int2), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_runs, runs.data(), runs.size() * sizeof(int2), hipMemcpyHostToDevice));
  b->blocks = nb;
  b->bx = bx;
  b->ty = ty;
  b->flat_pct = flat_pct;
  b->cap = cap;
  b->lag = lag;
  b->items = std::move(items);
  b->case_items = std::move(ci);
  b->runs = std::move(runs);
  return VCLB_OK;
}

// modelled cost (march iterations) of each run slot of the current cut
std::vector<double> run_costs(const vclb_batch* b) {
  std::vector<double> cost(b->runs.size(), 0.0);
  for (size_t r = 0; r < b->runs.size(); ++r)
    for (int i = b->runs[r].x; i < b->runs[r].x + b->runs[r].y; ++i) {
      const int4& w = b->items[size_t(i)];
      const ItemCost c = item_cost(b, w, b->bx, b->lag);
      cost[r] += c.over + (w.w - w.z) * c.row;
    }
  return cost;
}

vclb::BatchArgs batch_args(const vclb_batch* b, int64_t t, int reduce) {
  vclb::BatchArgs a{};
  a.items = b->d_items;
  a.nitems = int(b->items.size());
  a.runs = b->d_runs;
  a.case_items = b->d_case_items;
  a.ncases = b->n;
  a.part_w = b->part[t & 1];
  a.part_r = b->part[b->pend_buf];
  a.pend = b->pend ? 1 : 0;
  a.pend_step = long(b->pend_step);
  a.t = long(t);
  a.reduce = reduce;
  a.cap = b->cap;
  a.lag = b->lag;
  a.unit = b->unit ? 1 : 0;
  a.visc = b->visc ? 1 : 0;
  a.ticks = b->ticking ? b->d_ticks : nullptr;
  return a;
}

// enqueue nsteps batched steps (and the closing fold) on stream s
int batch_enqueue(vclb_batch* b, int64_t nsteps, bool reduce_on, hipStream_t s) {
  const int64_t t0 = b->cases[0]->t_host;
  for (int64_t k = 0; k < nsteps; ++k) {
    const int64_t t = t0 + k;
    const int reduce = (reduce_on && b->reduce_every > 0 && t % b->reduce_every == 0) ? 1 : 0;
    const vclb::BatchArgs a = batch_args(b, t, reduce);
    int rc = dispatch_storage(b->storage, [&](auto st) {
      return vclb::launch_batch_step<decltype(st)>(b->d_cases, a, b->blocks, b->bx, s);
    });
    if (rc) return fail(VCLB_EHIP, "batched step launch failed");
    b->pend = reduce != 0;
    b->pend_buf = int(t & 1);
    b->pend_step = t;
  }
  if (b->pend) {
    const vclb::BatchArgs a = batch_args(b, t0 + nsteps, 0);
    int rc = dispatch_storage(b->storage, [&](auto st) { return vclb::launch_batch_fold<decltype(st)>(b->d_cases, a, s); });
    if (rc) return fail(VCLB_EHIP, "batched fold launch failed");
    b->pend = false;
  }
  return VCLB_OK;
}

void batch_release_graph(vclb_batch* b) {
  if (b->gexec) {
    (void)hipEventSynchronize(b->ev_out);
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
}

}  // namespace

extern "C" {

int vclb_batch_create(const vclb_params* cases, int32_t ncases, vclb_batch** out) {
  if (!cases || !out || ncases < 1) return fail(VCLB_EINVAL, "bad batch arguments");
  *out = nullptr;
  bool any_visc = false;
  for (int k = 0; k < ncases; ++k) any_visc = any_visc || visc_ratio(cases[k]);
  for (int k = 0; k < ncases; ++k) {
    int rc = validate(&cases[k]);
    if (rc) return fail(rc, "case " + std::to_string(k) + ": " + g_last_error);
    if (cases[k].lattice != VCLB_D2Q9 || cases[k].mode != VCLB_COUPLED)
      return fail(VCLB_EINVAL, "batches hold coupled D2Q9 cases");
    if (cases[k].storage != cases[0].storage) return fail(VCLB_EINVAL, "every case of a batch has one storage");
    if (cases[k].nlabels > 1) return fail(VCLB_EINVAL, "batched cases have one observation label");
    // with unequal viscosities in any case, every case relaxes its f stress rows at the
    // per-node rate of Eq. 27 (its constant tau_f when its viscosities are equal)
    if (any_visc)
      for (int r = 0; r < 9; ++r)
        if (vclb::D2Q9::f_stress_row[r] && cases[k].s_f[r] != 0.0)
          return fail(VCLB_EINVAL, "case " + std::to_string(k) +
                                       ": in a batch with unequal viscosities the f stress rates follow Eq. 27 per "
                                       "node: leave them 0");
    if (cases[k].mass_fix > 0) return fail(VCLB_EINVAL, "batched cases take no global volume correction");
    if (double(cases[k].nx + 2) * (cases[k].ny + 2) >= double(1 << 24))
      return fail(VCLB_EINVAL, "batched cases hold fewer than 2^24 padded nodes");
  }
  vclb_batch* b = new (std::nothrow) vclb_batch();
  if (!b) return fail(VCLB_ENOMEM, "host allocation");
  b->n = ncases;
  b->storage = cases[0].storage;
  // the kernel indexes the table as an array of DevCase: the stride is exactly its size
  b->dcase_stride = size_t(dispatch_storage(b->storage, [&](auto st) {
    return int(sizeof(vclb::DevCase<vclb::D2Q9, decltype(st)>));
  }));
  size_t total = 0;
  std::vector<size_t> off(static_cast<size_t>(ncases), 0);
  size_t cap = 0;
  for (int k = 0; k < ncases; ++k) {
    off[size_t(k)] = total;
    total += align_up(layout_for(cases[k]).total);
    cap += size_t(cases[k].ny) * size_t((cases[k].nx + 63) / 64);   // at most one item per row and strip
    b->nodes += int64_t(cases[k].nx) * cases[k].ny;
  }
  const size_t o_cases = total;
  total += align_up(b->dcase_stride * size_t(ncases));
  const size_t runs_cap = 16384;   // resident workgroups: CUs x workgroups per CU
  cap += runs_cap;                  // each run end may split one item
  const size_t o_items = total;
  total += align_up(cap * sizeof(int4));
  const size_t o_ci = total;
  total += align_up(size_t(ncases) * sizeof(int2));
  const size_t o_runs = total;
  total += align_up(runs_cap * sizeof(int2));
  const size_t o_ticks = total;
  total += align_up(runs_cap * sizeof(unsigned));
  size_t o_part[2];
  for (int i = 0; i < 2; ++i) {
    o_part[i] = total;
    total += align_up(cap * 12 * sizeof(double));
  }
  void* m = nullptr;
  hipError_t e = hipMalloc(&m, total);
  if (e != hipSuccess) {
    delete b;
    return fail(e == hipErrorOutOfMemory ? VCLB_ENOMEM : VCLB_EHIP, "hipMalloc of the batch workspace failed");
  }
  b->ws = static_cast<char*>(m);
  b->items_cap = cap;
  b->d_cases = b->ws + o_cases;
  b->d_items = reinterpret_cast<int4*>(b->ws + o_items);
  b->d_case_items = reinterpret_cast<int2*>(b->ws + o_ci);
  b->d_runs = reinterpret_cast<int2*>(b->ws + o_runs);
  b->d_ticks = reinterpret_cast<unsigned*>(b->ws + o_ticks);
  b->runs_cap = runs_cap;
  for (int i = 0; i < 2; ++i) b->part[i] = reinterpret_cast<double*>(b->ws + o_part[i]);
  for (int k = 0; k < ncases; ++k) {
    vclb_case* c = nullptr;
    int rc = vclb_case_create(&cases[k], b->ws + off[size_t(k)], layout_for(cases[k]).total, &c);
    if (rc) {
      vclb_batch_destroy(b);
      return rc;
    }
    b->cases.push_back(c);
  }
  // device table of per-case descriptors (pointers and constants; the step index and the
  // partial-sum buffers are batch arguments)
  std::vector<char> table(b->dcase_stride * size_t(ncases));
  const int layout_rc = dispatch_storage(b->storage, [&](auto st) {
    using St = decltype(st);
    for (int k = 0; k < ncases; ++k) {
      auto d = make_dev<vclb::D2Q9, St>(*b->cases[size_t(k)]);
      b->unit = b->unit && d.unit_rates != 0;
      b->visc = b->visc || d.visc != 0;
      std::memcpy(table.data() + b->dcase_stride * size_t(k), &d, sizeof(d));
    }
    // the device reads entry k as cases[k]: check that indexing the table that way finds
    // each case's own buffers
    const auto* arr = reinterpret_cast<const vclb::DevCase<vclb::D2Q9, St>*>(table.data());
    for (int k = 0; k < ncases; ++k)
      if (static_cast<const void*>(arr[k].pop[0][0]) != b->cases[size_t(k)]->ws + b->cases[size_t(k)]->lay.pop[0][0])
        return -1;
    return 0;
  });
  if (layout_rc) {
    vclb_batch_destroy(b);
    return fail(VCLB_EINVAL, "internal: case table layout");
  }
  e = hipMemcpy(b->d_cases, table.data(), table.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
  if (e != hipSuccess) {
    vclb_batch_destroy(b);
    return hip_fail(e, "batch set-up");
  }
  int rc = batch_set_tile(b, 512, 1024, 100);   // whole-case items, 512-lane workgroups
  if (rc) {
    vclb_batch_destroy(b);
    return rc;
  }
  *out = b;
  return VCLB_OK;
}

void vclb_batch_destroy(vclb_batch* b) {
  if (!b) return;
  batch_release_graph(b);
  for (vclb_case* c : b->cases) vclb_case_destroy(c);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->own) (void)hipStreamDestroy(b->own);
  if (b->ws) (void)hipFree(b->ws);
  delete b;
}

int vclb_batch_case(vclb_batch* b, int32_t k, vclb_case** out) {
  if (!b || !out || k < 0 || k >= b->n) return fail(VCLB_EINVAL, "bad case index");
  *out = b->cases[size_t(k)];
  return VCLB_OK;
}

int vclb_batch_init(vclb_batch* b, const double* const* phi0s, const double* const* u0s, int ptr_kind,
                    void* stream) {
  if (!b || !phi0s) return fail(VCLB_EINVAL, "batch or phi0s is NULL");
  if (ptr_kind != VCLB_HOST && ptr_kind != VCLB_DEVICE) return fail(VCLB_EINVAL, "bad ptr_kind");
  for (int k = 0; k < b->n; ++k)
    if (!phi0s[k]) return fail(VCLB_EINVAL, "phi0 of case " + std::to_string(k) + " is NULL");
  for (int k = 0; k < b->n; ++k) {
    const int rc = vclb_case_init(b->cases[size_t(k)], phi0s[k], u0s ? u0s[k] : nullptr, ptr_kind, stream);
    if (rc) return fail(rc, "case " + std::to_string(k) + ": " + g_last_error);
  }
  return VCLB_OK;
}

int vclb_batch_nodes(const vclb_batch* b, int64_t* nodes) {
  if (!b || !nodes) return fail(VCLB_EINVAL, "NULL argument");
  *nodes = b->nodes;
  return VCLB_OK;
}

int vclb_batch_set_tile(vclb_batch* b, int32_t bx, int32_t ty) {
  if (!b) return fail(VCLB_EINVAL, "batch is NULL");
  batch_release_graph(b);
  return batch_set_tile(b, bx, ty, b->flat_pct);
}

int vclb_batch_get_tile(const vclb_batch* b, int32_t* bx, int32_t* ty, int32_t* blocks) {
  if (!b || !bx || !ty || !blocks) return fail(VCLB_EINVAL, "NULL argument");
  *bx = b->bx;
  *ty = b->ty;
  *blocks = b->blocks;
  return VCLB_OK;
}

int vclb_batch_set_schedule(vclb_batch* b, int32_t flat_pct) {
  if (!b) return fail(VCLB_EINVAL, "batch is NULL");
  batch_release_graph(b);
  return batch_set_tile(b, b->bx, b->ty, flat_pct);
}

int vclb_batch_get_schedule(const vclb_batch* b, int32_t* flat_pct) {
  if (!b || !flat_pct) return fail(VCLB_EINVAL, "NULL argument");
  *flat_pct = b->flat_pct;
  return VCLB_OK;
}

int vclb_batch_set_reduce_every(vclb_batch* b, int32_t every) {
  if (!b || every < 0) return fail(VCLB_EINVAL, "bad reduce_every");
  b->reduce_every = every;
  return VCLB_OK;
}

int vclb_batch_reduce(vclb_batch* b, vclb_obs* out, void* stream) {
  if (!b || !out) return fail(VCLB_EINVAL, "NULL argument");
  for (vclb_case* c : b->cases)
    if (!c->inited) return fail(VCLB_ESTATE, "reduce before every case is initialised");
  hipStream_t s = as_stream(stream);
  const size_t row = size_t(VCLB_MAX_LABELS) * vclb::kObsFields;
  std::vector<double> v(size_t(b->n) * row, 0.0);
  for (int k = 0; k < b->n; ++k) {
    vclb_case* c = b->cases[size_t(k)];
    if (int rc0 = flush_pending(c, s)) return rc0;
    const int rc = dispatch(*c, [&](auto dc, auto) {
      using DC = decltype(dc);
      return vclb::launch_reduce_state<typename DevTraits<DC>::L, typename DevTraits<DC>::St>(dc, s);
    });
    if (rc) return fail(VCLB_EHIP, "reduce kernel launch failed");
    const int nl = std::max(1, c->p.nlabels);
    HIP_TRY(hipMemcpyAsync(v.data() + size_t(k) * row, c->ws + c->lay.cur, size_t(nl) * vclb::kObsFields * sizeof(double),
                           hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  bool bad = false;
  for (int k = 0; k < b->n; ++k) {
    const vclb_case* c = b->cases[size_t(k)];
    const int nl = std::max(1, c->p.nlabels);
    vclb_obs* o = out + size_t(k) * VCLB_MAX_LABELS;
    std::memset(o, 0, sizeof(vclb_obs) * VCLB_MAX_LABELS);
    unpack_obs(v.data() + size_t(k) * row, nl, o);
    for (int l = 0; l < VCLB_MAX_LABELS; ++l) {
      o[l].step = c->t_host;
      o[l].label = l;
      bad = bad || o[l].nonfinite;
    }
  }
  if (bad) return fail(VCLB_ENONFINITE, "phi has a NaN/Inf");
  return VCLB_OK;
}

int vclb_batch_history(vclb_batch* b, int64_t t_first, int32_t count, vclb_obs* out, void* stream) {
  if (!b || !out || count < 0 || t_first < 0) return fail(VCLB_EINVAL, "bad argument");
  if (count > vclb::kHistory) return fail(VCLB_EINVAL, "count exceeds the history length");
  if (count == 0) return VCLB_OK;
  for (vclb_case* c : b->cases)
    for (int64_t t = t_first; t < t_first + count; ++t)
      if (c->recorded[size_t(t % vclb::kHistory)] != t) return fail(VCLB_ESTATE, "step not in the history");
  hipStream_t s = as_stream(stream);
  // per case, its slots of the device ring in step order (at most two copies: the ring wraps)
  std::vector<std::vector<double>> rows(size_t(b->n));
  for (int k = 0; k < b->n; ++k) {
    vclb_case* c = b->cases[size_t(k)];
    if (int rc0 = flush_pending(c, s)) return rc0;
    const size_t drow = size_t(std::max(1, c->p.nlabels)) * vclb::kObsFields;
    rows[size_t(k)].resize(size_t(count) * drow);
    for (int32_t j = 0; j < count;) {
      const int64_t slot = (t_first + j) % vclb::kHistory;
      const int32_t run = int32_t(std::min<int64_t>(count - j, vclb::kHistory - slot));
      HIP_TRY(hipMemcpyAsync(rows[size_t(k)].data() + size_t(j) * drow,
                             c->ws + c->lay.hist + size_t(slot) * drow * sizeof(double), size_t(run) * drow * sizeof(double),
                             hipMemcpyDeviceToHost, s));
      j += run;
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  bool bad = false;
  for (int32_t j = 0; j < count; ++j)
    for (int k = 0; k < b->n; ++k) {
      const vclb_case* c = b->cases[size_t(k)];
      const int nl = std::max(1, c->p.nlabels);
      vclb_obs* o = out + (size_t(j) * b->n + k) * VCLB_MAX_LABELS;
      std::memset(o, 0, sizeof(vclb_obs) * VCLB_MAX_LABELS);
      unpack_obs(rows[size_t(k)].data() + size_t(j) * nl * vclb::kObsFields, nl, o);
      for (int l = 0; l < nl; ++l) {
        if (o[l].step != t_first + j) return fail(VCLB_ESTATE, "history slot overwritten");
        bad = bad || o[l].nonfinite;
      }
      for (int l = nl; l < VCLB_MAX_LABELS; ++l) {
        o[l].step = t_first + j;
        o[l].label = l;
      }
    }
  if (bad) return fail(VCLB_ENONFINITE, "phi had a NaN/Inf");
  return VCLB_OK;
}

int vclb_batch_step(vclb_batch* b, int64_t nsteps, int32_t use_graph, void* stream) {
  if (!b || nsteps < 0) return fail(VCLB_EINVAL, "bad batch step arguments");
  const int64_t t0 = b->cases[0]->t_host;
  for (vclb_case* c : b->cases) {
    if (!c->inited) return fail(VCLB_ESTATE, "batch step before every case is initialised");
    if (c->t_host != t0) return fail(VCLB_ESTATE, "batched cases are at different steps");
    if (c->pending) return fail(VCLB_ESTATE, "a case has pending single-case reductions");
  }
  if (nsteps == 0) return VCLB_OK;
  hipStream_t s = as_stream(stream);
  batch_release_graph(b);
  int rc;
  if (use_graph) {
    // capture on the library's own stream, ordered after the caller's stream by events
    HIP_TRY(hipEventRecord(b->ev_in, s));
    HIP_TRY(hipStreamWaitEvent(b->own, b->ev_in, 0));
    HIP_TRY(hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal));
    rc = batch_enqueue(b, nsteps, true, b->own);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->own, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
    HIP_TRY(hipGraphLaunch(b->gexec, b->own));
    HIP_TRY(hipEventRecord(b->ev_out, b->own));
    HIP_TRY(hipStreamWaitEvent(s, b->ev_out, 0));
  } else {
    rc = batch_enqueue(b, nsteps, true, s);
    if (rc) return rc;
  }
  for (vclb_case* c : b->cases) {
    for (int64_t t = t0; t < t0 + nsteps; ++t)
      if (b->reduce_every > 0 && t % b->reduce_every == 0) c->recorded[size_t(t % vclb::kHistory)] = t;
    c->t_host = t0 + nsteps;
  }
  return VCLB_OK;
}

int vclb_batch_balance(vclb_batch* b, int32_t rounds, int32_t steps, double* gain, void* stream) {
  if (!b || rounds < 1 || rounds > 16 || steps < 1 || steps > 1000) return fail(VCLB_EINVAL, "bad balance arguments");
  if (gain) *gain = 1.0;
  for (vclb_case* c : b->cases)
    if (!c->inited) return fail(VCLB_ESTATE, "balance needs initialised cases (their state is restored)");
  hipStream_t s = as_stream(stream);
  batch_release_graph(b);
  HIP_TRY(hipStreamSynchronize(s));
  size_t bytes = 0;
  for (vclb_case* c : b->cases) bytes += c->lay.total;
  void* save = nullptr;
  HIP_TRY(hipMalloc(&save, bytes));
  size_t o = 0;
  for (vclb_case* c : b->cases) {
    HIP_TRY(hipMemcpyAsync(static_cast<char*>(save) + o, c->ws, c->lay.total, hipMemcpyDeviceToDevice, s));
    o += c->lay.total;
  }
  const int64_t t0 = b->cases[0]->t_host;
  int64_t t = t0;
  const int nb = b->blocks;
  std::vector<unsigned> tk(size_t(nb), 0u);
  // steps + 1 launches with per-slot ticks (the first not counted): each slot's mean
  // ticks, and the mean over launches of the slowest slot's
  auto measure = [&](std::vector<double>& mean, double& span) -> int {
    mean.assign(size_t(nb), 0.0);
    span = 0.0;
    for (int k = 0; k <= steps; ++k) {
      for (vclb_case* c : b->cases) c->t_host = t;
      b->ticking = true;
      const int rc = batch_enqueue(b, 1, false, s);
      b->ticking = false;
      if (rc) return rc;
      ++t;
      HIP_TRY(hipMemcpyAsync(tk.data(), b->d_ticks, size_t(nb) * sizeof(unsigned), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (k == 0) continue;
      unsigned mx = 0;
      for (int r = 0; r < nb; ++r) {
        mean[size_t(r)] += double(tk[size_t(r)]) / steps;
        mx = std::max(mx, tk[size_t(r)]);
      }
      span += double(mx) / steps;
    }
    return VCLB_OK;
  };
  std::vector<double> mean, best_w = b->weight;
  double span = 0.0, best = 0.0, first = 0.0;
  int rc = measure(mean, best);
  first = best;
  for (int round = 0; rc == VCLB_OK && round < rounds; ++round) {
    // a slot's speed: the modelled cost of its run over the time it took
    const std::vector<double> cost = run_costs(b);
    std::vector<double> w(size_t(nb), 0.0);
    double sum = 0.0;
    int cnt = 0;
    for (int r = 0; r < nb; ++r)
      if (cost[size_t(r)] > 0.0 && mean[size_t(r)] > 0.0) {
        w[size_t(r)] = cost[size_t(r)] / mean[size_t(r)];
        sum += w[size_t(r)];
        ++cnt;
      }
    if (cnt == 0) break;
    for (double& x : w) x = x > 0.0 ? x * cnt / sum : 1.0;
    b->weight = w;
    b->wbx = b->bx;
    b->wty = b->ty;
    b->wfp = b->flat_pct;
    if ((rc = batch_set_tile(b, b->bx, b->ty, b->flat_pct))) break;
    if ((rc = measure(mean, span))) break;
    if (span < best) {
      best = span;
      best_w = w;
    }
  }
  o = 0;
  for (vclb_case* c : b->cases) {
    (void)hipMemcpyAsync(c->ws, static_cast<char*>(save) + o, c->lay.total, hipMemcpyDeviceToDevice, s);
    c->t_host = t0;
    o += c->lay.total;
  }
  (void)hipStreamSynchronize(s);
  (void)hipFree(save);
  if (rc) {
    b->weight.clear();
    (void)batch_set_tile(b, b->bx, b->ty, b->flat_pct);
    return rc;
  }
  // keep the fastest cut seen (the uniform one if no weighting beat it)
  b->weight = best_w;
  if ((rc = batch_set_tile(b, b->bx, b->ty, b->flat_pct))) return rc;
  if (gain && best > 0.0) *gain = first / best;
  return VCLB_OK;
}

int vclb_batch_get_weights(const vclb_batch* b, double* weights, int32_t capacity, int32_t* count) {
  if (!b || !count || capacity < 0 || (capacity > 0 && !weights)) return fail(VCLB_EINVAL, "bad arguments");
  *count = b->blocks;
  for (int r = 0; r < std::min(capacity, b->blocks); ++r)
    weights[r] = b->weight.empty() ? 1.0 : b->weight[size_t(r)];
  return VCLB_OK;
}

int vclb_batch_set_weights(vclb_batch* b, const double* weights, int32_t count) {
  if (!b || count < 0 || (count > 0 && !weights)) return fail(VCLB_EINVAL, "bad arguments");
  if (count != 0 && count != b->blocks) return fail(VCLB_EINVAL, "one weight per run slot (see vclb_batch_get_tile)");
  for (int r = 0; r < count; ++r)
    if (!(weights[r] >= 1e-3 && weights[r] <= 1e3)) return fail(VCLB_EINVAL, "weights must lie in [1e-3, 1e3]");
  batch_release_graph(b);
  b->weight.assign(weights, weights + count);
  if (count) {
    double sum = 0.0;
    for (double w : b->weight) sum += w;
    for (double& w : b->weight) w *= count / sum;   // mean 1
  }
  b->wbx = b->bx;
  b->wty = b->ty;
  b->wfp = b->flat_pct;
  return batch_set_tile(b, b->bx, b->ty, b->flat_pct);
}

int vclb_batch_autotune(vclb_batch* b, const char* cache_path, int32_t steps, void* stream) {
  if (!b || steps < 1) return fail(VCLB_EINVAL, "bad autotune arguments");
  for (vclb_case* c : b->cases)
    if (!c->inited) return fail(VCLB_ESTATE, "autotune needs initialised cases (their state is restored)");
  // key: storage and every case's shape and boundary
  std::string desc = "s" + std::to_string(b->storage);
  for (vclb_case* c : b->cases)
    desc += ":" + std::to_string(c->p.nx) + "x" + std::to_string(c->p.ny) + (wall_y(c->p) ? "w" : "p");
  char key[32];
  std::snprintf(key, sizeof(key), "%016llx", static_cast<unsigned long long>(fnv1a(desc.data(), desc.size())));
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char line[4096];
      int bx = 0, ty = 0, fp = -1;
      while (std::fgets(line, sizeof(line), f)) {
        if (!std::strstr(line, key)) continue;
        const char* pb = std::strstr(line, "\"bx\": ");
        const char* pt = std::strstr(line, "\"ty\": ");
        const char* pf = std::strstr(line, "\"flat_pct\": ");
        if (pb && pt && pf) {
          bx = std::atoi(pb + 6);
          ty = std::atoi(pt + 6);
          fp = std::atoi(pf + 12);
        }
      }
      std::fclose(f);
      if (bx > 0 && ty > 0 && fp >= 0) {
        batch_release_graph(b);
        return batch_set_tile(b, bx, ty, fp);
      }
    }
  }
  hipStream_t s = as_stream(stream);
  batch_release_graph(b);
  HIP_TRY(hipStreamSynchronize(s));
  // save every case's device state; the timing steps run on it and it is restored after
  size_t bytes = 0;
  for (vclb_case* c : b->cases) bytes += c->lay.total;
  void* save = nullptr;
  HIP_TRY(hipMalloc(&save, bytes));
  size_t o = 0;
  for (vclb_case* c : b->cases) {
    HIP_TRY(hipMemcpyAsync(static_cast<char*>(save) + o, c->ws, c->lay.total, hipMemcpyDeviceToDevice, s));
    o += c->lay.total;
  }
  const int64_t t0 = b->cases[0]->t_host;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  struct Cand { int bx, ty, fp; float ms; };
  std::vector<Cand> cands;
  for (int fp : {0, 90, 100, 101})
    for (int bx : {64, 128, 256, 512, 1024})
      for (int ty : {8, 16, 32, 64, 1024}) cands.push_back({bx, ty, fp, -1.0f});
  int rc = VCLB_OK;
  // one warm-up step, then `n` timed steps of the current shape: ms per step
  auto time_shape = [&](int n, float& out) -> int {
    if (int r = batch_enqueue(b, 1, false, s)) return r;
    HIP_TRY(hipEventRecord(e0, s));
    for (vclb_case* c : b->cases) c->t_host = t0 + 1;
    if (int r = batch_enqueue(b, n, false, s)) return r;
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    out = ms / float(n);
    for (vclb_case* c : b->cases) c->t_host = t0;
    return VCLB_OK;
  };
  for (Cand& cd : cands) {
    if (batch_set_tile(b, cd.bx, cd.ty, cd.fp) == VCLB_EINVAL) continue;   // shape not valid for these cases
    if ((rc = time_shape(steps, cd.ms))) break;
  }
  // the leading shapes are often within timing noise of each other: time the best four
  // again, three times each in alternation with twice the steps, and keep each one's fastest
  std::vector<size_t> order;
  for (size_t i = 0; i < cands.size(); ++i)
    if (cands[i].ms > 0) order.push_back(i);
  std::sort(order.begin(), order.end(), [&](size_t a, size_t c) { return cands[a].ms < cands[c].ms; });
  if (order.size() > 4) order.resize(4);
  for (int pass = 0; rc == VCLB_OK && order.size() > 1 && pass < 3; ++pass)
    for (size_t i : order) {
      Cand& cd = cands[i];
      if ((rc = batch_set_tile(b, cd.bx, cd.ty, cd.fp))) break;
      float ms = 0;
      if ((rc = time_shape(2 * steps, ms))) break;
      cd.ms = std::min(cd.ms, ms);
    }
  o = 0;
  for (vclb_case* c : b->cases) {
    (void)hipMemcpyAsync(c->ws, static_cast<char*>(save) + o, c->lay.total, hipMemcpyDeviceToDevice, s);
    c->t_host = t0;
    o += c->lay.total;
  }
  (void)hipStreamSynchronize(s);
  (void)hipFree(save);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  Cand best{0, 0, 0, -1.0f};
  for (const Cand& cd : cands)
    if (cd.ms > 0 && (best.ms < 0 || cd.ms < best.ms)) best = cd;
  if (best.ms < 0) return fail(VCLB_EINVAL, "no batched launch shape fits these cases");
  rc = batch_set_tile(b, best.bx, best.ty, best.fp);
  if (rc) return rc;
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "a")) {
      std::fprintf(f, "{\"key\": \"%s\", \"cases\": %d, \"storage\": %d, \"bx\": %d, \"ty\": %d, \"flat_pct\": %d, \"ms_per_step\": %.6f, \"candidates\": [",
                   key, b->n, b->storage, best.bx, best.ty, best.fp, double(best.ms));
      for (size_t i = 0; i < cands.size(); ++i)
        std::fprintf(f, "%s[%d, %d, %d, %.6f]", i ? ", " : "", cands[i].bx, cands[i].ty, cands[i].fp, double(cands[i].ms));
      std::fprintf(f, "]}\n");
      std::fclose(f);
    }
  }
  return VCLB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- adjoint
// Device memory of one recorded forward pass: the initial fields, a state (g, f, Jprev:
// 20 N doubles) every `every` steps, room for the `every` states of the segment being
// recomputed, and the fields of the backward sweep.
struct AdjStore {
  char* mem = nullptr;
  int64_t nsteps = 0;
  int32_t every = 1;
  int64_t nckpt = 0;
  bool has_u0 = false;
  size_t n = 0, state = 0;   // nodes, doubles per state
  size_t phi0 = 0, u0 = 0, ckpt = 0, seg = 0, lg[2]{}, lf[2]{}, lJ[2]{}, lphi = 0, aux = 0, part = 0,
         seed = 0, out = 0, dphi = 0, total = 0;
  long blocks = 0;
};

namespace {

void adj_release(vclb_case* c) {
  if (!c->adj) return;
  if (c->adj->mem) (void)hipFree(c->adj->mem);
  delete c->adj;
  c->adj = nullptr;
}

int32_t adj_default_every(int64_t nsteps) {
  if (nsteps <= 1) return 1;
  return int32_t(std::ceil(std::sqrt(double(nsteps))));
}

AdjStore adj_layout(const vclb_params& p, int64_t nsteps, int32_t every) {
  AdjStore a;
  a.nsteps = nsteps;
  a.every = every;
  a.nckpt = nsteps > 0 ? (nsteps + every - 1) / every : 0;
  a.n = size_t(p.nx) * p.ny;
  a.state = 20 * size_t(vclb::plane_stride(long(a.n)));   // g, f, J in the case's padded planes
  a.blocks = vclb::adj_blocks(long(a.n));
  size_t off = 0;
  auto take = [&](size_t doubles) {
    const size_t o = off;
    off = align_up(off + doubles * sizeof(double));
    return o;
  };
  a.phi0 = take(a.n);
  a.u0 = take(2 * a.n);
  a.ckpt = take(size_t(a.nckpt) * a.state);
  a.seg = take(size_t(std::min<int64_t>(every, std::max<int64_t>(nsteps, 1))) * a.state);
  for (int b = 0; b < 2; ++b) {
    a.lg[b] = take(9 * a.n);
    a.lf[b] = take(9 * a.n);
    a.lJ[b] = take(2 * a.n);
  }
  a.lphi = take(a.n);
  a.aux = take(6 * a.n);
  a.part = take(2 * size_t(a.blocks));
  a.seed = take(size_t(vclb::kMaxLabels) * vclb::kSeedFields);
  a.out = take(2);
  a.dphi = take(a.n);
  a.total = off;
  return a;
}

int adj_check_case(const vclb_case* c) {
  if (c->p.lattice != VCLB_D2Q9 || c->p.storage != VCLB_FP64 || c->p.mode != VCLB_COUPLED)
    return fail(VCLB_EINVAL, "the adjoint covers FP64 D2Q9 coupled cases");
  if (c->p.mass_fix > 0) return fail(VCLB_EINVAL, "the adjoint covers cases without the global volume correction");
  return VCLB_OK;
}

// copy the case's current state (pulled populations of the current parity, Jprev)
int adj_save_state(vclb_case* c, double* dst, hipStream_t s) {
  const size_t ns = size_t(vclb::plane_stride(long(c->adj->n)));   // the case's plane stride
  const int par = int(c->t_host & 1);
  HIP_TRY(hipMemcpyAsync(dst, c->ws + c->lay.pop[0][par], 9 * ns * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(dst + 9 * ns, c->ws + c->lay.pop[1][par], 9 * ns * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(dst + 18 * ns, c->ws + c->lay.J, 2 * ns * sizeof(double), hipMemcpyDeviceToDevice, s));
  return VCLB_OK;
}

// derived observables of one label and their gradients with respect to the moments
// m = (sum, d[3], dd[6]): volume, centroid offset (3), deformation D of the in-plane
// second-moment tensor about the centroid
void derived_with_grad(const vclb_obs& o, double out[5], double grad[5][vclb::kSeedFields]) {
  for (int k = 0; k < 5; ++k)
    for (int j = 0; j < vclb::kSeedFields; ++j) grad[k][j] = 0.0;
  const double V = o.sum_phi;
  const double cx = o.sum_phi_d[0] / V, cy = o.sum_phi_d[1] / V, cz = o.sum_phi_d[2] / V;
  out[0] = V;
  out[1] = cx;
  out[2] = cy;
  out[3] = cz;
  grad[0][0] = 1.0;
  for (int a = 0; a < 3; ++a) {
    grad[1 + a][0] = -o.sum_phi_d[a] / (V * V);
    grad[1 + a][1 + a] = 1.0 / V;
  }
  const double dxx = o.sum_phi_dd[0] / V, dyy = o.sum_phi_dd[1] / V, dxy = o.sum_phi_dd[3] / V;
  const double ixx = dxx - cx * cx, iyy = dyy - cy * cy, ixy = dxy - cx * cy;
  // d(ixx, iyy, ixy)/dm over the entries m0, m1 (x), m2 (y), m4 (xx), m5 (yy), m7 (xy)
  double gi[3][vclb::kSeedFields] = {};
  gi[0][0] = (-dxx + 2.0 * cx * cx) / V;
  gi[0][1] = -2.0 * cx / V;
  gi[0][4] = 1.0 / V;
  gi[1][0] = (-dyy + 2.0 * cy * cy) / V;
  gi[1][2] = -2.0 * cy / V;
  gi[1][5] = 1.0 / V;
  gi[2][0] = (-dxy + 2.0 * cx * cy) / V;
  gi[2][1] = -cy / V;
  gi[2][2] = -cx / V;
  gi[2][7] = 1.0 / V;
  const double half = 0.5 * (ixx - iyy);
  const double disc = std::sqrt(half * half + ixy * ixy);
  const double lp = 0.5 * (ixx + iyy) + disc, lm = 0.5 * (ixx + iyy) - disc;
  const double a = std::sqrt(lp), b = std::sqrt(lm);
  out[4] = (a - b) / (a + b);
  // dD/dl+ = b / (a (a + b)^2), dD/dl- = -a / (b (a + b)^2); at a circle (disc = 0) the
  // one-sided derivatives differ and the terms in half/disc, ixy/disc are dropped
  const double s2 = (a + b) * (a + b);
  const double dlp = b / (a * s2), dlm = -a / (b * s2);
  const double hx = disc > 0.0 ? half / (2.0 * disc) : 0.0, hy = disc > 0.0 ? ixy / disc : 0.0;
  const double dIxx = dlp * (0.5 + hx) + dlm * (0.5 - hx);
  const double dIyy = dlp * (0.5 - hx) + dlm * (0.5 + hx);
  const double dIxy = dlp * hy - dlm * hy;
  for (int j = 0; j < vclb::kSeedFields; ++j) grad[4][j] = dIxx * gi[0][j] + dIyy * gi[1][j] + dIxy * gi[2][j];
}

}  // namespace

extern "C" {

int vclb_adjoint_bytes(const vclb_params* p, int64_t nsteps, int32_t every, size_t* bytes) {
  int rc = validate(p);
  if (rc) return rc;
  if (!bytes || nsteps < 0 || every < 0) return fail(VCLB_EINVAL, "bad argument");
  if (p->lattice != VCLB_D2Q9 || p->storage != VCLB_FP64 || p->mode != VCLB_COUPLED)
    return fail(VCLB_EINVAL, "the adjoint covers FP64 D2Q9 coupled cases");
  if (p->mass_fix > 0) return fail(VCLB_EINVAL, "the adjoint covers cases without the global volume correction");
  if (every == 0) every = adj_default_every(nsteps);
  *bytes = adj_layout(*p, nsteps, every).total;
  return VCLB_OK;
}

int vclb_adjoint_record(vclb_case* c, const double* phi0, const double* u0, int ptr_kind, int64_t nsteps,
                        int32_t every, void* stream) {
  if (!c || !phi0) return fail(VCLB_EINVAL, "case or phi0 is NULL");
  if (int rc = adj_check_case(c)) return rc;
  if (ptr_kind != VCLB_HOST && ptr_kind != VCLB_DEVICE) return fail(VCLB_EINVAL, "bad ptr_kind");
  if (nsteps < 0 || every < 0) return fail(VCLB_EINVAL, "nsteps and every must be >= 0");
  if (every == 0) every = adj_default_every(nsteps);
  const size_t n = size_t(c->p.nx) * c->p.ny;
  if (ptr_kind == VCLB_HOST)
    for (size_t i = 0; i < n; ++i)
      if (!std::isfinite(phi0[i])) return fail(VCLB_ENONFINITE, "phi0 has a NaN/Inf");
  hipStream_t s = as_stream(stream);
  adj_release(c);
  AdjStore lay = adj_layout(c->p, nsteps, every);
  void* m = nullptr;
  hipError_t e = hipMalloc(&m, lay.total);
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? VCLB_ENOMEM : VCLB_EHIP, "hipMalloc of the adjoint store failed");
  c->adj = new (std::nothrow) AdjStore(lay);
  if (!c->adj) {
    (void)hipFree(m);
    return fail(VCLB_ENOMEM, "host allocation");
  }
  AdjStore& a = *c->adj;
  a.mem = static_cast<char*>(m);
  a.has_u0 = u0 != nullptr;
  const hipMemcpyKind kind = ptr_kind == VCLB_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  double* dphi0 = reinterpret_cast<double*>(a.mem + a.phi0);
  double* du0 = reinterpret_cast<double*>(a.mem + a.u0);
  HIP_TRY(hipMemcpyAsync(dphi0, phi0, n * sizeof(double), kind, s));
  if (u0) HIP_TRY(hipMemcpyAsync(du0, u0, 2 * n * sizeof(double), kind, s));
  int rc = vclb_case_init(c, dphi0, u0 ? du0 : nullptr, VCLB_DEVICE, stream);
  if (rc) {
    adj_release(c);
    return rc;
  }
  for (int64_t k = 0; k < a.nckpt; ++k) {
    rc = adj_save_state(c, reinterpret_cast<double*>(a.mem + a.ckpt) + size_t(k) * a.state, s);
    if (!rc) rc = vclb_step(c, std::min<int64_t>(a.every, a.nsteps - k * a.every), stream);
    if (rc) {
      adj_release(c);
      return rc;
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  return VCLB_OK;
}

int vclb_adjoint_run(vclb_case* c, const double* seed, double normal_tau, double* dphi0, int ptr_kind,
                     double* dparams, void* stream) {
  if (!c || !seed) return fail(VCLB_EINVAL, "case or seed is NULL");
  if (!(normal_tau >= 0.0) || !std::isfinite(normal_tau)) return fail(VCLB_EINVAL, "normal_tau must be >= 0");
  if (int rc = adj_check_case(c)) return rc;
  if (!c->adj) return fail(VCLB_ESTATE, "adjoint run before vclb_adjoint_record");
  if (dphi0 && ptr_kind != VCLB_HOST && ptr_kind != VCLB_DEVICE) return fail(VCLB_EINVAL, "bad ptr_kind");
  const int nl = std::max(1, c->p.nlabels);
  for (int k = 0; k < nl * vclb::kSeedFields; ++k)
    if (!std::isfinite(seed[k])) return fail(VCLB_EINVAL, "seed has a NaN/Inf");
  hipStream_t s = as_stream(stream);
  AdjStore& st = *c->adj;
  char* M = st.mem;
  const size_t n = st.n;
  const size_t ns = size_t(vclb::plane_stride(long(n)));   // plane stride of the state snapshots
  auto dptr = [&](size_t off) { return reinterpret_cast<double*>(M + off); };
  HIP_TRY(hipMemcpyAsync(dptr(st.seed), seed, size_t(nl) * vclb::kSeedFields * sizeof(double),
                         hipMemcpyHostToDevice, s));
  if (vclb::launch_adj_zero(dptr(st.part), 2 * st.blocks, s)) return fail(VCLB_EHIP, "adjoint launch failed");

  vclb::DevCase<vclb::D2Q9, vclb::StoreF64> base = make_dev<vclb::D2Q9, vclb::StoreF64>(*c);
  base.t = 0;
  base.pend_nb = 0;
  base.part_r = nullptr;
  vclb::AdjArgs a{};
  a.lphi = dptr(st.lphi);
  a.aux = dptr(st.aux);
  a.param_part = dptr(st.part);
  a.seed = dptr(st.seed);
  a.beta4_per_sigma = 48.0 / c->p.W;
  a.kappa_per_sigma = 1.5 * c->p.W;
  a.normal_tau2 = normal_tau * normal_tau;
  a.mobility_rows = 0;
  for (int k = 0; k < 9; ++k)
    if (c->p.s_g[k] == 0.0 && vclb::D2Q9::g_flux_row[k]) a.mobility_rows |= 1u << k;
  int cur = 0;
  auto bind = [&](int in) {
    a.lg_in = dptr(st.lg[in]);
    a.lf_in = dptr(st.lf[in]);
    a.lJ_in = dptr(st.lJ[in]);
    a.lg_out = dptr(st.lg[in ^ 1]);
    a.lf_out = dptr(st.lf[in ^ 1]);
    a.lJ_out = dptr(st.lJ[in ^ 1]);
  };
  bind(1);   // the seed writes buffer 0
  int rc = vclb::launch_adj_seed(base, a, s);
  auto slot = [&](int64_t k) { return dptr(st.seg) + size_t(k) * st.state; };
  for (int64_t seg = st.nckpt - 1; seg >= 0 && !rc; --seg) {
    const int64_t t0 = seg * st.every, len = std::min<int64_t>(st.every, st.nsteps - t0);
    HIP_TRY(hipMemcpyAsync(slot(0), dptr(st.ckpt) + size_t(seg) * st.state, st.state * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
    // recompute the segment's states with the forward step (no reductions)
    for (int64_t k = 0; k + 1 < len && !rc; ++k) {
      HIP_TRY(hipMemcpyAsync(slot(k + 1) + 18 * ns, slot(k) + 18 * ns, 2 * ns * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
      auto f = base;
      f.pop[0][0] = slot(k);
      f.pop[1][0] = slot(k) + 9 * ns;
      f.pop[0][1] = slot(k + 1);
      f.pop[1][1] = slot(k + 1) + 9 * ns;
      f.J = slot(k + 1) + 18 * ns;
      rc = vclb::launch_step_fused<vclb::D2Q9, vclb::StoreF64, true>(f, c->tile, 0, s);
    }
    // backward through the segment
    for (int64_t k = len - 1; k >= 0 && !rc; --k) {
      auto b = base;
      b.pop[0][0] = slot(k);
      b.pop[1][0] = slot(k) + 9 * ns;
      b.pop[0][1] = nullptr;
      b.pop[1][1] = nullptr;
      b.J = slot(k) + 18 * ns;
      bind(cur);
      rc = vclb::launch_phi_psi<vclb::D2Q9, vclb::StoreF64>(b, s);
      if (!rc) rc = vclb::launch_adj_step(b, a, s);
      cur ^= 1;
    }
  }
  if (rc) return fail(VCLB_EHIP, "adjoint launch failed");
  bind(cur);
  double* dst = (dphi0 && ptr_kind == VCLB_DEVICE) ? dphi0 : dptr(st.dphi);
  rc = vclb::launch_adj_init(base, a, dptr(st.phi0), st.has_u0 ? dptr(st.u0) : nullptr, dst, s);
  if (!rc) rc = vclb::launch_adj_params(a, int(st.blocks), dptr(st.out), s);
  if (rc) return fail(VCLB_EHIP, "adjoint launch failed");
  double host_out[2] = {0.0, 0.0};
  HIP_TRY(hipMemcpyAsync(host_out, dptr(st.out), sizeof(host_out), hipMemcpyDeviceToHost, s));
  if (dphi0 && ptr_kind == VCLB_HOST) HIP_TRY(hipMemcpyAsync(dphi0, dst, n * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (dparams) {
    dparams[0] = host_out[0];
    dparams[1] = host_out[1];
  }
  return VCLB_OK;
}

int vclb_obs_derived(const vclb_obs* obs, int32_t nlabels, double* out) {
  if (!obs || !out || nlabels < 1 || nlabels > VCLB_MAX_LABELS) return fail(VCLB_EINVAL, "bad argument");
  for (int l = 0; l < nlabels; ++l) {
    double g[5][vclb::kSeedFields];
    derived_with_grad(obs[l], out + 5 * l, g);
  }
  return VCLB_OK;
}

int vclb_obs_seed(const vclb_obs* obs, int32_t nlabels, const double* weights, double* seed) {
  if (!obs || !weights || !seed || nlabels < 1 || nlabels > VCLB_MAX_LABELS)
    return fail(VCLB_EINVAL, "bad argument");
  for (int l = 0; l < nlabels; ++l) {
    double v[5], g[5][vclb::kSeedFields];
    derived_with_grad(obs[l], v, g);
    for (int j = 0; j < vclb::kSeedFields; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 5; ++k)
        if (weights[5 * l + k] != 0.0) acc += weights[5 * l + k] * g[k][j];
      seed[vclb::kSeedFields * l + j] = acc;
    }
  }
  return VCLB_OK;
}

}  // extern "C"
