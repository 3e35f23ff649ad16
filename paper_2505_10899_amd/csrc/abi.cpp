// Host side of the C ABI declared in include/vclb.h: parameter validation (no HIP call),
// workspace layout, per-case constants, launch dispatch over (lattice, storage, mode),
// observation history and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/vclb.h"
#include "launch.hpp"

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

// relaxation rates with defaults filled in (see lattice.hpp)
void fill_rates(const vclb_params& p, double* sg, double* sf) {
  const int Q = lattice_q(p.lattice);
  const double tau_g = 0.5 + p.mobility * 3.0;   // Eq. 34, c_s^2 = 1/3
  const double tau_f = 0.5 + p.nu * 3.0;         // Eq. 27 with mu = rho nu
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
  if (p->bc_y != VCLB_PERIODIC && p->bc_y != VCLB_WALL) return fail(VCLB_EINVAL, "unknown bc_y");
  if (p->bc_y == VCLB_WALL && p->lattice != VCLB_D2Q9) return fail(VCLB_EINVAL, "walls are D2Q9-only");
  if (p->bc_y == VCLB_WALL && p->ny < 2) return fail(VCLB_EINVAL, "walls need ny >= 2");
  if (p->nlabels < 0 || p->nlabels > VCLB_MAX_LABELS) return fail(VCLB_EINVAL, "nlabels out of range");
  if (!(finite(p->W) && p->W > 0)) return fail(VCLB_EINVAL, "W must be > 0");
  if (!(finite(p->sigma) && p->sigma >= 0)) return fail(VCLB_EINVAL, "sigma must be >= 0");
  if (!(finite(p->mobility) && p->mobility > 0)) return fail(VCLB_EINVAL, "mobility must be > 0");
  if (!(finite(p->lambda) && p->lambda >= 0)) return fail(VCLB_EINVAL, "lambda must be >= 0");
  if (!(finite(p->xi) && p->xi > 0)) return fail(VCLB_EINVAL, "xi must be > 0");
  if (!(finite(p->eps_n) && p->eps_n >= 0)) return fail(VCLB_EINVAL, "eps_n must be >= 0");
  if (!(finite(p->rho_heavy) && p->rho_heavy > 0)) return fail(VCLB_EINVAL, "rho_heavy must be > 0");
  if (!(finite(p->rho_light) && p->rho_light > 0)) return fail(VCLB_EINVAL, "rho_light must be > 0");
  if (!(finite(p->nu) && p->nu > 0)) return fail(VCLB_EINVAL, "nu must be > 0");
  const int Q = lattice_q(p->lattice);
  for (int k = 0; k < 19; ++k) {
    const bool used = k < Q;
    for (double s : {p->s_g[k], p->s_f[k]}) {
      if (!finite(s)) return fail(VCLB_EINVAL, "relaxation rate not finite");
      if (s != 0.0 && (!used || !(s > 0.0 && s < 2.0)))
        return fail(VCLB_EINVAL, "relaxation rates must lie in (0, 2)");
    }
  }
  double sg[19], sf[19];
  fill_rates(*p, sg, sf);
  for (int k = 0; k < Q; ++k)
    if (!(sg[k] > 0 && sg[k] < 2 && sf[k] > 0 && sf[k] < 2))
      return fail(VCLB_EINVAL, "derived relaxation rate outside (0, 2)");
  for (int a = 0; a < 3; ++a)
    if (!finite(p->wall_u_bottom[a]) || !finite(p->wall_u_top[a])) return fail(VCLB_EINVAL, "wall velocity");
  if (p->mode == VCLB_PRESCRIBED_VORTEX && !(finite(p->T) && p->T > 0 && finite(p->U0)))
    return fail(VCLB_EINVAL, "vortex needs T > 0 and a finite U0");
  for (int k = 0; k < p->nlabels; ++k)
    for (int a = 0; a < 3; ++a)
      if (!finite(p->label_centre[k][a])) return fail(VCLB_EINVAL, "label centre");
  return VCLB_OK;
}

struct Layout {
  size_t pop[2][2], J, phis[2], partials[2], hist, cur, tmp_phi, tmp_psi, total;
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
  for (int s = 0; s < 2; ++s)
    for (int b = 0; b < 2; ++b) {
      const bool need = s == 0 || p.mode == VCLB_COUPLED;
      L.pop[s][b] = need ? take(size_t(Q) * n * sb) : SIZE_MAX;
    }
  L.J = take(size_t(D) * n * rb);
  for (int b = 0; b < 2; ++b) L.phis[b] = p.storage != VCLB_FP64 ? take(n * 4) : SIZE_MAX;
  // every launch shape uses at least 64 nodes per workgroup, plus one partial row per
  // (y, z) line for tiles that are ragged in x
  L.partial_blocks = long(n / 64) + long(p.ny) * p.nz + 64;
  for (int b = 0; b < 2; ++b) L.partials[b] = take(size_t(L.partial_blocks) * nl * 12 * sizeof(double));
  L.hist = take(size_t(vclb::kHistory) * nl * vclb::kObsFields * sizeof(double));
  L.cur = take(size_t(nl) * vclb::kObsFields * sizeof(double));
  L.tmp_phi = take(n * rb);
  L.tmp_psi = take(n * rb);
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
};

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
  d.wall = p.bc_y == VCLB_WALL;
  d.nl = std::max(1, p.nlabels);
  for (int k = 0; k < vclb::kMaxLabels; ++k)
    for (int a = 0; a < 3; ++a) {
      double v;
      if (p.nlabels == 0) v = a == 0 ? (p.nx - 1) / 2.0 : (a == 1 ? (p.ny - 1) / 2.0 : (p.nz - 1) / 2.0);
      else v = p.label_centre[std::min(k, p.nlabels - 1)][a];
      // periodic axes: the minimum-image displacement is periodic in the centre, so the
      // centre is moved into [0, n) (the kernels rely on it to wrap without a division)
      const int na = a == 0 ? p.nx : (a == 1 ? p.ny : p.nz);
      const bool periodic = !(a == 1 && p.bc_y == VCLB_WALL);
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
  auto& np = d.np;
  const double sigma = p.sigma, W = p.W;
  np.W4 = R(W / 4.0);
  np.xi = R(p.xi);
  np.lamW = R(p.lambda / W);
  np.lam = R(p.lambda);
  np.beta4 = R(4.0 * (12.0 * sigma / W));
  np.kappa = R(1.5 * sigma * W);
  np.eps2 = R(p.eps_n * p.eps_n);
  np.rho_l = R(p.rho_light);
  np.drho = R(p.rho_heavy - p.rho_light);
  for (int k = 0; k < L::Q; ++k) {
    np.sg[k] = R(c.sg[k] / vclb::row_norm<L>(k));
    np.sf[k] = R(c.sf[k] / vclb::row_norm<L>(k));
    np.sgr[k] = R(c.sg[k]);
    np.sfr[k] = R(c.sf[k]);
    np.rest[k] = R(k == 0 ? 1.0 + (L::w[0] - 1.0) * p.lambda : L::w[k] * p.lambda);
    // moving-wall term 2 w_i rho (c_i . u_wall) / cs^2 of the incoming direction i = opp(k),
    // stored on the outgoing direction k at the first (bottom) / last (top) y row
    const int i = L::opp[k];
    const double cub = L::cx[i] * p.wall_u_bottom[0] + L::cy[i] * p.wall_u_bottom[1] + L::cz[i] * p.wall_u_bottom[2];
    const double cut = L::cx[i] * p.wall_u_top[0] + L::cy[i] * p.wall_u_top[1] + L::cz[i] * p.wall_u_top[2];
    np.wb[k] = R(L::cy[k] < 0 ? 2.0 * L::w[i] * cub * 3.0 : 0.0);
    np.wt[k] = R(L::cy[k] > 0 ? 2.0 * L::w[i] * cut * 3.0 : 0.0);
  }
  np.U0 = R(p.U0);
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

vclb::Tile default_tile(const vclb_params& p) {
  vclb::Tile t;
  if (p.lattice == VCLB_D2Q9) {
    // one lane per x column, rounded up to whole waves, at most 256
    int bx = std::min(256, (p.nx + 63) / 64 * 64);
    t.bx = bx;
    const long strips = (p.nx + bx - 1) / bx;
    // long marches amortise the two halo rows; keep >= 1024 workgroups (four per CU)
    // when the grid allows, with 8..64 rows each
    long ty = (long(p.ny) * strips) / 1024;
    t.ty = int(std::max(8L, std::min(64L, ty)));
    t.by3 = 1;
  } else {
    t.bx = std::min(64, (p.nx + 31) / 32 * 32);
    t.by3 = std::max(1, std::min(16, 256 / t.bx));
    t.ty = 16;
  }
  return t;
}

int check_tile(const vclb_params& p, const vclb::Tile& t) {
  if (p.lattice == VCLB_D2Q9) {
    if (t.bx < 64 || t.bx > 256 || t.bx % 64 != 0 || t.ty < 1) return fail(VCLB_EINVAL, "bad 2D tile");
  } else {
    if (t.bx < 1 || t.by3 < 1 || t.bx * t.by3 > 512 || (t.bx * t.by3) % 64 != 0 || t.ty < 1)
      return fail(VCLB_EINVAL, "bad 3D tile (bx * by3 must be a multiple of 64, at most 512)");
    const size_t lds = size_t(2) * 4 * (t.bx + 2) * (t.by3 + 2) * arith_bytes(p.storage);
    if (lds > 65536) return fail(VCLB_EINVAL, "3D tile needs more than 64 KiB of LDS");
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

int vclb_version(void) { return 10000; }

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
  c->tile = default_tile(c->p);
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

int vclb_reduce(vclb_case* c, vclb_obs* out, void* stream) {
  if (!c || !out) return fail(VCLB_EINVAL, "NULL argument");
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
  const int Q = lattice_q(c->p.lattice), D = lattice_d(c->p.lattice);
  std::vector<Span> v;
  v.push_back({c->lay.pop[0][par], size_t(Q) * n * storage_bytes(c->p.storage)});
  if (c->p.mode == VCLB_COUPLED) v.push_back({c->lay.pop[1][par], size_t(Q) * n * storage_bytes(c->p.storage)});
  v.push_back({c->lay.J, size_t(D) * n * arith_bytes(c->p.storage)});
  if (c->p.storage != VCLB_FP64) v.push_back({c->lay.phis[par], n * 4});
  return v;
}

uint64_t params_hash(const vclb_params& p) { return fnv1a(&p, sizeof(p)); }
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
  h.version = 1;
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
  if (std::memcmp(h.magic, "VCLBCKP1", 8) != 0 || h.version != 1) return fail(VCLB_EINVAL, "not a checkpoint");
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
