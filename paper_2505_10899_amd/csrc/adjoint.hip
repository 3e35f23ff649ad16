// Discrete adjoint of the FP64 coupled D2Q9 step (hand-written reverse sweep).
//
// The objective J is a function of the phase field after the last step, linearised as
// J = sum over labels of s0 sum(phi) + s1 . sum(phi d) + s2 : sum(phi d d^T).  The adjoint
// state of the populations pulled at step t is kept in two parts:
//     dJ/dg_i(t)(x) = lg_i(x) + lphi(x),   dJ/df_i(t)(x) = lf_i(x),   dJ/dJprev(t)(x) = lJ(x)
// where lphi is the adjoint of phi(x) = sum_i g_i(x) (Eq. 35), shared by the nine g_i.
// One backward step t+1 -> t is two launches:
//   k_adj_local    per node x: gather the adjoint of the node's post-collision
//                  populations (transpose of the pull streaming with half-way bounce-back
//                  and the moving-wall term), recompute the node's forward step from the
//                  stored state at t, and run it in reverse.  Writes lg, lf, lJ of step t
//                  and the adjoints of what the node read through stencils: its own phi,
//                  the Laplacian and gradient of phi and the gradient of psi (Eqs. 39-40).
//                  Accumulates dJ/dsigma and dJ/dM per workgroup.
//   k_adj_stencil  per node y: the transposed stencils (behind a wall, the ghost row is
//                  the wetting ghost of the edge row: its slope joins the chain),
//                  dpsi/dphi from Eq. 37, giving lphi of step t.
// Away from the interface psi saturates and |grad psi| falls to rounding level; the
// derivative of the unit normal there has a gain of order lambda / |grad psi| per step
// and grows without bound, so the normal is differentiated only where
// |grad psi| >= normal_tau (psi is a signed distance, |grad psi| = 1, across the
// interface); normal_tau = 0 gives the exact derivative of the discrete map.
// The initial state (g = g_eq(phi0), f = f_eq(0, rho(phi0), u0), Jprev = phi0 u0) has its
// own reverse pair giving dJ/dphi0.
#include <hip/hip_runtime.h>

#include "adjoint.hpp"

namespace vclb {

namespace {

using R = double;
using DC = DevCase<D2Q9, StoreF64>;

__device__ __forceinline__ int xwrap(int x, int nx) { return x < 0 ? x + nx : (x >= nx ? x - nx : x); }

// row of the neighbour y + dy for the phi/psi stencils: wrap, or the edge row itself
// behind a wall (mirrored ghost)
__device__ __forceinline__ int stencil_row(int y, int dy, int ny, bool wall) {
  const int v = y + dy;
  if (v < 0) return wall ? 0 : v + ny;
  if (v >= ny) return wall ? ny - 1 : v - ny;
  return v;
}

// v = M^T y with the integer matrix of Eq. 24
__device__ __forceinline__ void moments_T(const R (&y)[9], R (&v)[9]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    R acc = R(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const int m = D2Q9::M[k][i];
      if (m == 1) acc += y[k];
      else if (m == -1) acc -= y[k];
      else if (m != 0) acc += R(m) * y[k];
    }
    v[i] = acc;
  }
}

// d(mu)/d(sigma) at fixed phi: mu = 4 beta c(phi) - kappa lap, beta and kappa linear in sigma
__device__ __forceinline__ R dmu_dsigma(const AdjArgs& a, R cub, R lap) {
  return a.beta4_per_sigma * cub - a.kappa_per_sigma * lap;
}

// per-workgroup accumulation of (dJ/dsigma, dJ/dM) into this workgroup's own slot
__device__ __forceinline__ void add_params(const AdjArgs& a, double sig, double mob) {
  __shared__ double red[16 * 2];
  const double v[2] = {sig, mob};
  const double s = block_sum_fields<2>(v, 2, red);
  if (threadIdx.x < 2) a.param_part[long(threadIdx.x) * gridDim.x + blockIdx.x] += s;
}

// sum over the stencil readers m of node (x, y), m + c_i = (x, y): fn(i, m, side), with
// side 0 for a reader of the node itself and -1 / +1 for a reader of the ghost row behind
// the bottom / top wall, which holds the wetting ghost of this edge node (its mirror for
// a neutral wall)
template <class Fn>
__device__ __forceinline__ void stencil_readers(const DC& c, int x, int y, Fn&& fn) {
  const int nx = c.nx, ny = c.ny;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const int xs = xwrap(x - D2Q9::cx[i], nx);
    const int ys = y - D2Q9::cy[i];
    if (ys >= 0 && ys < ny) fn(i, xs + long(nx) * ys, 0);
    else if (!c.wall) fn(i, xs + long(nx) * (ys < 0 ? ys + ny : ys - ny), 0);
    if (c.wall && y == 0 && D2Q9::cy[i] < 0) fn(i, xs + long(nx) * y, -1);
    if (c.wall && y == ny - 1 && D2Q9::cy[i] > 0) fn(i, xs + long(nx) * y, 1);
  }
}

// the wetting-ghost coefficient of the wall on this side: phi_g = phi_e + w phi_e (1 - phi_e)
__device__ __forceinline__ R wet_coef(const DC& c, int side) { return side < 0 ? c.np.wet_lo : c.np.wet_hi; }

// d(phi_g)/d(phi_e) of the wetting ghost
__device__ __forceinline__ R wet_slope(R w, R phi) { return R(1) + w * (R(1) - R(2) * phi); }

// dpsi/dphi of Eq. 37 on the clipped range (zero where the clip holds psi fixed)
__device__ __forceinline__ R dpsi_dphi(const DC& c, R phi) {
  if (!(phi >= R(0) && phi <= R(1))) return R(0);
  const R aa = phi + c.np.xi, bb = (R(1) - phi) + c.np.xi;
  return c.np.W4 * (R(1) / aa + R(1) / bb);
}

}  // namespace

// -------------------------------------------------------------------------- seed
// dJ/dphi(x) at the final step from the per-label moment weights; lg = lf = lJ = 0.
__global__ void __launch_bounds__(256) k_adj_seed(DC c, AdjArgs a) {
  const long n = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (n >= c.n) return;
  const int x = int(n % c.nx), y = int(n / c.nx);
  double d[kMaxLabels][2];
#pragma unroll
  for (int k = 0; k < kMaxLabels; ++k) {
    d[k][0] = min_image(double(x) - c.cen[k][0], c.nx, true);
    d[k][1] = min_image(double(y) - c.cen[k][1], c.ny, !c.wall);
  }
  int lab = 0;
  if (c.nl > 1 && d[1][0] * d[1][0] + d[1][1] * d[1][1] < d[0][0] * d[0][0] + d[0][1] * d[0][1]) lab = 1;
  const double* s = a.seed + lab * kSeedFields;
  const double dx = d[lab][0], dy = d[lab][1];
  // moments: sum, d (x, y, z), d d^T (xx, yy, zz, xy, xz, yz); z terms vanish in 2D
  a.lphi[n] = s[0] + s[1] * dx + s[2] * dy + s[4] * dx * dx + s[5] * dy * dy + s[7] * dx * dy;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    a.lg_out[long(i) * c.n + n] = 0.0;
    a.lf_out[long(i) * c.n + n] = 0.0;
  }
  a.lJ_out[n] = 0.0;
  a.lJ_out[c.n + n] = 0.0;
}

// -------------------------------------------------------------------------- local reverse
__global__ void __launch_bounds__(256) k_adj_local(DC c, AdjArgs a) {
  const long n = blockIdx.x * long(blockDim.x) + threadIdx.x;
  double acc_sig = 0.0, acc_mob = 0.0;
  if (n < c.n) {
    const int nx = c.nx, ny = c.ny;
    const bool wall = c.wall;
    const int x = int(n % nx), y = int(n / nx);
    const auto& p = c.np;
    // ---- forward recomputation at node x (the arithmetic of node_update_d2q9)
    R q[9], s[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const long m = xwrap(x + D2Q9::cx[i], nx) + long(nx) * stencil_row(y, D2Q9::cy[i], ny, wall);
      const int yn = y + D2Q9::cy[i];
      const int side = wall ? (yn < 0 ? -1 : (yn >= ny ? 1 : 0)) : 0;
      if (side) {   // the ghost row behind a wall: the wetting ghost of the edge row
        q[i] = wet_ghost<R>(c.tmp_phi[m], wet_coef(c, side));
        s[i] = psi_of<R>(q[i], p.W4, p.xi);
      } else {
        q[i] = c.tmp_phi[m];
        s[i] = c.tmp_psi[m];
      }
    }
    R g[9], f[9];
    pull<D2Q9, StoreF64>(c, c.pop[0][0], nullptr, x, y, 0, g, nullptr);
    pull<D2Q9, StoreF64>(c, c.pop[1][0], nullptr, x, y, 0, f, nullptr);
    const R phi = q[0];
    const R rho = p.rho_l + phi * p.drho;
    const bool inside = phi >= R(0) && phi <= R(1);
    const R pc = clamp01(phi);
    const R aa = pc + p.xi, bb = (R(1) - pc) + p.xi;
    const R An = p.An4 * aa * bb;                       // a + b = 1 + 2 xi
    const R dAn = inside ? p.An4 * (bb - aa) : R(0);
    const R gpx = R(1.0 / 3.0) * (q[1] - q[3]) + R(1.0 / 12.0) * ((q[5] - q[7]) + (q[8] - q[6]));
    const R gpy = R(1.0 / 3.0) * (q[2] - q[4]) + R(1.0 / 12.0) * ((q[5] - q[7]) + (q[6] - q[8]));
    const R lap = R(2.0 / 3.0) * (((q[1] + q[3]) + (q[2] + q[4])) - R(4) * q[0]) +
                  R(1.0 / 6.0) * (((q[5] + q[7]) + (q[6] + q[8])) - R(4) * q[0]);
    const R gsx = R(1.0 / 3.0) * (s[1] - s[3]) + R(1.0 / 12.0) * ((s[5] - s[7]) + (s[8] - s[6]));
    const R gsy = R(1.0 / 3.0) * (s[2] - s[4]) + R(1.0 / 12.0) * ((s[5] - s[7]) + (s[6] - s[8]));
    const R cub = phi * (phi - R(1)) * (phi - R(0.5));
    const R mu = p.beta4 * cub - p.kappa * lap;
    const R Fx = mu * gpx, Fy = mu * gpy;
    const R grx = p.drho * gpx, gry = p.drho * gpy;
    R fm[9];
    d2q9_moments<R>(f, fm);
    const R ux = (fm[3] + R(0.5) * Fx) / rho, uy = (fm[5] + R(0.5) * Fy) / rho;
    const R uu = ux * ux + uy * uy;
    const R Jx = phi * ux, Jy = phi * uy;
    const R r = sqrt(gsx * gsx + gsy * gsy + p.eps2);
    const R nxn = gsx / r, nyn = gsy / r;
    const R Vx = R(3) * (Jx - c.J[n]) + An * nxn, Vy = R(3) * (Jy - c.J[c.ns + n]) + An * nyn;
    R gm[9];
    d2q9_moments<R>(g, gm);
    const R H = mu + p.lam * phi;
    const R geq[9] = {phi, R(-4) * phi + R(2) * H, R(4) * phi - R(3) * H, Jx, -Jx, Jy, -Jy, R(0), R(0)};
    const R Gx = Vx * R(1.0 / 3.0), Gy = Vy * R(1.0 / 3.0);
    const R gsrc[9] = {R(0), R(0), R(0), Gx, -Gx, Gy, -Gy, R(0), R(0)};

    // ---- transpose of the streaming: the reader of each post-collision population
    R lgs[9], lfs[9];
    R lrho = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int yd = y + D2Q9::cy[i];
      long dst;
      int di = i;
      if (yd < 0 || yd >= ny) {
        if (wall) {
          dst = n;                // bounced back: read by this node as the opposite direction
          di = D2Q9::opp[i];
        } else {
          dst = xwrap(x + D2Q9::cx[i], nx) + long(nx) * (yd < 0 ? yd + ny : yd - ny);
        }
      } else {
        dst = xwrap(x + D2Q9::cx[i], nx) + long(nx) * yd;
      }
      lgs[i] = a.lg_in[long(di) * c.n + dst] + a.lphi[dst];
      lfs[i] = a.lf_in[long(di) * c.n + dst];
      // moving-wall term added to the populations leaving through a wall
      if (wall && y == 0 && D2Q9::cy[i] < 0) lrho += p.wb[i] * lfs[i];
      if (wall && y == ny - 1 && D2Q9::cy[i] > 0) lrho += p.wt[i] * lfs[i];
    }

    // ---- f collision (Eq. 25) in reverse: f* = M^-1 [(1 - s) m + s m_eq + (1 - s/2) m_F],
    // M^-T = diag(1/|M_k|^2) M
    // With unequal viscosities the stress rows relax at the node's own rate
    // s = 1 / (1/2 + 3 mu / rho) (Eq. 27), mu = mu_l + phi dmu: their adjoint also reaches
    // phi and rho through s, with dm*_k/ds = m_eq,k - m_k - m_F,k / 2.
    const bool visc = c.visc != 0;
    const R irho = R(1) / rho;
    const R s_st = visc ? stress_rate<D2Q9, R>(p, phi, irho) : R(0);
    const R meq_st[2] = {rho * (ux * ux - uy * uy), rho * ux * uy};
    const R mF_st[2] = {R(2.0 / 3.0) * (ux * grx - uy * gry), R(1.0 / 3.0) * (ux * gry + uy * grx)};
    R ls_st = R(0);   // adjoint of s
    R lmf[9];
    d2q9_moments<R>(lfs, lmf);
    R lfm[9], leqf[9], lsrcf[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const R lms = lmf[k] / R(row_norm<D2Q9>(k));
      const bool st = visc && D2Q9::f_stress_row[k];
      const R sk = st ? s_st : p.sfr[k];
      lfm[k] = (R(1) - sk) * lms;
      leqf[k] = sk * lms;
      lsrcf[k] = (R(1) - R(0.5) * sk) * lms;
      if (st) ls_st += lms * (meq_st[k - 7] - fm[k] - R(0.5) * mF_st[k - 7]);
    }
    // s = 1 / (1/2 + 3 mu / rho): ds/dphi = -3 s^2 dmu / rho (through mu), ds/drho = 3 s^2 mu / rho^2
    const R lphi_st = visc ? ls_st * (R(-3) * s_st * s_st * p.dmu * irho) : R(0);
    if (visc) lrho += ls_st * (R(3) * s_st * s_st * (p.mu_l + phi * p.dmu) * irho * irho);
    // equilibrium moments (0, 6p + 3 rho uu, -9p - 3 rho uu, rho ux, -rho ux, rho uy, -rho uy,
    // rho (ux^2 - uy^2), rho ux uy)
    const R lpress = R(6) * leqf[1] - R(9) * leqf[2];
    const R l12 = leqf[1] - leqf[2];
    lrho += R(3) * uu * l12 + ux * (leqf[3] - leqf[4]) + uy * (leqf[5] - leqf[6]) +
            (ux * ux - uy * uy) * leqf[7] + ux * uy * leqf[8];
    R lux = R(6) * rho * ux * l12 + rho * (leqf[3] - leqf[4]) + R(2) * rho * ux * leqf[7] + rho * uy * leqf[8];
    R luy = R(6) * rho * uy * l12 + rho * (leqf[5] - leqf[6]) - R(2) * rho * uy * leqf[7] + rho * ux * leqf[8];
    // forcing moments (u.grad rho, 0, -u.grad rho, Fx, -Fx, Fy, -Fy, 2/3 (ux gx - uy gy), 1/3 (ux gy + uy gx))
    R lug = lsrcf[0] - lsrcf[2];
    R lFx = lsrcf[3] - lsrcf[4], lFy = lsrcf[5] - lsrcf[6];
    lux += R(2.0 / 3.0) * grx * lsrcf[7] + R(1.0 / 3.0) * gry * lsrcf[8];
    luy += R(-2.0 / 3.0) * gry * lsrcf[7] + R(1.0 / 3.0) * grx * lsrcf[8];
    R lgrx = R(2.0 / 3.0) * ux * lsrcf[7] + R(1.0 / 3.0) * uy * lsrcf[8];
    R lgry = R(-2.0 / 3.0) * uy * lsrcf[7] + R(1.0 / 3.0) * ux * lsrcf[8];

    // ---- g collision (Eq. 33) in reverse
    R lmg[9];
    d2q9_moments<R>(lgs, lmg);
    R lgm[9], leqg[9], lsrcg[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const R lms = lmg[k] / R(row_norm<D2Q9>(k));
      const R sk = p.sgr[k];
      lgm[k] = (R(1) - sk) * lms;
      leqg[k] = sk * lms;
      lsrcg[k] = (R(1) - R(0.5) * sk) * lms;
      // rates set by the mobility: s = 1 / (1/2 + 3 M), ds/dM = -3 s^2
      if ((a.mobility_rows >> k) & 1) acc_mob += lms * (geq[k] - gm[k] - R(0.5) * gsrc[k]) * (R(-3) * sk * sk);
    }
    const R lH = R(2) * leqg[1] - R(3) * leqg[2];
    R lphi = leqg[0] - R(4) * leqg[1] + R(4) * leqg[2] + p.lam * lH + lphi_st;
    R lmu = lH;
    R lJx = leqg[3] - leqg[4], lJy = leqg[5] - leqg[6];
    const R lVx = (lsrcg[3] - lsrcg[4]) * R(1.0 / 3.0), lVy = (lsrcg[5] - lsrcg[6]) * R(1.0 / 3.0);

    // ---- V = 3 (J - Jprev) + An n (Eq. 32), n = grad psi / sqrt(|grad psi|^2 + eps^2);
    // this step's J is the next step's Jprev
    lJx += R(3) * lVx + a.lJ_in[n];
    lJy += R(3) * lVy + a.lJ_in[c.n + n];
    const R lAn = lVx * nxn + lVy * nyn;
    // where psi has saturated (|grad psi| below the cut) the normal is held fixed
    const bool n_live = !(gsx * gsx + gsy * gsy < a.normal_tau2);
    const R lgsx = n_live ? An * (lVx - nxn * lAn) / r : R(0);
    const R lgsy = n_live ? An * (lVy - nyn * lAn) / r : R(0);

    // ---- J = phi u
    lphi += lJx * ux + lJy * uy;
    lux += phi * lJx;
    luy += phi * lJy;

    // ---- pressure (Eq. 29): p = 3/5 (sum_{i>0} f_i + u.grad rho / 2 - 2/3 rho uu)
    const R lP = R(0.6) * lpress;
    lug += R(0.3) * lpress;
    lrho += R(-0.4) * uu * lpress;
    lux += R(-0.8) * rho * ux * lpress + grx * lug;
    luy += R(-0.8) * rho * uy * lpress + gry * lug;
    lgrx += ux * lug;
    lgry += uy * lug;

    // ---- velocity (Eq. 28): u = (j + F/2) / rho
    lfm[3] += lux / rho;
    lfm[5] += luy / rho;
    lFx += R(0.5) * lux / rho;
    lFy += R(0.5) * luy / rho;
    lrho -= (ux * lux + uy * luy) / rho;

    // ---- F = mu grad phi, grad rho = drho grad phi
    lmu += lFx * gpx + lFy * gpy;
    const R lgpx = mu * lFx + p.drho * lgrx, lgpy = mu * lFy + p.drho * lgry;

    // ---- chemical potential (Eq. 2), density, correction amplitude
    lphi += lmu * p.beta4 * (R(3) * phi * phi - R(3) * phi + R(0.5));
    acc_sig += lmu * dmu_dsigma(a, cub, lap);
    lphi += p.drho * lrho + dAn * lAn;

    // ---- the pulled populations through m = M pop, and P = m_0 - f_0
    lfm[0] += lP;
    R lgd[9], lfd[9];
    moments_T(lgm, lgd);
    moments_T(lfm, lfd);
    lfd[0] -= lP;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      a.lg_out[long(i) * c.n + n] = lgd[i];
      a.lf_out[long(i) * c.n + n] = lfd[i];
    }
    a.lJ_out[n] = R(-3) * lVx;
    a.lJ_out[c.n + n] = R(-3) * lVy;
    // adjoints of what the stencils read: [phi (own), lap phi, d/dx phi, d/dy phi, d/dx psi, d/dy psi]
    a.aux[n] = lphi;
    a.aux[c.n + n] = -p.kappa * lmu;
    a.aux[2 * c.n + n] = lgpx;
    a.aux[3 * c.n + n] = lgpy;
    a.aux[4 * c.n + n] = lgsx;
    a.aux[5 * c.n + n] = lgsy;
  }
  add_params(a, acc_sig, acc_mob);
}

__global__ void __launch_bounds__(256) k_adj_stencil(DC c, AdjArgs a) {
  const long n = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (n >= c.n) return;
  const int x = int(n % c.nx), y = int(n / c.nx);
  const double* lph = a.aux;
  const double* llap = a.aux + c.n;
  const double* lgpx = a.aux + 2 * c.n;
  const double* lgpy = a.aux + 3 * c.n;
  const double* lgsx = a.aux + 4 * c.n;
  const double* lgsy = a.aux + 5 * c.n;
  // own node: the centre weight of the Laplacian, -sum_i 6 w_i = -6 (1 - w_0)
  R lphi = lph[n] + R(-6.0 * (1.0 - D2Q9::w[0])) * llap[n];
  R lpsi = R(0);
  R gphi[2] = {R(0), R(0)}, gpsi[2] = {R(0), R(0)};   // through the ghost rows (bottom, top)
  stencil_readers(c, x, y, [&](int i, long m, int side) {
    const R ax = R(3.0 * D2Q9::w[i] * D2Q9::cx[i]), ay = R(3.0 * D2Q9::w[i] * D2Q9::cy[i]);
    const R dphi = ax * lgpx[m] + ay * lgpy[m] + R(6.0 * D2Q9::w[i]) * llap[m];
    const R dpsi = ax * lgsx[m] + ay * lgsy[m];
    if (side == 0) {
      lphi += dphi;
      lpsi += dpsi;
    } else {
      gphi[side > 0] += dphi;
      gpsi[side > 0] += dpsi;
    }
  });
  const R phi = c.tmp_phi[n];
  lphi += lpsi * dpsi_dphi(c, phi);
  // the ghost value phi_g (and psi of it) depends on this edge node's phi
  for (int k = 0; k < 2; ++k) {
    if (gphi[k] == R(0) && gpsi[k] == R(0)) continue;
    const R w = wet_coef(c, k ? 1 : -1);
    const R phig = wet_ghost<R>(phi, w);
    lphi += wet_slope(w, phi) * (gphi[k] + gpsi[k] * dpsi_dphi(c, phig));
  }
  a.lphi[n] = lphi;
}

// -------------------------------------------------------------------------- initial state
// pass 1 at node x: dJ/d(phi0(x)) through g_eq, f_eq and Jprev at x, and the adjoint of
// lap phi0(x) (written to aux[1]); mu0 = 4 beta c(phi0) - kappa lap phi0
__global__ void __launch_bounds__(256) k_adj_init_local(DC c, AdjArgs a, const double* __restrict__ phi0,
                                                        const double* __restrict__ u0) {
  const long n = blockIdx.x * long(blockDim.x) + threadIdx.x;
  double acc_sig = 0.0;
  if (n < c.n) {
    const int nx = c.nx, ny = c.ny;
    const int x = int(n % nx), y = int(n / nx);
    const auto& p = c.np;
    R q[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      q[i] = phi0[xwrap(x + D2Q9::cx[i], nx) + long(nx) * stencil_row(y, D2Q9::cy[i], ny, c.wall)];
      const int yn = y + D2Q9::cy[i];
      if (c.wall && (yn < 0 || yn >= ny)) q[i] = wet_ghost<R>(q[i], wet_coef(c, yn < 0 ? -1 : 1));
    }
    const R phi = q[0];
    const R lap = R(2.0 / 3.0) * (((q[1] + q[3]) + (q[2] + q[4])) - R(4) * q[0]) +
                  R(1.0 / 6.0) * (((q[5] + q[7]) + (q[6] + q[8])) - R(4) * q[0]);
    const R cub = phi * (phi - R(1)) * (phi - R(0.5));
    const R ux = u0 ? u0[n] : R(0), uy = u0 ? u0[c.n + n] : R(0);
    const R uu = ux * ux + uy * uy;
    const R lph = a.lphi[n];
    R lH = R(0), lphi = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const R lg = a.lg_in[long(i) * c.n + n] + lph;
      const R lf = a.lf_in[long(i) * c.n + n];
      const R wi = R(D2Q9::w[i]);
      const R cu = R(D2Q9::cx[i]) * ux + R(D2Q9::cy[i]) * uy;
      // Eq. 31: g_0 = phi + (w_0 - 1) H, g_i = w_i H + 3 w_i c_i . (phi u)
      if (i == 0) {
        lH += R(D2Q9::w[0] - 1.0) * lg;
        lphi += lg;
      } else {
        lH += wi * lg;
        lphi += R(3) * wi * cu * lg;
      }
      // Eqs. 22-23 at p = 0: f_i = rho s_i(u)
      lphi += p.drho * wi * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu) * lf;
    }
    lphi += ux * a.lJ_in[n] + uy * a.lJ_in[c.n + n];
    lphi += p.lam * lH + lH * p.beta4 * (R(3) * phi * phi - R(3) * phi + R(0.5));
    acc_sig += lH * dmu_dsigma(a, cub, lap);
    a.aux[n] = lphi;
    a.aux[c.n + n] = -p.kappa * lH;
  }
  add_params(a, acc_sig, 0.0);
}

__global__ void __launch_bounds__(256) k_adj_init_stencil(DC c, AdjArgs a, const double* __restrict__ phi0,
                                                          double* __restrict__ dphi0) {
  const long n = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (n >= c.n) return;
  const int x = int(n % c.nx), y = int(n / c.nx);
  const double* llap = a.aux + c.n;
  R v = a.aux[n] + R(-6.0 * (1.0 - D2Q9::w[0])) * llap[n];
  stencil_readers(c, x, y, [&](int i, long m, int side) {
    const R t = R(6.0 * D2Q9::w[i]) * llap[m];
    v += side ? wet_slope(wet_coef(c, side), phi0[n]) * t : t;   // a ghost read: d(phi_g)/d(phi_e)
  });
  dphi0[n] = v;
}

// (dJ/dsigma, dJ/dM): the per-workgroup slots summed in workgroup order
__global__ void __launch_bounds__(256) k_adj_params(AdjArgs a, int nblocks, double* __restrict__ out) {
  __shared__ double red[16 * 2];
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
    v[0] += a.param_part[b];
    v[1] += a.param_part[long(nblocks) + b];
  }
  const double s = block_sum_fields<2>(v, 2, red);
  if (threadIdx.x < 2) out[threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_adj_zero(double* __restrict__ p, long count) {
  const long i = blockIdx.x * long(blockDim.x) + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

// -------------------------------------------------------------------------- launchers
namespace {
unsigned blocks_for(long n) { return unsigned((n + 255) / 256); }
int last_status() { return hipGetLastError() == hipSuccess ? 0 : -3; }
}  // namespace

long adj_blocks(long n) { return long(blocks_for(n)); }

int launch_adj_zero(double* p, long count, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_zero, dim3(blocks_for(count)), dim3(256), 0, s, p, count);
  return last_status();
}

int launch_adj_seed(const DC& c, const AdjArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_seed, dim3(blocks_for(c.n)), dim3(256), 0, s, c, a);
  return last_status();
}

int launch_adj_step(const DC& c, const AdjArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_local, dim3(blocks_for(c.n)), dim3(256), 0, s, c, a);
  hipLaunchKernelGGL(k_adj_stencil, dim3(blocks_for(c.n)), dim3(256), 0, s, c, a);
  return last_status();
}

int launch_adj_init(const DC& c, const AdjArgs& a, const double* phi0, const double* u0, double* dphi0,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_adj_init_local, dim3(blocks_for(c.n)), dim3(256), 0, s, c, a, phi0, u0);
  hipLaunchKernelGGL(k_adj_init_stencil, dim3(blocks_for(c.n)), dim3(256), 0, s, c, a, phi0, dphi0);
  return last_status();
}

int launch_adj_params(const AdjArgs& a, int nblocks, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_params, dim3(1), dim3(256), 0, s, a, nblocks, out);
  return last_status();
}

}  // namespace vclb
