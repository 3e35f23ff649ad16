// Per-node arithmetic of one time step (device code, shared by every step kernel).
//
// The order follows the time step of the paper's Sect. 3:
//   phi = sum g (Eq. 35) -> rho, psi (Eq. 37) -> grad/lap stencils (Eqs. 39-40)
//   -> chemical potential (Eq. 2) and F_s = mu grad phi -> u (Eq. 28), p (Eq. 29)
//   -> backward difference of phi u -> g collision (Eqs. 31-33) -> f collision
//   (Eqs. 21-25).
//
// Collision in moment space, m* = m - S (m - m_eq) + (I - S/2) M src, is evaluated as
//   pop* = pop + src - M^T [ diag(s_k / |M_k|^2) M (pop - eq + src / 2) ],
// which is the same expression: M^{-1} = M^T diag(1 / |M_k|^2) because the rows of M
// are orthogonal.  One forward and one backward product with the integer matrix.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include "lattice.hpp"

namespace vclb {

// ---------------------------------------------------------------- storage codecs
struct StoreF64 {
  using S = double;
  using R = double;
  static constexpr bool shifted = false;
  __device__ static R load(const S* p, long i) { return p[i]; }
  __device__ static void store(S* p, long i, R v) { p[i] = v; }
};
// FP32 storage uses the same deviation representation as FP16S (see below): the g
// arithmetic then never rounds at the magnitude of the rest populations (~0.7), which
// keeps the total of phi conserved to the rounding of small quantities.
struct StoreF32 {
  using S = float;
  using R = float;
  static constexpr bool shifted = true;
  __device__ static R load(const S* p, long i) { return p[i]; }
  __device__ static void store(S* p, long i, R v) { p[i] = v; }
};
// FP16 storage of deviations from the rest equilibrium: g_i - phi r_i with
// r_0 = 1 + (w_0 - 1) lambda, r_i = w_i lambda (g_eq at u = 0, mu = 0); f is stored
// as is (its rest equilibrium, f_eq at p = 0 and u = 0, vanishes).  phi of the node
// that wrote the value travels beside it in FP32.  Shifted storage also switches the
// g collision to deviation variables e_i = g_i - r_i phi (node_update, SH = true).
struct StoreF16S {
  using S = __half;
  using R = float;
  static constexpr bool shifted = true;
  __device__ static R load(const S* p, long i) { return __half2float(p[i]); }
  __device__ static void store(S* p, long i, R v) { p[i] = __float2half_rn(v); }
};

// ---------------------------------------------------------------- per-case constants
template <class L, class R>
struct NodeParams {
  R W4;          // W / 4
  R xi;          // regulariser of Eq. 37
  R lamW;        // lambda / W
  R lam;         // lambda
  R beta4;       // 4 beta, beta = 12 sigma / W
  R kappa;       // 3 sigma W / 2
  R eps2;        // eps_n^2
  R rho_l;       // rho at phi = 0
  R drho;        // rho_heavy - rho_light
  R sg[L::Q];    // s_k^g / |M_k|^2
  R sf[L::Q];    // s_k^f / |M_k|^2
  R wb[L::Q];    // moving-wall term for outgoing direction o at the first y row (times rho)
  R wt[L::Q];    // same at the last y row
  R rest[L::Q];  // FP16S rest-equilibrium coefficients r_i
  R U0;          // vortex amplitude
  double T;      // vortex period (steps)
};

template <class R>
__device__ __forceinline__ R clamp01(R v) {
  return v < R(0) ? R(0) : (v > R(1) ? R(1) : v);
}

// psi of Eq. 37 on the clipped order parameter
template <class R>
__device__ __forceinline__ R psi_of(R phi, R W4, R xi) {
  const R pc = clamp01(phi);
  return W4 * log((pc + xi) / ((R(1) - pc) + xi));
}

// grad (Eq. 39) and Laplacian (Eq. 40) of a field given at x + c_i, i = 0..Q-1
template <class L, class R>
__device__ __forceinline__ void stencil_grad(const R (&nb)[L::Q], R (&gr)[L::D]) {
#pragma unroll
  for (int d = 0; d < L::D; ++d) gr[d] = R(0);
#pragma unroll
  for (int i = 1; i < L::Q; ++i) {
    const int cc[3] = {L::cx[i], L::cy[i], L::cz[i]};
#pragma unroll
    for (int d = 0; d < L::D; ++d) {
      if (cc[d] != 0) gr[d] += R(3.0 * L::w[i] * cc[d]) * nb[i];
    }
  }
}

template <class L, class R>
__device__ __forceinline__ R stencil_lap(const R (&nb)[L::Q]) {
  R s = R(0);
#pragma unroll
  for (int i = 1; i < L::Q; ++i) s += R(6.0 * L::w[i]) * (nb[i] - nb[0]);
  return s;
}

// pop <- pop + src - M^T diag(srate) M (pop - eq + src/2); with CONSERVE the zeroth
// moment (sum of the populations, equal to that of the equilibrium) is not relaxed.
template <class L, class R, bool CONSERVE>
__device__ __forceinline__ void mrt_collide(R (&pop)[L::Q], const R (&eq)[L::Q], const R (&src)[L::Q],
                                            const R (&srate)[L::Q]) {
  R h[L::Q];
#pragma unroll
  for (int i = 0; i < L::Q; ++i) h[i] = pop[i] - eq[i] + R(0.5) * src[i];
  R y[L::Q];
#pragma unroll
  for (int k = 0; k < L::Q; ++k) {
    R acc = R(0);
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
      const int m = L::M[k][i];
      if (m == 1) acc += h[i];
      else if (m == -1) acc -= h[i];
      else if (m != 0) acc += R(m) * h[i];
    }
    y[k] = (CONSERVE && k == 0) ? R(0) : acc * srate[k];
  }
#pragma unroll
  for (int i = 0; i < L::Q; ++i) {
    R acc = R(0);
#pragma unroll
    for (int k = 0; k < L::Q; ++k) {
      const int m = L::M[k][i];
      if (m == 1) acc += y[k];
      else if (m == -1) acc -= y[k];
      else if (m != 0) acc += R(m) * y[k];
    }
    pop[i] = pop[i] + src[i] - acc;
  }
}

// Everything one node needs besides its own populations.
template <class L, class R>
struct NodeIn {
  R nphi[L::Q];   // phi at x + c_i (index 0: the node)
  R npsi[L::Q];   // psi at x + c_i
  R u[L::D];      // prescribed velocity (vortex mode only)
};

template <class L, class R>
struct NodeOut {
  R rho, mu, press;
  R u[L::D];
};

// One node of one time step.  g, f: pulled (time-t) populations in, post-collision out;
// J: previous phi u in, this step's phi u out.  With SH, g holds the deviations
// e_i = g_i - r_i phi from the node's rest state (in and out): the equilibrium enters as
// g_eq - r phi, and the relaxation of the conserved moment sum_i g_i (zero in exact
// arithmetic) is dropped, so no operation rounds at the magnitude of phi.
template <class L, class R, bool COUPLED, bool SH = false>
__device__ __forceinline__ void node_update(const NodeParams<L, R>& p, const NodeIn<L, R>& in,
                                            R (&g)[L::Q], R (&f)[L::Q], R (&J)[L::D],
                                            NodeOut<L, R>& out) {
  constexpr int Q = L::Q, D = L::D;
  const R phi = in.nphi[0];
  const R rho = p.rho_l + phi * p.drho;
  // factor (lambda/W)[1 - tanh^2(2 psi / W)] of Eq. 32 via tanh(0.5 ln(a/b)) = (a-b)/(a+b)
  const R pc = clamp01(phi);
  const R a = pc + p.xi, b = (R(1) - pc) + p.xi;
  const R An = p.lamW * (R(4) * a * b) / ((a + b) * (a + b));
  R gphi[D], gpsi[D];
  stencil_grad<L, R>(in.nphi, gphi);
  stencil_grad<L, R>(in.npsi, gpsi);
  const R lphi = stencil_lap<L, R>(in.nphi);
  const R mu = p.beta4 * phi * (phi - R(1)) * (phi - R(0.5)) - p.kappa * lphi;   // Eq. 2
  R Fs[D], grho[D], u[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    Fs[d] = mu * gphi[d];
    grho[d] = p.drho * gphi[d];
  }
  R press = R(0);
  if constexpr (COUPLED) {
    R j[D];
#pragma unroll
    for (int d = 0; d < D; ++d) j[d] = R(0);
    R P = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int cc[3] = {L::cx[i], L::cy[i], L::cz[i]};
#pragma unroll
      for (int d = 0; d < D; ++d) {
        if (cc[d] == 1) j[d] += f[i];
        else if (cc[d] == -1) j[d] -= f[i];
      }
      if (i > 0) P += f[i];
    }
    R uu = R(0), ug = R(0);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      u[d] = (j[d] + R(0.5) * Fs[d]) / rho;                                         // Eq. 28
      uu += u[d] * u[d];
      ug += u[d] * grho[d];
    }
    const R s0 = R(-1.5 * L::w[0]) * uu;                                            // Eq. 23, i = 0
    press = R((1.0 / 3.0) / (1.0 - L::w[0])) * (P + R(0.5) * ug + rho * s0);       // Eq. 29
  } else {
#pragma unroll
    for (int d = 0; d < D; ++d) u[d] = in.u[d];
  }
  // backward difference of phi u
  R dJ[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const R Jn = phi * u[d];
    dJ[d] = Jn - J[d];
    J[d] = Jn;
  }
  // V = d_t(phi u)/cs^2 + (lambda/W)(1 - tanh^2) grad psi / |grad psi|, G_i = w_i c_i . V (Eq. 32)
  R n2 = p.eps2;
#pragma unroll
  for (int d = 0; d < D; ++d) n2 += gpsi[d] * gpsi[d];
  const R inv = R(1) / sqrt(n2);
  R V[D];
#pragma unroll
  for (int d = 0; d < D; ++d) V[d] = R(3) * dJ[d] + An * (gpsi[d] * inv);
  // g: equilibrium Eq. 31 and collision Eq. 33
  {
    const R H = mu + p.lam * phi;
    R geq[Q], G[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int cc[3] = {L::cx[i], L::cy[i], L::cz[i]};
      R cJ = R(0), cV = R(0);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        if (cc[d] == 1) { cJ += J[d]; cV += V[d]; }
        else if (cc[d] == -1) { cJ -= J[d]; cV -= V[d]; }
      }
      const R wi = R(L::w[i]);
      if constexpr (SH) geq[i] = (i == 0) ? R(L::w[0] - 1.0) * mu : wi * mu + wi * (R(3) * cJ);
      else geq[i] = (i == 0) ? phi + R(L::w[0] - 1.0) * H : wi * H + wi * (R(3) * cJ);
      G[i] = wi * cV;
    }
    mrt_collide<L, R, SH>(g, geq, G, p.sg);
  }
  // f: equilibrium Eqs. 22-23, forcing Eq. 21 (in the exactly equivalent form
  // w_i [c_i.F + (c_i.u)(c_i.grad rho)] / cs^2) and collision Eq. 25
  if constexpr (COUPLED) {
    R uu = R(0);
#pragma unroll
    for (int d = 0; d < D; ++d) uu += u[d] * u[d];
    R feq[Q], Fi[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int cc[3] = {L::cx[i], L::cy[i], L::cz[i]};
      R cu = R(0), cF = R(0), cg = R(0);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        if (cc[d] == 1) { cu += u[d]; cF += Fs[d]; cg += grho[d]; }
        else if (cc[d] == -1) { cu -= u[d]; cF -= Fs[d]; cg -= grho[d]; }
      }
      const R wi = R(L::w[i]);
      const R si = wi * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu);
      feq[i] = (i == 0) ? R(3.0 * (L::w[0] - 1.0)) * press + rho * si : R(3.0 * L::w[i]) * press + rho * si;
      Fi[i] = R(3.0 * L::w[i]) * (cF + cu * cg);
    }
    mrt_collide<L, R, false>(f, feq, Fi, p.sf);
  }
  out.rho = rho;
  out.mu = mu;
  out.press = press;
#pragma unroll
  for (int d = 0; d < D; ++d) out.u[d] = u[d];
}

// Velocity of the prescribed single vortex, Eqs. 43-44, at node (x, y) and step t.
template <class R>
__device__ __forceinline__ void vortex_u(R U0, double T, int x, int y, int nx, int ny, long t, R& ux, R& uy) {
  const R pi = R(3.14159265358979323846);
  const R sx = sin(pi * R(x) / R(nx)), sy = sin(pi * R(y) / R(ny));
  const R s2x = sin(R(2) * pi * R(x) / R(nx)), s2y = sin(R(2) * pi * R(y) / R(ny));
  const R ct = R(cos(3.14159265358979323846 * double(t) / T));
  ux = U0 * (sx * sx) * s2y * ct;
  uy = -U0 * (sy * sy) * s2x * ct;
}

}  // namespace vclb
