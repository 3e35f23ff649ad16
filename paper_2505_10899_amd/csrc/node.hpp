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

#include <type_traits>

#include "lattice.hpp"

namespace vclb {

// ---------------------------------------------------------------- global memory access
// Every device buffer of the library lives in global memory.  Pointers that reach a
// kernel through a struct are generic to the compiler, which then emits flat memory
// instructions; flat accesses also wait on the LDS/scalar counter and so overlap less
// with the LDS traffic of the stencils.  These helpers cast to the global address
// space, so that the accesses compile to global_load / global_store.
// An unsigned index selects the 32-bit form: the caller guarantees i * sizeof(T) < 2^32,
// so the address is a uniform 64-bit base plus a 32-bit byte offset, which the hardware
// adds itself (global_load v, v_off, s_base): one multiply-shift per access instead of
// a sign extension and a 64-bit add.
#define VCLB_GLOBAL __attribute__((address_space(1)))
template <class T, class I>
__device__ __forceinline__ T ldg(const T* p, I i) {
  return ((const T VCLB_GLOBAL*)p)[i];
}
template <class T, class I>
__device__ __forceinline__ void stg(T* p, I i, T v) {
  ((T VCLB_GLOBAL*)p)[i] = v;
}
template <class T>
__device__ __forceinline__ T ldg(const T* p, unsigned i) {
  const unsigned b = i * unsigned(sizeof(T));
  return *(const T VCLB_GLOBAL*)((const char VCLB_GLOBAL*)p + b);
}
template <class T>
__device__ __forceinline__ void stg(T* p, unsigned i, T v) {
  const unsigned b = i * unsigned(sizeof(T));
  *(T VCLB_GLOBAL*)((char VCLB_GLOBAL*)p + b) = v;
}

// Non-temporal forms: the access carries the streaming hint, so that the line is not
// kept for reuse (a population is read once and written once per step).
template <class T, class I>
__device__ __forceinline__ T ldg_nt(const T* p, I i) {
  return __builtin_nontemporal_load((const T VCLB_GLOBAL*)p + i);
}
template <class T, class I>
__device__ __forceinline__ void stg_nt(T* p, I i, T v) {
  __builtin_nontemporal_store(v, (T VCLB_GLOBAL*)p + i);
}
template <class T>
__device__ __forceinline__ T ldg_nt(const T* p, unsigned i) {
  const unsigned b = i * unsigned(sizeof(T));
  return __builtin_nontemporal_load((const T VCLB_GLOBAL*)((const char VCLB_GLOBAL*)p + b));
}
template <class T>
__device__ __forceinline__ void stg_nt(T* p, unsigned i, T v) {
  const unsigned b = i * unsigned(sizeof(T));
  __builtin_nontemporal_store(v, (T VCLB_GLOBAL*)((char VCLB_GLOBAL*)p + b));
}

// ---------------------------------------------------------------- storage codecs
// load / store: plain accesses; load_nt / store_nt: with the non-temporal hint
// fold: the storage rounds coarsely enough that the phis entry a node writes for itself
// absorbs the sum of the rounding errors of the deviations it wrote (rounding(v): stored
// value minus v)
struct StoreF64 {
  using S = double;
  using R = double;
  static constexpr bool shifted = false;
  static constexpr bool fold = false;
  __device__ static R rounding(R) { return R(0); }
  template <class I>
  __device__ static R load(const S* p, I i) { return ldg(p, i); }
  template <class I>
  __device__ static void store(S* p, I i, R v) { stg(p, i, v); }
  template <class I>
  __device__ static R load_nt(const S* p, I i) { return ldg_nt(p, i); }
  template <class I>
  __device__ static void store_nt(S* p, I i, R v) { stg_nt(p, i, v); }
};
// FP32 storage uses the same deviation representation as FP16S (see below): the g
// arithmetic then never rounds at the magnitude of the rest populations (~0.7), which
// keeps the total of phi conserved to the rounding of small quantities.
struct StoreF32 {
  using S = float;
  using R = float;
  static constexpr bool shifted = true;
  static constexpr bool fold = false;
  __device__ static R rounding(R) { return R(0); }
  template <class I>
  __device__ static R load(const S* p, I i) { return ldg(p, i); }
  template <class I>
  __device__ static void store(S* p, I i, R v) { stg(p, i, v); }
  template <class I>
  __device__ static R load_nt(const S* p, I i) { return ldg_nt(p, i); }
  template <class I>
  __device__ static void store_nt(S* p, I i, R v) { stg_nt(p, i, v); }
};
// FP16 storage of deviations from the rest equilibrium: g_i - phi r_i with
// r_0 = 1 + (w_0 - 1) lambda, r_i = w_i lambda (g_eq at u = 0, mu = 0), where phi is that
// of the node that will read the value, kept in FP32 in the reader's own entry of a phi
// array (encode_dev); f is stored as is (its rest equilibrium, f_eq at p = 0 and u = 0,
// vanishes).  Shifted storage also switches the g collision to deviation variables
// e_i = g_i - r_i phi (node_update, SH = true).
struct StoreF16S {
  using S = __half;
  using R = float;
  static constexpr bool shifted = true;
  // A node's stored deviations, rounded to 2 bytes, change the total of g by the sum of
  // their rounding errors; at a node in a steady state that error is the same every step,
  // so the total of phi would drift steadily.  The node's own phi entry (FP32), which its
  // next pull adds back to every population it reads, is stored less that sum, so that the
  // total of the decoded populations stays the total of phi.
  static constexpr bool fold = true;
  __device__ static R rounding(R v) { return __half2float(__float2half_rn(v)) - v; }
  template <class I>
  __device__ static R load(const S* p, I i) {
    return __half2float(__ushort_as_half(ldg(reinterpret_cast<const unsigned short*>(p), i)));
  }
  template <class I>
  __device__ static void store(S* p, I i, R v) {
    stg(reinterpret_cast<unsigned short*>(p), i, __half_as_ushort(__float2half_rn(v)));
  }
  template <class I>
  __device__ static R load_nt(const S* p, I i) {
    return __half2float(__ushort_as_half(ldg_nt(reinterpret_cast<const unsigned short*>(p), i)));
  }
  template <class I>
  __device__ static void store_nt(S* p, I i, R v) {
    stg_nt(reinterpret_cast<unsigned short*>(p), i, __half_as_ushort(__float2half_rn(v)));
  }
};

// ---------------------------------------------------------------- per-case constants
template <class L, class R>
struct NodeParams {
  R W4;          // W / 4
  R xi;          // regulariser of Eq. 37
  R lamW;        // lambda / W
  R An4;         // 4 (lambda / W) / (1 + 2 xi)^2: the correction amplitude is An4 a b
  R lam;         // lambda
  R beta4;       // 4 beta, beta = 12 sigma / W
  R kappa;       // 3 sigma W / 2
  R eps2;        // eps_n^2
  R rho_l;       // rho at phi = 0
  R drho;        // rho_heavy - rho_light
  R mu_l;        // dynamic viscosity at phi = 0, rho_light nu_light
  R dmu;         // rho_heavy nu_heavy - rho_light nu_light
  R sg[L::Q];    // s_k^g / |M_k|^2
  R sf[L::Q];    // s_k^f / |M_k|^2
  R wb[L::Q];    // moving-wall term for outgoing direction o at the first y row (times rho)
  R wt[L::Q];    // same at the last y row
  R rest[L::Q];  // FP16S rest-equilibrium coefficients r_i
  R sgr[L::Q];   // s_k^g (unscaled)
  R sfr[L::Q];   // s_k^f (unscaled)
  R wet_lo;      // (4 / W) cos(theta) of the bottom wall (0: mirror ghosts)
  R wet_hi;      // same for the top wall
  R U0;          // vortex amplitude
  double T;      // vortex period (steps)
  double mass_fix;   // rate of the global volume correction (0: off)
};

template <class R>
__device__ __forceinline__ R clamp01(R v) {
  return v < R(0) ? R(0) : (v > R(1) ? R(1) : v);
}

// 1 / x and 1 / sqrt(x) for positive normal x: in FP32 the hardware instructions (about
// 1 ulp each, no denormal scaling, no Newton step in FP64), in FP64 correctly rounded
// division and the library rsqrt
template <class R>
__device__ __forceinline__ R recip(R x) {
  if constexpr (sizeof(R) == 4) return __builtin_amdgcn_rcpf(x);
  else return R(1) / x;
}
template <class R>
__device__ __forceinline__ R rsqrt_of(R x) {
  if constexpr (sizeof(R) == 4) return __builtin_amdgcn_rsqf(x);
  else return rsqrt(x);
}

// psi of Eq. 37 on the clipped order parameter
template <class R>
__device__ __forceinline__ R psi_of(R phi, R W4, R xi) {
  const R pc = clamp01(phi);
  if constexpr (sizeof(R) == 4) {
    // hardware reciprocal and base-2 logarithm (about 1 ulp each; ln = ln 2 log2): the
    // quotient lies in [xi / (1 + xi), (1 + xi) / xi], far from denormals, and psi's own
    // rounding at its magnitude (up to (W / 4) ln(1 / xi)) is larger than what they add
    return (W4 * R(0.693147180559945309)) * __builtin_amdgcn_logf((pc + xi) * __builtin_amdgcn_rcpf((R(1) - pc) + xi));
  } else {
    return W4 * log((pc + xi) / ((R(1) - pc) + xi));
  }
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

// Relaxation rate of the f stress moments at a node whose phases have different
// viscosities: 1 / tau_f with tau_f = 1/2 + mu / (rho c_s^2) (Eq. 27), where the dynamic
// viscosity mu is linear in phi between the light and heavy phases, like rho.
template <class L, class R>
__device__ __forceinline__ R stress_rate(const NodeParams<L, R>& p, R phi, R irho) {
  return recip(R(0.5) + R(3) * (p.mu_l + phi * p.dmu) * irho);
}

// ---------------------------------------------------------------- D2Q9 in closed form
// m = M g with the shared partial sums of the rows of Eq. 24
template <class R>
__device__ __forceinline__ void d2q9_moments(const R (&v)[9], R (&m)[9]) {
  const R a14 = (v[1] + v[3]) + (v[2] + v[4]);
  const R a58 = (v[5] + v[7]) + (v[6] + v[8]);
  m[0] = v[0] + a14 + a58;
  m[1] = R(-4) * v[0] - a14 + R(2) * a58;
  m[2] = R(4) * v[0] - R(2) * a14 + a58;
  const R d13 = v[1] - v[3], d24 = v[2] - v[4];
  const R x58 = (v[5] - v[7]) + (v[8] - v[6]);
  const R y58 = (v[5] - v[7]) + (v[6] - v[8]);
  m[3] = d13 + x58;
  m[4] = R(-2) * d13 + x58;
  m[5] = d24 + y58;
  m[6] = R(-2) * d24 + y58;
  m[7] = (v[1] + v[3]) - (v[2] + v[4]);
  m[8] = (v[5] + v[7]) - (v[6] + v[8]);
}

// v = M^{-1} m = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4) m
template <class R>
__device__ __forceinline__ void d2q9_from_moments(const R (&m)[9], R (&v)[9]) {
  const R a0 = m[0] * R(1.0 / 9.0), a1 = m[1] * R(1.0 / 36.0), a2 = m[2] * R(1.0 / 36.0);
  const R a3 = m[3] * R(1.0 / 6.0), a4 = m[4] * R(1.0 / 12.0), a5 = m[5] * R(1.0 / 6.0);
  const R a6 = m[6] * R(1.0 / 12.0), a7 = m[7] * R(0.25), a8 = m[8] * R(0.25);
  const R A = a0 - a1 - R(2) * a2, B = a0 + R(2) * a1 + a2;
  const R X1 = a3 - R(2) * a4, Y1 = a5 - R(2) * a6, X2 = a3 + a4, Y2 = a5 + a6;
  v[0] = a0 - R(4) * a1 + R(4) * a2;
  v[1] = A + X1 + a7;
  v[3] = A - X1 + a7;
  v[2] = A + Y1 - a7;
  v[4] = A - Y1 - a7;
  v[5] = B + X2 + Y2 + a8;
  v[7] = B - X2 - Y2 + a8;
  v[6] = B - X2 + Y2 - a8;
  v[8] = B + X2 - Y2 - a8;
}

// One D2Q9 node of one time step.  g, f: pulled (time-t) populations in, post-collision
// out; J: previous phi u in, this step's phi u out.  With SH, g holds the deviations
// e_i = g_i - r_i phi from the node's rest state (in and out): the equilibrium enters as
// g_eq - r phi, and the relaxation of the conserved moment sum_i g_i (zero in exact
// arithmetic) is dropped, so no operation rounds at the magnitude of phi.  The moments
// of the equilibria and sources are in closed form (M g_eq, M f_eq, M G and M F evaluated from
// Eqs. 21-24, 31-32), so that each population set costs one forward and one inverse
// moment transform.
// UNIT: every rate outside the g flux rows (3-6) and the f stress rows (7-8) is exactly 1
// (the defaults); those rows then relax straight to m_eq + src / 2 and their m is never
// formed.
// VISC: the two phases have different viscosities; the stress rows relax at the node's
// own 1 / tau_f (Eq. 27), see stress_rate.
template <class R, bool COUPLED, bool SH, bool UNIT = false, bool VISC = false>
__device__ __forceinline__ void node_update_d2q9(const NodeParams<D2Q9, R>& p, const NodeIn<D2Q9, R>& in,
                                                 R (&g)[9], R (&f)[9], R (&J)[2], NodeOut<D2Q9, R>& out) {
  const R* q = in.nphi;
  const R* s = in.npsi;
  const R phi = q[0];
  const R rho = p.rho_l + phi * p.drho;
  const R pc = clamp01(phi);
  const R a = pc + p.xi, b = (R(1) - pc) + p.xi;
  // (lambda/W)[1 - tanh^2(2 psi / W)] = (lambda/W) 4 a b / (a + b)^2, a + b = 1 + 2 xi
  const R An = p.An4 * a * b;
  // Eqs. 39-40 on D2Q9: 3 w_i c_i = 1/3 (axes), 1/12 (diagonals); 6 w_i = 2/3, 1/6
  const R gpx = R(1.0 / 3.0) * (q[1] - q[3]) + R(1.0 / 12.0) * ((q[5] - q[7]) + (q[8] - q[6]));
  const R gpy = R(1.0 / 3.0) * (q[2] - q[4]) + R(1.0 / 12.0) * ((q[5] - q[7]) + (q[6] - q[8]));
  const R lap = R(2.0 / 3.0) * (((q[1] + q[3]) + (q[2] + q[4])) - R(4) * q[0]) +
                R(1.0 / 6.0) * (((q[5] + q[7]) + (q[6] + q[8])) - R(4) * q[0]);
  const R gsx = R(1.0 / 3.0) * (s[1] - s[3]) + R(1.0 / 12.0) * ((s[5] - s[7]) + (s[8] - s[6]));
  const R gsy = R(1.0 / 3.0) * (s[2] - s[4]) + R(1.0 / 12.0) * ((s[5] - s[7]) + (s[6] - s[8]));
  const R mu = p.beta4 * phi * (phi - R(1)) * (phi - R(0.5)) - p.kappa * lap;   // Eq. 2
  const R Fx = mu * gpx, Fy = mu * gpy;                                          // F_s = mu grad phi
  const R grx = p.drho * gpx, gry = p.drho * gpy;
  R ux, uy, press = R(0);
  R fm[9];
  R s_stress = R(0);
  if constexpr (COUPLED) {
    d2q9_moments<R>(f, fm);
    const R irho = recip(rho);
    if constexpr (VISC) s_stress = stress_rate(p, phi, irho);
    ux = (fm[3] + R(0.5) * Fx) * irho;                                           // Eq. 28
    uy = (fm[5] + R(0.5) * Fy) * irho;
    const R P = fm[0] - f[0];
    const R uu = ux * ux + uy * uy, ug = ux * grx + uy * gry;
    press = R(0.6) * (P + R(0.5) * ug - R(2.0 / 3.0) * rho * uu);               // Eq. 29
  } else {
    ux = in.u[0];
    uy = in.u[1];
  }
  const R Jx = phi * ux, Jy = phi * uy;
  const R dJx = Jx - J[0], dJy = Jy - J[1];
  J[0] = Jx;
  J[1] = Jy;
  const R inv = rsqrt_of(gsx * gsx + gsy * gsy + p.eps2);
  const R Vx = R(3) * dJx + An * (gsx * inv), Vy = R(3) * dJy + An * (gsy * inv);  // Eq. 32: G_i = w_i c_i . V
  // g (Eq. 33): equilibrium moments (phi, -4 phi + 2H, 4 phi - 3H, Jx, -Jx, Jy, -Jy, 0, 0), H = mu + lambda phi;
  // in deviation variables (subtract M r phi) they are (0, 2 mu, -3 mu, Jx, -Jx, Jy, -Jy, 0, 0).
  // source moments (0, 0, 0, Vx/3, -Vx/3, Vy/3, -Vy/3, 0, 0).
  {
    R m[9];
    if constexpr (UNIT) {
      // only the conserved row (kept as is in deviation variables) and the flux rows
      const R d13 = g[1] - g[3], d24 = g[2] - g[4];
      const R x58 = (g[5] - g[7]) + (g[8] - g[6]);
      const R y58 = (g[5] - g[7]) + (g[6] - g[8]);
      m[0] = SH ? g[0] + ((g[1] + g[3]) + (g[2] + g[4])) + ((g[5] + g[7]) + (g[6] + g[8])) : R(0);
      m[1] = m[2] = m[7] = m[8] = R(0);
      m[3] = d13 + x58;
      m[4] = R(-2) * d13 + x58;
      m[5] = d24 + y58;
      m[6] = R(-2) * d24 + y58;
    } else {
      d2q9_moments<R>(g, m);
    }
    R eq[9];
    if constexpr (SH) {
      eq[0] = m[0];
      eq[1] = R(2) * mu;
      eq[2] = R(-3) * mu;
    } else {
      const R H = mu + p.lam * phi;
      eq[0] = phi;
      eq[1] = R(-4) * phi + R(2) * H;
      eq[2] = R(4) * phi - R(3) * H;
    }
    eq[3] = Jx; eq[4] = -Jx; eq[5] = Jy; eq[6] = -Jy; eq[7] = R(0); eq[8] = R(0);
    const R Gx = Vx * R(1.0 / 3.0), Gy = Vy * R(1.0 / 3.0);
    const R src[9] = {R(0), R(0), R(0), Gx, -Gx, Gy, -Gy, R(0), R(0)};
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      if (SH && k == 0) continue;
      if (UNIT && !D2Q9::g_flux_row[k]) m[k] = eq[k] + R(0.5) * src[k];
      else m[k] = m[k] - p.sgr[k] * (m[k] - eq[k]) + (R(1) - R(0.5) * p.sgr[k]) * src[k];
    }
    d2q9_from_moments<R>(m, g);
  }
  // f (Eq. 25): equilibrium moments (0, 6p + 3 rho u.u, -9p - 3 rho u.u, rho ux, -rho ux, rho uy,
  // -rho uy, rho (ux^2 - uy^2), rho ux uy); forcing moments (u.grad rho, 0, -u.grad rho, Fx, -Fx,
  // Fy, -Fy, 2/3 (ux gx - uy gy), 1/3 (ux gy + uy gx))
  if constexpr (COUPLED) {
    const R uu = ux * ux + uy * uy, ug = ux * grx + uy * gry;
    const R eq[9] = {R(0), R(6) * press + R(3) * rho * uu, R(-9) * press - R(3) * rho * uu,
                     rho * ux, -rho * ux, rho * uy, -rho * uy, rho * (ux * ux - uy * uy), rho * ux * uy};
    const R src[9] = {ug, R(0), -ug, Fx, -Fx, Fy, -Fy, R(2.0 / 3.0) * (ux * grx - uy * gry),
                      R(1.0 / 3.0) * (ux * gry + uy * grx)};
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const R sk = (VISC && D2Q9::f_stress_row[k]) ? s_stress : p.sfr[k];
      if (UNIT && !D2Q9::f_stress_row[k]) fm[k] = eq[k] + R(0.5) * src[k];
      else fm[k] = fm[k] - sk * (fm[k] - eq[k]) + (R(1) - R(0.5) * sk) * src[k];
    }
    d2q9_from_moments<R>(fm, f);
  }
  out.rho = rho;
  out.mu = mu;
  out.press = press;
  out.u[0] = ux;
  out.u[1] = uy;
}

// ---------------------------------------------------------------- any lattice, moment space
// Compile-time loop: f(integral_constant<int, K>) for K = B .. E - 1.
template <int B, int E, class Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  if constexpr (B < E) {
    fn(std::integral_constant<int, B>{});
    static_for<B + 1, E>(fn);
  }
}

// Every moment row of both bases has a definite parity under c -> -c: even rows see a
// pair of opposite populations only through their sum, odd rows only through their
// difference.  The transforms below work on those sums and differences, which halves
// the multiply-adds of a full matrix product (zero entries are skipped at compile time).
template <class L>
constexpr int row_parity(int k) {   // +1 even, -1 odd, 0 neither
  bool even = true, odd = true;
  for (int i = 0; i < L::Q; ++i) {
    even = even && L::M[k][i] == L::M[k][L::opp[i]];
    odd = odd && L::M[k][i] == -L::M[k][L::opp[i]];
  }
  return even ? 1 : (odd ? -1 : 0);
}
template <class L>
constexpr bool pair_lead(int i) {   // first member of an opposite pair
  return L::opp[i] > i;
}

// acc += c x for a compile-time integer c
template <int C, class R>
__device__ __forceinline__ void add_int_times(R& acc, R x) {
  if constexpr (C == 1) acc += x;
  else if constexpr (C == -1) acc -= x;
  else if constexpr (C != 0) acc += R(C) * x;
}

// Row selections for to_moments: every row, or only the rows whose relaxation rate is not
// fixed at 1 when the other rates are (then m*_k = m_k^eq + src_k / 2 needs no m_k): the
// g flux rows (and the conserved row, kept as is in deviation variables), the f stress rows.
struct AllRows {
  static constexpr bool need(int) { return true; }
};
template <class L>
struct GRateRows {
  static constexpr bool need(int k) { return k == 0 || L::g_flux_row[k]; }
};
template <class L>
struct FRateRows {
  static constexpr bool need(int k) { return L::f_stress_row[k]; }
};

// m = M v (rows outside `Rows` are left at zero)
template <class L, class R, class Rows = AllRows>
__device__ __forceinline__ void to_moments(const R (&v)[L::Q], R (&m)[L::Q]) {
  R sp[L::Q], dp[L::Q];   // pair sums and differences, at the lead index
  static_for<0, L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    if constexpr (pair_lead<L>(i)) {
      sp[i] = v[i] + v[L::opp[i]];
      dp[i] = v[i] - v[L::opp[i]];
    }
  });
  static_for<0, L::Q>([&](auto K) {
    constexpr int k = decltype(K)::value;
    constexpr int par = row_parity<L>(k);
    static_assert(par != 0, "moment rows must have a definite parity");
    R acc = R(0);
    if constexpr (Rows::need(k)) {
      add_int_times<L::M[k][0]>(acc, v[0]);
      static_for<1, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (pair_lead<L>(i)) add_int_times<L::M[k][i]>(acc, par > 0 ? sp[i] : dp[i]);
      });
    }
    m[k] = acc;
  });
}

// v = M^{-1} m = M^T diag(1 / |M_k|^2) m (m is scaled in place): for each pair the even
// rows give the common part and the odd rows the antisymmetric part
template <class L, class R>
__device__ __forceinline__ void from_moments(R (&m)[L::Q], R (&v)[L::Q]) {
  R (&a)[L::Q] = m;
  static_for<0, L::Q>([&](auto K) {
    constexpr int k = decltype(K)::value;
    a[k] = m[k] * R(1.0 / double(row_norm<L>(k)));
  });
  static_for<0, L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    if constexpr (i == 0 || pair_lead<L>(i)) {
      R ev = R(0), od = R(0);
      static_for<0, L::Q>([&](auto K) {
        constexpr int k = decltype(K)::value;
        if constexpr (row_parity<L>(k) > 0) add_int_times<L::M[k][i]>(ev, a[k]);
        else add_int_times<L::M[k][i]>(od, a[k]);
      });
      if constexpr (i == 0) {
        v[0] = ev + od;
      } else {
        v[i] = ev + od;
        v[L::opp[i]] = ev - od;
      }
    }
  });
}

// sum_d x_d T(k, d) and sum_{d,e} x_d y_e T(k, d, e) with compile-time tables
template <class L, class R, int k>
__device__ __forceinline__ R mom_lin(const R (&x)[L::D]) {
  R s = R(0);
  static_for<0, L::D>([&](auto D) {
    constexpr int d = decltype(D)::value;
    constexpr double t = mom_wc<L>(k, d);
    if constexpr (t != 0.0) s += R(t) * x[d];
  });
  return s;
}
template <class L, class R, int k>
__device__ __forceinline__ R mom_quad(const R (&x)[L::D], const R (&y)[L::D]) {
  R s = R(0);
  static_for<0, L::D>([&](auto D) {
    constexpr int d = decltype(D)::value;
    static_for<0, L::D>([&](auto E) {
      constexpr int e = decltype(E)::value;
      constexpr double t = mom_wcc<L>(k, d, e);
      if constexpr (t != 0.0) s += R(t) * (x[d] * y[e]);
    });
  });
  return s;
}

// One node on any lattice (used for D3Q19), with the collisions done in moment space and the moments of the equilibria and sources formed row by row
// from the tables above: with g_eq,i = w_i (H + 3 c_i . J) + delta_i0 (phi - H) (Eq. 31),
// G_i = w_i c_i . V (Eq. 32), f_eq,i = 3 w_i p + delta_i0 (-3 p) + rho w_i (3 c_i . u +
// 4.5 (c_i . u)^2 - 1.5 u . u) (Eqs. 22-23) and F_i = 3 w_i (c_i . F + (c_i . u)(c_i .
// grad rho)) (Eq. 21), no per-population equilibrium is ever stored.
// What the stencils of Eqs. 39-40 give at one node.
template <class L, class R>
struct StencilOut {
  R phi, lap;
  R gphi[L::D], gpsi[L::D];
  R u[L::D];   // prescribed velocity (vortex mode only)
};

// UNIT: every rate outside the g flux rows and the f stress rows is exactly 1 (the
// defaults); those rows then relax straight to m_eq + src / 2 without forming m.
// VISC: the stress rows relax at the node's own rate (stress_rate).
template <class L, class R, bool COUPLED, bool SH, bool UNIT = false, bool VISC = false>
__device__ __forceinline__ void node_update_mom_s(const NodeParams<L, R>& p, const StencilOut<L, R>& st,
                                                  R (&g)[L::Q], R (&f)[L::Q], R (&J)[L::D], NodeOut<L, R>& out) {
  constexpr int Q = L::Q, D = L::D;
  const R phi = st.phi;
  const R rho = p.rho_l + phi * p.drho;
  const R pc = clamp01(phi);
  const R a = pc + p.xi, b = (R(1) - pc) + p.xi;
  // (lambda/W)[1 - tanh^2(2 psi / W)] = (lambda/W) 4 a b / (a + b)^2, a + b = 1 + 2 xi
  const R An = p.An4 * a * b;
  const R* gphi = st.gphi;
  const R* gpsi = st.gpsi;
  const R lphi = st.lap;
  const R mu = p.beta4 * phi * (phi - R(1)) * (phi - R(0.5)) - p.kappa * lphi;   // Eq. 2
  R Fs[D], grho[D], u[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    Fs[d] = mu * gphi[d];
    grho[d] = p.drho * gphi[d];
  }
  R press = R(0);
  R s_stress = R(0);
  if constexpr (COUPLED) {
    // momentum and the sum of the moving populations; the full moments of f are formed
    // only at its collision, so that they are not live across the g collision
    R jj[3] = {R(0), R(0), R(0)}, P = R(0);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      P += f[i];
      if (L::cx[i] != 0) jj[0] += R(L::cx[i]) * f[i];
      if (L::cy[i] != 0) jj[1] += R(L::cy[i]) * f[i];
      if (D == 3 && L::cz[i] != 0) jj[2] += R(L::cz[i]) * f[i];
    }
    R uu = R(0), ug = R(0);
    const R irho = recip(rho);
    if constexpr (VISC) s_stress = stress_rate(p, phi, irho);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      u[d] = (jj[d] + R(0.5) * Fs[d]) * irho;                                       // Eq. 28
      uu += u[d] * u[d];
      ug += u[d] * grho[d];
    }
    press = R((1.0 / 3.0) / (1.0 - L::w[0])) * (P + R(0.5) * ug + rho * R(-1.5 * L::w[0]) * uu);   // Eq. 29
  } else {
#pragma unroll
    for (int d = 0; d < D; ++d) u[d] = st.u[d];
  }
  R Jn[D], V[D];
  R n2 = p.eps2;
#pragma unroll
  for (int d = 0; d < D; ++d) n2 += gpsi[d] * gpsi[d];
  const R inv = rsqrt_of(n2);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    Jn[d] = phi * u[d];
    V[d] = R(3) * (Jn[d] - J[d]) + An * (gpsi[d] * inv);
    J[d] = Jn[d];
  }
  // g (Eq. 33) in moment space; with SH the equilibrium enters as g_eq - r phi and the
  // conserved row is not relaxed
  {
    R m[Q];
    if constexpr (UNIT) to_moments<L, R, GRateRows<L>>(g, m);
    else to_moments<L, R>(g, m);
    const R H = mu + p.lam * phi;
    static_for<0, Q>([&](auto K) {
      constexpr int k = decltype(K)::value;
      if constexpr (!(SH && k == 0)) {
        constexpr double w0 = mom_w<L>(k);
        constexpr double rest = double(L::M[k][0]);
        R eq;
        if constexpr (SH) eq = R(w0 - rest) * mu;
        else eq = R(w0) * H + R(rest) * (phi - H);
        eq += R(3) * mom_lin<L, R, k>(Jn);
        const R src = mom_lin<L, R, k>(V);
        if constexpr (UNIT && !GRateRows<L>::need(k)) {
          m[k] = eq + R(0.5) * src;
        } else {
          const R s = p.sgr[k];
          m[k] = m[k] - s * (m[k] - eq) + (R(1) - R(0.5) * s) * src;
        }
      }
    });
    from_moments<L, R>(m, g);
  }
  // f (Eq. 25) in moment space
  if constexpr (COUPLED) {
    R fm[Q];
    if constexpr (UNIT) to_moments<L, R, FRateRows<L>>(f, fm);
    else to_moments<L, R>(f, fm);
    R uu = R(0);
#pragma unroll
    for (int d = 0; d < D; ++d) uu += u[d] * u[d];
    static_for<0, Q>([&](auto K) {
      constexpr int k = decltype(K)::value;
      constexpr double w0 = mom_w<L>(k);
      constexpr double rest = double(L::M[k][0]);
      const R eq = R(3.0 * (w0 - rest)) * press +
                   rho * (R(3) * mom_lin<L, R, k>(u) + R(4.5) * mom_quad<L, R, k>(u, u) - R(1.5 * w0) * uu);
      const R src = R(3) * mom_lin<L, R, k>(Fs) + R(3) * mom_quad<L, R, k>(u, grho);
      if constexpr (UNIT && !FRateRows<L>::need(k)) {
        fm[k] = eq + R(0.5) * src;
      } else {
        const R s = (VISC && L::f_stress_row[k]) ? s_stress : p.sfr[k];
        fm[k] = fm[k] - s * (fm[k] - eq) + (R(1) - R(0.5) * s) * src;
      }
    });
    from_moments<L, R>(fm, f);
  }
  out.rho = rho;
  out.mu = mu;
  out.press = press;
#pragma unroll
  for (int d = 0; d < D; ++d) out.u[d] = u[d];
}

template <class L, class R, bool COUPLED, bool SH, bool VISC = false>
__device__ __forceinline__ void node_update_mom(const NodeParams<L, R>& p, const NodeIn<L, R>& in,
                                                R (&g)[L::Q], R (&f)[L::Q], R (&J)[L::D], NodeOut<L, R>& out) {
  StencilOut<L, R> st;
  st.phi = in.nphi[0];
  st.lap = stencil_lap<L, R>(in.nphi);
  stencil_grad<L, R>(in.nphi, st.gphi);
  stencil_grad<L, R>(in.npsi, st.gpsi);
#pragma unroll
  for (int d = 0; d < L::D; ++d) st.u[d] = in.u[d];
  node_update_mom_s<L, R, COUPLED, SH, false, VISC>(p, st, g, f, J, out);
}

template <class L, class R, bool COUPLED, bool SH = false, bool VISC = false>
__device__ __forceinline__ void node_update(const NodeParams<L, R>& p, const NodeIn<L, R>& in, R (&g)[L::Q],
                                            R (&f)[L::Q], R (&J)[L::D], NodeOut<L, R>& out) {
  if constexpr (L::Q == 9) node_update_d2q9<R, COUPLED, SH, false, VISC>(p, in, g, f, J, out);
  else node_update_mom<L, R, COUPLED, SH, VISC>(p, in, g, f, J, out);
}
// the same with the viscosity choice made at run time (plain path and observe)
template <class L, class R, bool COUPLED, bool SH = false>
__device__ __forceinline__ void node_update_any(const NodeParams<L, R>& p, bool visc, const NodeIn<L, R>& in,
                                                R (&g)[L::Q], R (&f)[L::Q], R (&J)[L::D], NodeOut<L, R>& out) {
  if (COUPLED && visc) node_update<L, R, COUPLED, SH, COUPLED>(p, in, g, f, J, out);
  else node_update<L, R, COUPLED, SH, false>(p, in, g, f, J, out);
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
