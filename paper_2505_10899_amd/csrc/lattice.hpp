// Lattice tables for the HIP kernels (compile-time constants).
//
// D2Q9: velocities of the paper's Eq. 19 (rest, E, N, W, S, NE, NW, SW, SE), weights
// 4/9, 1/9, 1/36 and the transformation matrix of Eq. 24 (rows rho, e, eps, jx, qx,
// jy, qy, pxx, pxy).
// D3Q19 (3D workloads; not in the paper): standard velocity set, weights 1/3, 1/18,
// 1/36, and the orthogonal moment basis of d'Humieres et al. (2002), whose rows are
// evaluated here from that basis' polynomials.
#pragma once

namespace vclb {

struct D2Q9 {
  static constexpr int Q = 9;
  static constexpr int D = 2;
  static constexpr int cx[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static constexpr int cy[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  static constexpr int cz[Q] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr int opp[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  static constexpr double w[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                                  1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
  static constexpr int M[Q][Q] = {
      {1, 1, 1, 1, 1, 1, 1, 1, 1},     {-4, -1, -1, -1, -1, 2, 2, 2, 2},
      {4, -2, -2, -2, -2, 1, 1, 1, 1}, {0, 1, 0, -1, 0, 1, -1, -1, 1},
      {0, -2, 0, 2, 0, 1, -1, -1, 1},  {0, 0, 1, 0, -1, 1, 1, -1, -1},
      {0, 0, -2, 0, 2, 1, 1, -1, -1},  {0, 1, -1, 1, -1, 0, 0, 0, 0},
      {0, 0, 0, 0, 0, 1, -1, 1, -1}};
  // default rates: g relaxes the odd (flux) moments jx, qx, jy, qy at 1/tau_g,
  // f relaxes the stress moments pxx, pxy at 1/tau_f, every other rate is 1.
  static constexpr bool g_flux_row[Q] = {false, false, false, true, true, true, true, false, false};
  static constexpr bool f_stress_row[Q] = {false, false, false, false, false, false, false, true, true};
};

namespace detail {
struct Vel3 { int x, y, z; };
constexpr Vel3 d3q19_c[19] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                              {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                              {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                              {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
// Row k of the d'Humieres basis evaluated at velocity c.  Order: rho, e, eps, jx, qx,
// jy, qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz, pxz, mx, my, mz.  All integer-valued.
constexpr int d3q19_row(int k, Vel3 c) {
  const int x = c.x, y = c.y, z = c.z;
  const int c2 = x * x + y * y + z * z;
  switch (k) {
    case 0: return 1;
    case 1: return 19 * c2 - 30;
    case 2: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
    case 3: return x;
    case 4: return (5 * c2 - 9) * x;
    case 5: return y;
    case 6: return (5 * c2 - 9) * y;
    case 7: return z;
    case 8: return (5 * c2 - 9) * z;
    case 9: return 3 * x * x - c2;
    case 10: return (3 * c2 - 5) * (3 * x * x - c2);
    case 11: return y * y - z * z;
    case 12: return (3 * c2 - 5) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    default: return (x * x - y * y) * z;
  }
}
struct Table19 { int v[19][19]; };
constexpr Table19 d3q19_M() {
  Table19 t{};
  for (int k = 0; k < 19; ++k)
    for (int i = 0; i < 19; ++i) t.v[k][i] = d3q19_row(k, d3q19_c[i]);
  return t;
}
constexpr Table19 kM19 = d3q19_M();
}  // namespace detail

struct D3Q19 {
  static constexpr int Q = 19;
  static constexpr int D = 3;
  static constexpr int cx[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int cz[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr int opp[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
  static constexpr double w[Q] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                                  1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                  1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                  1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
  static constexpr auto& M = detail::kM19.v;
  static constexpr bool g_flux_row[Q] = {false, false, false, true,  true,  true,  true,
                                         true,  true,  false, false, false, false, false,
                                         false, false, false, false, false};
  static constexpr bool f_stress_row[Q] = {false, false, false, false, false, false, false,
                                           false, false, true,  false, true,  false, true,
                                           true,  true,  false, false, false};
};

// squared norm of moment row k (M M^T is diagonal for both bases)
template <class L>
constexpr int row_norm(int k) {
  int s = 0;
  for (int i = 0; i < L::Q; ++i) s += L::M[k][i] * L::M[k][i];
  return s;
}

// Moments of the weighted velocity monomials, sum_i M_ki w_i c_i^a: the building blocks
// of the moments of every equilibrium and source of the model, which are all of the
// form w_i (a + b . c_i + C : c_i c_i) plus a correction at the rest velocity.
template <class L>
constexpr int vel(int i, int d) {
  return d == 0 ? L::cx[i] : (d == 1 ? L::cy[i] : L::cz[i]);
}
template <class L>
constexpr double mom_w(int k) {
  double s = 0.0;
  for (int i = 0; i < L::Q; ++i) s += L::M[k][i] * L::w[i];
  return s;
}
template <class L>
constexpr double mom_wc(int k, int d) {
  double s = 0.0;
  for (int i = 0; i < L::Q; ++i) s += L::M[k][i] * L::w[i] * vel<L>(i, d);
  return s;
}
template <class L>
constexpr double mom_wcc(int k, int d, int e) {
  double s = 0.0;
  for (int i = 0; i < L::Q; ++i) s += L::M[k][i] * L::w[i] * vel<L>(i, d) * vel<L>(i, e);
  return s;
}

}  // namespace vclb
