// mevp_ref.hpp -- compile-time reference-element tables for the gfx950 kernels.
//
// The paper keeps the basis-at-Gauss-point matrices PSI<n, NGP> as compile-time
// constants selected by template parameters (Sec. 3.2, CUDA constant memory
// with `if constexpr`). Here they are constexpr arrays; after full unrolling
// every entry becomes an instruction immediate, so no table is ever loaded.
//
//   Gauss rule   NGP x NGP Gauss-Legendre on [0,1]^2, NGP = 2 for n_s = 3 and
//                3 for n_s = 6, 8 (appendix listing); point q = qy*NGP + qx.
//   DG basis     scaled Legendre products, s = xi - 1/2, t = eta - 1/2:
//                1, s, t, s^2 - 1/12, s t, t^2 - 1/12, (s^2 - 1/12) t, s (t^2 - 1/12),
//                orthogonal on the unit square with norms 1, 1/12, 1/12, 1/180,
//                1/144, 1/180, 1/2160, 1/2160.
//   CG2 basis    biquadratic Lagrange on {0, 1/2, 1}^2, local node a = 3 b + c.
#pragma once

namespace mevp {

template <int NS>
struct Ngp {
  static_assert(NS == 3 || NS == 6 || NS == 8, "n_s must be 3, 6 or 8");
  static constexpr int value = (NS == 3) ? 2 : 3;
};

// Gauss-Legendre abscissae on [0,1] (decimal expansions of 1/2 -+ 1/(2 sqrt 3)
// and 1/2 -+ sqrt(3/5)/2) and weights.
template <int NGP>
struct Gauss1D;
template <>
struct Gauss1D<2> {
  static constexpr double x[2] = {0.21132486540518711774542560974902,
                                  0.78867513459481288225457439025098};
  static constexpr double w[2] = {0.5, 0.5};
};
template <>
struct Gauss1D<3> {
  static constexpr double x[3] = {0.11270166537925831148207346002176, 0.5,
                                  0.88729833462074168851792653997824};
  static constexpr double w[3] = {5.0 / 18.0, 4.0 / 9.0, 5.0 / 18.0};
};

constexpr double dg_fn(int k, double xi, double eta) {
  const double s = xi - 0.5, t = eta - 0.5;
  switch (k) {
    case 0: return 1.0;
    case 1: return s;
    case 2: return t;
    case 3: return s * s - 1.0 / 12.0;
    case 4: return s * t;
    case 5: return t * t - 1.0 / 12.0;
    case 6: return (s * s - 1.0 / 12.0) * t;
    default: return s * (t * t - 1.0 / 12.0);
  }
}

// reference-square norms int psi_k^2
constexpr double dg_norm(int k) {
  switch (k) {
    case 0: return 1.0;
    case 1: case 2: return 1.0 / 12.0;
    case 3: case 5: return 1.0 / 180.0;
    case 4: return 1.0 / 144.0;
    default: return 1.0 / 2160.0;
  }
}

// quadratic Lagrange polynomials on {0, 1/2, 1} and derivatives
constexpr double q2_1d(int i, double t) {
  return i == 0 ? (2.0 * t - 1.0) * (t - 1.0) : (i == 1 ? 4.0 * t * (1.0 - t) : t * (2.0 * t - 1.0));
}
constexpr double q2_1d_d(int i, double t) {
  return i == 0 ? 4.0 * t - 3.0 : (i == 1 ? 4.0 - 8.0 * t : 4.0 * t - 1.0);
}

template <int NGP>
struct Quad {
  static constexpr int NG = NGP * NGP;
  static constexpr double xi(int q) { return Gauss1D<NGP>::x[q % NGP]; }
  static constexpr double eta(int q) { return Gauss1D<NGP>::x[q / NGP]; }
  static constexpr double w(int q) { return Gauss1D<NGP>::w[q % NGP] * Gauss1D<NGP>::w[q / NGP]; }
  // DG basis k at q
  static constexpr double psi(int k, int q) { return dg_fn(k, xi(q), eta(q)); }
  // CG2 basis a, d/dxi, d/deta at q
  static constexpr double phi(int a, int q) { return q2_1d(a % 3, xi(q)) * q2_1d(a / 3, eta(q)); }
  static constexpr double dxi(int a, int q) { return q2_1d_d(a % 3, xi(q)) * q2_1d(a / 3, eta(q)); }
  static constexpr double deta(int a, int q) { return q2_1d(a % 3, xi(q)) * q2_1d_d(a / 3, eta(q)); }
};

}  // namespace mevp

namespace mevp {

// ---------------------------------------------------------------------------
// Exact element operators of a parallelogram (affine) cell.
//
// With a constant Jacobian the strain projection and the weak divergence are
// constant matrices applied to the nodal velocities / DG coefficients, and
// every DG and CG2 function is a product of 1D polynomials, so each entry is a
// product of two exact 1D integrals over [0,1] (written with s = xi - 1/2):
//   P0 = 1, P1 = s, P2 = s^2 - 1/12;  L0 = 2s^2 - s, L1 = 1 - 4s^2, L2 = 2s^2 + s
//   I0[i][b] = int P_i L_b,   I1[i][c] = int P_i L_c'
// (the Gauss rules of the general path integrate the same polynomials exactly).
// ---------------------------------------------------------------------------
constexpr double kI0[3][3] = {{1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0},
                              {-1.0 / 12.0, 0.0, 1.0 / 12.0},
                              {1.0 / 90.0, -1.0 / 45.0, 1.0 / 90.0}};
constexpr double kI1[3][3] = {{-1.0, 0.0, 1.0},
                              {1.0 / 3.0, -2.0 / 3.0, 1.0 / 3.0},
                              {0.0, 0.0, 0.0}};
constexpr double kNorm1D[3] = {1.0, 1.0 / 12.0, 1.0 / 180.0};
// DG function k = P_kx(s) P_ky(t)
constexpr int kDgX[8] = {0, 1, 0, 2, 1, 0, 2, 1};
constexpr int kDgY[8] = {0, 0, 1, 0, 1, 2, 1, 2};

// 1D factors of the DG basis: psi_k(xi, eta) = dg_1d(kDgX[k], xi) dg_1d(kDgY[k], eta)
constexpr double dg_1d(int i, double x) {
  return i == 0 ? 1.0 : (i == 1 ? x - 0.5 : (x - 0.5) * (x - 0.5) - 1.0 / 12.0);
}

// Axi[k][a] = int psi_k dphi_a/dxi, Aeta[k][a] = int psi_k dphi_a/deta over the
// reference square (local node a = 3 b + c).
constexpr double a_xi(int k, int a) { return kI1[kDgX[k]][a % 3] * kI0[kDgY[k]][a / 3]; }
constexpr double a_eta(int k, int a) { return kI0[kDgX[k]][a % 3] * kI1[kDgY[k]][a / 3]; }

// The same with the coordinate of the derivative's direction as a weight,
// for bilinear cells, whose Jacobian entries are affine in one coordinate:
//   I1s[i][c] = int P_i s L_c',
//   AxiS[k][a] = int psi_k s dphi_a/dxi,  AetaT[k][a] = int psi_k t dphi_a/deta
// (exact: the integrands have degree <= 4 per direction, which the Gauss rules
// of the general path also integrate exactly).
constexpr double kI1s[3][3] = {{1.0 / 3.0, -2.0 / 3.0, 1.0 / 3.0},
                               {-1.0 / 12.0, 0.0, 1.0 / 12.0},
                               {1.0 / 45.0, -2.0 / 45.0, 1.0 / 45.0}};
constexpr double a_xi_s(int k, int a) { return kI1s[kDgX[k]][a % 3] * kI0[kDgY[k]][a / 3]; }
constexpr double a_eta_t(int k, int a) { return kI0[kDgX[k]][a % 3] * kI1s[kDgY[k]][a / 3]; }
constexpr double dg_mass(int k) { return kNorm1D[kDgX[k]] * kNorm1D[kDgY[k]]; }

}  // namespace mevp
