#pragma once
// mevp_device.hpp -- gfx950 device code of the mEVP momentum subcycle (included by
// the per-n_s kernel translation units and mevp_kernels.hip).
//
// One subcycle (Table 1 of the paper: strain, stress, divergence, velocity)
// has two parts:
//   element update  one element per lane (element_compute): gather the 9 CG2
//                   velocities, strain rates, L2 projection onto the DG
//                   stress space, the VP stress update of Listing 1, the new
//                   stress and the weak-form nodal forces of the element (18
//                   values). Three cell geometries: parallelograms (constant
//                   Jacobian, diagonal mass matrix, strain and divergence as
//                   exact constant operators), bilinear cells and curved
//                   isoparametric cells (Jacobian per Gauss point from the
//                   cell map, local mass matrix factorised per element).
//   node update     per CG2 node: sum the forces of the <= 4 elements around
//                   it in ascending element order (deterministic, no atomics),
//                   then the lumped-mass velocity update (NodeBatch).
// Kernels: k_fused runs both parts of one subcycle per tile with the forces
// in LDS; k_fused_multi runs K = 2 or 3 subcycles per tile (temporal
// blocking, recomputed halo); k_element + k_node run the parts as separate
// launches with the forces in a scratch array; k_fused_persist runs all
// subcycles of a call in one cooperative launch. All of them share the
// element and node arithmetic, so their results agree bit for bit.
// The cell maps are recomputed from the vertices (or CG2 node positions) in
// every subcycle (the paper's "on-the-fly map", Sec. 3.2) instead of being
// stored.
//
// Arrays are element- or node-fastest (structure of arrays), so consecutive
// lanes touch consecutive addresses for S, H, A, the forces and the node
// arrays; the 3x3 velocity gather of neighbouring elements overlaps and is
// served from L2 (or LDS inside a tile).
#include <hip/hip_cooperative_groups.h>

#include <type_traits>

#include "mevp_index.hpp"
#include "mevp_internal.hpp"
#include "mevp_ref.hpp"

namespace mevp {
namespace {

// An entry of the element matrices -- the operators that the strain,
// projection and divergence contractions apply to the velocities and stress
// coefficients: reference tables, Jacobian factors, quadrature weights times
// |J|, the local mass matrix's factors -- in the arithmetic type T. MP = 1 is
// the bfloat16 trial of the mixed form: each entry rounded to bfloat16 (8
// significant bits, round to nearest even), the arithmetic still in float.
template <class T, int MP>
__device__ __forceinline__ T mat(T x) {
  if constexpr (MP == 0) {
    return x;
  } else {
    static_assert(std::is_same<T, float>::value, "bfloat16 element matrices need float arithmetic");
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
  }
}

// Bilinear cell map from the vertices (0,0), (1,0), (0,1), (1,1) of the
// reference square: J(xi, eta) = [[J00, J01], [J10, J11]] with
//   J00 = (1-eta) ax + eta bx, J01 = (1-xi) cx + xi dx, and the same in y.
template <class T>
struct Cell {
  T ax, bx, cx, dx, ay, by, cy, dy;
  __device__ __forceinline__ void jac(double xi, double eta, T &J00, T &J01, T &J10,
                                      T &J11) const {
    J00 = T(1.0 - eta) * ax + T(eta) * bx;
    J01 = T(1.0 - xi) * cx + T(xi) * dx;
    J10 = T(1.0 - eta) * ay + T(eta) * by;
    J11 = T(1.0 - xi) * cy + T(xi) * dy;
  }
};

template <class T>
__device__ __forceinline__ Cell<T> load_cell(const DomDev &D, const double *vert, int ex, int ey) {
  const double *VX = vert + 2 * (size_t)D.vert_off;
  const double *VY = VX + D.nv;
  const int i0 = ey * (D.nx + 1) + ex, i2 = i0 + D.nx + 1;
  const double X0 = VX[i0], X1 = VX[i0 + 1], X2 = VX[i2], X3 = VX[i2 + 1];
  const double Y0 = VY[i0], Y1 = VY[i0 + 1], Y2 = VY[i2], Y3 = VY[i2 + 1];
  Cell<T> c;
  c.ax = T(X1 - X0);
  c.bx = T(X3 - X2);
  c.cx = T(X2 - X0);
  c.dx = T(X3 - X1);
  c.ay = T(Y1 - Y0);
  c.by = T(Y3 - Y2);
  c.cy = T(Y2 - Y0);
  c.dy = T(Y3 - Y1);
  return c;
}

// Jacobian of a bilinear cell in the form its passes use: each entry is
// affine in one reference coordinate, J00 = J00c + t tx, J10 = J10c + t ty,
// J01 = J01c + s tx, J11 = J11c + s ty (s = xi - 1/2, t = eta - 1/2; centre
// Jacobian and twist tx = (X3 - X2) - (X1 - X0), likewise ty), and the ξη terms
// of |J| cancel, so |J| = c0 + c1 s + c2 t exactly.
template <class T>
struct BilinearJ {
  static constexpr bool kLinearDet = true;
  T J00c, J01c, J10c, J11c, tx, ty, c0, c1, c2;
  __device__ __forceinline__ explicit BilinearJ(const Cell<T> &c) {
    J00c = T(0.5) * (c.ax + c.bx);
    J10c = T(0.5) * (c.ay + c.by);
    J01c = T(0.5) * (c.cx + c.dx);
    J11c = T(0.5) * (c.cy + c.dy);
    tx = c.bx - c.ax;
    ty = c.by - c.ay;
    c0 = J00c * J11c - J01c * J10c;
    c1 = J00c * ty - J10c * tx;
    c2 = J11c * tx - J01c * ty;
  }
  __device__ __forceinline__ void jac(double xi, double eta, T &J00, T &J01, T &J10,
                                      T &J11) const {
    const double sv = xi - 0.5, tv = eta - 0.5;
    J00 = J00c;
    J10 = J10c;
    J01 = J01c;
    J11 = J11c;
    if (tv != 0.0) {
      J00 = J00c + T(tv) * tx;
      J10 = J10c + T(tv) * ty;
    }
    if (sv != 0.0) {
      J01 = J01c + T(sv) * tx;
      J11 = J11c + T(sv) * ty;
    }
  }
  // w |J| at (xi, eta)
  __device__ __forceinline__ T wdet(double w, double xi, double eta) const {
    const double sv = xi - 0.5, tv = eta - 0.5;
    T r = T(w) * c0;
    if (sv != 0.0) r += T(w * sv) * c1;
    if (tv != 0.0) r += T(w * tv) * c2;
    return r;
  }
};

// Local mass matrix M_e = Psi W_e Psi^T (W_e = diag(w_q |J_q|)) factorised as
// L D L^T with unit lower L; solve() applies M_e^-1 in place.
template <int NS, class T>
struct Ldl {
  T L[NS][NS];
  T invd[NS];
  // sum_q w_q f_q psi_k(q) psi_l(q) with f = 1, s or t (which = 0, 1, 2)
  template <class Q>
  static constexpr double moment(int which, int k, int l) {
    double r = 0.0;
    for (int q = 0; q < Q::NG; ++q) {
      const double f = which == 0 ? 1.0 : which == 1 ? Q::xi(q) - 0.5 : Q::eta(q) - 0.5;
      r += Q::w(q) * f * Q::psi(k, q) * Q::psi(l, q);
    }
    return r;
  }
  template <class Q, class Map>
  __device__ __forceinline__ void build(const Map &c) {
    T M[NS][NS];
    if constexpr (Map::kLinearDet) {
      // |J| = c0 + c1 s + c2 t: M = c0 N + c1 S + c2 T with the quadrature's
      // moments (exact: the rule integrates these polynomials exactly)
#pragma unroll
      for (int k = 0; k < NS; ++k)
#pragma unroll
        for (int l = 0; l <= k; ++l) {
          T m = T(0);
          bool have = false;
          const double n0 = moment<Q>(0, k, l), n1 = moment<Q>(1, k, l), n2 = moment<Q>(2, k, l);
          if (n0 != 0.0) {
            m = T(n0) * c.c0;
            have = true;
          }
          if (n1 != 0.0) {
            m = have ? m + T(n1) * c.c1 : T(n1) * c.c1;
            have = true;
          }
          if (n2 != 0.0) m = have ? m + T(n2) * c.c2 : T(n2) * c.c2;
          M[k][l] = m;
        }
    } else {
#pragma unroll
      for (int k = 0; k < NS; ++k)
#pragma unroll
        for (int l = 0; l <= k; ++l) M[k][l] = T(0);
#pragma unroll
      for (int q = 0; q < Q::NG; ++q) {
        const T wd = c.wdet(Q::w(q), Q::xi(q), Q::eta(q));
#pragma unroll
        for (int k = 0; k < NS; ++k)
#pragma unroll
          for (int l = 0; l <= k; ++l) {
            const double pp = Q::psi(k, q) * Q::psi(l, q);
            if (pp != 0.0) M[k][l] += T(pp) * wd;
          }
      }
    }
    T dv[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      T dj = M[j][j];
#pragma unroll
      for (int k = 0; k < j; ++k) dj -= L[j][k] * L[j][k] * dv[k];
      dv[j] = dj;
      invd[j] = T(1) / dj;
#pragma unroll
      for (int i = j + 1; i < NS; ++i) {
        T s = M[i][j];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k] * dv[k];
        L[i][j] = s * invd[j];
      }
    }
  }
  __device__ __forceinline__ void solve(T (&x)[NS]) const {
#pragma unroll
    for (int i = 0; i < NS; ++i)
#pragma unroll
      for (int k = 0; k < i; ++k) x[i] -= L[i][k] * x[k];
#pragma unroll
    for (int i = 0; i < NS; ++i) x[i] *= invd[i];
#pragma unroll
    for (int i = NS - 1; i >= 0; --i)
#pragma unroll
      for (int k = i + 1; k < NS; ++k) x[i] -= L[k][i] * x[k];
  }
};

// The local mass matrix of a general cell factorised (entries rounded to
// bfloat16 for MP = 1, as the element update uses them).
template <int NS, class T, int MP, class Map>
__device__ __forceinline__ void factor_mass(const Map &cell, Ldl<NS, T> &mass) {
  using Q = Quad<Ngp<NS>::value>;
  mass.template build<Q>(cell);
  if constexpr (MP != 0) {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      mass.invd[i] = mat<T, MP>(mass.invd[i]);
#pragma unroll
      for (int k = 0; k < i; ++k) mass.L[i][k] = mat<T, MP>(mass.L[i][k]);
    }
  }
}

// Ice strength at Gauss point q: P = P* max(0, H Psi) exp(-C (1 - min(1, max(0, A Psi))))
// (clamps and formula of the stress listings), always in double.
template <int NA, class Q>
__device__ __forceinline__ double ice_strength(const KParams &p, const double (&Hc)[NA],
                                               const double (&Ac)[NA], int q) {
  double hs = 0.0, as = 0.0;
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    hs += Hc[k] * Q::psi(k, q);
    as += Ac[k] * Q::psi(k, q);
  }
  const double h = fmax(0.0, hs);
  const double a = fmin(1.0, fmax(0.0, as));
  return p.Pstar * h * exp(-p.C * (1.0 - a));
}

// The ice fields of one element as the stress update reads them: the DG
// coefficients of H and A, and with one coefficient each (constant fields)
// the ice strength, the same at every Gauss point, evaluated once when the
// element is loaded instead of in every subcycle.
template <int NA>
struct Ice {
  double H[NA], A[NA];
  double P0;
  template <class Q>
  __device__ __forceinline__ double P(const KParams &p, int q) const {
    if constexpr (NA == 1)
      return P0;
    else
      return ice_strength<NA, Q>(p, H, A, q);
  }
};

template <int NA>
__device__ __forceinline__ Ice<NA> load_ice(const DevArrays &d, const DomDev &D, const KParams &p,
                                            int el) {
  Ice<NA> ice;
  const size_t ne = (size_t)D.ne;
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    ice.H[k] = d.H[((size_t)NA * D.elem_off) + k * ne + el];
    ice.A[k] = d.A[((size_t)NA * D.elem_off) + k * ne + el];
  }
  // psi_0 = 1 at every point, so the rule does not matter for one coefficient
  ice.P0 = NA == 1 ? ice_strength<NA, Quad<3>>(p, ice.H, ice.A, 0) : 0.0;
  return ice;
}

// 1/sqrt(x) for a normal x > 0: the hardware estimate refined by two Newton
// steps y <- y + y (1 - x y^2) / 2, each doubling the number of correct bits.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-(x * y), y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-(x * y), y, 1.0);
  return fma(0.5 * y, e, y);
}

// VP stress at one Gauss point (Listing 1) from the strain in the variables
// A = (e11 + e22)/4, B = (e11 - e22)/8, Q = e12/4. The listing's
//   Delta^2 = Delta_min^2 + 1.25 (e11^2 + e22^2) + 1.5 e11 e22 + e12^2
// is 16 (A^2 + B^2 + Q^2) + Delta_min^2, so
//   P/Delta = (P/4) / sqrt(A^2 + B^2 + Q^2 + Delta_min^2/16)   (in double),
//   s11 = P/Delta (5/8 e11 + 3/8 e22) - P/2 = P/Delta (2A + B) - P/2,
//   s22 = P/Delta (2A - B) - P/2,   s12 = P/Delta e12/4 = P/Delta Q.
template <class T>
__device__ __forceinline__ void vp_stress(const KParams &p, double P, T A, T B, T Q, T &s11,
                                          T &s12, T &s22) {
  const double dA = A, dB = B, dQ = Q;
  const double inner = fma(dA, dA, fma(dB, dB, fma(dQ, dQ, p.dmin2_16)));
  const double PD = (0.25 * P) * rsqrt_nr(inner);  // inner >= Delta_min^2/16, a normal double
  const T tPD = T(PD), thP = T(0.5 * P);
  const T A2 = T(2) * A;
  s11 = tPD * (A2 + B) - thP;
  s22 = tPD * (A2 - B) - thP;
  s12 = tPD * Q;
}

// Velocities of the 9 local nodes of an element whose first node is j0 in
// the LDS table vs of row stride `stride` (interleaved per node). In float
// they are taken relative to local node 0 before narrowing (the gradient of a
// constant is zero), which keeps the strain free of cancellation.
template <class T>
__device__ __forceinline__ void gather_velocity(const double2 *vs, int j0, int stride, T (&vx)[9],
                                                T (&vy)[9]) {
  double2 u[9];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int c = 0; c < 3; ++c) u[3 * b + c] = vs[j0 + b * stride + c];
  double bx = 0.0, by = 0.0;
  if (sizeof(T) < sizeof(double)) {
    bx = u[0].x;
    by = u[0].y;
  }
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    vx[a] = T(u[a].x - bx);
    vy[a] = T(u[a].y - by);
  }
}

// the same for element (ex, ey) of a domain, from the global v array, whose
// velocities are interleaved per node (v[nn][2]: one 16-byte load a node)
template <class T>
__device__ __forceinline__ void load_velocity(const DomDev &D, const double *v, int ex, int ey,
                                              T (&vx)[9], T (&vy)[9]) {
  const double2 *V = reinterpret_cast<const double2 *>(v + 2 * (size_t)D.node_off);
  const int NX = 2 * D.nx + 1, j0 = 2 * ey * NX + 2 * ex;
  double2 u[9];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int c = 0; c < 3; ++c) u[3 * b + c] = V[j0 + b * NX + c];
  double bx = 0.0, by = 0.0;
  if (sizeof(T) < sizeof(double)) {
    bx = u[0].x;
    by = u[0].y;
  }
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    vx[a] = T(u[a].x - bx);
    vy[a] = T(u[a].y - by);
  }
}

// Isoparametric cell map: x(xi, eta) = sum_a X_a phi_a(xi, eta) over the 9
// CG2 nodes (positions relative to local node 0, so that the float variant
// keeps the Jacobian free of cancellation); J from the same reference
// derivative tables as the velocity gradient.
template <class T>
struct Q2Map {
  static constexpr bool kLinearDet = false;
  T x[9], y[9];
  // w |J| at (xi, eta)
  __device__ __forceinline__ T wdet(double w, double xi, double eta) const {
    T J00, J01, J10, J11;
    jac(xi, eta, J00, J01, J10, J11);
    return T(w) * (J00 * J11 - J01 * J10);
  }
  __device__ __forceinline__ void jac(double xi, double eta, T &J00, T &J01, T &J10,
                                      T &J11) const {
    J00 = J01 = J10 = J11 = T(0);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      const double dx = q2_1d_d(a % 3, xi) * q2_1d(a / 3, eta);
      const double dy = q2_1d(a % 3, xi) * q2_1d_d(a / 3, eta);
      if (dx != 0.0) {
        J00 += T(dx) * x[a];
        J10 += T(dx) * y[a];
      }
      if (dy != 0.0) {
        J01 += T(dy) * x[a];
        J11 += T(dy) * y[a];
      }
    }
  }
};

// the 9 node positions of element (ex, ey) relative to its node 0, in both
// precisions (the differences of nearby doubles are exact, and J then sums
// cell-sized terms instead of cancelling absolute coordinates)
template <class T>
__device__ __forceinline__ Q2Map<T> load_q2map(const DomDev &D, const double *xnode, int ex,
                                               int ey) {
  const double *XN = xnode + 2 * (size_t)D.node_off;
  const double *YN = XN + D.nn;
  const int NX = 2 * D.nx + 1, j0 = 2 * ey * NX + 2 * ex;
  const double x0 = XN[j0], y0 = YN[j0];
  Q2Map<T> m;
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int j = j0 + b * NX + c;
      m.x[3 * b + c] = T(XN[j] - x0);
      m.y[3 * b + c] = T(YN[j] - y0);
    }
  return m;
}

// Relaxation of Listing 1: R <- fac S_old + ainv R (R holds Pi_e(s) on entry);
// sold(c, k) is coefficient k of stress component c (11, 12, 22) before the
// update, in T.
template <int NS, class T, class SOld>
__device__ __forceinline__ void relax(const KParams &p, SOld sold, T (&R11)[NS], T (&R12)[NS],
                                      T (&R22)[NS]) {
  const T fac = T(p.fac), ainv = T(p.ainv);
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    R11[k] = fac * sold(0, k) + ainv * R11[k];
    R12[k] = fac * sold(1, k) + ainv * R12[k];
    R22[k] = fac * sold(2, k) + ainv * R22[k];
  }
}

// The stress inside the library is [3][ne][NS]: a component's NS coefficients
// of one element are contiguous (the public layout [3][NS][ne] is converted
// at set_state / get_state), so an element's row moves as 16-byte vectors
// when its size allows (FP64 at n_s = 6, 8; float at n_s = 8), else as
// 8-byte ones (float at n_s = 6) or words.
template <int NS, class TS>
struct StressRow {
  static constexpr int kBytes = NS * (int)sizeof(TS);
  static constexpr int kVec = kBytes % 16 == 0 ? 16 : kBytes % 8 == 0 ? 8 : (int)sizeof(TS);
  static constexpr int kPer = kVec / (int)sizeof(TS);  // coefficients per access
  template <class T>
  __device__ __forceinline__ static void load(const TS *p, T (&r)[NS]) {
    if constexpr (kPer == 1) {
#pragma unroll
      for (int k = 0; k < NS; ++k) r[k] = T(p[k]);
    } else if constexpr (sizeof(TS) == 8) {
      const double2 *q = reinterpret_cast<const double2 *>(p);
#pragma unroll
      for (int i = 0; i < NS / 2; ++i) {
        const double2 v = q[i];
        r[2 * i] = T(v.x);
        r[2 * i + 1] = T(v.y);
      }
    } else if constexpr (kPer == 4) {
      const float4 *q = reinterpret_cast<const float4 *>(p);
#pragma unroll
      for (int i = 0; i < NS / 4; ++i) {
        const float4 v = q[i];
        r[4 * i] = T(v.x);
        r[4 * i + 1] = T(v.y);
        r[4 * i + 2] = T(v.z);
        r[4 * i + 3] = T(v.w);
      }
    } else {
      const float2 *q = reinterpret_cast<const float2 *>(p);
#pragma unroll
      for (int i = 0; i < NS / 2; ++i) {
        const float2 v = q[i];
        r[2 * i] = T(v.x);
        r[2 * i + 1] = T(v.y);
      }
    }
  }
  template <class T>
  __device__ __forceinline__ static void store(TS *p, const T (&r)[NS]) {
    if constexpr (kPer == 1) {
#pragma unroll
      for (int k = 0; k < NS; ++k) p[k] = TS(r[k]);
    } else if constexpr (sizeof(TS) == 8) {
      double2 *q = reinterpret_cast<double2 *>(p);
#pragma unroll
      for (int i = 0; i < NS / 2; ++i) q[i] = double2{double(r[2 * i]), double(r[2 * i + 1])};
    } else if constexpr (kPer == 4) {
      float4 *q = reinterpret_cast<float4 *>(p);
#pragma unroll
      for (int i = 0; i < NS / 4; ++i)
        q[i] = float4{TS(r[4 * i]), TS(r[4 * i + 1]), TS(r[4 * i + 2]), TS(r[4 * i + 3])};
    } else {
      float2 *q = reinterpret_cast<float2 *>(p);
#pragma unroll
      for (int i = 0; i < NS / 2; ++i) q[i] = float2{TS(r[2 * i]), TS(r[2 * i + 1])};
    }
  }
};

// the new stress of element el; vectors for parallelogram cells (kVec), word
// by word for general cells, whose larger update has no registers to spare
template <int NS, class T, class TS, bool kVec = true>
__device__ __forceinline__ void store_stress(TS *S_out, size_t ne, int el, const T (&R11)[NS],
                                             const T (&R12)[NS], const T (&R22)[NS]) {
  if constexpr (kVec) {
    StressRow<NS, TS>::store(S_out + (0 * ne + (size_t)el) * NS, R11);
    StressRow<NS, TS>::store(S_out + (1 * ne + (size_t)el) * NS, R12);
    StressRow<NS, TS>::store(S_out + (2 * ne + (size_t)el) * NS, R22);
  } else {
    TS *row = S_out + (size_t)el * NS;  // the lane's part; components ne * NS apart
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      row[k] = TS(R11[k]);
      row[ne * NS + k] = TS(R12[k]);
      row[2 * ne * NS + k] = TS(R22[k]);
    }
  }
}

// the stress of element el before the update, as stored
template <int NS, class TS>
__device__ __forceinline__ void load_stress(const TS *S_in, size_t ne, int el, TS (&r)[3][NS]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) StressRow<NS, TS>::load(S_in + (c * ne + (size_t)el) * NS, r[c]);
}

// Per-domain base pointers of the buffers a subcycle reads and writes.
template <class TS>
struct DomBufs {
  const double *v_in;
  double *v_out;
  const TS *S_in;
  TS *S_out;
  __device__ __forceinline__ DomBufs(const Bufs &b, const DomDev &D, int ns) {
    v_in = b.v_in + 2 * (size_t)D.node_off;
    v_out = b.v_out + 2 * (size_t)D.node_off;
    S_in = static_cast<const TS *>(b.S_in) + (size_t)3 * ns * D.elem_off;
    S_out = static_cast<TS *>(b.S_out) + (size_t)3 * ns * D.elem_off;
  }
};

// ---------------------------------------------------------------------------
// A DG function sum_k c[k] psi_k at the Gauss points, by sum factorisation
// over the tensor-product basis psi_k = P_kx(xi) P_ky(eta):
//   w[ky][i] = sum_{k: kDgY[k] = ky} c[k] P_kDgX[k](x_i),
//   at(i, j) = sum_ky w[ky][i] P_ky(x_j),
// with the zero factors (P_1 at the centre point) skipped at compile time
// (every index is a constant after unrolling).
// ---------------------------------------------------------------------------
template <int NS, int NGP, class T, int MP = 0>
struct DgGauss {
  T w[3][NGP];
  bool hw[3][NGP];
  __device__ __forceinline__ explicit DgGauss(const T (&c)[NS]) {
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
      for (int i = 0; i < NGP; ++i) {
        T acc = T(0);
        bool have = false;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const double f = dg_1d(kDgX[k], Gauss1D<NGP>::x[i]);
          if (kDgY[k] != ky || f == 0.0) continue;
          acc = have ? acc + c[k] * mat<T, MP>(T(f)) : c[k] * mat<T, MP>(T(f));
          have = true;
        }
        w[ky][i] = acc;
        hw[ky][i] = have;
      }
  }
  __device__ __forceinline__ T at(int i, int j) const {
    T acc = T(0);
    bool have = false;
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
      const double f = dg_1d(ky, Gauss1D<NGP>::x[j]);
      if (!hw[ky][i] || f == 0.0) continue;
      acc = have ? acc + w[ky][i] * mat<T, MP>(T(f)) : w[ky][i] * mat<T, MP>(T(f));
      have = true;
    }
    return acc;
  }
};

// ---------------------------------------------------------------------------
// Geometry of one element as the element update needs it: the constant
// Jacobian of a parallelogram cell, or the bilinear map of a general cell.
// ---------------------------------------------------------------------------
template <class T, int GK>
struct Geo;
template <class T>
struct Geo<T, kGeoAffine> {
  T J00, J01, J10, J11;
  T idet;  // 1 / |J|
};
template <class T>
struct Geo<T, kGeoBilinear> {
  Cell<T> map;
};
template <class T>
struct Geo<T, kGeoIso> {
  Q2Map<T> map;
};

template <class T, int GK>
__device__ __forceinline__ Geo<T, GK> load_geo(const DevArrays &d, const DomDev &D, int ex,
                                               int ey) {
  if constexpr (GK == kGeoAffine) {
    const double *VX = d.vert + 2 * (size_t)D.vert_off;
    const double *VY = VX + D.nv;
    const int i0 = ey * (D.nx + 1) + ex, i2 = i0 + D.nx + 1;
    const double X0 = VX[i0], Y0 = VY[i0];
    Geo<T, kGeoAffine> g;
    g.J00 = T(VX[i0 + 1] - X0);
    g.J10 = T(VY[i0 + 1] - Y0);
    g.J01 = T(VX[i2] - X0);
    g.J11 = T(VY[i2] - Y0);
    g.idet = T(1) / (g.J00 * g.J11 - g.J01 * g.J10);
    return g;
  } else if constexpr (GK == kGeoBilinear) {
    return Geo<T, kGeoBilinear>{load_cell<T>(D, d.vert, ex, ey)};
  } else {
    return Geo<T, kGeoIso>{load_q2map<T>(D, d.xnode, ex, ey)};
  }
}

// ---------------------------------------------------------------------------
// Element update, parallelogram cells: strain -> stress update -> nodal forces.
// J = [[J00, J01], [J10, J11]] is constant, |J| cancels from the projections
// (M_e = |J| diag(int psi_k^2)), and
//   w|J| grad v projected:  R11[k] = J11 (Axi vx)[k] - J10 (Aeta vx)[k], ...
//   divergence:            f_x[a] = -(J11 (Axi^T S11)[a] - J01 (Axi^T S12)[a]
//                                     + J00 (Aeta^T S12)[a] - J10 (Aeta^T S11)[a])
// with the exact reference operators a_xi, a_eta of mevp_ref.hpp.
// Inputs: the geometry, the ice fields, the 9 nodal velocities and sold(c, k)
// (the stress before the update). On return R holds the new stress
// coefficients and fx, fy the forces.
// ---------------------------------------------------------------------------
template <int NS, int NA, class T, int MP = 0, class SOld>
__device__ __forceinline__ void element_affine(const KParams &p, const Geo<T, kGeoAffine> &g,
                                               const Ice<NA> &ice,
                                               const T (&vx)[9], const T (&vy)[9], SOld sold,
                                               T (&R11)[NS], T (&R12)[NS], T (&R22)[NS],
                                               T (&fx)[9], T (&fy)[9]) {
  using Q = Quad<Ngp<NS>::value>;
  constexpr int NG = Q::NG;
  const T J00 = g.J00, J01 = g.J01, J10 = g.J10, J11 = g.J11;
  const T idet = g.idet;

  // ---- strain, projected, in the stress update's variables (vp_stress):
  // EA = (E11 + E22)/4, EB = (E11 - E22)/8, EQ = E12/4 per coefficient, with
  // E11 = (J11 Gxx - J10 Gxe)/|J|, E22 = (J00 Gye - J01 Gyx)/|J|,
  // E12 = ((J00 Gxe - J01 Gxx) + (J11 Gyx - J10 Gye))/(2|J|), G = the
  // reference operators applied to v and divided by the DG norm ----
  const T s4 = T(0.25) * idet, s8 = T(0.125) * idet;
  const T a00 = mat<T, MP>(J00 * s4), a01 = mat<T, MP>(J01 * s4);
  const T a10 = mat<T, MP>(J10 * s4), a11 = mat<T, MP>(J11 * s4);
  const T b00 = mat<T, MP>(J00 * s8), b01 = mat<T, MP>(J01 * s8);
  const T b10 = mat<T, MP>(J10 * s8), b11 = mat<T, MP>(J11 * s8);
  T EA[NS], EB[NS], EQ[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    T gxx = 0, gxe = 0, gyx = 0, gye = 0;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      if (a_xi(k, a) != 0.0) {
        const T c = mat<T, MP>(T(a_xi(k, a) / dg_mass(k)));
        gxx += c * vx[a];
        gyx += c * vy[a];
      }
      if (a_eta(k, a) != 0.0) {
        const T c = mat<T, MP>(T(a_eta(k, a) / dg_mass(k)));
        gxe += c * vx[a];
        gye += c * vy[a];
      }
    }
    // left to right: one multiply and three fused multiply-adds each
    EA[k] = a11 * gxx - a10 * gxe + a00 * gye - a01 * gyx;
    EB[k] = b11 * gxx - b10 * gxe - b00 * gye + b01 * gyx;
    EQ[k] = b00 * gxe - b01 * gxx + b11 * gyx - b10 * gye;
  }

  // ---- stress update ----
  const DgGauss<NS, Ngp<NS>::value, T, MP> gA(EA), gB(EB), gQ(EQ);
#pragma unroll
  for (int k = 0; k < NS; ++k) R11[k] = R12[k] = R22[k] = T(0);
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    const int i = q % Ngp<NS>::value, j = q / Ngp<NS>::value;
    const double P = ice.template P<Q>(p, q);
    T s11, s12, s22;
    vp_stress<T>(p, P, gA.at(i, j), gB.at(i, j), gQ.at(i, j), s11, s12, s22);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      if (Q::psi(k, q) != 0.0) {
        const T pw = mat<T, MP>(T(Q::w(q) * Q::psi(k, q) / dg_mass(k)));
        R11[k] += pw * s11;
        R12[k] += pw * s12;
        R22[k] += pw * s22;
      }
    }
  }
  relax<NS, T>(p, sold, R11, R12, R22);

  // ---- divergence, element part: the adjugate-weighted stress per
  // coefficient first, then the transposed reference operators ----
  T Gxx[NS], Gxe[NS], Gyx[NS], Gye[NS];
  const T m00 = mat<T, MP>(J00), m01 = mat<T, MP>(J01), m10 = mat<T, MP>(J10),
          m11 = mat<T, MP>(J11);
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    Gxx[k] = m11 * R11[k] - m01 * R12[k];
    Gxe[k] = m00 * R12[k] - m10 * R11[k];
    Gyx[k] = m11 * R12[k] - m01 * R22[k];
    Gye[k] = m00 * R22[k] - m10 * R12[k];
  }
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    T bx = 0, by = 0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      if (a_xi(k, a) != 0.0) {
        const T c = mat<T, MP>(T(a_xi(k, a)));
        bx += c * Gxx[k];
        by += c * Gyx[k];
      }
      if (a_eta(k, a) != 0.0) {
        const T c = mat<T, MP>(T(a_eta(k, a)));
        bx += c * Gxe[k];
        by += c * Gye[k];
      }
    }
    fx[a] = -bx;
    fy[a] = -by;
  }
}

// ---------------------------------------------------------------------------
// Element update, general cells (bilinear or isoparametric map): Jacobian per
// Gauss point from the map, local mass matrix M_e = Psi W_e Psi^T factorised
// per element. Same inputs and outputs as element_affine.
// ---------------------------------------------------------------------------
template <int NS, int NA, class T, int MP, class Map, class SOld>
__device__ __forceinline__ void element_general_core(const KParams &p, const Map &cell,
                                                     const Ice<NA> &ice, const T (&vx)[9],
                                                     const T (&vy)[9], SOld sold, T (&R11)[NS],
                                                     T (&R12)[NS], T (&R22)[NS], T (&fx)[9],
                                                     T (&fy)[9], const Ldl<NS, T> *pre);

template <int NS, int NA, class T, int MP = 0, class Map, class SOld>
__device__ __forceinline__ void element_general(const KParams &p, const Map &cell,
                                                const Ice<NA> &ice,
                                                const T (&vx)[9], const T (&vy)[9], SOld sold,
                                                T (&R11)[NS], T (&R12)[NS], T (&R22)[NS],
                                                T (&fx)[9], T (&fy)[9],
                                                const Ldl<NS, T> *pre = nullptr) {
  if constexpr (std::is_same<Map, Cell<T>>::value)
    element_general_core<NS, NA, T, MP>(p, BilinearJ<T>(cell), ice, vx, vy, sold, R11, R12, R22,
                                        fx, fy, pre);
  else
    element_general_core<NS, NA, T, MP>(p, cell, ice, vx, vy, sold, R11, R12, R22, fx, fy, pre);
}

// Map: BilinearJ or Q2Map (jac, wdet, and the mass-matrix build).
template <int NS, int NA, class T, int MP, class Map, class SOld>
__device__ __forceinline__ void element_general_core(const KParams &p, const Map &cell,
                                                     const Ice<NA> &ice, const T (&vx)[9],
                                                     const T (&vy)[9], SOld sold, T (&R11)[NS],
                                                     T (&R12)[NS], T (&R22)[NS], T (&fx)[9],
                                                     T (&fy)[9], const Ldl<NS, T> *pre) {
  using Q = Quad<Ngp<NS>::value>;
  constexpr int NG = Q::NG;

  // ---- strain ----
  T E11[NS], E12[NS], E22[NS];
  if constexpr (Map::kLinearDet) {
    // bilinear cell: J00 = J00c + t tx, J10 = J10c + t ty, J01 = J01c + s tx,
    // J11 = J11c + s ty, so the moments sum_q w psi_k adj(J)^T grad v are the
    // exact constant operators a_xi, a_xi_s, a_eta, a_eta_t applied to v and
    // combined with the cell's coefficients (no Gauss-point loop)
    const T J00c = mat<T, MP>(cell.J00c), J01c = mat<T, MP>(cell.J01c);
    const T J10c = mat<T, MP>(cell.J10c), J11c = mat<T, MP>(cell.J11c);
    const T tx = mat<T, MP>(cell.tx), ty = mat<T, MP>(cell.ty);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      T xi_x = 0, xis_x = 0, eta_x = 0, etat_x = 0, xi_y = 0, xis_y = 0, eta_y = 0, etat_y = 0;
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        if (a_xi(k, a) != 0.0) {
          const T c = mat<T, MP>(T(a_xi(k, a)));
          xi_x += c * vx[a];
          xi_y += c * vy[a];
        }
        if (a_xi_s(k, a) != 0.0) {
          const T c = mat<T, MP>(T(a_xi_s(k, a)));
          xis_x += c * vx[a];
          xis_y += c * vy[a];
        }
        if (a_eta(k, a) != 0.0) {
          const T c = mat<T, MP>(T(a_eta(k, a)));
          eta_x += c * vx[a];
          eta_y += c * vy[a];
        }
        if (a_eta_t(k, a) != 0.0) {
          const T c = mat<T, MP>(T(a_eta_t(k, a)));
          etat_x += c * vx[a];
          etat_y += c * vy[a];
        }
      }
      // int psi_k (J11 dvx/dxi - J10 dvx/deta) and the like
      E11[k] = (J11c * xi_x + ty * xis_x) - (J10c * eta_x + ty * etat_x);
      E22[k] = (J00c * eta_y + tx * etat_y) - (J01c * xi_y + tx * xis_y);
      E12[k] = T(0.5) * (((J00c * eta_x + tx * etat_x) - (J01c * xi_x + tx * xis_x)) +
                         ((J11c * xi_y + ty * xis_y) - (J10c * eta_y + ty * etat_y)));
    }
  } else {
#pragma unroll
  for (int k = 0; k < NS; ++k) E11[k] = E12[k] = E22[k] = T(0);
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    T gxx = 0, gxe = 0, gyx = 0, gye = 0;  // d/dxi and d/deta of vx, vy
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      if (Q::dxi(a, q) != 0.0) {
        gxx += mat<T, MP>(T(Q::dxi(a, q))) * vx[a];
        gyx += mat<T, MP>(T(Q::dxi(a, q))) * vy[a];
      }
      if (Q::deta(a, q) != 0.0) {
        gxe += mat<T, MP>(T(Q::deta(a, q))) * vx[a];
        gye += mat<T, MP>(T(Q::deta(a, q))) * vy[a];
      }
    }
    T J00, J01, J10, J11;
    cell.jac(Q::xi(q), Q::eta(q), J00, J01, J10, J11);
    J00 = mat<T, MP>(J00);
    J01 = mat<T, MP>(J01);
    J10 = mat<T, MP>(J10);
    J11 = mat<T, MP>(J11);
    // w_q |J_q| grad v = w_q adj(J)^T (d/dxi, d/deta) v: the determinant cancels
    const T w = mat<T, MP>(T(Q::w(q)));
    const T e11 = w * (J11 * gxx - J10 * gxe);
    const T e22 = w * (J00 * gye - J01 * gyx);
    const T e12 = T(0.5) * w * ((J00 * gxe - J01 * gxx) + (J11 * gyx - J10 * gye));
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      if (Q::psi(k, q) != 0.0) {
        const T ps = mat<T, MP>(T(Q::psi(k, q)));
        E11[k] += ps * e11;
        E12[k] += ps * e12;
        E22[k] += ps * e22;
      }
    }
  }
  }
  // factorised only now: the velocities are dead, so the factor and the strain
  // moments are the only large arrays live
  Ldl<NS, T> built;
  if (!pre) factor_mass<NS, T, MP>(cell, built);
  const Ldl<NS, T> &mass = pre ? *pre : built;
  mass.solve(E11);
  mass.solve(E12);
  mass.solve(E22);
  // the stress update's variables (vp_stress)
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const T a = T(0.25) * (E11[k] + E22[k]), b = T(0.125) * (E11[k] - E22[k]);
    E11[k] = a;
    E22[k] = b;
    E12[k] = T(0.25) * E12[k];
  }

  // ---- stress update ----
  const DgGauss<NS, Ngp<NS>::value, T, MP> gA(E11), gB(E22), gQ(E12);
#pragma unroll
  for (int k = 0; k < NS; ++k) R11[k] = R12[k] = R22[k] = T(0);
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    const int i = q % Ngp<NS>::value, j = q / Ngp<NS>::value;
    const double P = ice.template P<Q>(p, q);
    T s11, s12, s22;
    vp_stress<T>(p, P, gA.at(i, j), gB.at(i, j), gQ.at(i, j), s11, s12, s22);
    const T wd = mat<T, MP>(cell.wdet(Q::w(q), Q::xi(q), Q::eta(q)));
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      if (Q::psi(k, q) != 0.0) {
        const T pw = mat<T, MP>(T(Q::psi(k, q))) * wd;
        R11[k] += pw * s11;
        R12[k] += pw * s12;
        R22[k] += pw * s22;
      }
    }
  }
  mass.solve(R11);
  mass.solve(R12);
  mass.solve(R22);
  relax<NS, T>(p, sold, R11, R12, R22);

  // ---- divergence, element part: f[a] = -sum_q w_q |J_q| sigma(q) grad phi_a(q)
  //      = -sum_q (dphi_a/dxi Gxi + dphi_a/deta Geta) with G = w_q sigma adj(J)^T ----
  if constexpr (Map::kLinearDet) {
    // bilinear cell: with sigma = sum_k R[k] psi_k and the affine Jacobian
    // entries, f[a] = -sum_k (a_xi Gc + a_xi_s Gt + a_eta Hc + a_eta_t Ht)[k][a]
    // with per-coefficient combinations G, H of the new stress
    const T J00c = mat<T, MP>(cell.J00c), J01c = mat<T, MP>(cell.J01c);
    const T J10c = mat<T, MP>(cell.J10c), J11c = mat<T, MP>(cell.J11c);
    const T tx = mat<T, MP>(cell.tx), ty = mat<T, MP>(cell.ty);
    // coefficient by coefficient (eight combinations live at a time), each
    // node's sums accumulated over k
    T bx[9], by[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) bx[a] = by[a] = T(0);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const T Gxc = J11c * R11[k] - J01c * R12[k], Gxt = ty * R11[k] - tx * R12[k];
      const T Hxc = J00c * R12[k] - J10c * R11[k], Hxt = tx * R12[k] - ty * R11[k];
      const T Gyc = J11c * R12[k] - J01c * R22[k], Gyt = ty * R12[k] - tx * R22[k];
      const T Hyc = J00c * R22[k] - J10c * R12[k], Hyt = tx * R22[k] - ty * R12[k];
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        if (a_xi(k, a) != 0.0) {
          const T c = mat<T, MP>(T(a_xi(k, a)));
          bx[a] += c * Gxc;
          by[a] += c * Gyc;
        }
        if (a_xi_s(k, a) != 0.0) {
          const T c = mat<T, MP>(T(a_xi_s(k, a)));
          bx[a] += c * Gxt;
          by[a] += c * Gyt;
        }
        if (a_eta(k, a) != 0.0) {
          const T c = mat<T, MP>(T(a_eta(k, a)));
          bx[a] += c * Hxc;
          by[a] += c * Hyc;
        }
        if (a_eta_t(k, a) != 0.0) {
          const T c = mat<T, MP>(T(a_eta_t(k, a)));
          bx[a] += c * Hxt;
          by[a] += c * Hyt;
        }
      }
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      fx[a] = -bx[a];
      fy[a] = -by[a];
    }
    return;
  }
#pragma unroll
  for (int a = 0; a < 9; ++a) fx[a] = fy[a] = T(0);
  const DgGauss<NS, Ngp<NS>::value, T, MP> r11(R11), r12(R12), r22(R22);
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    const int i = q % Ngp<NS>::value, j = q / Ngp<NS>::value;
    const T s11 = r11.at(i, j), s12 = r12.at(i, j), s22 = r22.at(i, j);
    T J00, J01, J10, J11;
    cell.jac(Q::xi(q), Q::eta(q), J00, J01, J10, J11);
    J00 = mat<T, MP>(J00);
    J01 = mat<T, MP>(J01);
    J10 = mat<T, MP>(J10);
    J11 = mat<T, MP>(J11);
    const T w = mat<T, MP>(T(Q::w(q)));
    const T gxxi = w * (s11 * J11 - s12 * J01);
    const T gxet = w * (s12 * J00 - s11 * J10);
    const T gyxi = w * (s12 * J11 - s22 * J01);
    const T gyet = w * (s22 * J00 - s12 * J10);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      if (Q::dxi(a, q) != 0.0) {
        fx[a] -= mat<T, MP>(T(Q::dxi(a, q))) * gxxi;
        fy[a] -= mat<T, MP>(T(Q::dxi(a, q))) * gyxi;
      }
      if (Q::deta(a, q) != 0.0) {
        fx[a] -= mat<T, MP>(T(Q::deta(a, q))) * gxet;
        fy[a] -= mat<T, MP>(T(Q::deta(a, q))) * gyet;
      }
    }
  }
}

template <int NS, int NA, class T, int GK, int MP = 0, class SOld>
__device__ __forceinline__ void element_compute(const KParams &p, const Geo<T, GK> &g,
                                                const Ice<NA> &ice,
                                                const T (&vx)[9], const T (&vy)[9], SOld sold,
                                                T (&R11)[NS], T (&R12)[NS], T (&R22)[NS],
                                                T (&fx)[9], T (&fy)[9],
                                                const Ldl<NS, T> *pre = nullptr) {
  if constexpr (GK == kGeoAffine)
    element_affine<NS, NA, T, MP>(p, g, ice, vx, vy, sold, R11, R12, R22, fx, fy);
  else
    element_general<NS, NA, T, MP>(p, g.map, ice, vx, vy, sold, R11, R12, R22, fx, fy, pre);
}

// Element update of element el = (ex, ey) with every input read from global
// memory (v and S of the current subcycle).
template <int NS, int NA, class T, class TS, int GK, int MP = 0>
__device__ __forceinline__ void element_update(const DevArrays &d, const DomDev &D,
                                               const KParams &p, const double *v_in,
                                               const TS *S_in, int el, int ex, int ey,
                                               T (&R11)[NS], T (&R12)[NS], T (&R22)[NS],
                                               T (&fx)[9], T (&fy)[9]) {
  const Geo<T, GK> g = load_geo<T, GK>(d, D, ex, ey);
  T vx[9], vy[9];
  load_velocity<T>(D, v_in - 2 * (size_t)D.node_off, ex, ey, vx, vy);
  const Ice<NA> ice = load_ice<NA>(d, D, p, el);
  const size_t ne = (size_t)D.ne;
  if constexpr (GK == kGeoAffine) {
    // parallelogram cells: the old stress as vectors, up front
    TS so[3][NS];
    load_stress<NS, TS>(S_in, ne, el, so);
    auto sold = [&](int c, int k) { return T(so[c][k]); };
    element_compute<NS, NA, T, GK, MP>(p, g, ice, vx, vy, sold, R11, R12, R22, fx, fy);
  } else {
    // general cells: coefficient by coefficient, where the relaxation needs
    // it (held across their larger update, the row costs an occupancy step)
    const TS *row = S_in + (size_t)el * NS;  // the lane's part; components ne * NS apart
    auto sold = [&](int c, int k) { return T(row[(size_t)c * ne * NS + k]); };
    element_compute<NS, NA, T, GK, MP>(p, g, ice, vx, vy, sold, R11, R12, R22, fx, fy);
  }
}

// Velocity update of one interior node:
//   (c (1+beta) + d) v + b k x v = c beta v^{p-1} + g + d v_o + F
// with c = M^H/dt, b = f M^H, d = m^A rho_o C_o |v_o - v^{p-1}| and
// g = c v^n + m^A tau_a, closed form. The node constants of the step are
// interleaved per node, nc[nn][6] = {c, m^A rho_o C_o, g_x, g_y, v_o,x, v_o,y}
// (48 bytes a node: three 16-byte loads).
__device__ __forceinline__ void velocity_update6(const KParams &p, const double (&o)[6], double ux,
                                                 double uy, double Fx, double Fy, double &vx,
                                                 double &vy);
__device__ __forceinline__ void velocity_update(const KParams &p, const double *nc, int j,
                                                double ux, double uy, double Fx, double Fy,
                                                double &vx, double &vy) {
  const double2 *r = reinterpret_cast<const double2 *>(nc + 6 * (size_t)j);
  const double2 a = r[0], b = r[1], c = r[2];
  const double o[6] = {a.x, a.y, b.x, b.y, c.x, c.y};
  velocity_update6(p, o, ux, uy, Fx, Fy, vx, vy);
}

// velocity_update with the six node constants already loaded
__device__ __forceinline__ void velocity_update6(const KParams &p, const double (&o)[6], double ux,
                                                 double uy, double Fx, double Fy, double &vx,
                                                 double &vy) {
  const double c = o[0], ko = o[1], gx = o[2], gy = o[3], ox = o[4], oy = o[5];
  const double dox = ox - ux, doy = oy - uy;
  const double dd = ko * sqrt(dox * dox + doy * doy);
  const double bb = c * p.f_dt;
  const double cb = c * p.beta;
  const double rx = cb * ux + gx + dd * ox + Fx;
  const double ry = cb * uy + gy + dd * oy + Fy;
  const double aa = c * (1.0 + p.beta) + dd;
  const double den = aa * aa + bb * bb;
  if (den == 0.0) {
    vx = 0.0;
    vy = 0.0;
  } else {
    const double inv = 1.0 / den;
    vx = (aa * rx + bb * ry) * inv;
    vy = (aa * ry - bb * rx) * inv;
  }
}

// ---------------------------------------------------------------------------
// Two-phase subcycle, element kernel: element update, S written in place
// (each lane reads and writes only its own element), forces to scratch.
// ---------------------------------------------------------------------------
template <int NS, int NA, class T, class TS, int GK>
__global__ void __launch_bounds__(kElemBlock) k_element(DevArrays d, KParams p, const Blk *blks,
                                                        Bufs b) {
  const Blk blk = blks[blockIdx.x];
  const DomDev D = d.doms[blk.dom];
  const int el = blk.first + (int)threadIdx.x;
  if (el >= D.ne) return;
  const int ex = el % D.nx, ey = el / D.nx;
  const DomBufs<TS> B(b, D, NS);
  T R11[NS], R12[NS], R22[NS], fx[9], fy[9];
  element_update<NS, NA, T, TS, GK>(d, D, p, B.v_in, B.S_in, el, ex, ey, R11, R12, R22, fx, fy);
  store_stress<NS, T, TS, GK == kGeoAffine>(B.S_out, (size_t)D.ne, el, R11, R12, R22);
  const size_t ne = (size_t)D.ne;
  TS *fe = static_cast<TS *>(d.fe) + (size_t)18 * D.elem_off;
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    fe[a * ne + el] = TS(fx[a]);
    fe[(9 + a) * ne + el] = TS(fy[a]);
  }
}

// ---------------------------------------------------------------------------
// Two-phase subcycle, node kernel: deterministic gather of the element forces
// (ascending element order, no atomics) + velocity update, v in place.
// ---------------------------------------------------------------------------
template <class TF>
__global__ void __launch_bounds__(kNodeBlock) k_node(DevArrays d, KParams p, Bufs b) {
  const Blk blk = d.nblk[blockIdx.x];
  const DomDev D = d.doms[blk.dom];
  const int j = blk.first + (int)threadIdx.x;
  if (j >= D.nn) return;
  const int NX = 2 * D.nx + 1, NY = 2 * D.ny + 1;
  const int ix = j % NX, iy = j / NX;
  const double *vin = b.v_in + 2 * (size_t)D.node_off;
  double *vout = b.v_out + 2 * (size_t)D.node_off;
  if (ix == 0 || iy == 0 || ix == NX - 1 || iy == NY - 1) {
    reinterpret_cast<double2 *>(vout)[j] = double2{0.0, 0.0};
    return;
  }
  // elements around node (ix, iy): for an odd index the one element whose
  // middle node it is, for an even index the elements on both sides
  const int ney = (iy & 1) ? 1 : 2, nex = (ix & 1) ? 1 : 2;
  const int ey0 = (iy & 1) ? (iy - 1) / 2 : iy / 2 - 1;
  const int ex0 = (ix & 1) ? (ix - 1) / 2 : ix / 2 - 1;
  const int b0 = (iy & 1) ? 1 : 2, c0 = (ix & 1) ? 1 : 2;
  const TF *fe = static_cast<const TF *>(d.fe) + (size_t)18 * D.elem_off;
  const size_t ne = (size_t)D.ne;
  double Fx = 0.0, Fy = 0.0;
  for (int t = 0; t < ney; ++t) {
    const int ey = ey0 + t, bb = b0 - 2 * t;
    for (int s = 0; s < nex; ++s) {
      const int ex = ex0 + s, c = c0 - 2 * s;
      const size_t e = (size_t)ey * D.nx + ex;
      const int a = 3 * bb + c;
      Fx += (double)fe[a * ne + e];
      Fy += (double)fe[(9 + a) * ne + e];
    }
  }
  double vx, vy;
  const double2 u = reinterpret_cast<const double2 *>(vin)[j];
  velocity_update(p, d.nc + (size_t)6 * D.node_off, j, u.x, u.y, Fx, Fy, vx, vy);
  reinterpret_cast<double2 *>(vout)[j] = double2{vx, vy};
}

// ---------------------------------------------------------------------------
// Node part of a tile: the velocity update of the CG2 nodes (ix, iy) in
// [ix0, ix1) x [iy0, iy1) of one domain, row-major (consecutive lanes,
// consecutive nodes), each lane taking up to R of them and issuing all their
// loads before the first update. The forces of element (ex, ey) are at
// fl[.][(ey - ey0) * FW + ex - ex0] (every element around an interior node of
// the range must be there); each interior node sums them in ascending element
// order. uin(ix, iy, j, ux, uy) reads v^{p-1} of node j = iy * NX + ix,
// out(ix, iy, j, vx, vy) stores v^p; boundary nodes get v = 0 (Dirichlet).
// ---------------------------------------------------------------------------
template <int R, int NT>
struct NodeBatch {
  int jn[R], ixs[R], iys[R];
  bool act[R], bnd[R];
  double ux[R], uy[R], o[R][6];

  // index the nodes and issue all their loads (v^{p-1} through uin, the six
  // node constants); nothing here reads the element forces, so a kernel may
  // call it before the barrier that publishes them
  template <class UIn>
  __device__ __forceinline__ void load(const DomDev &D, const double *nc, int ix0, int ix1,
                                       int iy0, int iy1, UIn uin) {
    const int tid = (int)threadIdx.x;
    const int NX = 2 * D.nx + 1, NY = 2 * D.ny + 1;
    const int w = ix1 - ix0, n = w * (iy1 - iy0);
    static_assert(R * NT <= 8192, "node rounds beyond the exact float division");
    const float rw = 1.0f / (float)w;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int k = tid + m * NT;
      act[m] = k < n;
      int dx, dy;
      node_in_range(act[m] ? k : 0, w, rw, dx, dy);
      ixs[m] = ix0 + dx;
      iys[m] = iy0 + dy;
      jn[m] = iys[m] * NX + ixs[m];
      bnd[m] = ixs[m] == 0 || iys[m] == 0 || ixs[m] == NX - 1 || iys[m] == NY - 1;
      if (act[m] && !bnd[m]) {
        uin(ixs[m], iys[m], jn[m], ux[m], uy[m]);
        // the node's six constants, interleaved: three 16-byte loads
        const double2 *r = reinterpret_cast<const double2 *>(nc + 6 * (size_t)jn[m]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double2 t = r[c];
          o[m][2 * c] = t.x;
          o[m][2 * c + 1] = t.y;
        }
      }
    }
  }

  // sum the forces of the <= 4 elements around each node in ascending element
  // order (element (ex, ey) at fl[.][(ey - ey0) * FW + ex - ex0]), update and
  // store through out; boundary nodes get v = 0 (Dirichlet)
  template <int NF, int FW, class T, class Out>
  __device__ __forceinline__ void finish(const KParams &p, int ex0, int ey0, const T (*fl)[NF],
                                         Out out) const {
#pragma unroll
    for (int m = 0; m < R; ++m) {
      if (!act[m]) continue;
      if (bnd[m]) {
        out(ixs[m], iys[m], jn[m], 0.0, 0.0);
        continue;
      }
      const int ix = ixs[m], iy = iys[m];
      // the elements around the node: one (odd ix and iy, the centre node),
      // two (an edge node) or four (a vertex node), ((ix-1)/2, (iy-1)/2) the
      // first of them; the node is local node a = 3 b + c of each, b = 1 or 2
      // (odd or even iy) in the first row of elements and 0 in the second,
      // likewise c. All reads are issued at once: a missing element's read
      // stays inside fl (any row, le + FW + 1 < NF + FW) and its value is
      // replaced by +0.0, so the sum, in ascending element order, is the one
      // over the elements that exist.
      int off[4];
      bool two_x, two_y;
      node_force_offsets(ix, iy, ex0, ey0, FW, NF, off, two_x, two_y);
      const T *f = &fl[0][0];
      const T x00 = f[off[0]], x01 = f[off[1]], x10 = f[off[2]], x11 = f[off[3]];
      const T y00 = f[9 * NF + off[0]], y01 = f[9 * NF + off[1]], y10 = f[9 * NF + off[2]],
              y11 = f[9 * NF + off[3]];
      double Fx = 0.0 + (double)x00, Fy = 0.0 + (double)y00;
      Fx += two_x ? (double)x01 : 0.0;
      Fy += two_x ? (double)y01 : 0.0;
      Fx += two_y ? (double)x10 : 0.0;
      Fy += two_y ? (double)y10 : 0.0;
      Fx += (two_x && two_y) ? (double)x11 : 0.0;
      Fy += (two_x && two_y) ? (double)y11 : 0.0;
      double vx, vy;
      velocity_update6(p, o[m], ux[m], uy[m], Fx, Fy, vx, vy);
      out(ix, iy, jn[m], vx, vy);
    }
  }
};

// ---------------------------------------------------------------------------
// Fused subcycle on one tile of EX x EY elements. The tile's first column
// and row are a halo (the elements left of and below the owned
// (EX-1) x (EY-1) block): their forces are recomputed here (their stress is
// not stored; its owner stores it), so every node the tile owns -- CG2
// columns [2 x0, 2 x0 + 2 (EX-1)) and rows likewise, plus the last column /
// row of the domain for the last tile -- finds the forces of all its elements
// in LDS. The forces never leave the chip. v and S are read from the *_in
// buffers and written to the *_out buffers (double buffering: neighbouring
// tiles read the old values while this one writes the new).
// ---------------------------------------------------------------------------
template <int NS, int NA, class T, class TS, int GK, int EX, int EY, int MP = 0>
__device__ __forceinline__ void fused_tile(const DevArrays &d, const KParams &p, const Tile t,
                                           const Bufs &b, T (*fl)[EX * EY]) {
  constexpr int TX = EX - 1, TY = EY - 1, NT = EX * EY;
  const DomDev D = d.doms[t.dom];
  const DomBufs<TS> B(b, D, NS);
  const int tid = (int)threadIdx.x;
  {
    const int lx = tid % EX, ly = tid / EX;
    const int ex = t.x0 - 1 + lx, ey = t.y0 - 1 + ly;
    if (ex >= 0 && ey >= 0 && ex < D.nx && ey < D.ny) {
      const int el = ey * D.nx + ex;
      T R11[NS], R12[NS], R22[NS], fx[9], fy[9];
      element_update<NS, NA, T, TS, GK, MP>(d, D, p, B.v_in, B.S_in, el, ex, ey, R11, R12, R22,
                                            fx, fy);
      if (lx > 0 && ly > 0) store_stress<NS, T, TS, GK == kGeoAffine>(B.S_out, (size_t)D.ne, el, R11, R12, R22);
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        fl[a][tid] = fx[a];
        fl[9 + a][tid] = fy[a];
      }
    }
  }
  // ---- nodes owned by the tile: loads before the barrier, update after ----
  const int NX = 2 * D.nx + 1, NY = 2 * D.ny + 1;
  const NodeRange own = owned_nodes(t.x0, t.y0, TX, TY, D.nx, D.ny, NX, NY);
  const int ix0 = own.ix0, ix1 = own.ix1, iy0 = own.iy0, iy1 = own.iy1;
  constexpr int R = ((2 * EX - 1) * (2 * EY - 1) + NT - 1) / NT;
  auto uin = [&](int, int, int j, double &ux, double &uy) {
    const double2 u = reinterpret_cast<const double2 *>(B.v_in)[j];
    ux = u.x;
    uy = u.y;
  };
  auto out = [&](int, int, int j, double vx, double vy) {
    reinterpret_cast<double2 *>(B.v_out)[j] = double2{vx, vy};
  };
  NodeBatch<R, NT> nb;
  nb.load(D, d.nc + (size_t)6 * D.node_off, ix0, ix1, iy0, iy1, uin);
  __syncthreads();
  nb.template finish<NT, EX, T>(p, t.x0 - 1, t.y0 - 1, fl, out);
}

// ---------------------------------------------------------------------------
// K subcycles on one tile in one pass (temporal blocking, K = 2 or 3). The
// tile of owned (EX-1) x (EY-1) elements (the same tiles as fused_tile) takes
// a halo of K elements on its low sides and K-1 on its high sides; lane
// (lx, ly) holds element (x0-K+lx, y0-K+ly) for the whole pass. Subcycle i:
//   element phase  elements [x0-K+i, x0+TX+K-2-i] (likewise in y): element
//                  update from v in global memory (i = 0) or LDS, and S in
//                  global memory (i = 0) or in the lane's registers; forces
//                  to LDS, the new stress kept in registers (the owned
//                  elements' stress stored at i = K-1);
//   node phase     i < K-1: the nodes of the next element phase, velocity
//                  update in place in LDS; i = K-1: the owned nodes, stored.
// Each node phase's loads (v^{p-1}, node constants) are issued before the
// barrier that publishes the forces when the registers allow (kEarly).
// Every element and node update is the arithmetic of fused_tile, so a pass
// equals K single subcycles bit for bit. Only v^{p-1} / S^{p-1} are read
// and only v^{p+K-1} / S^{p+K-1} written (double buffering as in fused_tile).
// ---------------------------------------------------------------------------
template <int NS, int NA, class T, class TS, int GK, int EX, int EY, int K, int MP = 0>
__global__ void __launch_bounds__((EX + 2 * K - 2) * (EY + 2 * K - 2))
    k_fused_multi(DevArrays d, KParams p, const Tile *tiles, Bufs b) {
  static_assert(K == 2 || K == 3, "two or three subcycles per pass");
  constexpr int TX = EX - 1, TY = EY - 1;
  constexpr int FX = EX + 2 * K - 2, FY = EY + 2 * K - 2, NT = FX * FY;  // lanes = elements
  // nodes of element phase 1, in LDS: [2 (x0-K+1), 2 (x0+TX+K-2)]
  constexpr int VW = 2 * TX + 4 * K - 5, VH = 2 * TY + 4 * K - 5;
  // node loads before the barrier only where the registers allow it: up to 8
  // waves per workgroup (2 per SIMD, 256 VGPRs); larger workgroups need 3
  // waves per SIMD and would spill
  constexpr bool kEarly = (NT + 63) / 64 <= 8;
  __shared__ T fl[18][NT];
  __shared__ double2 vl[VW * VH];  // velocities, interleaved per node
  const Tile t = tiles[blockIdx.x];
  const DomDev D = d.doms[t.dom];
  const DomBufs<TS> B(b, D, NS);
  const int tid = (int)threadIdx.x;
  const int NX = 2 * D.nx + 1, NY = 2 * D.ny + 1;
  const size_t ne = (size_t)D.ne;
  const double *nc = d.nc + (size_t)6 * D.node_off;
  const int ex0 = t.x0 - K, ey0 = t.y0 - K;  // element of lane (0, 0)
  const int jx0 = 2 * (ex0 + 1), jy0 = 2 * (ey0 + 1);  // node of LDS entry (0, 0)
  const int lx = tid % FX, ly = tid / FX;
  const int ex = ex0 + lx, ey = ey0 + ly;
  const bool exists = ex >= 0 && ey >= 0 && ex < D.nx && ey < D.ny;
  const int el = exists ? ey * D.nx + ex : 0;

  Geo<T, GK> g{};
  Ice<NA> ice{};
  Ldl<NS, T> lmass;  // bilinear cells: the local mass factor, once per pass
  T S11[NS], S12[NS], S22[NS];  // the lane's stress, as stored (rounded to TS)
  auto vlds = [&](int ix, int iy) { return (iy - jy0) * VW + (ix - jx0); };
#pragma unroll
  for (int i = 0; i < K; ++i) {
    // ---- element phase i ----
    if (exists && lx >= i && ly >= i && lx < FX - i && ly < FY - i) {
      T vx[9], vy[9];
      T R11[NS], R12[NS], R22[NS], fx[9], fy[9];
      if (i == 0) {
        g = load_geo<T, GK>(d, D, ex, ey);
        ice = load_ice<NA>(d, D, p, el);
        load_velocity<T>(D, B.v_in - 2 * (size_t)D.node_off, ex, ey, vx, vy);
        if constexpr (GK == kGeoBilinear) {
          // general cells: the old stress coefficient by coefficient (see
          // element_update)
          const TS *row = B.S_in + (size_t)el * NS;
          auto sold = [&](int c, int k) { return T(row[(size_t)c * ne * NS + k]); };
          factor_mass<NS, T, MP>(BilinearJ<T>(g.map), lmass);
          element_compute<NS, NA, T, GK, MP>(p, g, ice, vx, vy, sold, R11, R12, R22, fx, fy,
                                             &lmass);
        } else {
          TS so[3][NS];
          load_stress<NS, TS>(B.S_in, ne, el, so);
          auto sold = [&](int c, int k) { return T(so[c][k]); };
          element_compute<NS, NA, T, GK, MP>(p, g, ice, vx, vy, sold, R11, R12, R22, fx, fy);
        }
      } else {
        gather_velocity<T>(vl, vlds(2 * ex, 2 * ey), VW, vx, vy);
        auto sold = [&](int c, int k) { return c == 0 ? S11[k] : c == 1 ? S12[k] : S22[k]; };
        if constexpr (GK == kGeoBilinear)
          element_compute<NS, NA, T, GK, MP>(p, g, ice, vx, vy, sold, R11, R12, R22, fx, fy,
                                             &lmass);
        else
          element_compute<NS, NA, T, GK, MP>(p, g, ice, vx, vy, sold, R11, R12, R22, fx, fy);
      }
      if (i == K - 1) {
        if (lx >= K && ly >= K) store_stress<NS, T, TS, GK == kGeoAffine>(B.S_out, ne, el, R11, R12, R22);
      } else {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          S11[k] = T(TS(R11[k]));
          S12[k] = T(TS(R12[k]));
          S22[k] = T(TS(R22[k]));
        }
      }
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        fl[a][tid] = fx[a];
        fl[9 + a][tid] = fy[a];
      }
    }
    // ---- node phase i: loads before the barrier, update after (kEarly) ----
    if constexpr (!kEarly) __syncthreads();
    if (i < K - 1) {
      // nodes of element phase i+1: [2 (x0-K+i+1), 2 (x0+TX+K-2-i)]
      const NodeRange nr = multi_phase_nodes(t.x0, t.y0, TX, TY, K, i, NX, NY);
      const int ix0 = nr.ix0, ix1 = nr.ix1, iy0 = nr.iy0, iy1 = nr.iy1;
      constexpr int R = (VW * VH + NT - 1) / NT;
      auto out = [&](int ix, int iy, int, double vx, double vy) {
        const int q = vlds(ix, iy);
        vl[q] = double2{vx, vy};
      };
      if (i == 0) {
        auto uin = [&](int, int, int j, double &ux, double &uy) {
          const double2 u = reinterpret_cast<const double2 *>(B.v_in)[j];
          ux = u.x;
          uy = u.y;
        };
        NodeBatch<R, NT> nb;
        nb.load(D, nc, ix0, ix1, iy0, iy1, uin);
        if constexpr (kEarly) __syncthreads();
        nb.template finish<NT, FX, T>(p, ex0, ey0, fl, out);
      } else {
        auto uin = [&](int ix, int iy, int, double &ux, double &uy) {
          const int q = vlds(ix, iy);
          const double2 u = vl[q];
          ux = u.x;
          uy = u.y;
        };
        NodeBatch<R, NT> nb;
        nb.load(D, nc, ix0, ix1, iy0, iy1, uin);
        if constexpr (kEarly) __syncthreads();
        nb.template finish<NT, FX, T>(p, ex0, ey0, fl, out);
      }
    } else {
      // the owned nodes, v to global memory
      const NodeRange own = owned_nodes(t.x0, t.y0, TX, TY, D.nx, D.ny, NX, NY);
      const int ix0 = own.ix0, ix1 = own.ix1, iy0 = own.iy0, iy1 = own.iy1;
      constexpr int R = ((2 * EX - 1) * (2 * EY - 1) + NT - 1) / NT;
      auto uin = [&](int ix, int iy, int, double &ux, double &uy) {
        const int q = vlds(ix, iy);
        const double2 u = vl[q];
        ux = u.x;
        uy = u.y;
      };
      auto out = [&](int, int, int j, double vx, double vy) {
        reinterpret_cast<double2 *>(B.v_out)[j] = double2{vx, vy};
      };
      NodeBatch<R, NT> nb;
      nb.load(D, nc, ix0, ix1, iy0, iy1, uin);
      if constexpr (kEarly) __syncthreads();
      nb.template finish<NT, FX, T>(p, ex0, ey0, fl, out);
    }
    if (i < K - 1) __syncthreads();
  }
}

// Fused subcycle kernel: one tile per workgroup, one subcycle.
// (at least two waves per SIMD: the curved-cell FP64 update would otherwise
// take a few registers past 256 and run one wave per SIMD)
template <int NS, int NA, class T, class TS, int GK, int EX, int EY, int MP = 0>
__global__ void __launch_bounds__(EX *EY) __attribute__((amdgpu_waves_per_eu(2)))
    k_fused(DevArrays d, KParams p, const Tile *tiles,
                                                   Bufs b) {
  __shared__ T fl[18][EX * EY];
  fused_tile<NS, NA, T, TS, GK, EX, EY, MP>(d, p, tiles[blockIdx.x], b, fl);
}

// Persistent form (cooperative launch): the workgroups stay resident for n_sub
// subcycles; in subcycle i every workgroup takes the tiles blockIdx.x,
// blockIdx.x + gridDim.x, ... (the grid is a multiple of 8, so a workgroup
// stays on one XCD's band of the XCD-ordered tile table), with buffers b0 for
// even i and b1 (= b0 swapped) for odd i, and a grid-wide barrier between
// subcycles. Every workgroup runs the same number of barriers, so the grid
// always drains. A kernel of its own: the subcycle loop lets the compiler
// keep loop-invariant constants in registers, which the single-tile kernel
// should not pay for.
template <int NS, int NA, class T, class TS, int GK, int EX, int EY>
__global__ void __launch_bounds__(EX *EY) k_fused_persist(DevArrays d, KParams p,
                                                           const Tile *tiles, int ntiles,
                                                           Bufs b0, Bufs b1, int n_sub) {
  __shared__ T fl[18][EX * EY];
  cooperative_groups::grid_group g = cooperative_groups::this_grid();
  for (int it = 0; it < n_sub; ++it) {
    const Bufs &b = (it & 1) ? b1 : b0;
    for (int i = blockIdx.x; i < ntiles; i += gridDim.x) {
      fused_tile<NS, NA, T, TS, GK, EX, EY>(d, p, tiles[i], b, fl);
      __syncthreads();  // the next tile reuses the LDS
    }
    if (it + 1 < n_sub) g.sync();
  }
}

// ---------------------------------------------------------------------------
// Start of a time step, on the fused kernels' tiles: every element of the
// tile (with its one-element low halo) integrates rho_i h and a against the
// basis functions of its 9 CG2 nodes into LDS, then every interior node the
// tile owns gathers its lumped masses M^H, m^A from the <= 4 elements around
// it in ascending element order and writes the six node constants of the
// velocity update: c = M^H/dt, m^A rho_o C_o, g = c v^n + m^A tau_a (2),
// ocean velocity (2). Boundary nodes (Dirichlet, never updated) get zeros.
// ---------------------------------------------------------------------------

// int rho_i h phi_a and int a phi_a over element (ex, ey) for its 9 local
// nodes a = 3 b + c (phi_a = L_c(xi) L_b(eta)), with h, a clamped at the
// Gauss points as in the stress listings
template <int NS, int NA>
__device__ __forceinline__ void element_masses(const DevArrays &d, const DomDev &D,
                                               const KParams &p, int ex, int ey, double (&mh)[9],
                                               double (&ma)[9]) {
  using Q = Quad<Ngp<NS>::value>;
  constexpr int NGP = Ngp<NS>::value;
  const size_t ne = (size_t)D.ne, e = (size_t)ey * D.nx + ex;
  const double *Hd = d.H + (size_t)NA * D.elem_off;
  const double *Ad = d.A + (size_t)NA * D.elem_off;
  double Hc[NA], Ac[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    Hc[k] = Hd[k * ne + e];
    Ac[k] = Ad[k * ne + e];
  }
  if (NA == 1 && D.kind == kGeoAffine) {
    // parallelogram cell, constant fields: |J|, h and a are constants, and
    // the rule integrates the product of the two quadratics L_c, L_b exactly,
    // to the Simpson weights 1/6, 2/3, 1/6 of [0, 1]
    const Cell<double> cell = load_cell<double>(D, d.vert, ex, ey);
    double J00, J01, J10, J11;
    cell.jac(0.5, 0.5, J00, J01, J10, J11);
    const double det = J00 * J11 - J01 * J10;
    const double h = fmax(0.0, Hc[0]), ac = fmin(1.0, fmax(0.0, Ac[0]));
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      const double wa = (a % 3 == 1 ? 2.0 / 3.0 : 1.0 / 6.0) * (a / 3 == 1 ? 2.0 / 3.0 : 1.0 / 6.0);
      mh[a] = wa * det * p.rho_i * h;
      ma[a] = wa * det * ac;
    }
    return;
  }
  auto integrals = [&](const auto &cell) {
#pragma unroll
    for (int a = 0; a < 9; ++a) mh[a] = ma[a] = 0.0;
#pragma unroll
    for (int q = 0; q < Q::NG; ++q) {
      double J00, J01, J10, J11;
      cell.jac(Q::xi(q), Q::eta(q), J00, J01, J10, J11);
      const double wd = Q::w(q) * (J00 * J11 - J01 * J10);
      double hs = 0.0, as = 0.0;
#pragma unroll
      for (int k = 0; k < NA; ++k) {
        hs += Hc[k] * Q::psi(k, q);
        as += Ac[k] * Q::psi(k, q);
      }
      const double h = fmax(0.0, hs), ac = fmin(1.0, fmax(0.0, as));
      const double x = Gauss1D<NGP>::x[q % NGP], y = Gauss1D<NGP>::x[q / NGP];
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        const double phi = q2_1d(a % 3, x) * q2_1d(a / 3, y);
        mh[a] += wd * p.rho_i * h * phi;
        ma[a] += wd * ac * phi;
      }
    }
  };
  if (D.kind == kGeoIso)
    integrals(load_q2map<double>(D, d.xnode, ex, ey));
  else
    integrals(load_cell<double>(D, d.vert, ex, ey));
}

template <int NS, int NA, int EX, int EY>
__global__ void __launch_bounds__(EX *EY) k_begin_tile(DevArrays d, KParams p, const Tile *tiles,
                                                        const double *v) {
  constexpr int TX = EX - 1, TY = EY - 1, NT = EX * EY;
  constexpr int R = ((2 * EX - 1) * (2 * EY - 1) + NT - 1) / NT;  // node rounds per lane
  __shared__ double fl[18][NT];  // the elements' nodal integrals: rho_i h (0..8), a (9..17)
  const Tile t = tiles[blockIdx.x];
  const DomDev D = d.doms[t.dom];
  const int tid = (int)threadIdx.x;
  {
    const int ex = t.x0 - 1 + tid % EX, ey = t.y0 - 1 + tid / EX;
    if (ex >= 0 && ey >= 0 && ex < D.nx && ey < D.ny) {
      double mh[9], ma[9];
      element_masses<NS, NA>(d, D, p, ex, ey, mh, ma);
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        fl[a][tid] = mh[a];
        fl[9 + a][tid] = ma[a];
      }
    }
  }
  // the owned nodes, up to R per lane: index them and issue their loads
  // (wind, ocean, v^n) before the barrier, as they do not depend on it
  const int NX = 2 * D.nx + 1, NY = 2 * D.ny + 1;
  const size_t nn = (size_t)D.nn, o = 2 * (size_t)D.node_off;
  const NodeRange own = owned_nodes(t.x0, t.y0, TX, TY, D.nx, D.ny, NX, NY);
  const int w = own.ix1 - own.ix0, n = w * (own.iy1 - own.iy0);
  static_assert(R * NT <= 8192, "node rounds beyond the exact float division");
  const float rw = 1.0f / (float)w;
  int ixs[R], iys[R];
  bool act[R], bnd[R];
  double in[R][6];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int k = tid + m * NT;
    act[m] = k < n;
    int dx, dy;
    node_in_range(act[m] ? k : 0, w, rw, dx, dy);
    ixs[m] = own.ix0 + dx;
    iys[m] = own.iy0 + dy;
    bnd[m] = ixs[m] == 0 || iys[m] == 0 || ixs[m] == NX - 1 || iys[m] == NY - 1;
    if (act[m] && !bnd[m]) {
      const size_t j = (size_t)iys[m] * NX + ixs[m];
      in[m][0] = d.wind[o + j];
      in[m][1] = d.wind[o + nn + j];
      in[m][2] = d.ocean[o + j];
      in[m][3] = d.ocean[o + nn + j];
      const double2 u = reinterpret_cast<const double2 *>(v + o)[j];
      in[m][4] = u.x;
      in[m][5] = u.y;
    }
  }
  __syncthreads();
  double *nc = d.nc + (size_t)6 * D.node_off;
  const double *f = &fl[0][0];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    if (!act[m]) continue;
    const int ix = ixs[m], iy = iys[m];
    const size_t j = (size_t)iy * NX + ix;
    if (bnd[m]) {
#pragma unroll
      for (int c = 0; c < 6; ++c) nc[6 * j + c] = 0.0;
      continue;
    }
    // the <= 4 elements around the node, in ascending element order (the
    // force table's layout; a missing element adds +0.0)
    int off[4];
    bool two_x, two_y;
    node_force_offsets(ix, iy, t.x0 - 1, t.y0 - 1, EX, NT, off, two_x, two_y);
    double MH = 0.0 + f[off[0]], mA = 0.0 + f[9 * NT + off[0]];
    MH += two_x ? f[off[1]] : 0.0;
    mA += two_x ? f[9 * NT + off[1]] : 0.0;
    MH += two_y ? f[off[2]] : 0.0;
    mA += two_y ? f[9 * NT + off[2]] : 0.0;
    MH += (two_x && two_y) ? f[off[3]] : 0.0;
    mA += (two_x && two_y) ? f[9 * NT + off[3]] : 0.0;
    const double wx = in[m][0], wy = in[m][1];
    const double sp = sqrt(wx * wx + wy * wy);
    const double c = MH * p.inv_dt;
    // interleaved per node (see velocity_update)
    double2 *r = reinterpret_cast<double2 *>(nc + 6 * j);
    r[0] = double2{c, mA * p.rhoCo};
    r[1] = double2{c * in[m][4] + mA * (p.rhoCa * sp * wx), c * in[m][5] + mA * (p.rhoCa * sp * wy)};
    r[2] = double2{in[m][2], in[m][3]};
  }
}

__global__ void __launch_bounds__(kElemBlock) k_cell_shape(DevArrays d, int dom, int *flag) {
  const DomDev D = d.doms[dom];
  for (int el = blockIdx.x * blockDim.x + threadIdx.x; el < D.ne; el += gridDim.x * blockDim.x) {
    const int ex = el % D.nx, ey = el / D.nx;
    const double *VX = d.vert + 2 * (size_t)D.vert_off;
    const double *VY = VX + D.nv;
    const int i0 = ey * (D.nx + 1) + ex, i2 = i0 + D.nx + 1;
    const bool par = (VX[i0 + 1] - VX[i0] == VX[i2 + 1] - VX[i2]) &&
                     (VY[i0 + 1] - VY[i0] == VY[i2 + 1] - VY[i2]) &&
                     (VX[i2] - VX[i0] == VX[i2 + 1] - VX[i0 + 1]) &&
                     (VY[i2] - VY[i0] == VY[i2 + 1] - VY[i0 + 1]);
    if (!par) *flag = 0;
  }
}

// ---------------------------------------------------------------------------
// Advection of H and A (Sec. 2, Eq. (si:ad); DG with the upwind flux):
// one stage of the three-stage SSP Runge-Kutta scheme,
//   U_out = a U^n + b (U_in + dt M^-1 R(U_in)),
//   R_k = int_K U v.grad psi_k - sum_edges int_edge (v.n) U_up psi_k,
// U_up the trace of K where v.n >= 0 and of the neighbour otherwise (of K on
// the domain boundary), v the CG2 velocity held fixed, 3x3 Gauss points in the
// cell and 3 per edge. One element per lane, both fields, bilinear cells.
// ---------------------------------------------------------------------------
constexpr double kAdvW[3] = {5.0 / 18.0, 4.0 / 9.0, 5.0 / 18.0};
constexpr double kAdvX[3] = {0.11270166537925831148207346002176, 0.5,
                             0.88729833462074168851792653997824};

// gradient of DG function k in reference coordinates
__device__ __forceinline__ void dg_grad_ref(int k, double xi, double eta, double &gx, double &ge) {
  const double s = xi - 0.5, t = eta - 0.5;
  gx = (k == 1) ? 1.0 : (k == 3) ? 2.0 * s : (k == 4) ? t : 0.0;
  ge = (k == 2) ? 1.0 : (k == 5) ? 2.0 * t : (k == 4) ? s : 0.0;
}

// Point values at compile-time points (after unrolling every basis value is a
// constant): terms whose basis value is zero are skipped, which leaves every
// sum of finite values unchanged bit for bit (a CG2 function on an edge
// depends on the edge's three nodes only).
template <int NA>
__device__ __forceinline__ double dg_eval(const double (&c)[NA], double xi, double eta) {
  double u = 0.0;
#pragma unroll
  for (int k = 0; k < NA; ++k)
    if (dg_fn(k, xi, eta) != 0.0) u += c[k] * dg_fn(k, xi, eta);
  return u;
}

__device__ __forceinline__ void cg2_eval(const double (&vx)[9], const double (&vy)[9], double xi,
                                         double eta, double &ux, double &uy) {
  ux = 0.0;
  uy = 0.0;
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const double ph = q2_1d(a % 3, xi) * q2_1d(a / 3, eta);
    if (ph == 0.0) continue;
    ux += vx[a] * ph;
    uy += vy[a] * ph;
  }
}

template <int NA, class Map>
__device__ __forceinline__ void advect_element(const DevArrays &d, const DomDev &D, const Map &cell,
                                               bool curved, int el, int ex, int ey,
                                               const double *v, const double *Hn,
                                               const double *An, const double *Hin,
                                               const double *Ain, double *Hout, double *Aout,
                                               double dt, double ca, double cb);

// One kernel per cell geometry (GK: vertex cells or curved cells), launched on
// that kind's element blocks, so that each keeps its own register budget.
template <int NA, int GK>
__global__ void __launch_bounds__(kElemBlock) k_advect(DevArrays d, const Blk *blks,
                                                       const double *v, const double *Hn,
                                                       const double *An, const double *Hin,
                                                       const double *Ain, double *Hout,
                                                       double *Aout, double dt, double ca,
                                                       double cb) {
  const Blk blk = blks[blockIdx.x];
  const DomDev D = d.doms[blk.dom];
  const int el = blk.first + (int)threadIdx.x;
  if (el >= D.ne) return;
  const int ex = el % D.nx, ey = el / D.nx;
  if constexpr (GK == kGeoIso)
    advect_element<NA>(d, D, load_q2map<double>(D, d.xnode, ex, ey), true, el, ex, ey, v, Hn,
                       An, Hin, Ain, Hout, Aout, dt, ca, cb);
  else
    advect_element<NA>(d, D, load_cell<double>(D, d.vert, ex, ey), false, el, ex, ey, v, Hn, An,
                       Hin, Ain, Hout, Aout, dt, ca, cb);
}

// One stage for element el with cell map `cell`; curved: edge normals from
// the map's tangent at each edge point, else from the edge vector.
template <int NA, class Map>
__device__ __forceinline__ void advect_element(const DevArrays &d, const DomDev &D, const Map &cell,
                                               bool curved, int el, int ex, int ey,
                                               const double *v, const double *Hn,
                                               const double *An, const double *Hin,
                                               const double *Ain, double *Hout, double *Aout,
                                               double dt, double ca, double cb) {
  const size_t ne = (size_t)D.ne, off = (size_t)NA * D.elem_off;
  double vx[9], vy[9];
  load_velocity<double>(D, v, ex, ey, vx, vy);
  double Ue[2][NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    Ue[0][k] = Hin[off + k * ne + el];
    Ue[1][k] = Ain[off + k * ne + el];
  }
  double R[2][NA], M[NA][NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    R[0][k] = R[1][k] = 0.0;
#pragma unroll
    for (int l = 0; l < NA; ++l) M[k][l] = 0.0;
  }
  // ---- cell integral and mass matrix ----
#pragma unroll
  for (int qy = 0; qy < 3; ++qy)
#pragma unroll
    for (int qx = 0; qx < 3; ++qx) {
      const double xi = kAdvX[qx], eta = kAdvX[qy], w = kAdvW[qx] * kAdvW[qy];
      double J00, J01, J10, J11;
      cell.jac(xi, eta, J00, J01, J10, J11);
      const double det = J00 * J11 - J01 * J10;
      double ux, uy;
      cg2_eval(vx, vy, xi, eta, ux, uy);
      // w |J| v.grad psi_k = w v . adj(J)^T grad_ref psi_k
      const double uh = dg_eval<NA>(Ue[0], xi, eta), ua = dg_eval<NA>(Ue[1], xi, eta);
#pragma unroll
      for (int k = 0; k < NA; ++k) {
        double gx, ge;
        dg_grad_ref(k, xi, eta, gx, ge);
        if (gx != 0.0 || ge != 0.0) {  // psi_0 is constant: no volume term
          const double vg = w * (ux * (J11 * gx - J10 * ge) + uy * (J00 * ge - J01 * gx));
          R[0][k] += uh * vg;
          R[1][k] += ua * vg;
        }
#pragma unroll
        for (int l = 0; l < NA; ++l) M[k][l] += w * det * dg_fn(k, xi, eta) * dg_fn(l, xi, eta);
      }
    }
  // ---- edge fluxes: bottom, right, top, left, counter-clockwise ----
  const double *VX = d.vert + 2 * (size_t)D.vert_off;
  const double *VY = VX + D.nv;
  const int i0 = ey * (D.nx + 1) + ex, i2 = i0 + D.nx + 1;
  const int vid[4] = {i0, i0 + 1, i2, i2 + 1};
  const int from[4] = {0, 1, 3, 2}, to[4] = {1, 3, 2, 0};
  const int ddx[4] = {0, 1, 0, -1}, ddy[4] = {-1, 0, 1, 0};
  const double dxu[4] = {1.0, 0.0, -1.0, 0.0}, deu[4] = {0.0, 1.0, 0.0, -1.0};
#pragma unroll
  for (int ed = 0; ed < 4; ++ed) {
    const double ex_t = VX[vid[to[ed]]] - VX[vid[from[ed]]];
    const double ey_t = VY[vid[to[ed]]] - VY[vid[from[ed]]];
    const int fx = ex + ddx[ed], fy = ey + ddy[ed];
    const bool nb = fx >= 0 && fy >= 0 && fx < D.nx && fy < D.ny;
    double Un[2][NA];
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      const size_t f = nb ? (size_t)fy * D.nx + fx : (size_t)el;
      Un[0][k] = Hin[off + k * ne + f];
      Un[1][k] = Ain[off + k * ne + f];
    }
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      const double u = kAdvX[g];
      const double xi = ed == 0 ? u : ed == 1 ? 1.0 : ed == 2 ? 1.0 - u : 0.0;
      const double eta = ed == 0 ? 0.0 : ed == 1 ? u : ed == 2 ? 1.0 : 1.0 - u;
      // outward normal times the edge's length element: (t_y, -t_x) of the
      // tangent t = dx/du along the counter-clockwise edge
      double tx = ex_t, ty = ey_t;
      if (curved) {
        double J00, J01, J10, J11;
        cell.jac(xi, eta, J00, J01, J10, J11);
        tx = J00 * dxu[ed] + J01 * deu[ed];
        ty = J10 * dxu[ed] + J11 * deu[ed];
      }
      const double nlx = ty, nly = -tx;
      double ux, uy;
      cg2_eval(vx, vy, xi, eta, ux, uy);
      const double vn = ux * nlx + uy * nly;
      double uh, ua;
      if (vn >= 0.0 || !nb) {
        uh = dg_eval<NA>(Ue[0], xi, eta);
        ua = dg_eval<NA>(Ue[1], xi, eta);
      } else {  // the same point in the neighbour's reference coordinates
        const double xn = ed == 0 ? u : ed == 1 ? 0.0 : ed == 2 ? 1.0 - u : 1.0;
        const double en = ed == 0 ? 1.0 : ed == 1 ? u : ed == 2 ? 0.0 : 1.0 - u;
        uh = dg_eval<NA>(Un[0], xn, en);
        ua = dg_eval<NA>(Un[1], xn, en);
      }
#pragma unroll
      for (int k = 0; k < NA; ++k) {
        const double wp = kAdvW[g] * vn * dg_fn(k, xi, eta);
        R[0][k] -= wp * uh;
        R[1][k] -= wp * ua;
      }
    }
  }
  // ---- M^-1 R (Cholesky-free LDL^T of the small SPD matrix) and the stage ----
  double L[NA][NA], dv[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    double dj = M[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) dj -= L[j][k] * L[j][k] * dv[k];
    dv[j] = dj;
#pragma unroll
    for (int i = j + 1; i < NA; ++i) {
      double sum = M[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) sum -= L[i][k] * L[j][k] * dv[k];
      L[i][j] = sum / dj;
    }
  }
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    double x[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      x[i] = R[f][i];
#pragma unroll
      for (int k = 0; k < i; ++k) x[i] -= L[i][k] * x[k];
    }
#pragma unroll
    for (int i = 0; i < NA; ++i) x[i] /= dv[i];
#pragma unroll
    for (int i = NA - 1; i >= 0; --i)
#pragma unroll
      for (int k = i + 1; k < NA; ++k) x[i] -= L[k][i] * x[k];
    const double *Un0 = f == 0 ? Hn : An;
    double *Uo = f == 0 ? Hout : Aout;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      const size_t i = off + k * ne + el;
      Uo[i] = ca * Un0[i] + cb * (Ue[f][k] + dt * x[k]);
    }
  }
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
template <int NS, int NA>
inline hipError_t begin_step_t(const DevArrays &d, const KParams &p, const double *v, int shape,
                               int ntiles, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
#define MEVP_BT(SH_)                                                                          \
  if (shape == SH_) {                                                                         \
    constexpr int EX = kTileShapes[SH_][0], EY = kTileShapes[SH_][1];                          \
    hipLaunchKernelGGL((k_begin_tile<NS, NA, EX, EY>), dim3(ntiles), dim3(EX * EY), 0, s, d, p, \
                       d.tiles, v);                                                          \
    return hipGetLastError();                                                                 \
  }
  MEVP_BT(0) MEVP_BT(1) MEVP_BT(2) MEVP_BT(3)
#undef MEVP_BT
  return hipErrorInvalidValue;
}

// Two-phase subcycle: element kernel(s) per geometry kind, then the node kernel.
template <int NS, int NA, class T>
inline hipError_t two_phase_t(const DevArrays &d, const KParams &p, const Launch &L, Bufs b,
                              hipStream_t s) {
  const Blk *blk = d.eblk;
  if (L.n[kGeoAffine] > 0)
    hipLaunchKernelGGL((k_element<NS, NA, T, T, kGeoAffine>), dim3(L.n[kGeoAffine]),
                       dim3(kElemBlock), 0, s, d, p, blk, b);
  blk += L.n[kGeoAffine];
  if (L.n[kGeoBilinear] > 0)
    hipLaunchKernelGGL((k_element<NS, NA, T, T, kGeoBilinear>), dim3(L.n[kGeoBilinear]),
                       dim3(kElemBlock), 0, s, d, p, blk, b);
  blk += L.n[kGeoBilinear];
  if (L.n[kGeoIso] > 0)
    hipLaunchKernelGGL((k_element<NS, NA, T, T, kGeoIso>), dim3(L.n[kGeoIso]), dim3(kElemBlock),
                       0, s, d, p, blk, b);
  return hipGetLastError();
}

// Fused subcycle(s): tile kernel(s) per geometry kind, in GeoKind order; f.depth 2 or 3:
// the kernel that runs that many subcycles per pass.
template <int NS, int NA, class T, int GK, int EX, int EY, int MP = 0>
inline hipError_t fused_one(const DevArrays &d, const KParams &p, const Tile *tiles, int ntiles,
                            const FusedArgs &f, hipStream_t s) {
  if (f.depth == 2) {
    // two subcycles per pass: parallelogram and bilinear cells (the
    // isoparametric map's 18 coordinates per lane do not fit beside them)
    if constexpr (GK != kGeoIso) {
      hipLaunchKernelGGL((k_fused_multi<NS, NA, T, T, GK, EX, EY, 2, MP>), dim3(ntiles),
                         dim3((EX + 2) * (EY + 2)), 0, s, d, p, tiles, f.b0);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  if (f.depth == 3) {
    // three subcycles per pass: built for parallelogram cells and one ice dof
    // only (the general-cell update would spill at this occupancy)
    if constexpr (NA == 1 && GK == kGeoAffine) {
      hipLaunchKernelGGL((k_fused_multi<NS, NA, T, T, GK, EX, EY, 3, MP>), dim3(ntiles),
                         dim3((EX + 4) * (EY + 4)), 0, s, d, p, tiles, f.b0);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  if (!f.persist) {
    hipLaunchKernelGGL((k_fused<NS, NA, T, T, GK, EX, EY, MP>), dim3(ntiles), dim3(EX * EY), 0, s,
                       d, p, tiles, f.b0);
    return hipGetLastError();
  }
  if constexpr (MP != 0) {
    return hipErrorInvalidValue;  // no persistent form of the trial
  } else {
    auto kern = k_fused_persist<NS, NA, T, T, GK, EX, EY>;
    int per_cu = 0, dev = 0, n_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, EX * EY, 0);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    int grid = per_cu * n_cu;
    if (grid > ntiles) grid = ntiles;
    if (grid >= kNumXcd) grid -= grid % kNumXcd;
    if (grid < 1) return hipErrorInvalidValue;
    DevArrays dd = d;
    KParams pp = p;
    const Tile *tt = tiles;
    int nt = ntiles, ns = f.n_sub;
    Bufs b0 = f.b0, b1 = f.b1;
    void *args[] = {&dd, &pp, &tt, &nt, &b0, &b1, &ns};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kern), dim3(grid), dim3(EX * EY),
                                      args, 0, s);
  }
}

// MP = 1 (the bfloat16 trial): parallelogram and bilinear cells, launched from
// the unit that instantiates fused_t with it
template <int NS, int NA, class T, int EX, int EY, int MP = 0>
inline hipError_t fused_shape(const DevArrays &d, const KParams &p, const Launch &L,
                              const FusedArgs &f, hipStream_t s) {
  hipError_t e = hipSuccess;
  const Tile *t = d.tiles;
  if (L.n[kGeoAffine] > 0) {
    if constexpr (MP == 0)
      e = fused_affine<NS, NA, T, EX, EY>(d, p, t, L.n[kGeoAffine], f, s);
    else
      e = fused_one<NS, NA, T, kGeoAffine, EX, EY, MP>(d, p, t, L.n[kGeoAffine], f, s);
  }
  t += L.n[kGeoAffine];
  if (e == hipSuccess && L.n[kGeoBilinear] > 0)
    e = fused_one<NS, NA, T, kGeoBilinear, EX, EY, MP>(d, p, t, L.n[kGeoBilinear], f, s);
  t += L.n[kGeoBilinear];
  if (e == hipSuccess && L.n[kGeoIso] > 0) {
    if constexpr (MP == 0)
      e = fused_one<NS, NA, T, kGeoIso, EX, EY>(d, p, t, L.n[kGeoIso], f, s);
    else
      e = hipErrorInvalidValue;
  }
  return e;
}

template <int NS, int NA, class T, int MP = 0>
inline hipError_t fused_t(const DevArrays &d, const KParams &p, const Launch &L,
                          const FusedArgs &f, hipStream_t s) {
  if (f.shape == 0)
    return fused_shape<NS, NA, T, kTileShapes[0][0], kTileShapes[0][1], MP>(d, p, L, f, s);
  if constexpr (NA == 1) {  // the other tile shapes are built for one ice dof only
    if (f.shape == 1)
      return fused_shape<NS, NA, T, kTileShapes[1][0], kTileShapes[1][1], MP>(d, p, L, f, s);
    if (f.shape == 2)
      return fused_shape<NS, NA, T, kTileShapes[2][0], kTileShapes[2][1], MP>(d, p, L, f, s);
    if (f.shape == 3)
      return fused_shape<NS, NA, T, kTileShapes[3][0], kTileShapes[3][1], MP>(d, p, L, f, s);
  }
  return hipErrorInvalidValue;
}


// Launchers of one n_s for every n_a and precision; each kernel translation
// unit instantiates them for its n_s.
template <int NS>
inline hipError_t begin_step_ns(const DevArrays &d, const KParams &p, int n_a, const double *v,
                                int shape, int ntiles, hipStream_t s) {
  static_assert(kNumTileShapes == 4, "begin_step_t dispatches on the four tile shapes");
  if (n_a == 1) return begin_step_t<NS, 1>(d, p, v, shape, ntiles, s);
  if (n_a == 3) return begin_step_t<NS, 3>(d, p, v, shape, ntiles, s);
  if (n_a == 6) return begin_step_t<NS, 6>(d, p, v, shape, ntiles, s);
  return hipErrorInvalidValue;
}

template <int NS>
inline hipError_t two_phase_ns(const DevArrays &d, const KParams &p, int n_a, bool mixed,
                               const Launch &L, Bufs b, hipStream_t s) {
#define MEVP_TP(NA_) \
  if (n_a == NA_) return mixed ? two_phase_t<NS, NA_, float>(d, p, L, b, s) : two_phase_t<NS, NA_, double>(d, p, L, b, s);
  MEVP_TP(1) MEVP_TP(3) MEVP_TP(6)
#undef MEVP_TP
  return hipErrorInvalidValue;
}

template <int NS>
inline hipError_t fused_ns(const DevArrays &d, const KParams &p, int n_a, bool mixed,
                           const Launch &L, const FusedArgs &f, hipStream_t s) {
#define MEVP_FU(NA_) \
  if (n_a == NA_) return mixed ? fused_t<NS, NA_, float>(d, p, L, f, s) : fused_t<NS, NA_, double>(d, p, L, f, s);
  MEVP_FU(1) MEVP_FU(3) MEVP_FU(6)
#undef MEVP_FU
  return hipErrorInvalidValue;
}

}  // namespace
}  // namespace mevp
