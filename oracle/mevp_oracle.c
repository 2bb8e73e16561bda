/*
 * mevp_oracle.c -- plain FP64 CPU reference of the mEVP momentum subcycle.
 *
 * TEST INFRASTRUCTURE ONLY: called by the test suite, the smoke check and the
 * CPU baseline leg of the benchmark, never by the product path. Plain loops in
 * the order the method states them; nothing is blocked, fused or reordered.
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off [-fopenmp]. OpenMP only
 * splits independent elements or nodes across threads; every sum is taken in
 * the same order for any thread count.
 *
 * Readings of the paper (where it is silent or inconsistent), all chosen here:
 *  R1 relaxation: the listings' (1 - 1/alpha) S + (1/alpha) M^-1(...) by
 *     default; Eq. (si:mevp)'s alpha/(1+alpha), 1/(1+alpha) via relax_form=1.
 *  R2 Delta uses the strain-rate values at the Gauss points (appendix listing),
 *     not the DG coefficients printed in Listing 1.
 *  R3 viscous law: the listings' constants, i.e. Hibler's ellipse with e = 2.
 *  R4 Delta = sqrt(Delta_min^2 + ...), the form both listings print.
 *  R5 Gauss rule: NGP x NGP tensor Gauss-Legendre, NGP = 3 for ns in {6,8},
 *     2 for ns = 3 (appendix listing).
 *  R6 DG basis: scaled Legendre products on the reference square [0,1]^2,
 *     orthogonal there: 1, s, t, s^2-1/12, s t, t^2-1/12, (s^2-1/12) t,
 *     s (t^2-1/12) with s = xi-1/2, t = eta-1/2.
 *  R7 velocity: biquadratic (Q2) Lagrange on the 3x3 local nodes {0,1/2,1}^2,
 *     local node a = 3 b + c (c along xi, b along eta).
 *  R8 geometry: bilinear map of the 4 element vertices (the "on-the-fly map"
 *     of Sec. 3.2, four vertices with two values each); planar coordinates.
 *     Isoparametric variant (Sec. 2.1: the cell map in the velocity's finite
 *     element space): x(xi, eta) = sum_a X_a phi_a(xi, eta) over the 9 CG2
 *     nodes of the cell, so cell edges may be curved (quadratic).
 *  R9 strain: eps11 = dvx/dx, eps22 = dvy/dy, eps12 = (dvx/dy + dvy/dx)/2 at
 *     the Gauss points, L2-projected onto the DG stress space (same projection
 *     M^-1 Psi W as the stress update's iMJwPSI).
 *  R10 divergence: weak form, f_e[a] = -sum_q w_q|J_q| sigma(q) grad phi_a(q)
 *     with the new stress; nodal sums in ascending element order.
 *  R11 velocity update: lumped-mass semi-discrete form of Eq. (si:momentum)
 *     under the mEVP pseudo-time relaxation beta:
 *       (M^H/dt)[beta (v^p - v^{p-1}) + v^p - v^n] = F + m^A tau_a
 *          + m^A rho_o C_o |v_o - v^{p-1}| (v_o - v^p) - f M^H k x v^p,
 *     with M^H_j = int rho_i h phi_j and m^A_j = int a phi_j (lumped),
 *     tau_a = rho_a C_a |v_a| v_a, the ocean drag magnitude lagged and the
 *     Coriolis term implicit (a closed-form 2x2 solve).
 *  R12 boundary: v = 0 on all CG2 nodes of the outer boundary.
 *  R13 state: S persists between time steps, v^n is v at the start of a step.
 *  R14 advection (Sec. 2 and Eq. (si:ad): DG in space with the standard upwind
 *     flux, explicit Runge-Kutta in time; sources S_H = S_A = 0): for each DG
 *     test function psi_k of the n_a-dof space,
 *       M_e dU/dt = int_K U v.grad psi_k - sum over the 4 edges of
 *                   int_edge (v.n) U_up psi_k,
 *     with U_up the trace of K where v.n >= 0 and of the neighbour otherwise
 *     (the trace of K on the domain boundary, where v = 0 anyway), v the
 *     CG2 velocity at the start of the step, held fixed, 3x3 Gauss points in
 *     the cell and 3 per edge, and the three-stage SSP Runge-Kutta scheme
 *     U1 = U + dt L(U), U2 = 3/4 U + 1/4 (U1 + dt L(U1)),
 *     U^{n+1} = 1/3 U + 2/3 (U2 + dt L(U2)).
 */
#include "mevp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXG 9 /* max Gauss points per element */
#define MAXS 8 /* max DG stress dofs */

struct or_mesh {
  int nx, ny, ns, na, ngp, ng;
  double gp[3], gw[3];
  double psiS[MAXS][MAXG];
  double psiA[6][MAXG];
  double phi[9][MAXG];
  /* per element: w_q|J_q|, gradients of the 9 CG2 basis functions, Cholesky factor of M_e */
  double *wdet;  /* [ne][ng] */
  double *dphix; /* [ne][9][ng] */
  double *dphiy; /* [ne][9][ng] */
  double *chol;  /* [ne][ns][ns], lower triangle */
  double *vx, *vy; /* copy of the vertices [(nx+1)(ny+1)] */
  int iso;         /* 1: isoparametric CG2 map from the node coordinates below */
  double *nx_, *ny_; /* CG2 node coordinates [(2nx+1)(2ny+1)] (iso only) */
};

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads for the following calls (n >= 1). The results do not depend on it:
 * every parallel loop writes disjoint outputs and sums in a fixed order. */
void or_set_num_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ---------------------------------------------------------------------------
 * Reference element (R5-R7)
 * ------------------------------------------------------------------------- */

static int ngp_for(int ns) { return ns == 3 ? 2 : ((ns == 6 || ns == 8) ? 3 : -1); }

/* Gauss-Legendre points and weights mapped to [0,1]. */
static void gauss_rule(int ngp, double *x, double *w) {
  if (ngp == 2) {
    double d = 0.5 / sqrt(3.0);
    x[0] = 0.5 - d;
    x[1] = 0.5 + d;
    w[0] = 0.5;
    w[1] = 0.5;
  } else {
    double d = 0.5 * sqrt(0.6);
    x[0] = 0.5 - d;
    x[1] = 0.5;
    x[2] = 0.5 + d;
    w[0] = 5.0 / 18.0;
    w[1] = 4.0 / 9.0;
    w[2] = 5.0 / 18.0;
  }
}

/* DG basis function k at (xi, eta) (R6). */
static double dg_basis(int k, double xi, double eta) {
  double s = xi - 0.5, t = eta - 0.5;
  switch (k) {
    case 0: return 1.0;
    case 1: return s;
    case 2: return t;
    case 3: return s * s - 1.0 / 12.0;
    case 4: return s * t;
    case 5: return t * t - 1.0 / 12.0;
    case 6: return (s * s - 1.0 / 12.0) * t;
    case 7: return s * (t * t - 1.0 / 12.0);
  }
  return 0.0;
}

/* 1D quadratic Lagrange polynomials on {0, 1/2, 1} and their derivatives (R7). */
static double lag2(int i, double t) {
  if (i == 0) return (1.0 - t) * (1.0 - 2.0 * t);
  if (i == 1) return 4.0 * t * (1.0 - t);
  return t * (2.0 * t - 1.0);
}
static double dlag2(int i, double t) {
  if (i == 0) return 4.0 * t - 3.0;
  if (i == 1) return 4.0 - 8.0 * t;
  return 4.0 * t - 1.0;
}

/* Gauss point q = qy*ngp + qx -> (xi, eta), weight. */
static void gauss_point(const or_mesh *m, int q, double *xi, double *eta, double *w) {
  int qx = q % m->ngp, qy = q / m->ngp;
  *xi = m->gp[qx];
  *eta = m->gp[qy];
  *w = m->gw[qx] * m->gw[qy];
}

int or_tables(int ns, int na, double *gpts, double *gwts, double *psiS, double *psiA,
              double *phi, double *dxi, double *deta) {
  int ngp = ngp_for(ns);
  if (ngp < 0) return -1;
  double x[3], w[3];
  gauss_rule(ngp, x, w);
  int ng = ngp * ngp;
  for (int i = 0; i < ngp; ++i) {
    if (gpts) gpts[i] = x[i];
    if (gwts) gwts[i] = w[i];
  }
  for (int q = 0; q < ng; ++q) {
    double xi = x[q % ngp], eta = x[q / ngp];
    if (psiS)
      for (int k = 0; k < ns; ++k) psiS[k * ng + q] = dg_basis(k, xi, eta);
    if (psiA)
      for (int k = 0; k < na; ++k) psiA[k * ng + q] = dg_basis(k, xi, eta);
    for (int a = 0; a < 9; ++a) {
      int b = a / 3, c = a % 3;
      if (phi) phi[a * ng + q] = lag2(c, xi) * lag2(b, eta);
      if (dxi) dxi[a * ng + q] = dlag2(c, xi) * lag2(b, eta);
      if (deta) deta[a * ng + q] = lag2(c, xi) * dlag2(b, eta);
    }
  }
  return ng;
}

/* ---------------------------------------------------------------------------
 * Mesh, bilinear element map and local mass matrix (R8; Listing 1 caption:
 * M_i^-1 is the inverse local mass matrix scaled by the transformation weights)
 * ------------------------------------------------------------------------- */

static int vert_index(const or_mesh *m, int ix, int iy) { return iy * (m->nx + 1) + ix; }
static int node_index(const or_mesh *m, int ix, int iy) { return iy * (2 * m->nx + 1) + ix; }

/* global CG2 node of local node a of element e */
static int local_to_global(const or_mesh *m, int e, int a) {
  int ex = e % m->nx, ey = e / m->nx;
  int b = a / 3, c = a % 3;
  return node_index(m, 2 * ex + c, 2 * ey + b);
}

/* Cholesky factorisation A = L L^T of an n x n SPD matrix (lower triangle). */
static int cholesky(int n, const double *A, double *L) {
  memset(L, 0, sizeof(double) * n * n);
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
    if (!(d > 0.0)) return -1;
    L[j * n + j] = sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = s / L[j * n + j];
    }
  }
  return 0;
}

/* Solve L L^T x = b in place. */
static void chol_solve(int n, const double *L, double *x) {
  for (int i = 0; i < n; ++i) {
    double s = x[i];
    for (int k = 0; k < i; ++k) s -= L[i * n + k] * x[k];
    x[i] = s / L[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * x[k];
    x[i] = s / L[i * n + i];
  }
}

/* J = d(x, y)/d(xi, eta) of element e at (xi, eta): J[0] = dx/dxi,
 * J[1] = dx/deta, J[2] = dy/dxi, J[3] = dy/deta. Bilinear map of the 4
 * vertices (R8), or the isoparametric map of the 9 CG2 nodes. */
static void map_jacobian(const or_mesh *m, int e, double xi, double eta, double *J) {
  int ex = e % m->nx, ey = e / m->nx;
  if (!m->iso) {
    int vi[4] = {vert_index(m, ex, ey), vert_index(m, ex + 1, ey), vert_index(m, ex, ey + 1),
                 vert_index(m, ex + 1, ey + 1)};
    double X[4], Y[4];
    for (int i = 0; i < 4; ++i) {
      X[i] = m->vx[vi[i]];
      Y[i] = m->vy[vi[i]];
    }
    J[0] = (1.0 - eta) * (X[1] - X[0]) + eta * (X[3] - X[2]);
    J[1] = (1.0 - xi) * (X[2] - X[0]) + xi * (X[3] - X[1]);
    J[2] = (1.0 - eta) * (Y[1] - Y[0]) + eta * (Y[3] - Y[2]);
    J[3] = (1.0 - xi) * (Y[2] - Y[0]) + xi * (Y[3] - Y[1]);
    return;
  }
  /* positions relative to the cell's local node 0: the derivatives of the
   * CG2 basis sum to zero, so J is unchanged, and the sum no longer cancels
   * absolute coordinates far larger than the cell */
  int j0 = local_to_global(m, e, 0);
  double x0 = m->nx_[j0], y0 = m->ny_[j0];
  J[0] = J[1] = J[2] = J[3] = 0.0;
  for (int a = 0; a < 9; ++a) {
    int j = local_to_global(m, e, a);
    double dx = dlag2(a % 3, xi) * lag2(a / 3, eta);
    double dy = lag2(a % 3, xi) * dlag2(a / 3, eta);
    J[0] += (m->nx_[j] - x0) * dx;
    J[1] += (m->nx_[j] - x0) * dy;
    J[2] += (m->ny_[j] - y0) * dx;
    J[3] += (m->ny_[j] - y0) * dy;
  }
}

/* Mesh record with the reference tables, without geometry. */
static or_mesh *mesh_alloc(int nx, int ny, int ns, int na) {
  if (nx < 1 || ny < 1) return NULL;
  if (ngp_for(ns) < 0 || !(na == 1 || na == 3 || na == 6)) return NULL;
  or_mesh *m = (or_mesh *)calloc(1, sizeof(or_mesh));
  if (!m) return NULL;
  m->nx = nx;
  m->ny = ny;
  m->ns = ns;
  m->na = na;
  m->ngp = ngp_for(ns);
  m->ng = m->ngp * m->ngp;
  gauss_rule(m->ngp, m->gp, m->gw);
  for (int q = 0; q < m->ng; ++q) {
    double xi, eta, w;
    gauss_point(m, q, &xi, &eta, &w);
    for (int k = 0; k < ns; ++k) m->psiS[k][q] = dg_basis(k, xi, eta);
    for (int k = 0; k < na; ++k) m->psiA[k][q] = dg_basis(k, xi, eta);
    for (int a = 0; a < 9; ++a) m->phi[a][q] = lag2(a % 3, xi) * lag2(a / 3, eta);
  }
  size_t ne = (size_t)nx * ny, ng = m->ng;
  m->wdet = (double *)malloc(sizeof(double) * ne * ng);
  m->dphix = (double *)malloc(sizeof(double) * ne * 9 * ng);
  m->dphiy = (double *)malloc(sizeof(double) * ne * 9 * ng);
  m->chol = (double *)malloc(sizeof(double) * ne * ns * ns);
  size_t nv = (size_t)(nx + 1) * (ny + 1);
  m->vx = (double *)malloc(sizeof(double) * nv);
  m->vy = (double *)malloc(sizeof(double) * nv);
  if (!m->wdet || !m->dphix || !m->dphiy || !m->chol || !m->vx || !m->vy) {
    or_mesh_destroy(m);
    return NULL;
  }
  return m;
}

/* Per-element geometry at the Gauss points and the Cholesky factor of M_e;
 * -1 if some Jacobian determinant is not positive. */
static int mesh_geometry(or_mesh *m) {
  size_t ne = (size_t)m->nx * m->ny, ng = m->ng;
  int ns = m->ns;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (long e = 0; e < (long)ne; ++e) {
    double *wd = m->wdet + e * ng, *gx = m->dphix + e * 9 * ng, *gy = m->dphiy + e * 9 * ng;
    for (int q = 0; q < m->ng; ++q) {
      double xi, eta, w, J[4];
      gauss_point(m, q, &xi, &eta, &w);
      map_jacobian(m, (int)e, xi, eta, J);
      double J00 = J[0], J01 = J[1], J10 = J[2], J11 = J[3];
      double det = J00 * J11 - J01 * J10;
      if (!(det > 0.0)) bad = 1;
      wd[q] = w * det;
      /* grad phi = J^{-T} (dphi/dxi, dphi/deta) */
      for (int a = 0; a < 9; ++a) {
        double dx = dlag2(a % 3, xi) * lag2(a / 3, eta);
        double dy = lag2(a % 3, xi) * dlag2(a / 3, eta);
        gx[a * ng + q] = (J11 * dx - J10 * dy) / det;
        gy[a * ng + q] = (-J01 * dx + J00 * dy) / det;
      }
    }
    /* M_e = Psi W Psi^T, W = diag(w_q |J_q|) */
    double M[MAXS * MAXS];
    for (int k = 0; k < ns; ++k)
      for (int l = 0; l < ns; ++l) {
        double s = 0.0;
        for (int q = 0; q < m->ng; ++q) s += m->psiS[k][q] * wd[q] * m->psiS[l][q];
        M[k * ns + l] = s;
      }
    if (cholesky(ns, M, m->chol + e * ns * ns) != 0) bad = 1;
  }
  return bad ? -1 : 0;
}

or_mesh *or_mesh_create(int nx, int ny, int ns, int na, const double *vertices) {
  if (!vertices) return NULL;
  or_mesh *m = mesh_alloc(nx, ny, ns, na);
  if (!m) return NULL;
  size_t nv = (size_t)(nx + 1) * (ny + 1);
  memcpy(m->vx, vertices, sizeof(double) * nv);
  memcpy(m->vy, vertices + nv, sizeof(double) * nv);
  if (mesh_geometry(m) != 0) {
    or_mesh_destroy(m);
    return NULL;
  }
  return m;
}

or_mesh *or_mesh_create_iso(int nx, int ny, int ns, int na, const double *nodes) {
  if (!nodes) return NULL;
  or_mesh *m = mesh_alloc(nx, ny, ns, na);
  if (!m) return NULL;
  size_t nn = (size_t)(2 * nx + 1) * (2 * ny + 1);
  m->iso = 1;
  m->nx_ = (double *)malloc(sizeof(double) * nn);
  m->ny_ = (double *)malloc(sizeof(double) * nn);
  if (!m->nx_ || !m->ny_) {
    or_mesh_destroy(m);
    return NULL;
  }
  memcpy(m->nx_, nodes, sizeof(double) * nn);
  memcpy(m->ny_, nodes + nn, sizeof(double) * nn);
  /* the vertices are the corner nodes */
  for (int iy = 0; iy <= ny; ++iy)
    for (int ix = 0; ix <= nx; ++ix) {
      m->vx[vert_index(m, ix, iy)] = m->nx_[node_index(m, 2 * ix, 2 * iy)];
      m->vy[vert_index(m, ix, iy)] = m->ny_[node_index(m, 2 * ix, 2 * iy)];
    }
  if (mesh_geometry(m) != 0) {
    or_mesh_destroy(m);
    return NULL;
  }
  return m;
}

void or_mesh_destroy(or_mesh *m) {
  if (!m) return;
  free(m->wdet);
  free(m->dphix);
  free(m->dphiy);
  free(m->chol);
  free(m->vx);
  free(m->vy);
  free(m->nx_);
  free(m->ny_);
  free(m);
}

void or_element_geometry(const or_mesh *m, int e, double *wdet, double *dphix, double *dphiy) {
  int ng = m->ng;
  memcpy(wdet, m->wdet + (size_t)e * ng, sizeof(double) * ng);
  memcpy(dphix, m->dphix + (size_t)e * 9 * ng, sizeof(double) * 9 * ng);
  memcpy(dphiy, m->dphiy + (size_t)e * 9 * ng, sizeof(double) * 9 * ng);
}

/* L2 projection of Gauss values g[q] onto the DG stress space of element e:
 * c = M_e^-1 Psi W_e g, the operator the listings call iMJwPSI. */
static void project(const or_mesh *m, size_t e, const double *g, double *c) {
  const double *wd = m->wdet + e * m->ng;
  for (int k = 0; k < m->ns; ++k) {
    double s = 0.0;
    for (int q = 0; q < m->ng; ++q) s += m->psiS[k][q] * wd[q] * g[q];
    c[k] = s;
  }
  chol_solve(m->ns, m->chol + e * m->ns * m->ns, c);
}

/* Value at Gauss point q of the DG function with coefficients c[k*stride]. */
static double eval_dg(const or_mesh *m, const double *c, size_t stride, int q) {
  double s = 0.0;
  for (int k = 0; k < m->ns; ++k) s += c[k * stride] * m->psiS[k][q];
  return s;
}

/* ---------------------------------------------------------------------------
 * Per time step quantities (R11; clamps of h and a from the stress listings)
 * ------------------------------------------------------------------------- */

/* h and a at Gauss point q: max(0, H Psi_A), min(1, max(0, A Psi_A)). */
static void ice_at_gauss(const or_mesh *m, const double *H, const double *A, size_t e, int q,
                         double *h, double *a) {
  size_t ne = (size_t)m->nx * m->ny;
  double hs = 0.0, as = 0.0;
  for (int k = 0; k < m->na; ++k) {
    hs += H[k * ne + e] * m->psiA[k][q];
    as += A[k * ne + e] * m->psiA[k][q];
  }
  *h = fmax(0.0, hs);
  *a = fmin(1.0, fmax(0.0, as));
}

void or_node_masses(const or_mesh *m, const or_params *p, const double *H, const double *A,
                    double *MH, double *mA) {
  size_t ne = (size_t)m->nx * m->ny, nn = (size_t)(2 * m->nx + 1) * (2 * m->ny + 1);
  double *me = (double *)malloc(sizeof(double) * ne * 18);
#pragma omp parallel for schedule(static)
  for (long e = 0; e < (long)ne; ++e) {
    const double *wd = m->wdet + e * m->ng;
    for (int a = 0; a < 9; ++a) {
      double sh = 0.0, sa = 0.0;
      for (int q = 0; q < m->ng; ++q) {
        double h, c;
        ice_at_gauss(m, H, A, e, q, &h, &c);
        sh += wd[q] * p->rho_i * h * m->phi[a][q];
        sa += wd[q] * c * m->phi[a][q];
      }
      me[e * 18 + a] = sh;
      me[e * 18 + 9 + a] = sa;
    }
  }
  memset(MH, 0, sizeof(double) * nn);
  memset(mA, 0, sizeof(double) * nn);
  for (size_t e = 0; e < ne; ++e) /* ascending element order */
    for (int a = 0; a < 9; ++a) {
      int j = local_to_global(m, (int)e, a);
      MH[j] += me[e * 18 + a];
      mA[j] += me[e * 18 + 9 + a];
    }
  free(me);
}

void or_air_stress(const or_params *p, int nn, const double *wind, double *tau) {
  for (int j = 0; j < nn; ++j) {
    double ux = wind[j], uy = wind[nn + j];
    double sp = sqrt(ux * ux + uy * uy);
    tau[j] = p->rho_a * p->C_a * sp * ux;
    tau[nn + j] = p->rho_a * p->C_a * sp * uy;
  }
}

/* ---------------------------------------------------------------------------
 * Subcycle phases (Table 1: strain, stress, divergence, velocity)
 * ------------------------------------------------------------------------- */

void or_strain_gauss(const or_mesh *m, const double *v, double *eps) {
  size_t ne = (size_t)m->nx * m->ny, nn = (size_t)(2 * m->nx + 1) * (2 * m->ny + 1);
  int ng = m->ng;
#pragma omp parallel for schedule(static)
  for (long e = 0; e < (long)ne; ++e) {
    const double *gx = m->dphix + e * 9 * ng, *gy = m->dphiy + e * 9 * ng;
    double vx[9], vy[9];
    for (int a = 0; a < 9; ++a) {
      int j = local_to_global(m, (int)e, a);
      vx[a] = v[j];
      vy[a] = v[nn + j];
    }
    for (int q = 0; q < ng; ++q) {
      double dvxdx = 0, dvxdy = 0, dvydx = 0, dvydy = 0;
      for (int a = 0; a < 9; ++a) {
        dvxdx += vx[a] * gx[a * ng + q];
        dvxdy += vx[a] * gy[a * ng + q];
        dvydx += vy[a] * gx[a * ng + q];
        dvydy += vy[a] * gy[a * ng + q];
      }
      eps[(0 * ng + q) * ne + e] = dvxdx;
      eps[(1 * ng + q) * ne + e] = 0.5 * (dvxdy + dvydx);
      eps[(2 * ng + q) * ne + e] = dvydy;
    }
  }
}

void or_project(const or_mesh *m, const double *g, int ncomp, double *coef) {
  size_t ne = (size_t)m->nx * m->ny;
  int ng = m->ng, ns = m->ns;
#pragma omp parallel for schedule(static)
  for (long e = 0; e < (long)ne; ++e) {
    for (int c = 0; c < ncomp; ++c) {
      double gq[MAXG], cf[MAXS];
      for (int q = 0; q < ng; ++q) gq[q] = g[((size_t)c * ng + q) * ne + e];
      project(m, e, gq, cf);
      for (int k = 0; k < ns; ++k) coef[((size_t)c * ns + k) * ne + e] = cf[k];
    }
  }
}

/* Strain (R9): E^{ij} = Pi_e(eps^{ij}). */
void or_strain(const or_mesh *m, const double *v, double *E) {
  size_t ne = (size_t)m->nx * m->ny;
  double *eps = (double *)malloc(sizeof(double) * 3 * m->ng * ne);
  or_strain_gauss(m, v, eps);
  or_project(m, eps, 3, E);
  free(eps);
}

void or_eval_gauss(const or_mesh *m, const double *coef, int ncomp, double *out) {
  size_t ne = (size_t)m->nx * m->ny;
  int ng = m->ng, ns = m->ns;
  for (int c = 0; c < ncomp; ++c)
    for (size_t e = 0; e < ne; ++e)
      for (int q = 0; q < ng; ++q)
        out[((size_t)c * ng + q) * ne + e] = eval_dg(m, coef + (size_t)c * ns * ne + e, ne, q);
}

/* VP stress at one Gauss point, in the order of the stress listings:
 * P = P* h exp(-C(1-a)); Delta = sqrt(Dmin^2 + 5/4 (e11^2+e22^2) + 3/2 e11 e22 + e12^2);
 * s11 = P/Delta (5/8 e11 + 3/8 e22) - P/2; s12 = P/Delta e12/4; s22 symmetric. */
static void vp_stress_point(const or_params *p, double h, double a, double e11, double e12,
                            double e22, double s[3], double *Pout, double *Dout) {
  double P = p->Pstar * h * exp(-p->C * (1.0 - a));
  double D = sqrt(p->DeltaMin * p->DeltaMin + 1.25 * (e11 * e11 + e22 * e22) + 1.5 * e11 * e22 +
                  e12 * e12);
  double PD = P / D;
  s[0] = PD * (5.0 / 8.0 * e11 + 3.0 / 8.0 * e22) - 0.5 * P;
  s[1] = PD * (1.0 / 4.0) * e12;
  s[2] = PD * (5.0 / 8.0 * e22 + 3.0 / 8.0 * e11) - 0.5 * P;
  if (Pout) *Pout = P;
  if (Dout) *Dout = D;
}

void or_stress_gauss(const or_mesh *m, const or_params *p, const double *E, const double *H,
                     const double *A, double *s, double *P, double *Delta) {
  size_t ne = (size_t)m->nx * m->ny;
  int ng = m->ng, ns = m->ns;
  for (size_t e = 0; e < ne; ++e)
    for (int q = 0; q < ng; ++q) {
      double h, a, sq[3], Pq, Dq;
      ice_at_gauss(m, H, A, e, q, &h, &a);
      double e11 = eval_dg(m, E + 0 * ns * ne + e, ne, q);
      double e12 = eval_dg(m, E + 1 * ns * ne + e, ne, q);
      double e22 = eval_dg(m, E + 2 * ns * ne + e, ne, q);
      vp_stress_point(p, h, a, e11, e12, e22, sq, &Pq, &Dq);
      for (int c = 0; c < 3; ++c) s[((size_t)c * ng + q) * ne + e] = sq[c];
      if (P) P[(size_t)q * ne + e] = Pq;
      if (Delta) Delta[(size_t)q * ne + e] = Dq;
    }
}

/* Stress update (Listing 1; appendix listing): S <- fac S + ainv Pi_e(s). */
void or_stress(const or_mesh *m, const or_params *p, const double *E, const double *H,
               const double *A, double *S) {
  size_t ne = (size_t)m->nx * m->ny;
  int ng = m->ng, ns = m->ns;
  double fac, ainv;
  if (p->relax_form == 1) {
    fac = p->alpha / (1.0 + p->alpha);
    ainv = 1.0 / (1.0 + p->alpha);
  } else {
    ainv = 1.0 / p->alpha;
    fac = 1.0 - ainv;
  }
#pragma omp parallel for schedule(static)
  for (long e = 0; e < (long)ne; ++e) {
    double sg[3][MAXG];
    for (int q = 0; q < ng; ++q) {
      double h, a, sq[3];
      ice_at_gauss(m, H, A, e, q, &h, &a);
      double e11 = eval_dg(m, E + 0 * ns * ne + e, ne, q);
      double e12 = eval_dg(m, E + 1 * ns * ne + e, ne, q);
      double e22 = eval_dg(m, E + 2 * ns * ne + e, ne, q);
      vp_stress_point(p, h, a, e11, e12, e22, sq, NULL, NULL);
      for (int c = 0; c < 3; ++c) sg[c][q] = sq[c];
    }
    for (int c = 0; c < 3; ++c) {
      double pc[MAXS];
      project(m, e, sg[c], pc);
      for (int k = 0; k < ns; ++k) {
        double *Sk = S + ((size_t)c * ns + k) * ne + e;
        *Sk = fac * *Sk + ainv * pc[k];
      }
    }
  }
}

/* Divergence (R10): F_j = sum over elements e containing j, ascending e, of
 * f_e[a] = -sum_q w_q|J_q| (s11 dphi_a/dx + s12 dphi_a/dy, s12 dphi_a/dx + s22 dphi_a/dy). */
void or_divergence(const or_mesh *m, const double *S, double *F) {
  size_t ne = (size_t)m->nx * m->ny, nn = (size_t)(2 * m->nx + 1) * (2 * m->ny + 1);
  int ng = m->ng, ns = m->ns;
  double *fe = (double *)malloc(sizeof(double) * ne * 18);
#pragma omp parallel for schedule(static)
  for (long e = 0; e < (long)ne; ++e) {
    const double *wd = m->wdet + e * ng, *gx = m->dphix + e * 9 * ng, *gy = m->dphiy + e * 9 * ng;
    double s11[MAXG], s12[MAXG], s22[MAXG];
    for (int q = 0; q < ng; ++q) {
      s11[q] = eval_dg(m, S + 0 * ns * ne + e, ne, q);
      s12[q] = eval_dg(m, S + 1 * ns * ne + e, ne, q);
      s22[q] = eval_dg(m, S + 2 * ns * ne + e, ne, q);
    }
    for (int a = 0; a < 9; ++a) {
      double fx = 0.0, fy = 0.0;
      for (int q = 0; q < ng; ++q) {
        fx += wd[q] * (s11[q] * gx[a * ng + q] + s12[q] * gy[a * ng + q]);
        fy += wd[q] * (s12[q] * gx[a * ng + q] + s22[q] * gy[a * ng + q]);
      }
      fe[e * 18 + a] = -fx;
      fe[e * 18 + 9 + a] = -fy;
    }
  }
  memset(F, 0, sizeof(double) * 2 * nn);
  for (size_t e = 0; e < ne; ++e) /* ascending element order */
    for (int a = 0; a < 9; ++a) {
      int j = local_to_global(m, (int)e, a);
      F[j] += fe[e * 18 + a];
      F[nn + j] += fe[e * 18 + 9 + a];
    }
  free(fe);
}

/* Velocity update (R11, R12), node by node. */
void or_velocity(const or_mesh *m, const or_params *p, const double *F, const double *MH,
                 const double *mA, const double *tau, const double *ocean, const double *vn,
                 double *v) {
  int NX = 2 * m->nx + 1, NY = 2 * m->ny + 1;
  size_t nn = (size_t)NX * NY;
#pragma omp parallel for schedule(static)
  for (long j = 0; j < (long)nn; ++j) {
    int ix = (int)(j % NX), iy = (int)(j / NX);
    if (ix == 0 || iy == 0 || ix == NX - 1 || iy == NY - 1) {
      v[j] = 0.0;
      v[nn + j] = 0.0;
      continue;
    }
    double vx = v[j], vy = v[nn + j];
    double ox = ocean[j], oy = ocean[nn + j];
    double c = MH[j] / p->dt;
    double d = mA[j] * p->rho_o * p->C_o * sqrt((ox - vx) * (ox - vx) + (oy - vy) * (oy - vy));
    double b = p->f_cor * MH[j];
    double rx = c * (p->beta * vx + vn[j]) + mA[j] * tau[j] + d * ox + F[j];
    double ry = c * (p->beta * vy + vn[nn + j]) + mA[j] * tau[nn + j] + d * oy + F[nn + j];
    double a = c * (1.0 + p->beta) + d;
    double den = a * a + b * b;
    if (den == 0.0) {
      v[j] = 0.0;
      v[nn + j] = 0.0;
    } else {
      v[j] = (a * rx + b * ry) / den;
      v[nn + j] = (a * ry - b * rx) / den;
    }
  }
}

/* ---------------------------------------------------------------------------
 * Advection of H and A (R14)
 * ------------------------------------------------------------------------- */

/* d psi_k / d xi and d psi_k / d eta (R6). */
static void dg_basis_grad(int k, double xi, double eta, double *dxi, double *deta) {
  double s = xi - 0.5, t = eta - 0.5;
  switch (k) {
    case 0: *dxi = 0.0; *deta = 0.0; return;
    case 1: *dxi = 1.0; *deta = 0.0; return;
    case 2: *dxi = 0.0; *deta = 1.0; return;
    case 3: *dxi = 2.0 * s; *deta = 0.0; return;
    case 4: *dxi = t; *deta = s; return;
    case 5: *dxi = 0.0; *deta = 2.0 * t; return;
  }
  *dxi = 0.0;
  *deta = 0.0;
}

/* reference point of parameter u in [0,1] on edge ed of the reference square,
 * traversed counter-clockwise: 0 bottom, 1 right, 2 top, 3 left */
static void edge_point(int ed, double u, double *xi, double *eta) {
  switch (ed) {
    case 0: *xi = u; *eta = 0.0; return;
    case 1: *xi = 1.0; *eta = u; return;
    case 2: *xi = 1.0 - u; *eta = 1.0; return;
    default: *xi = 0.0; *eta = 1.0 - u; return;
  }
}

/* the same physical point seen from the neighbour across edge ed */
static void edge_point_nb(int ed, double u, double *xi, double *eta) {
  switch (ed) {
    case 0: *xi = u; *eta = 1.0; return;
    case 1: *xi = 0.0; *eta = u; return;
    case 2: *xi = 1.0 - u; *eta = 0.0; return;
    default: *xi = 1.0; *eta = 1.0 - u; return;
  }
}

static double dg_value(int na, const double *U, size_t ne, size_t e, double xi, double eta) {
  double s = 0.0;
  for (int k = 0; k < na; ++k) s += U[k * ne + e] * dg_basis(k, xi, eta);
  return s;
}

/* L(U) = M_e^-1 R_e(U) for one field, all elements. */
static void advect_rate(const or_mesh *m, const double *v, const double *U, double *L) {
  size_t ne = (size_t)m->nx * m->ny, nn = (size_t)(2 * m->nx + 1) * (2 * m->ny + 1);
  int na = m->na;
  double gp[3], gw[3];
  gauss_rule(3, gp, gw);
  const double *VX = m->vx, *VY = m->vy;
#pragma omp parallel for schedule(static)
  for (long e = 0; e < (long)ne; ++e) {
    int ex = (int)(e % m->nx), ey = (int)(e / m->nx);
    int vi[4] = {vert_index(m, ex, ey), vert_index(m, ex + 1, ey), vert_index(m, ex, ey + 1),
                 vert_index(m, ex + 1, ey + 1)};
    double X[4], Y[4], vxe[9], vye[9];
    for (int i = 0; i < 4; ++i) {
      X[i] = VX[vi[i]];
      Y[i] = VY[vi[i]];
    }
    for (int a = 0; a < 9; ++a) {
      int j = local_to_global(m, (int)e, a);
      vxe[a] = v[j];
      vye[a] = v[nn + j];
    }
    double R[6] = {0, 0, 0, 0, 0, 0}, M[36];
    memset(M, 0, sizeof M);
    /* cell integral and mass matrix */
    for (int qy = 0; qy < 3; ++qy)
      for (int qx = 0; qx < 3; ++qx) {
        double xi = gp[qx], eta = gp[qy], w = gw[qx] * gw[qy], J[4];
        map_jacobian(m, (int)e, xi, eta, J);
        double J00 = J[0], J01 = J[1], J10 = J[2], J11 = J[3];
        double det = J00 * J11 - J01 * J10;
        double ux = 0.0, uy = 0.0;
        for (int a = 0; a < 9; ++a) {
          double ph = lag2(a % 3, xi) * lag2(a / 3, eta);
          ux += vxe[a] * ph;
          uy += vye[a] * ph;
        }
        double Uq = dg_value(na, U, ne, (size_t)e, xi, eta);
        for (int k = 0; k < na; ++k) {
          double dxi, deta;
          dg_basis_grad(k, xi, eta, &dxi, &deta);
          double gx = (J11 * dxi - J10 * deta) / det; /* grad psi = J^-T (d/dxi, d/deta) */
          double gy = (-J01 * dxi + J00 * deta) / det;
          R[k] += w * det * Uq * (ux * gx + uy * gy);
          for (int l = 0; l < na; ++l)
            M[k * na + l] += w * det * dg_basis(k, xi, eta) * dg_basis(l, xi, eta);
        }
      }
    /* edge fluxes; scaled outward normal n L = (t_y, -t_x) of the tangent t =
     * dx/du of the counter-clockwise edge: the edge vector for the bilinear
     * map (straight edges), J (dxi/du, deta/du) at the point for the
     * isoparametric map (curved edges) */
    const int from[4] = {0, 1, 3, 2}, to[4] = {1, 3, 2, 0};
    const int nbx[4] = {0, 1, 0, -1}, nby[4] = {-1, 0, 1, 0};
    const double dxu[4] = {1.0, 0.0, -1.0, 0.0}, deu[4] = {0.0, 1.0, 0.0, -1.0};
    for (int ed = 0; ed < 4; ++ed) {
      double tx = X[to[ed]] - X[from[ed]], ty = Y[to[ed]] - Y[from[ed]];
      int fx = ex + nbx[ed], fy = ey + nby[ed];
      int has_nb = fx >= 0 && fy >= 0 && fx < m->nx && fy < m->ny;
      size_t f = has_nb ? (size_t)fy * m->nx + fx : 0;
      for (int g = 0; g < 3; ++g) {
        double xi, eta;
        edge_point(ed, gp[g], &xi, &eta);
        if (m->iso) {
          double J[4];
          map_jacobian(m, (int)e, xi, eta, J);
          tx = J[0] * dxu[ed] + J[1] * deu[ed];
          ty = J[2] * dxu[ed] + J[3] * deu[ed];
        }
        double nlx = ty, nly = -tx;
        double ux = 0.0, uy = 0.0;
        for (int a = 0; a < 9; ++a) {
          double ph = lag2(a % 3, xi) * lag2(a / 3, eta);
          ux += vxe[a] * ph;
          uy += vye[a] * ph;
        }
        double vn = ux * nlx + uy * nly;
        double Uup;
        if (vn >= 0.0 || !has_nb) {
          Uup = dg_value(na, U, ne, (size_t)e, xi, eta);
        } else {
          double xn, en;
          edge_point_nb(ed, gp[g], &xn, &en);
          Uup = dg_value(na, U, ne, f, xn, en);
        }
        for (int k = 0; k < na; ++k) R[k] -= gw[g] * vn * Uup * dg_basis(k, xi, eta);
      }
    }
    double Lc[36];
    if (cholesky(na, M, Lc) != 0) { /* cells were validated at mesh creation */
      for (int k = 0; k < na; ++k) L[k * ne + e] = 0.0;
      continue;
    }
    chol_solve(na, Lc, R);
    for (int k = 0; k < na; ++k) L[k * ne + e] = R[k];
  }
}

/* One advection step of one field with the three-stage SSP Runge-Kutta scheme. */
static void advect_field(const or_mesh *m, double dt, const double *v, double *U) {
  size_t n = (size_t)m->na * m->nx * m->ny;
  double *L = (double *)malloc(sizeof(double) * n);
  double *U1 = (double *)malloc(sizeof(double) * n);
  double *U2 = (double *)malloc(sizeof(double) * n);
  advect_rate(m, v, U, L);
  for (size_t i = 0; i < n; ++i) U1[i] = U[i] + dt * L[i];
  advect_rate(m, v, U1, L);
  for (size_t i = 0; i < n; ++i) U2[i] = 0.75 * U[i] + 0.25 * (U1[i] + dt * L[i]);
  advect_rate(m, v, U2, L);
  for (size_t i = 0; i < n; ++i) U[i] = U[i] / 3.0 + 2.0 / 3.0 * (U2[i] + dt * L[i]);
  free(L), free(U1), free(U2);
}

void or_advect_rate(const or_mesh *m, const double *v, const double *U, double *L) {
  advect_rate(m, v, U, L);
}

void or_advect(const or_mesh *m, double dt, const double *v, double *H, double *A) {
  advect_field(m, dt, v, H);
  advect_field(m, dt, v, A);
}

/* ---------------------------------------------------------------------------
 * Drivers (Sec. 2: advection at a large step, momentum + mEVP subcycled)
 * ------------------------------------------------------------------------- */

int or_subcycles(const or_mesh *m, const or_params *p, const double *H, const double *A,
                 const double *wind, const double *ocean, const double *vn, double *v,
                 double *S, int n_sub) {
  if (!m || !p || n_sub < 0) return -1;
  size_t ne = (size_t)m->nx * m->ny, nn = (size_t)(2 * m->nx + 1) * (2 * m->ny + 1);
  double *MH = (double *)malloc(sizeof(double) * nn);
  double *mA = (double *)malloc(sizeof(double) * nn);
  double *tau = (double *)malloc(sizeof(double) * 2 * nn);
  double *E = (double *)malloc(sizeof(double) * 3 * m->ns * ne);
  double *F = (double *)malloc(sizeof(double) * 2 * nn);
  if (!MH || !mA || !tau || !E || !F) {
    free(MH), free(mA), free(tau), free(E), free(F);
    return -2;
  }
  or_node_masses(m, p, H, A, MH, mA);
  or_air_stress(p, (int)nn, wind, tau);
  for (int it = 0; it < n_sub; ++it) {
    or_strain(m, v, E);                                /* sigma^(p) from v^(p-1) ... */
    or_stress(m, p, E, H, A, S);
    or_divergence(m, S, F);                            /* ... then v^(p) from sigma^(p) */
    or_velocity(m, p, F, MH, mA, tau, ocean, vn, v);
  }
  free(MH), free(mA), free(tau), free(E), free(F);
  return 0;
}

int or_step(const or_mesh *m, const or_params *p, const double *H, const double *A,
            const double *wind, const double *ocean, double *v, double *S, int n_sub) {
  if (!m) return -1;
  size_t nn = (size_t)(2 * m->nx + 1) * (2 * m->ny + 1);
  double *vn = (double *)malloc(sizeof(double) * 2 * nn);
  if (!vn) return -2;
  memcpy(vn, v, sizeof(double) * 2 * nn);
  int rc = or_subcycles(m, p, H, A, wind, ocean, vn, v, S, n_sub);
  free(vn);
  return rc;
}
