/*
 * mevp_oracle.h -- plain FP64 CPU reference of the mEVP momentum subcycle.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may call this library. The product path (the
 * HIP library) never links, includes or executes anything from here, and this
 * code includes nothing from the product path.
 *
 * What it computes (Jendersie, Lessig, Richter, "Towards a GPU-Parallelization
 * of the neXtSIM-DG Dynamical Core", PASC 2024):
 *   Sec. 2, Eq. (si:momentum) and Eq. (si:mevp): the momentum equation solved
 *   by the mEVP pseudo-time iteration, subcycled n_sub times per time step;
 *   Sec. 2.1: CG velocity, tensor-valued DG stress, quadrilateral mesh mapped
 *   from a reference element;
 *   Table 1: one subcycle = strain, stress, divergence, velocity;
 *   Listing 1 and the appendix listing: the stress update.
 * The strain, divergence and velocity formulas are only named in the paper;
 * the oracle uses the standard finite-element weak form of Eq. (si:momentum)
 * with the readings listed in mevp_oracle.c.
 *
 * Parity status: every function below is pinned by the CPU test suite
 * (closed forms, invariants, an exact-arithmetic brute-force assembly). The
 * full-run field values have no printed worked example in the paper and are
 * checked only through those pins.
 *
 * Arrays are host, float64, C order:
 *   vertices [2][(ny+1)(nx+1)]  vertex (ix,iy) -> iy*(nx+1)+ix
 *   H, A     [na][nx*ny]        element (ex,ey) -> ey*nx+ex
 *   S, E     [3][ns][nx*ny]     component order 11, 12, 22
 *   v, F, wind, ocean, tau [2][(2nx+1)(2ny+1)]  CG2 node (ix,iy) -> iy*(2nx+1)+ix
 */
#ifndef MEVP_ORACLE_H
#define MEVP_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double Pstar;    /* ice strength P* [N/m^2] */
  double C;        /* concentration parameter (20 in the stress listing) */
  double DeltaMin; /* Delta_min [1/s] */
  double alpha;    /* mEVP stress relaxation */
  double beta;     /* mEVP velocity relaxation */
  double rho_i;    /* ice density [kg/m^3] */
  double rho_a;    /* air density */
  double C_a;      /* air drag coefficient */
  double rho_o;    /* ocean density */
  double C_o;      /* ocean drag coefficient */
  double f_cor;    /* Coriolis parameter [1/s] */
  double dt;       /* advection time step [s] */
  int relax_form;  /* 0: (1-1/alpha, 1/alpha) as in the listings; 1: (alpha/(1+alpha), 1/(1+alpha)) as in Eq. (si:mevp) */
} or_params;

typedef struct or_mesh or_mesh;

/* Mesh and per-element geometry. Returns NULL on invalid arguments
 * (nx, ny < 1; ns not in {3,6,8}; na not in {1,3,6}) or a degenerate element. */
or_mesh *or_mesh_create(int nx, int ny, int ns, int na, const double *vertices);
/* The same with the isoparametric CG2 map (reading R8): nodes [2][(2nx+1)(2ny+1)]
 * are the positions of the CG2 nodes in the node order of v; the vertices are
 * the corner nodes. */
or_mesh *or_mesh_create_iso(int nx, int ny, int ns, int na, const double *nodes);
void or_mesh_destroy(or_mesh *m);

/* Reference-element tables. Sizes: ngp from ns (2 for ns=3, else 3), nG=ngp^2.
 * gpts[ngp], gwts[ngp]; psiS[ns][nG]; psiA[na][nG]; phi, dxi, deta [9][nG]. */
int or_tables(int ns, int na, double *gpts, double *gwts, double *psiS, double *psiA,
              double *phi, double *dxi, double *deta);

/* Per-element Gauss data: wdet[nG] = w_q |J_q|; dphix, dphiy [9][nG]. */
void or_element_geometry(const or_mesh *m, int e, double *wdet, double *dphix, double *dphiy);

/* Per time step: lumped ice mass M^H, lumped concentration m^A [nn], air stress tau [2][nn]. */
void or_node_masses(const or_mesh *m, const or_params *p, const double *H, const double *A,
                    double *MH, double *mA);
void or_air_stress(const or_params *p, int nn, const double *wind, double *tau);

/* Subcycle phases. */
void or_strain(const or_mesh *m, const double *v, double *E);
void or_stress(const or_mesh *m, const or_params *p, const double *E, const double *H,
               const double *A, double *S);
void or_divergence(const or_mesh *m, const double *S, double *F);
void or_velocity(const or_mesh *m, const or_params *p, const double *F, const double *MH,
                 const double *mA, const double *tau, const double *ocean, const double *vn,
                 double *v);

/* Advection of H and A over dt with the CG2 velocity v held fixed
 * (Sec. 2, Eq. (si:ad); reading R14 in mevp_oracle.c). H, A in/out. */
void or_advect(const or_mesh *m, double dt, const double *v, double *H, double *A);
/* Test hook: the advection rate L(U) = M^-1 R(U) of one field [na][ne]. */
void or_advect_rate(const or_mesh *m, const double *v, const double *U, double *L);

/* One time step = snapshot v^n, masses, air stress, then n_sub subcycles. */
int or_step(const or_mesh *m, const or_params *p, const double *H, const double *A,
            const double *wind, const double *ocean, double *v, double *S, int n_sub);
/* Subcycles only, with a caller-held v^n (no snapshot, masses from H, A). */
int or_subcycles(const or_mesh *m, const or_params *p, const double *H, const double *A,
                 const double *wind, const double *ocean, const double *vn, double *v,
                 double *S, int n_sub);

/* Test hooks: Gauss-point values. */
void or_strain_gauss(const or_mesh *m, const double *v, double *eps);          /* [3][nG][ne] */
void or_eval_gauss(const or_mesh *m, const double *coef, int ncomp, double *out); /* [ncomp][ns][ne] -> [ncomp][nG][ne] */
void or_stress_gauss(const or_mesh *m, const or_params *p, const double *E, const double *H,
                     const double *A, double *s, double *P, double *Delta); /* s [3][nG][ne]; P, Delta [nG][ne] */
void or_project(const or_mesh *m, const double *g, int ncomp, double *coef);   /* [ncomp][nG][ne] -> [ncomp][ns][ne] */

int or_num_threads(void);
void or_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
