/*
 * mevp.h -- C ABI of the MI355X (gfx950) mEVP momentum-subcycle library.
 *
 * The library advances the sea-ice momentum equation of the neXtSIM-DG
 * dynamical core (Jendersie, Lessig, Richter, "Towards a GPU-Parallelization
 * of the neXtSIM-DG Dynamical Core", PASC 2024) by mEVP pseudo-time
 * subcycles: Sec. 2, Eq. (si:momentum) and Eq. (si:mevp); Table 1 names the
 * four phases of one subcycle (strain, stress, divergence, velocity); the
 * stress phase is the one printed in Listing 1 and in the appendix listing.
 * Discretisation (Sec. 2.1): structured quadrilateral mesh, biquadratic
 * continuous (CG2) velocity, discontinuous (DG) stress with n_s local dofs
 * per component, DG ice height H and concentration A with n_a dofs.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers. Every array argument is a caller-owned DEVICE pointer (host
 * pointers are accepted by the copy-in/out calls, which then block the
 * host). The library never calls a device allocator: a context's state lives
 * in the workspace the caller passes to mevp_create, and mevp_step_static
 * works in a file-scope device array (MEVP_STATIC_SCRATCH_BYTES per GPU, part
 * of the library's code object on that GPU).
 * Errors. Every call returns a mevp_status; no call aborts or throws. All
 * argument validation happens on the host before anything is enqueued.
 * Asynchronous HIP failures surface at the next mevp_sync / mevp_check_*.
 * Streams. A context enqueues all its work on the stream given at creation
 * (NULL = the default stream). Calls on one context are stream-ordered;
 * a context is not thread-safe. Contexts on one device are independent.
 * Logging. With the environment variable MEVP_LOG=1 (read once per
 * process) the library writes host-side lines "[mevp] ..." to stderr: each
 * context created, every autotuning trial with its time and the choice (or
 * the cache entry used), a step-graph capture that failed (the context then
 * launches directly), and every create / step / subcycles / begin_step /
 * advect / tune / check / step_static / set_config call that returns an
 * error, with its status. MEVP_LOG=2 adds each launch configuration set and
 * each step graph captured. Unset or 0: nothing is written. Logging changes
 * no result and no status.
 * Precision. MEVP_FP64 computes everything in IEEE double. MEVP_MIXED stores
 * the DG stress in float and runs the strain, stress and divergence
 * contractions in float, keeping the ice-strength exponential, the Delta
 * denominator, the nodal sums and the velocity update in double. The API
 * takes and returns double in both modes.
 * Layouts (C order, element index e = ey*nx + ex, CG2 node index
 * j = iy*(2nx+1) + ix, vertex index iy*(nx+1) + ix):
 *   vertex_xy  [2][(nx+1)(ny+1)]     metres, planar coordinates
 *   H, A       [n_a][nx*ny]          DG coefficients (scaled Legendre basis)
 *   wind_xy, ocean_xy, v_xy [2][(2nx+1)(2ny+1)]   m/s
 *   S          [3][n_s][nx*ny]       components 11, 12, 22 of the DG stress
 * DG basis on the reference square [0,1]^2 with s = xi-1/2, t = eta-1/2:
 *   1, s, t, s^2-1/12, s t, t^2-1/12, (s^2-1/12) t, s (t^2-1/12)
 * (the first n_s, resp. n_a, of them). CG2 local node a = 3 b + c sits at
 * (c/2, b/2) of the reference square.
 */
#ifndef MEVP_H
#define MEVP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MEVP_OK = 0,
  MEVP_EINVAL = -1,       /* bad argument: null pointer, size, domain index, alignment, parameter */
  MEVP_ENOMEM = -2,       /* workspace smaller than mevp_workspace_size reports */
  MEVP_EDEVICE = -3,      /* HIP error: no device, launch failure, asynchronous fault */
  MEVP_ESTATE = -4,       /* call out of order, e.g. a step before geometry/fields/forcing are set */
  MEVP_ENONFINITE = -5,   /* non-finite or invalid values found by a check call */
  MEVP_EUNSUPPORTED = -6, /* the current device is not gfx950 */
  MEVP_EINTERNAL = -7,    /* a self-check failed (the tuner's bitwise comparison) */
  MEVP_EHOSTMEM = -8      /* host memory allocation failed (context, tables, tuner copies) */
} mevp_status;

/* MEVP_MIXED_BF16: the bfloat16 trial of the mixed form. As MEVP_MIXED, with
 * every entry of the element matrices -- the operators that the strain,
 * projection and divergence contractions apply (reference basis and
 * gradient tables, Jacobian factors, quadrature weights times |J|, the
 * local mass matrix's factors; the listings' PSI and iMJwPSI) -- rounded to
 * bfloat16 (8 significant bits, round to nearest even) and the arithmetic
 * in float. n_s = 6 and n_a = 1 only (EINVAL otherwise), vertex geometry
 * (parallelogram and bilinear cells), strategies FUSED, FUSED_PAIR and
 * FUSED_TRIPLE. Its error against FP64 is set by the 2^-9 relative rounding
 * of the matrices, far above the mixed form's. */
typedef enum {
  MEVP_FP64 = 0,
  MEVP_MIXED = 1,
  MEVP_MIXED_BF16 = 2,
  /* not precisions: they give the enum the range of int, so that any int a
   * caller passes is a value of the type and the library rejects it (EINVAL)
   * instead of reading an out-of-range enum */
  MEVP_PRECISION_RANGE_MIN_ = -2147483647 - 1,
  MEVP_PRECISION_RANGE_MAX_ = 2147483647
} mevp_precision;

/* Physical and iteration parameters (mevp_default_params fills the values
 * the paper uses: P* and the factor 20 of the stress listings, 100 subcycles
 * per 120 s step of Sec. 4, alpha = beta = 300; the rest are conventional
 * viscous-plastic constants the paper does not state). */
typedef struct {
  double Pstar;    /* ice strength P* [N m^-2] */
  double C;        /* concentration exponent factor (20 in the listings) */
  double DeltaMin; /* Delta_min [s^-1], regularises the viscosities, >= 1e-100 */
  double alpha;    /* mEVP stress relaxation, > 0 */
  double beta;     /* mEVP velocity relaxation, >= 0 */
  double rho_i;    /* ice density [kg m^-3] */
  double rho_a;    /* air density */
  double C_a;      /* air drag coefficient */
  double rho_o;    /* ocean density */
  double C_o;      /* ocean drag coefficient */
  double f_cor;    /* Coriolis parameter [s^-1] */
  double dt;       /* time step of one mevp_step [s], > 0 */
  int relax_form;  /* 0: S <- (1-1/alpha) S + (1/alpha) M^-1(...) as in both listings;
                      1: alpha/(1+alpha) and 1/(1+alpha) as in Eq. (si:mevp) */
} mevp_params;

/* One independent domain: nx x ny elements, n_s in {3, 6, 8} stress dofs
 * (Gauss rule 2x2 for n_s = 3, 3x3 otherwise, as in the appendix listing),
 * n_a in {1, 3, 6} dofs for H and A. All domains of one context must share
 * n_s and n_a. */
typedef struct {
  int nx, ny, n_s, n_a;
} mevp_domain_desc;

/* How subcycles are mapped to launches. All strategies and tile shapes
 * compute the same values and sum each node's forces in the same order, so
 * their results agree bitwise.
 * FUSED (default): one launch per subcycle; a workgroup owns a tile of
 * elements and the CG2 nodes at its low edges, recomputes the forces of a
 * one-element halo, keeps all element forces in LDS and updates its nodes;
 * v and S are double-buffered in the workspace.
 * PERSISTENT: the fused subcycle, with all subcycles of one mevp_subcycles
 * call in a single cooperative launch (a grid-wide barrier between
 * subcycles). Used when all domains take the same element kernel; otherwise,
 * or if the device cannot hold the grid, it falls back to FUSED.
 * TWO_PHASE: an element launch writing the element forces to the workspace,
 * then a node launch gathering them.
 * FUSED_PAIR: two subcycles per launch on the FUSED tiles (temporal
 * blocking): each workgroup recomputes a halo of two elements, keeps the
 * intermediate velocity in LDS and the intermediate stress in registers, so
 * v and S cross HBM once per two subcycles; an odd count ends with one FUSED
 * launch.
 * FUSED_TRIPLE: three subcycles per launch likewise (halo of three elements;
 * n_a = 1 only); a remainder of one or two subcycles ends the call. If any
 * domain has general (non-parallelogram) cells it runs two per launch.
 * All strategies give bitwise-identical results. */
typedef enum {
  MEVP_STRATEGY_FUSED = 0,
  MEVP_STRATEGY_TWO_PHASE = 1,
  MEVP_STRATEGY_PERSISTENT = 2,
  MEVP_STRATEGY_FUSED_PAIR = 3,
  MEVP_STRATEGY_FUSED_TRIPLE = 4,
  /* not strategies: the range of int, as for mevp_precision */
  MEVP_STRATEGY_RANGE_MIN_ = -2147483647 - 1,
  MEVP_STRATEGY_RANGE_MAX_ = 2147483647
} mevp_strategy;

/* Launch configuration: strategy and the fused kernels' tile of owned
 * elements per workgroup (16 x 14; with n_a = 1 also 16 x 16, 32 x 15 and
 * 13 x 13). */
typedef struct {
  int strategy;  /* a mevp_strategy */
  int tile_nx;
  int tile_ny;
} mevp_config;

typedef struct mevp_ctx mevp_ctx;

/* Fill *out with the default parameters. EINVAL if out is NULL. */
mevp_status mevp_default_params(mevp_params *out);

/* Bytes of device workspace a context for these domains needs (Sec. 3.2: the
 * per-element inverse mass maps are recomputed from the four vertices of each
 * cell, so the workspace holds fields and state only). EINVAL on bad
 * descriptors, n_domains < 1, mixed n_s / n_a, or more than 2^31-1 elements
 * or nodes in total. */
mevp_status mevp_workspace_size(const mevp_domain_desc *domains, int n_domains,
                                mevp_precision precision, size_t *bytes);

/* Create a context: the device-resident counterpart of the arguments the
 * appendix listing's stress update takes besides the fields (the VP
 * parameters P*, Delta_min, the relaxation parameters alpha, beta, and the
 * mesh the element loop runs over), for one or more domains. The paper's
 * ports copy those buffers host <-> device around every kernel call
 * (Sec. 3.2, Sec. 4); a context instead keeps them, the state and the forcing
 * in the caller's workspace between calls.
 * `workspace` is a caller-owned device buffer of at least
 * mevp_workspace_size bytes, 256-byte aligned, that must outlive the context.
 * `hip_stream` is a hipStream_t (NULL = default stream). Checks that the
 * current device is gfx950 (EUNSUPPORTED otherwise). Enqueues the zeroing of
 * the state (v = 0, S = 0) on the stream and waits for it. On success *out
 * owns host memory released by mevp_destroy (*out is NULL on any error).
 * Errors: EINVAL (out, params, domains or workspace pointer/alignment),
 * ENOMEM (ws_bytes below the required size), EDEVICE, EUNSUPPORTED,
 * EHOSTMEM (the context's host tables could not be allocated). */
mevp_status mevp_create(const mevp_params *params, mevp_precision precision,
                        const mevp_domain_desc *domains, int n_domains, void *workspace,
                        size_t ws_bytes, void *hip_stream, mevp_ctx **out);

/* Select how subcycles are launched (default MEVP_STRATEGY_FUSED, tile
 * 16 x 14). set_config: EINVAL for an unknown strategy or tile, or FUSED_TRIPLE
 * or a tile other than 16 x 14 with n_a != 1; it waits for
 * the stream when the tile changes. */
mevp_status mevp_set_strategy(mevp_ctx *ctx, mevp_strategy strategy);
mevp_status mevp_set_config(mevp_ctx *ctx, const mevp_config *config);
mevp_status mevp_get_config(mevp_ctx *ctx, mevp_config *config);

/* Subcycles one launch of the subcycle kernel runs under the current
 * configuration and geometry (Eq. (si:mevp): each subcycle needs the previous
 * one's velocity, so a launch covers whole subcycles): 1 for FUSED and
 * TWO_PHASE; 2 or 3 for FUSED_PAIR / FUSED_TRIPLE, less where the cells do not
 * allow it (a bilinear domain: at most 2; a curved domain: 1); 0 for
 * PERSISTENT when it runs all subcycles of a call in one launch (every domain
 * of one geometry kind), else 1. A call of n subcycles then takes n / depth
 * launches plus one for the remainder. EINVAL if ctx or depth is NULL. */
mevp_status mevp_get_launch_depth(mevp_ctx *ctx, int *depth);

/* Replace the parameters (validated as in mevp_create). */
mevp_status mevp_set_params(mevp_ctx *ctx, const mevp_params *params);

/* Copy-in calls (stream-ordered; the caller may reuse its buffer once the
 * stream has passed the call). Layouts as above. mevp_set_geometry also
 * classifies the cells of the domain (all parallelograms or not, which picks
 * the element kernel; Sec. 2.1: cells are mapped from a reference element) and
 * waits for the stream to do so. */
mevp_status mevp_set_geometry(mevp_ctx *ctx, int dom, const double *vertex_xy);
/* Curved cells (Sec. 2.1: the cell map in the velocity's finite element
 * space): `node_xy` [2][(2nx+1)(2ny+1)] holds the positions of the CG2 nodes in
 * the node order of v, and every cell of the domain uses the isoparametric map
 * x(xi, eta) = sum_a X_a phi_a(xi, eta) of its 9 nodes (Jacobian per Gauss
 * point, local mass matrix per cell, edge normals from the map in
 * mevp_advect). Replaces a vertex geometry set before (and vice versa); the
 * corner nodes become the domain's vertices. Stream-ordered copy, then waits
 * for the stream. With this geometry in a context, FUSED_PAIR and
 * FUSED_TRIPLE run one subcycle per launch. EINVAL on a bad domain or a NULL
 * pointer. */
mevp_status mevp_set_geometry_cg2(mevp_ctx *ctx, int dom, const double *node_xy);
/* Ice height H and concentration A of domain `dom`, [n_a][nx*ny] DG
 * coefficients each: the H and A arguments of the appendix listing's stress
 * update, clamped at the Gauss points there and in Listing 1 (h >= 0,
 * 0 <= a <= 1) and advected by Eq. (si:ad). Stream-ordered copy (device or
 * host pointers); EINVAL on a bad domain or a NULL pointer. Values are not
 * checked here (mevp_check_inputs does). */
mevp_status mevp_set_fields(mevp_ctx *ctx, int dom, const double *H, const double *A);
/* Wind and ocean velocities of domain `dom` at the CG2 nodes,
 * [2][(2nx+1)(2ny+1)] m/s each: they enter the external forcing F of
 * Eq. (si:momentum), which the paper names as the combination of all external
 * forcings without stating it; here F is quadratic air drag
 * rho_a C_a |v_a| v_a weighted by the lumped concentration, and quadratic
 * ocean drag rho_o C_o |v_o - v| (v_o - v) weighted likewise, its magnitude
 * taken at the previous subcycle. Stream-ordered copy; EINVAL on a bad domain
 * or a NULL pointer. */
mevp_status mevp_set_forcing(mevp_ctx *ctx, int dom, const double *wind_xy,
                             const double *ocean_xy);
/* State of domain `dom`: the CG2 velocity v [2][(2nx+1)(2ny+1)] of
 * Eq. (si:momentum) and the DG stress S [3][n_s][nx*ny], the S11, S12, S22
 * coefficients that the stress update of Listing 1 and the appendix listing
 * reads and relaxes in place (Eq. (si:mevp) carries sigma^(p) from one
 * subcycle to the next; the state also carries S from one step to the next).
 * Stream-ordered copy into the current state buffers: the arrays are copied
 * to the device and reordered there into the library's internal layouts
 * (velocities interleaved per node, each element's coefficients of one
 * stress component contiguous), with the context's second state buffer as
 * staging. In MEVP_MIXED and
 * MEVP_MIXED_BF16, S is rounded to float on the device, so S must be a device pointer there
 * (EINVAL otherwise). EINVAL on a bad domain or a NULL pointer. */
mevp_status mevp_set_state(mevp_ctx *ctx, int dom, const double *v_xy, const double *S);

/* One time step of every domain (Sec. 2: momentum and mEVP subcycled inside
 * one advection step): mevp_begin_step, then mevp_subcycles(n_subcycles).
 * ESTATE unless geometry, fields and forcing of every domain were set.
 * By default the step's launches are captured once into a HIP graph (per
 * n_subcycles and state-buffer parity) on a private stream and replayed on
 * the context's stream; kernel timing, the persistent strategy or a failed
 * capture launch them one by one instead. Results are identical. */
mevp_status mevp_step(mevp_ctx *ctx, int n_subcycles);

/* Enable (default) or disable graph replay of mevp_step; drops the captured
 * graphs. */
mevp_status mevp_set_graph(mevp_ctx *ctx, int enable);

/* Start a time step: v^n <- v, and per node the lumped ice mass
 * M^H = int rho_i h phi, lumped concentration m^A = int a phi (h, a clamped
 * as in the stress listings) and air stress rho_a C_a |v_a| v_a. */
mevp_status mevp_begin_step(mevp_ctx *ctx);

/* n >= 0 mEVP subcycles (Eq. (si:mevp)) using the v^n of the last
 * mevp_begin_step: strain E from v^(p-1); stress update of Listing 1,
 * S <- fac S + ainv M^-1 Psi W s(E); divergence F_j = sum over the elements
 * around node j, in ascending element order, of -int sigma grad phi_j;
 * lumped-mass velocity update with beta relaxation, air drag, lagged ocean
 * drag and implicit Coriolis; v = 0 on the outer boundary. */
mevp_status mevp_subcycles(mevp_ctx *ctx, int n);

/* Autotuner: pick the fastest launch configuration for this context's
 * domains. Runs mevp_begin_step on the current state, then times every
 * candidate (FUSED, FUSED_PAIR and FUSED_TRIPLE with each tile shape available
 * for n_a, and TWO_PHASE; not PERSISTENT, whose grid-wide barrier costs more
 * than the gap between two launches of a replayed graph) on
 * n_trial >= 1 subcycles from that same state, restoring the state after each
 * trial, and checks that every candidate reproduces the first one bit for bit
 * (EINTERNAL if one does not; the previous configuration is kept). Leaves
 * the state as it was and the winner selected (*chosen, may be NULL).
 * cache_path (may be NULL): a text file of "key strategy tile_nx tile_ny"
 * lines, the key naming precision, n_s, n_a and the domain sizes; a matching
 * line is applied without timing, a new result is appended. Synchronous;
 * copies the state through host memory (EHOSTMEM if that cannot be
 * allocated). */
mevp_status mevp_tune(mevp_ctx *ctx, int n_trial, const char *cache_path, mevp_config *chosen);

/* Advect H and A of every domain over one step dt (Sec. 2: the advection
 * equations Eq. (si:ad) are solved at the large step, before the momentum
 * subcycles; no sources): DG with the upwind flux, three-stage SSP
 * Runge-Kutta, the current CG2 velocity held fixed. Per cell, for each DG
 * test function psi_k: M dU/dt = int_K U v.grad psi_k - sum over edges of
 * int (v.n) U_up psi_k, U_up the upwind trace (the cell's own trace on the
 * domain boundary), 3x3 Gauss points in the cell and 3 per edge. Stream-ordered;
 * no clamping of A (the stress and mass computations clamp h and a). */
mevp_status mevp_advect(mevp_ctx *ctx);

/* Copy out H and A of domain `dom` ([n_a][ne] each; either may be NULL). */
mevp_status mevp_get_fields(mevp_ctx *ctx, int dom, double *H, double *A);

/* Copy out the state of domain `dom` in the layouts of mevp_set_state: the
 * velocity v and the DG stress S after the last subcycle (Eq. (si:mevp);
 * the in-out stress arguments of the appendix listing). Either pointer may be
 * NULL. The state is reordered from the internal layouts on the device (the
 * second state buffer as staging), then copied out. Stream-ordered: the
 * values are valid once the stream has passed the call (mevp_sync). In MEVP_MIXED and MEVP_MIXED_BF16, S is widened from
 * float on the device and must be a device pointer (EINVAL otherwise). EINVAL on a bad domain. */
mevp_status mevp_get_state(mevp_ctx *ctx, int dom, double *v_xy, double *S);

/* Wait for the context's stream; EDEVICE if any enqueued work failed. */
mevp_status mevp_sync(mevp_ctx *ctx);

/* Synchronous device checks. check_inputs: every vertex, H, A, wind and
 * ocean value finite and every element Jacobian positive at every Gauss
 * point; check_state: every v and S value finite. ENONFINITE if not. */
mevp_status mevp_check_inputs(mevp_ctx *ctx);
mevp_status mevp_check_state(mevp_ctx *ctx);

/* Kernel timing for measurement (the paper times kernels alone, with
 * barriers around them, Sec. 4). enable: record a HIP event pair around each
 * of the next `max_launches` launches of every phase on the context's stream
 * (0 disables and frees the events). read: wait for the stream, then return
 * per phase (0 = element phase, 1 = node phase, 2 = start of step) the number
 * of timed launches and their summed duration in milliseconds, and restart
 * the count. Arrays have 3 entries; either may be NULL. */
mevp_status mevp_timing_enable(mevp_ctx *ctx, int max_launches);
mevp_status mevp_timing_read(mevp_ctx *ctx, int *count, double *total_ms);

/* Bytes of the device array that mevp_step_static works in, per GPU. */
#define MEVP_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate memory: code that must not call hipMalloc
 * or create HIP objects, tight serving loops, harnesses that forbid
 * allocation. One time step (mevp_begin_step, then n_subcycles >= 0 mEVP
 * subcycles) of ONE domain with vertex geometry, without a context or a
 * workspace: the values are those of mevp_create + mevp_set_geometry /
 * _fields / _forcing / _state + mevp_step(n_subcycles) + mevp_get_state on
 * the same inputs (bit for bit, in every precision).
 * Arguments: params and precision as in mevp_create; `domain` one descriptor;
 * vertex_xy, H, A, wind_xy, ocean_xy the inputs in the layouts above, read in
 * place by the kernels; v_xy [2][(2nx+1)(2ny+1)] and S [3][n_s][nx*ny] the
 * state, read at the start and overwritten with the state after the step.
 * Every array must be device memory on the current device (EINVAL
 * otherwise), 8-byte aligned, of the stated size, and stay valid until the
 * stream has passed the call. `hip_stream` as in mevp_create.
 * Working memory: a file-scope device array of MEVP_STATIC_SCRATCH_BYTES, one
 * per GPU, held from the library's first use on that GPU until the process
 * ends; it takes the tables, both velocity and stress buffers and the node
 * constants (at n_s = 6 about 610 bytes per element in FP64, 470 in mixed
 * precision: up to ~1.1e5 / ~1.4e5 elements). ENOMEM if the domain needs more.
 * The call allocates no device or host memory and creates no HIP object: no
 * hipMalloc / hipFree, no graph, no event. It classifies the cells on the
 * device as mevp_set_geometry does and waits for the stream once to read the
 * result (so it cannot be captured into a graph); everything after that is
 * stream-ordered and the outputs are valid once the stream has passed the
 * call. Every call on a GPU shares that GPU's array, which keeps the last
 * call's contents (this call clears what it uses first): calls that overlap
 * on one GPU (other host threads, or other streams not ordered with this
 * one) race and give wrong results; the caller serialises them.
 * Errors: EINVAL (NULL or non-device pointer, bad params or descriptor,
 * n_subcycles < 0), ENOMEM (the domain does not fit the array), EDEVICE,
 * EUNSUPPORTED (not gfx950), EHOSTMEM. */
mevp_status mevp_step_static(const mevp_params *params, mevp_precision precision,
                             const mevp_domain_desc *domain, const double *vertex_xy,
                             const double *H, const double *A, const double *wind_xy,
                             const double *ocean_xy, double *v_xy, double *S, int n_subcycles,
                             void *hip_stream);

/* Release the context's host memory (the workspace stays the caller's).
 * Does not synchronise. NULL is a no-op. */
void mevp_destroy(mevp_ctx *ctx);

/* Static description of a status code. */
const char *mevp_status_string(mevp_status s);

/* Library version string. */
const char *mevp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MEVP_H */
