// mevp_internal.hpp -- types shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mevp {

// One domain as the kernels see it. Every per-domain array is a contiguous
// block inside a context-wide array, at the offsets below (in elements,
// nodes or vertices), in the public layout of mevp.h.
struct DomDev {
  int nx, ny;
  int ne, nn, nv;      // elements, CG2 nodes, vertices
  int elem_off;        // first element of this domain in the context
  int node_off;        // first node
  int vert_off;        // first vertex
};

// A block of work: domain index and the first local element (or node).
struct Blk {
  int dom;
  int first;
};

// Scalars the kernels need, derived once from mevp_params on the host.
struct KParams {
  double Pstar, C, dmin2;  // P*, concentration factor, Delta_min^2
  double fac, ainv;        // stress relaxation weights
  double beta, inv_dt;     // velocity relaxation, 1/dt
  double rho_i, rhoCa, rhoCo, f_dt;  // densities x drag coefficients, Coriolis x dt
};

// Device pointers of one context (all carved from the caller's workspace).
struct DevArrays {
  const DomDev *doms;
  const Blk *eblk;  // element blocks: parallelogram-cell domains first, then general
  const Blk *nblk;  // node blocks
  const double *vert;  // [dom][2][nv]
  const double *H;     // [dom][n_a][ne]
  const double *A;
  const double *wind;  // [dom][2][nn]
  const double *ocean;
  double *v;           // [dom][2][nn]
  double *nc;          // [dom][6][nn] node constants of the velocity update
  void *S;             // [dom][3][n_s][ne], double or float
  void *fe;            // [dom][18][ne] element nodal forces, double or float
  int *flag;           // check results
};

constexpr int kElemBlock = 256;
constexpr int kNodeBlock = 256;

// Launchers (mevp_kernels.hip). Return hipSuccess or the launch error.
hipError_t launch_begin_step(const DevArrays &d, const KParams &p, int n_a, int n_s,
                             int n_nblk, hipStream_t s);
hipError_t launch_element_phase(const DevArrays &d, const KParams &p, int n_s, int n_a,
                                bool mixed, int n_aff, int n_gen, hipStream_t s);
hipError_t launch_cell_shape(const DevArrays &d, int dom, int ne, int *flag, hipStream_t s);
hipError_t launch_node_phase(const DevArrays &d, const KParams &p, bool mixed, int n_nblk,
                             hipStream_t s);
hipError_t launch_fill(void *dst, size_t n_words32, uint32_t value, hipStream_t s);
hipError_t launch_convert_d2f(const double *src, float *dst, size_t n, hipStream_t s);
hipError_t launch_convert_f2d(const float *src, double *dst, size_t n, hipStream_t s);
hipError_t launch_check_finite(const double *p, size_t n, int *flag, int bit, hipStream_t s);
hipError_t launch_check_finite_f(const float *p, size_t n, int *flag, int bit, hipStream_t s);
hipError_t launch_check_jacobian(const DevArrays &d, int n_s, int n_eblk, int bit, hipStream_t s);

}  // namespace mevp
