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
  int kind;            // cell geometry, a GeoKind
};

// Cell geometry of a domain, which picks the element update: parallelogram
// cells (constant Jacobian), bilinear map of the 4 vertices, isoparametric
// map of the 9 CG2 nodes (curved cells).
enum GeoKind { kGeoAffine = 0, kGeoBilinear = 1, kGeoIso = 2 };
constexpr int kNumGeo = 3;

// A block of work: domain index and the first local element (or node).
struct Blk {
  int dom;
  int first;
};

// A tile of the fused subcycle kernel: domain and the first owned element.
struct Tile {
  int dom;
  int x0, y0;
  int pad;
};

// Buffers one subcycle reads and writes (context-wide bases; the fused kernel
// double-buffers v and S, the two-phase kernels update them in place).
struct Bufs {
  const double *v_in;
  double *v_out;
  const void *S_in;
  void *S_out;
};

// Launch arguments of the fused subcycle kernel.
struct FusedArgs {
  Bufs b0, b1;     // buffers of even / odd subcycles (b1 = b0 swapped)
  int shape;       // index into kTileShapes
  int persist;     // 1: one cooperative launch for n_sub subcycles
  int n_sub;
  int depth;       // subcycles per launch of k_fused_multi (2, 3; buffers b0), else 1
};

// Blocks (or tiles) grouped by the geometry kind of their domain, in GeoKind
// order: n[k] of kind k.
struct Launch {
  int n[kNumGeo];
};

// Scalars the kernels need, derived once from mevp_params on the host.
struct KParams {
  double Pstar, C, dmin2;  // P*, concentration factor, Delta_min^2
  double dmin2_16;         // Delta_min^2 / 16
  double fac, ainv;        // stress relaxation weights
  double beta, inv_dt;     // velocity relaxation, 1/dt
  double rho_i, rhoCa, rhoCo, f_dt;  // densities x drag coefficients, Coriolis x dt
};

// Device pointers of one context (all carved from the caller's workspace).
struct DevArrays {
  const DomDev *doms;
  const Blk *eblk;  // element blocks: parallelogram-cell domains first, then general
  const Blk *nblk;  // node blocks
  const Tile *tiles;  // fused-kernel tiles: parallelogram-cell domains first
  const double *vert;  // [dom][2][nv]
  const double *xnode; // [dom][2][nn] CG2 node positions (isoparametric domains)
  const double *H;     // [dom][n_a][ne]
  const double *A;
  double *adv;         // advection stages: [4][dom][n_a][ne] (H1, A1, H2, A2)
  const double *wind;  // [dom][2][nn]
  const double *ocean;
  double *v;           // [dom][nn][2], interleaved per node (two buffers: v and v + 2 * total nodes)
  double *nc;          // [dom][nn][6] node constants of the velocity update, per node
  void *S;             // [dom][3][ne][n_s], double or float (two buffers)
  void *fe;            // [dom][18][ne] element nodal forces, double or float
  int *flag;           // check results
};

constexpr int kElemBlock = 256;
constexpr int kNodeBlock = 256;
// fused kernel tile shapes (elements per workgroup including the one-element
// halo; the owned block is one smaller in each direction): 17 x 15 (16 x 14
// owned, 16 owned elements = one 128-byte line of a double array per row),
// 17 x 17, 33 x 16 (32 x 15 owned: three subcycles per launch take 37 x 20
// lanes, twelve waves, all that three waves per SIMD allow, and 149 KB of LDS)
// and 14 x 14 (13 x 13 owned: two subcycles per launch take 16 x 16 lanes,
// exactly four waves, so that two workgroups share a CU at the general-cell
// update's two waves per SIMD)
constexpr int kNumTileShapes = 4;
constexpr int kTileShapes[kNumTileShapes][2] = {{17, 15}, {17, 17}, {33, 16}, {14, 14}};
// workgroups are dealt to the 8 XCDs of the chip in turn
constexpr int kNumXcd = 8;
// A domain's tiles are listed in column strips about kStripElems elements
// wide (strip_width tiles), row by row within a strip, before the list is cut
// into one contiguous band per XCD: the workgroups an XCD runs at once then
// cover a few consecutive rows of one strip, so the tiles beside and below a
// tile (which read the same halo elements and nodes) run with it or just
// before it, while those lines are in the XCD's L2
constexpr int kStripElems = 256;

// Launchers (mevp_kernels.hip). Return hipSuccess or the launch error.
// start of a time step on the ntiles fused-kernel tiles of tile shape `shape`
// (d.tiles: every tile of every domain)
hipError_t launch_begin_step(const DevArrays &d, const KParams &p, int n_a, int n_s,
                             const double *v, int shape, int ntiles, hipStream_t s);
// prec: a mevp_precision (0 FP64, 1 mixed, 2 mixed with bfloat16 element
// matrices, fused kernels at n_s = 6 and n_a = 1 only)
hipError_t launch_element_phase(const DevArrays &d, const KParams &p, int n_s, int n_a,
                                int prec, const Launch &L, Bufs b, hipStream_t s);
hipError_t launch_node_phase(const DevArrays &d, const KParams &p, bool mixed, int n_nblk, Bufs b,
                             hipStream_t s);
hipError_t launch_fused_subcycle(const DevArrays &d, const KParams &p, int n_s, int n_a,
                                 int prec, const Launch &L, const FusedArgs &f, hipStream_t s);
hipError_t launch_cell_shape(const DevArrays &d, int dom, int ne, int *flag, hipStream_t s);
hipError_t launch_corner_vertices(const DevArrays &d, int dom, int nv, hipStream_t s);
// one advection stage over the element blocks, grouped by geometry kind as in L
hipError_t launch_advect_stage(const DevArrays &d, int n_a, const Launch &L, const double *v,
                               const double *Hn, const double *An, const double *Hin,
                               const double *Ain, double *Hout, double *Aout, double dt, double ca,
                               double cb, hipStream_t s);
hipError_t launch_fill(void *dst, size_t n_words32, uint32_t value, hipStream_t s);
// Tables of a one-domain context written on the device (no host staging):
// doms[0] = D, element and node blocks of that domain in order, and its
// fused-kernel tiles of tx x ty owned elements in the XCD band order of the
// host-built tables.
hipError_t launch_single_tables(const DomDev &D, int tx, int ty, DomDev *doms, Blk *eblk,
                                int n_eblk, Blk *nblk, int n_nblk, Tile *tiles, int n_tiles,
                                hipStream_t s);
// Fused subcycle launch of the parallelogram-cell tiles of one tile shape
// (defined in mevp_affine.hpp and instantiated, for every n_s, n_a, precision
// and tile shape the dispatch reaches, in mevp_kernels_affine*.hip: units of
// their own, so that each can be scheduled as measured best).
template <int NS, int NA, class T, int EX, int EY>
hipError_t fused_affine(const DevArrays &d, const KParams &p, const Tile *tiles, int ntiles,
                        const FusedArgs &f, hipStream_t s);
// per-n_s launchers (mevp_kernels_ns{3,6,8}.hip)
hipError_t begin_step_ns3(const DevArrays &, const KParams &, int, const double *, int, int,
                          hipStream_t);
hipError_t begin_step_ns6(const DevArrays &, const KParams &, int, const double *, int, int,
                          hipStream_t);
hipError_t begin_step_ns8(const DevArrays &, const KParams &, int, const double *, int, int,
                          hipStream_t);
hipError_t two_phase_ns3(const DevArrays &, const KParams &, int, bool, const Launch &, Bufs, hipStream_t);
hipError_t two_phase_ns6(const DevArrays &, const KParams &, int, bool, const Launch &, Bufs, hipStream_t);
hipError_t two_phase_ns8(const DevArrays &, const KParams &, int, bool, const Launch &, Bufs, hipStream_t);
hipError_t fused_ns3(const DevArrays &, const KParams &, int, bool, const Launch &, const FusedArgs &, hipStream_t);
hipError_t fused_ns6(const DevArrays &, const KParams &, int, bool, const Launch &, const FusedArgs &, hipStream_t);
hipError_t fused_ns8(const DevArrays &, const KParams &, int, bool, const Launch &, const FusedArgs &, hipStream_t);
// the bfloat16 element-matrix trial (mevp_kernels_bf16.hip)
hipError_t fused_bf16(const DevArrays &, const KParams &, int n_s, int n_a, const Launch &,
                      const FusedArgs &, hipStream_t);
// velocities between the public layout [2][n] and the kernels' [n][2]
hipError_t launch_interleave2(const double *src, double *dst, size_t n, hipStream_t s);
hipError_t launch_deinterleave2(const double *src, double *dst, size_t n, hipStream_t s);
// the stress of one domain between the public layout [3][ns][ne] (double)
// and the kernels' [3][ne][ns] (double, or float when fp32)
hipError_t launch_stress_in(const double *src, void *dst, bool fp32, size_t ne, int ns,
                            hipStream_t s);
hipError_t launch_stress_out(const void *src, bool fp32, double *dst, size_t ne, int ns,
                             hipStream_t s);
hipError_t launch_convert_d2f(const double *src, float *dst, size_t n, hipStream_t s);
hipError_t launch_convert_f2d(const float *src, double *dst, size_t n, hipStream_t s);
hipError_t launch_check_finite(const double *p, size_t n, int *flag, int bit, hipStream_t s);
hipError_t launch_check_finite_f(const float *p, size_t n, int *flag, int bit, hipStream_t s);
hipError_t launch_check_jacobian(const DevArrays &d, int n_s, int n_eblk, int bit, hipStream_t s);

}  // namespace mevp
