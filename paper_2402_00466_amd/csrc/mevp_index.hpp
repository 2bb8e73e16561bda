// mevp_index.hpp -- index arithmetic of the fused tile kernels, shared by the
// kernels (mevp_device.hpp), the host runtime (mevp_api.hip) and the host-side
// index check (tests/index_check.hip): the node ranges of each node phase, the
// node-to-lane mapping of a node phase, the LDS offsets of the element forces
// a node sums, and the order of a domain's tiles. Host and device run the
// same functions, so the check covers the kernels' own arithmetic.
#pragma once

#include <hip/hip_runtime.h>

namespace mevp {

// A half-open range of CG2 nodes [ix0, ix1) x [iy0, iy1).
struct NodeRange {
  int ix0, ix1, iy0, iy1;
};

// Nodes a tile of TX x TY owned elements with first owned element (x0, y0)
// updates and stores: CG2 columns [2 x0, 2 (x0 + TX)), rows likewise, and the
// last column / row of the domain for the last tile (NX x NY nodes, nx x ny
// elements).
__host__ __device__ inline NodeRange owned_nodes(int x0, int y0, int TX, int TY, int nx, int ny,
                                                int NX, int NY) {
  NodeRange r;
  r.ix0 = 2 * x0;
  r.iy0 = 2 * y0;
  r.ix1 = (x0 + TX >= nx) ? NX : r.ix0 + 2 * TX;
  r.iy1 = (y0 + TY >= ny) ? NY : r.iy0 + 2 * TY;
  return r;
}

// Nodes of element phase i+1 of a K-subcycle pass (node phase i < K-1):
// elements [x0-K+i+1, x0+TX+K-2-i] (likewise in y), clipped to the domain.
__host__ __device__ inline NodeRange multi_phase_nodes(int x0, int y0, int TX, int TY, int K,
                                                      int i, int NX, int NY) {
  const int ex0 = x0 - K, ey0 = y0 - K;
  const int a = 2 * (ex0 + i + 1), b = 2 * (ey0 + i + 1);
  const int c = 2 * (x0 + TX + K - 2 - i) + 1, e = 2 * (y0 + TY + K - 2 - i) + 1;
  NodeRange r;
  r.ix0 = a > 0 ? a : 0;
  r.iy0 = b > 0 ? b : 0;
  r.ix1 = c < NX ? c : NX;
  r.iy1 = e < NY ? e : NY;
  return r;
}

// Tiles per strip for tiles of tx owned elements in x: about kStripElems
// elements (at least one tile).
__host__ __device__ inline int strip_width(int tx, int strip_elems) {
  const int w = (strip_elems + tx / 2) / tx;
  return w > 0 ? w : 1;
}

// Tile k of a domain's tile list of ntx x nty tiles in strip order: column
// strips `strip` tiles wide (the last one narrower), row by row within a
// strip, left to right within a row; (col, row) of that tile.
__host__ __device__ inline void strip_tile(int k, int ntx, int nty, int strip, int &col, int &row) {
  const int j = k / (strip * nty);
  const int w = ntx - strip * j < strip ? ntx - strip * j : strip;
  const int off = k - strip * j * nty;
  row = off / w;
  col = strip * j + off % w;
}

// Node k of a range w nodes wide, row-major: (k mod w, k div w), the
// division through the float reciprocal rw = 1/w: for k < 2^13 and w < 2^7
// the product (k + 1/2) rw is within 1e-3 of (k + 1/2) / w, which lies at
// least 1/(2w) from an integer, so the truncation is exact.
__host__ __device__ inline void node_in_range(int k, int w, float rw, int &dx, int &dy) {
  dy = (int)(((float)k + 0.5f) * rw);
  dx = k - dy * w;
}

// The forces of the <= 4 elements around interior node (ix, iy), in a table
// fl[18][NF] (x components in rows 0..8, y in 9..17, one column per element,
// element (ex, ey) at column (ey - ey0) * FW + ex - ex0): off[0..3] are the
// x-component offsets of the four reads in ascending element order (first
// element, its right neighbour, the one above, the one above-right; add
// 9 NF for y), two_x / two_y say whether the second and third exist (an even
// node index: the node lies on an element boundary in that direction); the
// fourth exists when both do. The node is local node a = 3 b + c of each
// element (b = 1 or 2 for odd or even iy in the first row of elements, 0 in
// the second; likewise c).
__host__ __device__ inline void node_force_offsets(int ix, int iy, int ex0, int ey0, int FW, int NF,
                                                   int (&off)[4], bool &two_x, bool &two_y) {
  two_x = !(ix & 1);
  two_y = !(iy & 1);
  const int b3 = two_y ? 6 : 3, c0 = two_x ? 2 : 1;
  const int base = (((iy - 1) >> 1) - ey0) * FW + ((ix - 1) >> 1) - ex0;
  off[0] = base + (b3 + c0) * NF;
  off[1] = base + b3 * NF + 1;
  off[2] = base + c0 * NF + FW;
  off[3] = base + FW + 1;
}

}  // namespace mevp
