// mevp_kernels.hip -- n_s-independent kernels (node phase, utilities) and the
// dispatch of the per-n_s launchers (mevp_kernels_ns{3,6,8}.hip).
#include "mevp_device.hpp"

namespace mevp {
namespace {

// ---------------------------------------------------------------------------
// Small utility kernels
// ---------------------------------------------------------------------------
__global__ void k_fill(uint32_t *dst, size_t n, uint32_t value) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = value;
}
__global__ void k_d2f(const double *src, float *dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}
// [2][n] <-> [n][2] (the velocities' public and internal layouts)
__global__ void k_interleave2(const double *src, double *dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    reinterpret_cast<double2 *>(dst)[i] = double2{src[i], src[n + i]};
}
__global__ void k_deinterleave2(const double *src, double *dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const double2 u = reinterpret_cast<const double2 *>(src)[i];
    dst[i] = u.x;
    dst[n + i] = u.y;
  }
}
// the stress between the public layout [3][ns][ne] (double) and the kernels'
// [3][ne][ns] (double or float)
template <class TD>
__global__ void k_stress_in(const double *src, TD *dst, size_t ne, int ns) {
  const size_t n = 3 * (size_t)ns * ne;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t k = i % ns, e = (i / ns) % ne, c = i / (ns * ne);
    dst[i] = TD(src[(c * ns + k) * ne + e]);
  }
}
template <class TS>
__global__ void k_stress_out(const TS *src, double *dst, size_t ne, int ns) {
  const size_t n = 3 * (size_t)ns * ne;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t k = i % ns, e = (i / ns) % ne, c = i / (ns * ne);
    dst[(c * ns + k) * ne + e] = double(src[i]);
  }
}
__global__ void k_f2d(const float *src, double *dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (double)src[i];
}
template <class T>
__global__ void k_check_finite(const T *p, size_t n, int *flag, int bit) {
  int bad = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    bad |= !isfinite(p[i]);
  if (bad) atomicOr(flag, bit);
}
template <int NS>
__global__ void __launch_bounds__(kElemBlock) k_check_jacobian(DevArrays d, int bit) {
  using Q = Quad<Ngp<NS>::value>;
  const Blk blk = d.eblk[blockIdx.x];
  const DomDev D = d.doms[blk.dom];
  const int el = blk.first + (int)threadIdx.x;
  if (el >= D.ne) return;
  bool bad = false;
  auto check = [&](const auto &c) {
#pragma unroll
    for (int q = 0; q < Q::NG; ++q) {
      double J00, J01, J10, J11;
      c.jac(Q::xi(q), Q::eta(q), J00, J01, J10, J11);
      bad |= !(J00 * J11 - J01 * J10 > 0.0);
    }
  };
  if (D.kind == kGeoIso)
    check(load_q2map<double>(D, d.xnode, el % D.nx, el / D.nx));
  else
    check(load_cell<double>(D, d.vert, el % D.nx, el / D.nx));
  if (bad) atomicOr(d.flag, bit);
}

// Vertices of an isoparametric domain: its corner CG2 nodes.
__global__ void __launch_bounds__(kElemBlock) k_corner_vertices(DevArrays d, int dom) {
  const DomDev D = d.doms[dom];
  double *VX = const_cast<double *>(d.vert) + 2 * (size_t)D.vert_off;
  const double *XN = d.xnode + 2 * (size_t)D.node_off;
  const int NX = 2 * D.nx + 1;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < D.nv; i += gridDim.x * blockDim.x) {
    const int ix = i % (D.nx + 1), iy = i / (D.nx + 1);
    const int j = 2 * iy * NX + 2 * ix;
    VX[i] = XN[j];
    VX[D.nv + i] = XN[D.nn + j];
  }
}

// Tables of a one-domain context (see launch_single_tables). Tile i of the
// launch runs on XCD i % 8 and takes tile `start + s` of the strip-ordered
// tile list, s = i / 8, start = the tiles dealt to the lower XCDs: every XCD
// gets one contiguous band, as in the host-built tables.
__global__ void k_single_tables(DomDev D, int tx, int ty, DomDev *doms, Blk *eblk, int n_eblk,
                                Blk *nblk, int n_nblk, Tile *tiles, int n_tiles) {
  const int stride = gridDim.x * blockDim.x;
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 == 0) doms[0] = D;
  for (int i = i0; i < n_eblk; i += stride) eblk[i] = Blk{0, i * kElemBlock};
  for (int i = i0; i < n_nblk; i += stride) nblk[i] = Blk{0, i * kNodeBlock};
  const int ntx = (D.nx + tx - 1) / tx, nty = (D.ny + ty - 1) / ty;
  for (int i = i0; i < n_tiles; i += stride) {
    const int x = i % kNumXcd, s = i / kNumXcd;
    int start = 0;
    for (int xx = 0; xx < x; ++xx) start += (n_tiles - xx + kNumXcd - 1) / kNumXcd;
    int col, row;
    strip_tile(start + s, ntx, nty, strip_width(tx, kStripElems), col, row);
    tiles[i] = Tile{0, col * tx, row * ty, 0};
  }
}

inline unsigned grid_for(size_t n, unsigned block) {
  size_t g = (n + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g == 0) g = 1;
  return (unsigned)g;
}

}  // namespace


// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_begin_step(const DevArrays &d, const KParams &p, int n_a, int n_s,
                             const double *v, int shape, int ntiles, hipStream_t s) {
  if (n_s == 3) return begin_step_ns3(d, p, n_a, v, shape, ntiles, s);
  if (n_s == 6) return begin_step_ns6(d, p, n_a, v, shape, ntiles, s);
  if (n_s == 8) return begin_step_ns8(d, p, n_a, v, shape, ntiles, s);
  return hipErrorInvalidValue;
}

hipError_t launch_element_phase(const DevArrays &d, const KParams &p, int n_s, int n_a, int prec,
                                const Launch &L, Bufs b, hipStream_t s) {
  if (prec != 0 && prec != 1) return hipErrorInvalidValue;
  const bool mixed = prec == 1;
  if (n_s == 3) return two_phase_ns3(d, p, n_a, mixed, L, b, s);
  if (n_s == 6) return two_phase_ns6(d, p, n_a, mixed, L, b, s);
  if (n_s == 8) return two_phase_ns8(d, p, n_a, mixed, L, b, s);
  return hipErrorInvalidValue;
}

hipError_t launch_fused_subcycle(const DevArrays &d, const KParams &p, int n_s, int n_a, int prec,
                                 const Launch &L, const FusedArgs &f, hipStream_t s) {
  if (prec == 2) return fused_bf16(d, p, n_s, n_a, L, f, s);
  if (prec != 0 && prec != 1) return hipErrorInvalidValue;
  const bool mixed = prec == 1;
  if (n_s == 3) return fused_ns3(d, p, n_a, mixed, L, f, s);
  if (n_s == 6) return fused_ns6(d, p, n_a, mixed, L, f, s);
  if (n_s == 8) return fused_ns8(d, p, n_a, mixed, L, f, s);
  return hipErrorInvalidValue;
}

hipError_t launch_node_phase(const DevArrays &d, const KParams &p, bool mixed, int n_nblk, Bufs b,
                             hipStream_t s) {
  if (mixed)
    hipLaunchKernelGGL((k_node<float>), dim3(n_nblk), dim3(kNodeBlock), 0, s, d, p, b);
  else
    hipLaunchKernelGGL((k_node<double>), dim3(n_nblk), dim3(kNodeBlock), 0, s, d, p, b);
  return hipGetLastError();
}

hipError_t launch_advect_stage(const DevArrays &d, int n_a, const Launch &L, const double *v,
                               const double *Hn, const double *An, const double *Hin,
                               const double *Ain, double *Hout, double *Aout, double dt, double ca,
                               double cb, hipStream_t s) {
  if (n_a != 1 && n_a != 3 && n_a != 6) return hipErrorInvalidValue;
  // element blocks grouped by geometry kind: vertex cells (parallelogram and
  // bilinear), then curved cells
  const int n_vert = L.n[kGeoAffine] + L.n[kGeoBilinear], n_iso = L.n[kGeoIso];
  const Blk *bv = d.eblk, *bi = d.eblk + n_vert;
#define MEVP_AD(NA_)                                                                          \
  if (n_a == NA_) {                                                                           \
    if (n_vert > 0)                                                                           \
      hipLaunchKernelGGL((k_advect<NA_, kGeoBilinear>), dim3(n_vert), dim3(kElemBlock), 0, s, d, \
                         bv, v, Hn, An, Hin, Ain, Hout, Aout, dt, ca, cb);                   \
    if (n_iso > 0)                                                                            \
      hipLaunchKernelGGL((k_advect<NA_, kGeoIso>), dim3(n_iso), dim3(kElemBlock), 0, s, d, bi, \
                         v, Hn, An, Hin, Ain, Hout, Aout, dt, ca, cb);                       \
  }
  MEVP_AD(1) MEVP_AD(3) MEVP_AD(6)
#undef MEVP_AD
  return hipGetLastError();
}

hipError_t launch_cell_shape(const DevArrays &d, int dom, int ne, int *flag, hipStream_t s) {
  hipLaunchKernelGGL(k_cell_shape, dim3(grid_for((size_t)ne, kElemBlock)), dim3(kElemBlock), 0, s, d,
                     dom, flag);
  return hipGetLastError();
}

hipError_t launch_fill(void *dst, size_t n_words32, uint32_t value, hipStream_t s) {
  if (n_words32 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n_words32, 256)), dim3(256), 0, s,
                     static_cast<uint32_t *>(dst), n_words32, value);
  return hipGetLastError();
}
hipError_t launch_single_tables(const DomDev &D, int tx, int ty, DomDev *doms, Blk *eblk,
                                int n_eblk, Blk *nblk, int n_nblk, Tile *tiles, int n_tiles,
                                hipStream_t s) {
  int most = n_eblk > n_nblk ? n_eblk : n_nblk;
  if (n_tiles > most) most = n_tiles;
  hipLaunchKernelGGL(k_single_tables, dim3(grid_for((size_t)most, 256)), dim3(256), 0, s, D, tx, ty,
                     doms, eblk, n_eblk, nblk, n_nblk, tiles, n_tiles);
  return hipGetLastError();
}
hipError_t launch_interleave2(const double *src, double *dst, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_interleave2, dim3(grid_for(n, 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}
hipError_t launch_deinterleave2(const double *src, double *dst, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_deinterleave2, dim3(grid_for(n, 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}
hipError_t launch_stress_in(const double *src, void *dst, bool fp32, size_t ne, int ns,
                            hipStream_t s) {
  const size_t n = 3 * (size_t)ns * ne;
  if (n == 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL((k_stress_in<float>), dim3(grid_for(n, 256)), dim3(256), 0, s, src,
                       static_cast<float *>(dst), ne, ns);
  else
    hipLaunchKernelGGL((k_stress_in<double>), dim3(grid_for(n, 256)), dim3(256), 0, s, src,
                       static_cast<double *>(dst), ne, ns);
  return hipGetLastError();
}
hipError_t launch_stress_out(const void *src, bool fp32, double *dst, size_t ne, int ns,
                             hipStream_t s) {
  const size_t n = 3 * (size_t)ns * ne;
  if (n == 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL((k_stress_out<float>), dim3(grid_for(n, 256)), dim3(256), 0, s,
                       static_cast<const float *>(src), dst, ne, ns);
  else
    hipLaunchKernelGGL((k_stress_out<double>), dim3(grid_for(n, 256)), dim3(256), 0, s,
                       static_cast<const double *>(src), dst, ne, ns);
  return hipGetLastError();
}
hipError_t launch_convert_d2f(const double *src, float *dst, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_d2f, dim3(grid_for(n, 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}
hipError_t launch_convert_f2d(const float *src, double *dst, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_f2d, dim3(grid_for(n, 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}
hipError_t launch_check_finite(const double *p, size_t n, int *flag, int bit, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_check_finite<double>), dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, flag, bit);
  return hipGetLastError();
}
hipError_t launch_check_finite_f(const float *p, size_t n, int *flag, int bit, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_check_finite<float>), dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, flag, bit);
  return hipGetLastError();
}
hipError_t launch_corner_vertices(const DevArrays &d, int dom, int nv, hipStream_t s) {
  hipLaunchKernelGGL(k_corner_vertices, dim3(grid_for((size_t)nv, kElemBlock)), dim3(kElemBlock), 0,
                     s, d, dom);
  return hipGetLastError();
}

hipError_t launch_check_jacobian(const DevArrays &d, int n_s, int n_eblk, int bit, hipStream_t s) {
  if (n_s == 3)
    hipLaunchKernelGGL((k_check_jacobian<3>), dim3(n_eblk), dim3(kElemBlock), 0, s, d, bit);
  else
    hipLaunchKernelGGL((k_check_jacobian<6>), dim3(n_eblk), dim3(kElemBlock), 0, s, d, bit);
  return hipGetLastError();
}

}  // namespace mevp
