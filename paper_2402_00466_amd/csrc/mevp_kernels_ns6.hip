// mevp_kernels_ns6.hip -- kernels with 6 DG stress dofs per component
// (one translation unit per n_s so that the kernels compile in parallel).
#include "mevp_device.hpp"

namespace mevp {

hipError_t begin_step_ns6(const DevArrays &d, const KParams &p, int n_a, const double *v,
                          int shape, int ntiles, hipStream_t s) {
  return begin_step_ns<6>(d, p, n_a, v, shape, ntiles, s);
}

hipError_t two_phase_ns6(const DevArrays &d, const KParams &p, int n_a, bool mixed,
                         const Launch &L, Bufs b, hipStream_t s) {
  return two_phase_ns<6>(d, p, n_a, mixed, L, b, s);
}

hipError_t fused_ns6(const DevArrays &d, const KParams &p, int n_a, bool mixed, const Launch &L,
                     const FusedArgs &f, hipStream_t s) {
  return fused_ns<6>(d, p, n_a, mixed, L, f, s);
}

}  // namespace mevp
