// mevp_kernels_bf16.hip -- the bfloat16 trial of the mixed form: the fused
// subcycle kernels (one, two or three subcycles per launch, every tile shape)
// at n_s = 6 with one ice dof, parallelogram and bilinear cells, with every
// element-matrix entry rounded to bfloat16 and the arithmetic in float
// (mat<T, 1> in mevp_device.hpp).
#include "mevp_device.hpp"

namespace mevp {

hipError_t fused_bf16(const DevArrays &d, const KParams &p, int n_s, int n_a, const Launch &L,
                      const FusedArgs &f, hipStream_t s) {
  if (n_s != 6 || n_a != 1 || f.persist) return hipErrorInvalidValue;
  return fused_t<6, 1, float, 1>(d, p, L, f, s);
}

}  // namespace mevp
