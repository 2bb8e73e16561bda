// mevp_kernels_affine_ns6_fp64.hip -- parallelogram-cell fused kernels, FP64
// at n_s = 6, built with the machine scheduler set to form memory clauses
// (loads issued in groups): measured faster for these kernels only.
#include "mevp_affine.hpp"

namespace mevp {
MEVP_FA_ALL(6, double)
}  // namespace mevp
