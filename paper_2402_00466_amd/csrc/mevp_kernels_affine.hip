// mevp_kernels_affine.hip -- parallelogram-cell fused kernels, default
// schedule: n_s = 3 and 8, and mixed precision at n_s = 6.
#include "mevp_affine.hpp"

namespace mevp {
MEVP_FA_ALL(3, double)
MEVP_FA_ALL(3, float)
MEVP_FA_ALL(6, float)
MEVP_FA_ALL(8, double)
MEVP_FA_ALL(8, float)
}  // namespace mevp
