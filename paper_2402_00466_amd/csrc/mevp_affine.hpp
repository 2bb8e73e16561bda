// mevp_affine.hpp -- definition of fused_affine (declared in mevp_internal.hpp)
// for the translation units that instantiate it: the fused subcycle kernels of
// parallelogram cells (one, two and three subcycles per launch, and the
// persistent form). Two units, so that each can be scheduled as measured best.
#pragma once
#include "mevp_device.hpp"

namespace mevp {

template <int NS, int NA, class T, int EX, int EY>
hipError_t fused_affine(const DevArrays &d, const KParams &p, const Tile *tiles, int ntiles,
                        const FusedArgs &f, hipStream_t s) {
  return fused_one<NS, NA, T, kGeoAffine, EX, EY>(d, p, tiles, ntiles, f, s);
}

static_assert(kNumTileShapes == 4 && kTileShapes[0][0] == 17 && kTileShapes[0][1] == 15 &&
                  kTileShapes[1][0] == 17 && kTileShapes[1][1] == 17 && kTileShapes[2][0] == 33 &&
                  kTileShapes[2][1] == 16 && kTileShapes[3][0] == 14 && kTileShapes[3][1] == 14,
              "the instantiations follow kTileShapes");

}  // namespace mevp

// one instantiation; fused_t dispatches to tile shape 0 for every n_a and to
// shapes 1 to 3 for n_a = 1
#define MEVP_FA(NS_, NA_, T_, EX_, EY_)                                                   \
  template hipError_t fused_affine<NS_, NA_, T_, EX_, EY_>(const DevArrays &, const KParams &, \
                                                           const Tile *, int,               \
                                                           const FusedArgs &, hipStream_t);
// every n_a and tile shape of one n_s and precision
#define MEVP_FA_ALL(NS_, T_)                                                              \
  MEVP_FA(NS_, 1, T_, 17, 15) MEVP_FA(NS_, 3, T_, 17, 15) MEVP_FA(NS_, 6, T_, 17, 15)     \
  MEVP_FA(NS_, 1, T_, 17, 17) MEVP_FA(NS_, 1, T_, 33, 16) MEVP_FA(NS_, 1, T_, 14, 14)
