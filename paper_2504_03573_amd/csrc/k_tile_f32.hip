// Multi-element gather-fold apply tiles (float).
#include "k_tile.hpp"

namespace sipdg {

template <>
hipError_t launch_gfold3d_tile<float>(int P, int geo, int tile, int budget, const g3::Args &A,
                                      const g3::Data<float> &D, hipStream_t st) {
    return tile_detail::dispatch<float>(P, geo, tile, budget, A, D, st);
}

}  // namespace sipdg
