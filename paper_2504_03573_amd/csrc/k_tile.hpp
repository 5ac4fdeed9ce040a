// Launchers of the multi-element gather-fold apply tiles (one translation
// unit per precision).
#pragma once

#include "gfold_tile.hpp"
#include "tile_shapes.hpp"

namespace sipdg {

// geo: GEO_POINT or GEO_MAP.  Returns hipErrorInvalidValue for a shape the
// library is not built with.
template <class R>
hipError_t launch_gfold3d_tile(int P, int geo, int tile, int budget, const g3::Args &A, const g3::Data<R> &D,
                               hipStream_t st);

namespace tile_detail {

template <class R, int P, int E, int BUD, int GEO>
hipError_t run(const g3::Args &A, const g3::Data<R> &D, hipStream_t st) {
    constexpr int NW = (E * (P + 2) * (P + 2) + 63) / 64;
    using M = g3::MSz<P, E, NW>;
    const int grid = (A.count + E - 1) / E;
    const size_t lds = sizeof(R) * M::TOTAL;
    hipLaunchKernelGGL((g3::k3gm<R, P, E, NW, GEO, BUD>), dim3(grid), dim3(64 * NW), lds, st, A, D);
    return hipGetLastError();
}

template <class R>
hipError_t dispatch(int P, int geo, int tile, int budget, const g3::Args &A, const g3::Data<R> &D,
                    hipStream_t st) {
    if (A.count <= 0) return hipSuccess;
#define SIPDG_TILE_CASE(PP, EE, BB)                                                          \
    if (P == PP && tile == EE && budget == BB) {                                             \
        if (geo == g3::GEO_POINT) return run<R, PP, EE, BB, g3::GEO_POINT>(A, D, st);        \
        if (geo == g3::GEO_MAP) return run<R, PP, EE, BB, g3::GEO_MAP>(A, D, st);            \
        return hipErrorInvalidValue;                                                         \
    }
    SIPDG_TILE_SHAPES(SIPDG_TILE_CASE)
#undef SIPDG_TILE_CASE
    return hipErrorInvalidValue;
}

}  // namespace tile_detail
}  // namespace sipdg
