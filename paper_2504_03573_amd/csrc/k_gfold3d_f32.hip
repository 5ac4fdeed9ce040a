// Gather-fold hexahedron kernel (float), orders 1..6: one launch per order group.
#include "gfold3d.hpp"

namespace sipdg {

template <class R>
hipError_t launch_gfold3d(int P, int mode, const g3::Args &A, const g3::Data<R> &D, hipStream_t st);
template <class R>
hipError_t launch_gfold3d_persistent(int mode, int grid, const g3::Args &A, const g3::Data<R> &D, hipStream_t st);

namespace {
template <int P>
hipError_t gfold_p(int mode, const g3::Args &A, const g3::Data<float> &D, hipStream_t st) {
    if (A.count <= 0) return hipSuccess;
    const size_t lds = sizeof(float) * g3::lds_total<P>(mode);
    if (mode == 0) hipLaunchKernelGGL((g3::k3g<float, P, 0>), dim3(A.count), dim3(g3::W), lds, st, A, D);
    else if (mode == 1) hipLaunchKernelGGL((g3::k3g<float, P, 1>), dim3(A.count), dim3(g3::W), lds, st, A, D);
    else hipLaunchKernelGGL((g3::k3g<float, P, 2>), dim3(A.count), dim3(g3::W), lds, st, A, D);
    return hipGetLastError();
}
}  // namespace

template <>
hipError_t launch_gfold3d<float>(int P, int mode, const g3::Args &A, const g3::Data<float> &D, hipStream_t st) {
    switch (P) {
    case 1: return gfold_p<1>(mode, A, D, st);
    case 2: return gfold_p<2>(mode, A, D, st);
    case 3: return gfold_p<3>(mode, A, D, st);
    case 4: return gfold_p<4>(mode, A, D, st);
    case 5: return gfold_p<5>(mode, A, D, st);
    case 6: return gfold_p<6>(mode, A, D, st);
    default: return hipErrorInvalidValue;
    }
}

template <>
hipError_t launch_gfold3d_persistent<float>(int mode, int grid, const g3::Args &A, const g3::Data<float> &D,
                                          hipStream_t st) {
    if (A.count <= 0) return hipSuccess;
    if (grid <= 0 || grid > A.count) grid = A.count;
    if (mode == 0) {
        const size_t lds = sizeof(float) * g3::lds_persistent<0>();
        hipLaunchKernelGGL((g3::k3g_persistent<float, 0>), dim3(grid), dim3(g3::W), lds, st, A, D);
    } else {
        const size_t lds = sizeof(float) * g3::lds_persistent<1>();
        hipLaunchKernelGGL((g3::k3g_persistent<float, 1>), dim3(grid), dim3(g3::W), lds, st, A, D);
    }
    return hipGetLastError();
}

}  // namespace sipdg
