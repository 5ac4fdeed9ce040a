// Gather-fold hexahedron kernel (double), orders 1..8: one launch per order group.
#include "gfold3d.hpp"

namespace sipdg {

template <class R>
hipError_t launch_gfold3d(int P, int mode, int nfmax, const g3::Args &A, const g3::Data<R> &D, hipStream_t st);
template <class R>
hipError_t launch_gfold3d_persistent(int mode, int grid, const g3::Args &A, const g3::Data<R> &D, hipStream_t st);
template <class R>
hipError_t launch_gfold3d_trace_all(const g3::Args &A, const g3::Data<R> &D, hipStream_t st);

namespace {
template <int P>
hipError_t gfold_p(int mode, int nfmax, const g3::Args &A, const g3::Data<double> &D, hipStream_t st) {
    // the lane grid covers traces up to NFMAX x NFMAX points
    if (nfmax > g3::Geo<P>::NFMAX) return hipErrorInvalidValue;
    if (A.count <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * g3::lds_mode<P>(mode >= 5 ? 3 : (mode >= 3 ? 1 : mode));
    const dim3 blk(g3::Geo<P>::W);
    if (mode == 0 && A.side && A.basis) hipLaunchKernelGGL((g3::k3t<double, P, 1, true>), dim3(A.count), blk, lds, st, A, D);
    else if (mode == 0 && A.side) hipLaunchKernelGGL((g3::k3t<double, P, 0, true>), dim3(A.count), blk, lds, st, A, D);
    else if (mode == 0 && A.basis) hipLaunchKernelGGL((g3::k3t<double, P, 1>), dim3(A.count), blk, lds, st, A, D);
    else if (mode == 0) hipLaunchKernelGGL((g3::k3t<double, P>), dim3(A.count), blk, lds, st, A, D);
    else if (mode == 1) hipLaunchKernelGGL((g3::k3g<double, P, 1>), dim3(A.count), blk, lds, st, A, D);
    else if (mode == 3) hipLaunchKernelGGL((g3::k3g<double, P, 1, g3::GEO_AFFINE>), dim3(A.count), blk, lds, st, A, D);
    else if (mode == 4) hipLaunchKernelGGL((g3::k3g<double, P, 1, g3::GEO_MAP>), dim3(A.count), blk, lds, st, A, D);
    // Gauss volume points: map geometry (5) or affine constants (6)
    else if (mode == 5) hipLaunchKernelGGL((g3::k3g<double, P, 3, g3::GEO_MAP>), dim3(A.count), blk, lds, st, A, D);
    else if (mode == 6) hipLaunchKernelGGL((g3::k3g<double, P, 3, g3::GEO_AFFINE>), dim3(A.count), blk, lds, st, A, D);
    else if (A.basis) return hipErrorInvalidValue;   // the fused kernel: Legendre endpoint values
    else if constexpr (P <= 6) hipLaunchKernelGGL((g3::k3g<double, P, 2>), dim3(A.count), blk, lds, st, A, D);
    else return hipErrorInvalidValue;   // the fused kernel covers orders <= 6
    return hipGetLastError();
}
}  // namespace

template <>
hipError_t launch_gfold3d<double>(int P, int mode, int nfmax, const g3::Args &A, const g3::Data<double> &D, hipStream_t st) {
    switch (P) {
    case 1: return gfold_p<1>(mode, nfmax, A, D, st);
    case 2: return gfold_p<2>(mode, nfmax, A, D, st);
    case 3: return gfold_p<3>(mode, nfmax, A, D, st);
    case 4: return gfold_p<4>(mode, nfmax, A, D, st);
    case 5: return gfold_p<5>(mode, nfmax, A, D, st);
    case 6: return gfold_p<6>(mode, nfmax, A, D, st);
    case 7: return gfold_p<7>(mode, nfmax, A, D, st);
    case 8: return gfold_p<8>(mode, nfmax, A, D, st);
    default: return hipErrorInvalidValue;
    }
}

template <>
hipError_t launch_gfold3d_persistent<double>(int mode, int grid, const g3::Args &A, const g3::Data<double> &D,
                                          hipStream_t st) {
    if (A.basis) return hipErrorInvalidValue;   // Legendre endpoint values in closed form
    if (A.count <= 0) return hipSuccess;
    if (grid <= 0 || grid > A.count) grid = A.count;
    if (mode == 0) {
        const size_t lds = sizeof(double) * g3::lds_persistent<0>();
        hipLaunchKernelGGL((g3::k3g_persistent<double, 0>), dim3(grid), dim3(g3::W), lds, st, A, D);
    } else {
        const size_t lds = sizeof(double) * g3::lds_persistent<1>();
        hipLaunchKernelGGL((g3::k3g_persistent<double, 1>), dim3(grid), dim3(g3::W), lds, st, A, D);
    }
    return hipGetLastError();
}

template <>
hipError_t launch_gfold3d_trace_all<double>(const g3::Args &A, const g3::Data<double> &D, hipStream_t st) {
    if (A.count <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * g3::lds_trace_all();
    if (A.side && A.basis) hipLaunchKernelGGL((g3::k3t_all<double, 1, true>), dim3(A.count), dim3(g3::W), lds, st, A, D);
    else if (A.side) hipLaunchKernelGGL((g3::k3t_all<double, 0, true>), dim3(A.count), dim3(g3::W), lds, st, A, D);
    else if (D.fold_p && A.basis) hipLaunchKernelGGL((g3::k3t_all<double, 1, false, true>), dim3(A.count), dim3(g3::W), lds, st, A, D);
    else if (D.fold_p) hipLaunchKernelGGL((g3::k3t_all<double, 0, false, true>), dim3(A.count), dim3(g3::W), lds, st, A, D);
    else if (A.basis) hipLaunchKernelGGL((g3::k3t_all<double, 1>), dim3(A.count), dim3(g3::W), lds, st, A, D);
    else hipLaunchKernelGGL((g3::k3t_all<double>), dim3(A.count), dim3(g3::W), lds, st, A, D);
    return hipGetLastError();
}

}  // namespace sipdg
