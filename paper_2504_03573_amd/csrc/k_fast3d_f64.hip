// Wavefront-per-element hexahedron kernels (FP64), orders 1..6.
#include "fast3d.hpp"

namespace sipdg {

template <class R>
hipError_t launch_fast3d(int P, int kind, const f3::Args3 &A, const f3::Data3<R> &D, hipStream_t st);

namespace {
template <int P>
hipError_t fast_p(int kind, const f3::Args3 &A, const f3::Data3<double> &D, hipStream_t st) {
    if (A.count <= 0) return hipSuccess;
    size_t lds;
    if (kind == 0) {
        lds = sizeof(double) * f3::Lds<P>::trace_total;
        hipLaunchKernelGGL((f3::k3_trace<double, P>), dim3(A.count), dim3(f3::W), lds, st, A, D);
    } else if (kind == 1) {
        lds = sizeof(double) * f3::Lds<P>::apply_total;
        hipLaunchKernelGGL((f3::k3_apply<double, P, false>), dim3(A.count), dim3(f3::W), lds, st, A, D);
    } else {
        lds = sizeof(double) * f3::Lds<P>::fused_total;
        hipLaunchKernelGGL((f3::k3_apply<double, P, true>), dim3(A.count), dim3(f3::W), lds, st, A, D);
    }
    return hipGetLastError();
}
}  // namespace

template <>
hipError_t launch_fast3d<double>(int P, int kind, const f3::Args3 &A, const f3::Data3<double> &D, hipStream_t st) {
    switch (P) {
    case 1: return fast_p<1>(kind, A, D, st);
    case 2: return fast_p<2>(kind, A, D, st);
    case 3: return fast_p<3>(kind, A, D, st);
    case 4: return fast_p<4>(kind, A, D, st);
    case 5: return fast_p<5>(kind, A, D, st);
    case 6: return fast_p<6>(kind, A, D, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sipdg
