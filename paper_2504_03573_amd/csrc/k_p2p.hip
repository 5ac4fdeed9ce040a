// Point-to-point interpolation flux kernels (hexahedra), FP64 and FP32, orders 1..8.
#include "op_instances.hpp"
#include "p2p3d.hpp"

namespace sipdg {

template <class R>
hipError_t launch_p2p(int P, int stage, const OpArgs<R> &A, int nfm, hipStream_t st);

namespace {
template <class R, int P>
hipError_t p2p_p(int stage, const OpArgs<R> &A, int nfm, hipStream_t st) {
    using C = Cfg<3, P>;
    if (A.count <= 0) return hipSuccess;
    const int blocks = (A.count + C::EPB - 1) / C::EPB;
    const size_t lds = lds_bytes<3, P>(A.tsz, stage == 2, sizeof(R));
    if (stage == 1) {
        ensure_lds(k_p2p_trace<R, P>, lds);
        hipLaunchKernelGGL((k_p2p_trace<R, P>), dim3(blocks), dim3(BLOCK), lds, st, A);
    } else {
        ensure_lds(k_p2p_apply<R, P>, lds);
        hipLaunchKernelGGL((k_p2p_apply<R, P>), dim3(blocks), dim3(BLOCK), lds, st, A, nfm);
    }
    return hipGetLastError();
}

}  // namespace

template <>
hipError_t launch_p2p<double>(int P, int stage, const OpArgs<double> &A, int nfm, hipStream_t st) {
#define CALL(p) p2p_p<double, p>(stage, A, nfm, st)
    SIPDG_DISPATCH_P(P, CALL)
#undef CALL
}

template <>
hipError_t launch_p2p<float>(int P, int stage, const OpArgs<float> &A, int nfm, hipStream_t st) {
#define CALL(p) p2p_p<float, p>(stage, A, nfm, st)
    SIPDG_DISPATCH_P(P, CALL)
#undef CALL
}

hipError_t launch_p2p_factors(int64_t nfaces, const FaceTopo *faces, const int *order, const int64_t *side,
                              const double *emap, const double *tab, double *fg, hipStream_t st) {
    if (nfaces <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_p2p_factors, dim3((unsigned)nfaces, 2), dim3(BLOCK), 0, st, faces, order, side, emap, tab, fg);
    return hipGetLastError();
}

}  // namespace sipdg
