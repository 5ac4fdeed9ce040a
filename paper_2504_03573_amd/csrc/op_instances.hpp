// Per-order instantiation and dispatch of the operator kernels for one
// dimension / precision (included by the k_op*.hip translation units, so
// that the instantiations compile in parallel).
#pragma once

#include "aux_kernels.hpp"
#include "launch.hpp"

namespace sipdg {

template <class K>
static inline void ensure_lds(K kernel, size_t lds) {
    if (lds > 65536) (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <class R, int DIM, int P>
static hipError_t op_p(int kind, const OpArgs<R> &A, int nfm, hipStream_t st) {
    using C = Cfg<DIM, P>;
    if (A.count <= 0) return hipSuccess;
    const int blocks = (A.count + C::EPB - 1) / C::EPB;
    const size_t lds = lds_bytes<DIM, P>(A.tsz, kind == OP_APPLY, sizeof(R));
    if (kind == OP_TRACE) {
        ensure_lds(k_trace<R, DIM, P>, lds);
        hipLaunchKernelGGL((k_trace<R, DIM, P>), dim3(blocks), dim3(BLOCK), lds, st, A, nfm);
    } else {
        ensure_lds(k_apply<R, DIM, P>, lds);
        hipLaunchKernelGGL((k_apply<R, DIM, P>), dim3(blocks), dim3(BLOCK), lds, st, A, nfm);
    }
    return hipGetLastError();
}

template <int DIM, int P>
static hipError_t load_p(const OpArgs<double> &A, const int64_t *qoff, const int64_t *boff,
                         const double *src, const double *gdir, hipStream_t st) {
    using C = Cfg<DIM, P>;
    if (A.count <= 0) return hipSuccess;
    const int blocks = (A.count + C::EPB - 1) / C::EPB;
    const size_t lds = lds_bytes<DIM, P>(A.tsz, false, sizeof(double));
    ensure_lds(k_load<DIM, P>, lds);
    hipLaunchKernelGGL((k_load<DIM, P>), dim3(blocks), dim3(BLOCK), lds, st, A, qoff, boff, src, gdir);
    return hipGetLastError();
}

template <int DIM, int P>
static hipError_t pgrad_p(const OpArgs<double> &A, const double *a, const double *b,
                          const double *tau0, double *dlam, double *bsig, hipStream_t st) {
    using C = Cfg<DIM, P>;
    if (A.count <= 0) return hipSuccess;
    const int blocks = (A.count + C::EPB - 1) / C::EPB;
    const size_t lds = lds_bytes<DIM, P>(A.tsz, false, sizeof(double));
    ensure_lds(k_pgrad_elem<DIM, P>, lds);
    hipLaunchKernelGGL((k_pgrad_elem<DIM, P>), dim3(blocks), dim3(BLOCK), lds, st, A, a, b, tau0, dlam, bsig);
    return hipGetLastError();
}

#define SIPDG_DISPATCH_P(P_, CALL) \
    switch (P_) {                  \
    case 1: return CALL(1);        \
    case 2: return CALL(2);        \
    case 3: return CALL(3);        \
    case 4: return CALL(4);        \
    case 5: return CALL(5);        \
    case 6: return CALL(6);        \
    case 7: return CALL(7);        \
    case 8: return CALL(8);        \
    default: return hipErrorInvalidValue; \
    }

}  // namespace sipdg
