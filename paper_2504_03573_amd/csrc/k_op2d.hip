// Operator kernels, 2-D quadrilaterals, FP64 and FP32; load vector and
// parameter-gradient kernels (FP64).
#include "op_instances.hpp"

namespace sipdg {

template <class R>
hipError_t launch_op_2d(int P, int kind, const OpArgs<R> &A, int nfm, hipStream_t st) {
#define CALL(p) op_p<R, 2, p>(kind, A, nfm, st)
    SIPDG_DISPATCH_P(P, CALL)
#undef CALL
}
template hipError_t launch_op_2d<double>(int, int, const OpArgs<double> &, int, hipStream_t);
template hipError_t launch_op_2d<float>(int, int, const OpArgs<float> &, int, hipStream_t);

hipError_t launch_load_2d(int P, const OpArgs<double> &A, const int64_t *qoff, const int64_t *boff,
                          const double *src, const double *gdir, hipStream_t st) {
#define CALL(p) load_p<2, p>(A, qoff, boff, src, gdir, st)
    SIPDG_DISPATCH_P(P, CALL)
#undef CALL
}

hipError_t launch_pgrad_2d(int P, const OpArgs<double> &A, const double *a, const double *b,
                           const double *tau0, double *dlam, double *bsig, hipStream_t st) {
#define CALL(p) pgrad_p<2, p>(A, a, b, tau0, dlam, bsig, st)
    SIPDG_DISPATCH_P(P, CALL)
#undef CALL
}

}  // namespace sipdg
