// 3-D load vector and parameter-gradient kernels (FP64).
#include "op_instances.hpp"

namespace sipdg {

hipError_t launch_load_3d(int P, const OpArgs<double> &A, const int64_t *qoff, const int64_t *boff,
                          const double *src, const double *gdir, hipStream_t st) {
#define CALL(p) load_p<3, p>(A, qoff, boff, src, gdir, st)
    SIPDG_DISPATCH_P(P, CALL)
#undef CALL
}

hipError_t launch_pgrad_3d(int P, const OpArgs<double> &A, const double *a, const double *b,
                           const double *tau0, double *dlam, double *bsig, hipStream_t st) {
#define CALL(p) pgrad_p<3, p>(A, a, b, tau0, dlam, bsig, st)
    SIPDG_DISPATCH_P(P, CALL)
#undef CALL
}

}  // namespace sipdg
