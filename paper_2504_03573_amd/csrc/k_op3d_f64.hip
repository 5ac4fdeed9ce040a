// Operator kernels, 3-D hexahedra, FP64.
#include "op_instances.hpp"

namespace sipdg {

template <class R>
hipError_t launch_op_3d(int P, int kind, const OpArgs<R> &A, int nfm, hipStream_t st);

template <>
hipError_t launch_op_3d<double>(int P, int kind, const OpArgs<double> &A, int nfm, hipStream_t st) {
#define CALL(p) op_p<double, 3, p>(kind, A, nfm, st)
    SIPDG_DISPATCH_P(P, CALL)
#undef CALL
}

}  // namespace sipdg
