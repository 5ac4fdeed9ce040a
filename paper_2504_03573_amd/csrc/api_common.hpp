// Helpers shared by the host translation units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "context.hpp"
#include "launch.hpp"

namespace sipdg {

int fail(int code, const std::string &msg);

#define HIPCHK(call)                                                                         \
    do {                                                                                     \
        hipError_t _e = (call);                                                              \
        if (_e != hipSuccess) {                                                              \
            (void)hipGetLastError();                                                         \
            return ::sipdg::fail(SIPDG_EHIP, std::string(#call) + ": " + hipGetErrorString(_e)); \
        }                                                                                    \
    } while (0)

template <class R>
OpArgs<R> make_args(const sipdg_ctx *c, const Group &g, const R *x, R *y, R *tbuf, const int *skip);

// One CG step folded into the apply's trace stage (see g3::Data): x of the
// apply is the search direction p.
template <class R>
struct CgFold {
    R *p, *x;
    const R *r, *dinv;   // dinv null: no preconditioner
    const double *alpha, *beta;
    const int *conv;
};

template <class R>
int apply_impl(sipdg_ctx *c, const R *x, R *y, R *tbuf, const int *skip, hipStream_t st, int stages = 3,
               LaunchRec *rec = nullptr, const CgFold<R> *fold = nullptr);
// Can the handle's current apply take a folded CG step?  (3-D gather-fold
// structure, shared-trace flux, every element in the one trace launch.)
bool fold_ok(const sipdg_ctx *c);

int refresh_diag(sipdg_ctx *c, hipStream_t st);
void free_cg(sipdg_ctx *c);
// CG work vectors (FP64 and FP32) and reduction partials, allocated at create
int alloc_cg(sipdg_ctx *c);
// device pointers of two CG work vectors of n_dofs doubles (autotuner timing)
void cg_scratch(sipdg_ctx *c, double **a, double **b);
// device address of the allocation-free apply's scratch array on `device`
// (the current device), looked up once per device
int noalloc_setup(int device);

}  // namespace sipdg
