// Krylov solver internals: device-side per-problem scalars and the vector
// kernels' launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sipdg {

// Block decomposition of a (batched) vector: block b covers
// [blk_start[b], blk_start[b+1]) inside problem blk_prob[b]; problem p owns
// blocks [prob_blk[p], prob_blk[p+1]).
struct VecCtx {
    int nblk;
    int nprob;
    const int64_t *blk_start;
    const int *blk_prob;
    const int *prob_blk;
    int *done;   // set once every problem has stopped; kernels then return at once
};

// Per-problem recurrence scalars (device arrays of length nprob).
struct CgScalars {
    double *rho, *alpha, *beta, *bnorm, *rel;
    int *conv;      // 0 running, 1 converged, 2 breakdown
    int *iters;     // iterations per problem
    int *counter;   // [1] iterations executed by the whole batch
    int *flags;     // [1] bit 1: breakdown seen
    double *tol;    // [1] relative tolerance of the running solve (set by the start kernel)
    int *nact, *nfin;   // [1] each: vote counters of the finalisation launches (zero between launches)
};

template <class R>
hipError_t vec_dot(const VecCtx &V, const R *a, const R *b, double *partial, hipStream_t st);
// alpha of each problem from the p.q partials ppq (every block forms the same
// fixed-order sum; the problem's first block records it), then x += alpha p,
// r -= alpha q, z = M r with the partials of r.r and r.z.  ppq must not alias
// prr or prz (blocks read ppq while others write their r.r partials).
template <class R>
hipError_t vec_update(const VecCtx &V, const CgScalars &S, R *x, R *r, const R *p, const R *q,
                      const R *dinv, R *z, const double *ppq, double *prr, double *prz, hipStream_t st);
template <class R>
hipError_t vec_pupdate(const VecCtx &V, const CgScalars &S, const R *z, R *p, hipStream_t st);
// folded CG step (x and p updated in the next application's trace stage):
// alpha as in vec_update, r -= alpha q with the partials of r.r and r.z, and
// the deferred x update
template <class R>
hipError_t vec_update_fold(const VecCtx &V, const CgScalars &S, R *r, const R *q, const R *dinv,
                           const double *ppq, double *prr, double *prz, hipStream_t st);
template <class R>
hipError_t vec_flush(const VecCtx &V, const CgScalars &S, R *x, const R *p, hipStream_t st);
template <class R>
hipError_t vec_start(const VecCtx &V, const R *r, const R *dinv, R *z, R *p, R *x, double *prr,
                     double *prz, hipStream_t st);
template <class R>
hipError_t vec_fill(R *v, int64_t n, R val, hipStream_t st);
hipError_t vec_fin_beta(const VecCtx &V, const CgScalars &S, const double *prr, const double *prz,
                        hipStream_t st);
hipError_t vec_fin_start(const VecCtx &V, const CgScalars &S, const double *prr, const double *prz,
                         const double *bnorm_src, const int *preconv, double tol, hipStream_t st);
hipError_t vec_fin_cont(const VecCtx &V, const CgScalars &S, const double *prr, const double *prz,
                        const int *preconv, const double *ratio, double tol, hipStream_t st);
hipError_t vec_fin_norm(const VecCtx &V, const double *part, double *out, hipStream_t st);
hipError_t vec_resid(const VecCtx &V, const double *b, const double *q, double *r, double *prr,
                     hipStream_t st);
hipError_t vec_scale32(const VecCtx &V, const double *r, const double *nrm, float *r32, hipStream_t st);
hipError_t vec_correct(const VecCtx &V, const float *d32, const double *nrm, double *x, hipStream_t st);

}  // namespace sipdg
