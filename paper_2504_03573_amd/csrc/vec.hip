// Vector kernels of the Krylov solver.  Every reduction is two-stage with a
// fixed block-to-range assignment and a fixed tree order, so results are
// bitwise reproducible.  Scalars of the recurrences live on the device, one
// per problem, so a CG iteration needs no host round trip.
#include "solver.hpp"

namespace sipdg {

constexpr int VB = 256;   // threads per vector block
// Entries per thread whose loads are issued together, by precision (FP64
// vectors: 8; FP32: 4 in the updates, 1 in the dot product, which measured
// fastest on the 32^3 workload and the 64-problem batch)
template <class R>
struct Ub {
    static constexpr int UPD = sizeof(R) == 8 ? 8 : 4;
    static constexpr int DOT = sizeof(R) == 8 ? 8 : 1;
};

__device__ inline double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = VB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// partial[b] = sum over block b's range of a_i b_i
template <class R>
__global__ __launch_bounds__(VB) void k_dot(VecCtx V, const R *a, const R *b, double *partial) {
    if (V.done && *V.done) return;
    __shared__ double red[VB];
    const int64_t s = V.blk_start[blockIdx.x], e = V.blk_start[blockIdx.x + 1];
    double acc = 0.0;
    // UB entries per thread loaded before they are added (in the same order)
    constexpr int UB = Ub<R>::DOT;
    for (int64_t i0 = s + threadIdx.x; i0 < e; i0 += UB * VB) {
        R av[UB], bv[UB];
#pragma unroll
        for (int j = 0; j < UB; ++j) {
            const int64_t i = i0 + j * VB;
            av[j] = i < e ? a[i] : R(0);
            bv[j] = i < e ? b[i] : R(0);
        }
#pragma unroll
        for (int j = 0; j < UB; ++j)
            if (i0 + j * VB < e) acc += (double)av[j] * (double)bv[j];
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// The deferred x update of the folded CG step: x += alpha p (every block;
// never skipped), then alpha = 0 (k_alpha_zero) so that it is applied once.
template <class R>
__global__ __launch_bounds__(VB) void k_flush(VecCtx V, const CgScalars S, R *x, const R *p) {
    const int prob = V.blk_prob[blockIdx.x];
    const int64_t s = V.blk_start[blockIdx.x], e = V.blk_start[blockIdx.x + 1];
    const double alpha = S.alpha[prob];
    for (int64_t i = s + threadIdx.x; i < e; i += VB) x[i] = (R)((double)x[i] + alpha * (double)p[i]);
}
__global__ void k_alpha_zero(CgScalars S, int nprob) {
    for (int p = threadIdx.x; p < nprob; p += blockDim.x) S.alpha[p] = 0.0;
}

// p = z + beta p; a stopped problem keeps its last direction
template <class R>
__global__ __launch_bounds__(VB) void k_pupdate(VecCtx V, const CgScalars S, const R *z, R *p) {
    if (V.done && *V.done) return;
    const int prob = V.blk_prob[blockIdx.x];
    if (S.conv[prob]) return;
    const int64_t s = V.blk_start[blockIdx.x], e = V.blk_start[blockIdx.x + 1];
    const double beta = S.beta[prob];
    for (int64_t i = s + threadIdx.x; i < e; i += VB) p[i] = (R)((double)z[i] + beta * (double)p[i]);
}

// Sum of part[b0, b1) by the whole block in a fixed order: thread t adds
// b0 + t, b0 + t + VB, ..., then the fixed tree of block_sum.
//
// The partials are loaded 8 per thread at a time before they are added (in
// the same order), so a thread waits on one round of loads per 8 values
// instead of one per value.
constexpr int SEG_BATCH = 8;
__device__ inline double seg_acc(const double *part, int b0, int b1) {
    double acc = 0.0;
    for (int b = b0 + threadIdx.x; b < b1; b += SEG_BATCH * VB) {
        double v[SEG_BATCH];
#pragma unroll
        for (int j = 0; j < SEG_BATCH; ++j) v[j] = b + j * VB < b1 ? part[b + j * VB] : 0.0;
#pragma unroll
        for (int j = 0; j < SEG_BATCH; ++j)
            if (b + j * VB < b1) acc += v[j];
    }
    return acc;
}
__device__ inline double seg_sum(const double *part, int b0, int b1, double *red) {
    return block_sum(seg_acc(part, b0, b1), red);
}
// Two segmented sums over the same range, with the loads of both in flight
// together.
__device__ inline void seg_sum2(const double *pa, const double *pb, int b0, int b1, double *red, double &sa,
                                double &sb) {
    double aa = 0.0, ab = 0.0;
    for (int b = b0 + threadIdx.x; b < b1; b += SEG_BATCH * VB) {
        double va[SEG_BATCH], vb[SEG_BATCH];
#pragma unroll
        for (int j = 0; j < SEG_BATCH; ++j) {
            va[j] = b + j * VB < b1 ? pa[b + j * VB] : 0.0;
            vb[j] = b + j * VB < b1 ? pb[b + j * VB] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < SEG_BATCH; ++j)
            if (b + j * VB < b1) {
                aa += va[j];
                ab += vb[j];
            }
    }
    sa = block_sum(aa, red);
    sb = block_sum(ab, red);
}

// Batch-wide vote of the per-problem blocks of a finalisation launch (thread
// 0 of each block): the block that finishes last gets true and the number of
// active problems, and zeroes both counters for the next launch.
__device__ inline bool last_vote(int *nact, int *nfin, bool active, int &total) {
    if (active) atomicAdd(nact, 1);
    __threadfence();
    if (atomicAdd(nfin, 1) != (int)gridDim.x - 1) return false;
    __threadfence();
    total = atomicExch(nact, 0);
    atomicExch(nfin, 0);
    return true;
}

// alpha = rho / p.q of problem p (0 once converged, and on a breakdown,
// p.q <= 0), from the problem's p.q partials: every block of the problem
// forms the same fixed-order sum, so every block has the same alpha without a
// separate launch; the problem's first block records alpha (for the next trace
// stage and k_flush) and a breakdown.  A breakdown gives alpha = 0 whether or
// not a block already sees the breakdown mark.
__device__ inline double block_alpha(const VecCtx &V, const CgScalars &S, const double *ppq, int p, double *red) {
    const double pq = seg_sum(ppq, V.prob_blk[p], V.prob_blk[p + 1], red);
    const int c = S.conv[p];
    const double alpha = (c || !(pq > 0.0)) ? 0.0 : S.rho[p] / pq;
    if (threadIdx.x == 0 && (int)blockIdx.x == V.prob_blk[p]) {
        S.alpha[p] = alpha;
        if (!c && !(pq > 0.0)) {
            S.conv[p] = 2;   // breakdown
            atomicOr(S.flags, 2);
        }
    }
    return alpha;
}

// alpha from the p.q partials (block_alpha); x += alpha p, r -= alpha q,
// z = dinv r; partials of r.r and r.z
template <class R>
__global__ __launch_bounds__(VB) void k_update(VecCtx V, const CgScalars S, R *x, R *r, const R *p,
                                               const R *q, const R *dinv, R *z, const double *ppq,
                                               double *prr, double *prz) {
    if (V.done && *V.done) return;
    __shared__ double red[VB];
    const int prob = V.blk_prob[blockIdx.x];
    const int64_t s = V.blk_start[blockIdx.x], e = V.blk_start[blockIdx.x + 1];
    const double alpha = block_alpha(V, S, ppq, prob, red);
    double rr = 0.0, rz = 0.0;
    constexpr int UB = Ub<R>::UPD;
    for (int64_t i0 = s + threadIdx.x; i0 < e; i0 += UB * VB) {
        R xv[UB], pv[UB], rv[UB], qv[UB], dv[UB];
#pragma unroll
        for (int j = 0; j < UB; ++j) {
            const int64_t i = i0 + j * VB;
            const bool in = i < e;
            xv[j] = in ? x[i] : R(0);
            pv[j] = in ? p[i] : R(0);
            rv[j] = in ? r[i] : R(0);
            qv[j] = in ? q[i] : R(0);
            dv[j] = in && dinv ? dinv[i] : R(1);
        }
#pragma unroll
        for (int j = 0; j < UB; ++j) {
            const int64_t i = i0 + j * VB;
            if (i < e) {
                const R xi = (R)((double)xv[j] + alpha * (double)pv[j]);
                const R ri = (R)((double)rv[j] - alpha * (double)qv[j]);
                const R zi = dinv ? (R)((double)dv[j] * (double)ri) : ri;
                x[i] = xi;
                r[i] = ri;
                z[i] = zi;
                rr += (double)ri * (double)ri;
                rz += (double)ri * (double)zi;
            }
        }
    }
    rr = block_sum(rr, red);
    rz = block_sum(rz, red);
    if (threadIdx.x == 0) {
        prr[blockIdx.x] = rr;
        prz[blockIdx.x] = rz;
    }
}

// alpha from the p.q partials (block_alpha); r -= alpha q; partials of r.r
// and r.z with z = dinv r (not stored): the update of the folded CG step,
// whose x and p updates happen in the next application's trace stage (or in
// k_flush)
template <class R>
__global__ __launch_bounds__(VB) void k_update_fold(VecCtx V, const CgScalars S, R *r, const R *q, const R *dinv,
                                                    const double *ppq, double *prr, double *prz) {
    if (V.done && *V.done) return;
    __shared__ double red[VB];
    const int prob = V.blk_prob[blockIdx.x];
    const int64_t s = V.blk_start[blockIdx.x], e = V.blk_start[blockIdx.x + 1];
    // the first UB entries per thread are requested before alpha is formed
    constexpr int UB = Ub<R>::UPD;
    int64_t i0 = s + threadIdx.x;
    R rv[UB], qv[UB], dv[UB];
#pragma unroll
    for (int j = 0; j < UB; ++j) {
        const int64_t i = i0 + j * VB;
        const bool in = i < e;
        rv[j] = in ? r[i] : R(0);
        qv[j] = in ? q[i] : R(0);
        dv[j] = in && dinv ? dinv[i] : R(1);
    }
    const double alpha = block_alpha(V, S, ppq, prob, red);
    double rr = 0.0, rz = 0.0;
    for (; i0 < e; i0 += UB * VB) {
#pragma unroll
        for (int j = 0; j < UB; ++j) {
            const int64_t i = i0 + j * VB;
            if (i < e) {
                const R ri = (R)((double)rv[j] - alpha * (double)qv[j]);
                const R zi = dinv ? (R)((double)dv[j] * (double)ri) : ri;
                r[i] = ri;
                rr += (double)ri * (double)ri;
                rz += (double)ri * (double)zi;
            }
        }
        // the next UB entries per thread
#pragma unroll
        for (int j = 0; j < UB; ++j) {
            const int64_t i = i0 + UB * VB + j * VB;
            const bool in = i < e;
            rv[j] = in ? r[i] : R(0);
            qv[j] = in ? q[i] : R(0);
            dv[j] = in && dinv ? dinv[i] : R(1);
        }
    }
    rr = block_sum(rr, red);
    rz = block_sum(rz, red);
    if (threadIdx.x == 0) {
        prr[blockIdx.x] = rr;
        prz[blockIdx.x] = rz;
    }
}

// residual test and beta per problem (one block each); the last block sets
// *done when every problem has stopped.
__global__ __launch_bounds__(VB) void k_fin_beta(VecCtx V, CgScalars S, const double *prr, const double *prz) {
    if (V.done && *V.done) return;
    __shared__ double red[VB];
    const int p = blockIdx.x;
    const bool run = S.conv[p] == 0;   // the same on every thread
    double rr = 0.0, rz = 0.0;
    if (run) {
        seg_sum2(prr, prz, V.prob_blk[p], V.prob_blk[p + 1], red, rr, rz);
    }
    if (threadIdx.x != 0) return;
    bool active = false;
    if (!run) {
        S.beta[p] = 0.0;
    } else {
        S.iters[p] += 1;
        const double rel = sqrt(rr) / S.bnorm[p];
        S.rel[p] = rel;
        if (rel <= S.tol[0] || !(S.bnorm[p] > 0.0)) {
            S.conv[p] = 1;
            S.beta[p] = 0.0;
        } else {
            S.beta[p] = rz / S.rho[p];
            S.rho[p] = rz;
            active = true;
        }
    }
    int total = 0;
    if (last_vote(S.nact, S.nfin, active, total)) {
        S.counter[0] += 1;
        if (total == 0) *V.done = 1;
    }
}

// Start of a (P)CG solve from x = 0 with residual r already set:
// z = dinv r, p = z; partials of r.r and r.z
template <class R>
__global__ __launch_bounds__(VB) void k_start(VecCtx V, const R *r, const R *dinv, R *z, R *p, R *x,
                                              double *prr, double *prz) {
    __shared__ double red[VB];
    const int64_t s = V.blk_start[blockIdx.x], e = V.blk_start[blockIdx.x + 1];
    double rr = 0.0, rz = 0.0;
    for (int64_t i = s + threadIdx.x; i < e; i += VB) {
        const R ri = r[i];
        const R zi = dinv ? (R)((double)dinv[i] * (double)ri) : ri;
        z[i] = zi;
        if (p) p[i] = zi;   // null: keep the search direction (reliable update)
        if (x) x[i] = (R)0;
        rr += (double)ri * (double)ri;
        rz += (double)ri * (double)zi;
    }
    rr = block_sum(rr, red);
    rz = block_sum(rz, red);
    if (threadIdx.x == 0) {
        prr[blockIdx.x] = rr;
        prz[blockIdx.x] = rz;
    }
}

// rho = r.z, bnorm given by bnorm_src (or ||r|| when null), conv = (||r|| <= tol bnorm);
// one block per problem, the last one sets *done and the batch counters.
__global__ __launch_bounds__(VB) void k_fin_start(VecCtx V, CgScalars S, const double *prr, const double *prz,
                                                   const double *bnorm_src, const int *preconv, double tol) {
    __shared__ double red[VB];
    const int p = blockIdx.x;
    double rr, rz;
    seg_sum2(prr, prz, V.prob_blk[p], V.prob_blk[p + 1], red, rr, rz);
    if (threadIdx.x != 0) return;
    const double bn = bnorm_src ? bnorm_src[p] : sqrt(rr);
    S.bnorm[p] = bn;
    S.rho[p] = rz;
    S.alpha[p] = 0.0;
    S.beta[p] = 0.0;
    S.iters[p] = 0;
    S.rel[p] = bn > 0.0 ? sqrt(rr) / bn : 0.0;
    const bool c = (preconv && preconv[p]) || !(bn > 0.0) || sqrt(rr) <= tol * bn;
    S.conv[p] = c ? 1 : 0;
    int total = 0;
    if (last_vote(S.nact, S.nfin, !c, total)) {
        *V.done = total == 0 ? 1 : 0;
        S.counter[0] = 0;
        S.flags[0] = 0;
        S.tol[0] = tol;
    }
}

// Continuation after a reliable update (one block per problem): r was
// replaced by the true residual, renormalised by ratio = ||r_new|| / ||r_old||
// of the unnormalised residuals, and z = M r recomputed; the search direction
// p is kept.  rho' = r.z; beta = (rho' / rho) ratio makes p = z + beta p the
// next conjugate direction in the new normalisation (rho from the last step
// that used p); conv as in k_fin_start.
__global__ __launch_bounds__(VB) void k_fin_cont(VecCtx V, CgScalars S, const double *prr, const double *prz,
                                                  const int *preconv, const double *ratio, double tol) {
    __shared__ double red[VB];
    const int p = blockIdx.x;
    double rr, rz;
    seg_sum2(prr, prz, V.prob_blk[p], V.prob_blk[p + 1], red, rr, rz);
    if (threadIdx.x != 0) return;
    const double bn = sqrt(rr);
    const double rho = S.rho[p];
    const bool c = (preconv && preconv[p]) || !(bn > 0.0) || sqrt(rr) <= tol * bn;
    S.bnorm[p] = bn;
    S.beta[p] = (!c && rho > 0.0) ? (rz / rho) * ratio[p] : 0.0;
    S.rho[p] = rz;
    S.alpha[p] = 0.0;
    S.rel[p] = bn > 0.0 ? 1.0 : 0.0;
    S.conv[p] = c ? 1 : 0;
    int total = 0;
    if (last_vote(S.nact, S.nfin, !c, total)) {
        *V.done = total == 0 ? 1 : 0;
        S.counter[0] = 0;
        S.flags[0] = 0;
        S.tol[0] = tol;
    }
}

// out_p = sqrt(sum of partials) per problem (one block each)
__global__ __launch_bounds__(VB) void k_fin_norm(VecCtx V, const double *part, double *out) {
    __shared__ double red[VB];
    const int p = blockIdx.x;
    const double s = seg_sum(part, V.prob_blk[p], V.prob_blk[p + 1], red);
    if (threadIdx.x == 0) out[p] = sqrt(s);
}

// r = b - q  (FP64) with partials of r.r
__global__ __launch_bounds__(VB) void k_resid(VecCtx V, const double *b, const double *q, double *r,
                                              double *prr) {
    __shared__ double red[VB];
    const int64_t s = V.blk_start[blockIdx.x], e = V.blk_start[blockIdx.x + 1];
    double rr = 0.0;
    for (int64_t i = s + threadIdx.x; i < e; i += VB) {
        const double ri = b[i] - q[i];
        r[i] = ri;
        rr += ri * ri;
    }
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) prr[blockIdx.x] = rr;
}

// r32 = r / ||r||_p   (problems with a zero norm get zero)
__global__ __launch_bounds__(VB) void k_scale32(VecCtx V, const double *r, const double *nrm, float *r32) {
    const int prob = V.blk_prob[blockIdx.x];
    const int64_t s = V.blk_start[blockIdx.x], e = V.blk_start[blockIdx.x + 1];
    const double inv = nrm[prob] > 0.0 ? 1.0 / nrm[prob] : 0.0;
    for (int64_t i = s + threadIdx.x; i < e; i += VB) r32[i] = (float)(r[i] * inv);
}

// x += ||r||_p d32
__global__ __launch_bounds__(VB) void k_correct(VecCtx V, const float *d32, const double *nrm, double *x) {
    const int prob = V.blk_prob[blockIdx.x];
    const int64_t s = V.blk_start[blockIdx.x], e = V.blk_start[blockIdx.x + 1];
    const double sc = nrm[prob];
    for (int64_t i = s + threadIdx.x; i < e; i += VB) x[i] += sc * (double)d32[i];
}

template <class R>
__global__ void k_fill(R *v, int64_t n, R val) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) v[i] = val;
}

// ------------------------------------------------------------------ launchers
#define LCHK() return hipGetLastError()

template <class R>
hipError_t vec_dot(const VecCtx &V, const R *a, const R *b, double *partial, hipStream_t st) {
    if (V.nblk == 0) return hipSuccess;   // no DOFs
    hipLaunchKernelGGL(k_dot<R>, dim3(V.nblk), dim3(VB), 0, st, V, a, b, partial);
    LCHK();
}
template <class R>
hipError_t vec_update(const VecCtx &V, const CgScalars &S, R *x, R *r, const R *p, const R *q,
                      const R *dinv, R *z, const double *ppq, double *prr, double *prz, hipStream_t st) {
    if (V.nblk == 0) return hipSuccess;   // no DOFs
    hipLaunchKernelGGL(k_update<R>, dim3(V.nblk), dim3(VB), 0, st, V, S, x, r, p, q, dinv, z, ppq, prr, prz);
    LCHK();
}
template <class R>
hipError_t vec_update_fold(const VecCtx &V, const CgScalars &S, R *r, const R *q, const R *dinv,
                           const double *ppq, double *prr, double *prz, hipStream_t st) {
    if (V.nblk == 0) return hipSuccess;   // no DOFs
    hipLaunchKernelGGL(k_update_fold<R>, dim3(V.nblk), dim3(VB), 0, st, V, S, r, q, dinv, ppq, prr, prz);
    LCHK();
}
template <class R>
hipError_t vec_flush(const VecCtx &V, const CgScalars &S, R *x, const R *p, hipStream_t st) {
    if (V.nblk > 0) hipLaunchKernelGGL(k_flush<R>, dim3(V.nblk), dim3(VB), 0, st, V, S, x, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_alpha_zero, dim3(1), dim3(64), 0, st, S, V.nprob);
    LCHK();
}
template <class R>
hipError_t vec_pupdate(const VecCtx &V, const CgScalars &S, const R *z, R *p, hipStream_t st) {
    if (V.nblk == 0) return hipSuccess;   // no DOFs
    hipLaunchKernelGGL(k_pupdate<R>, dim3(V.nblk), dim3(VB), 0, st, V, S, z, p);
    LCHK();
}
template <class R>
hipError_t vec_start(const VecCtx &V, const R *r, const R *dinv, R *z, R *p, R *x, double *prr,
                     double *prz, hipStream_t st) {
    if (V.nblk == 0) return hipSuccess;   // no DOFs
    hipLaunchKernelGGL(k_start<R>, dim3(V.nblk), dim3(VB), 0, st, V, r, dinv, z, p, x, prr, prz);
    LCHK();
}
template <class R>
hipError_t vec_fill(R *v, int64_t n, R val, hipStream_t st) {
    int64_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_fill<R>, dim3(g), dim3(256), 0, st, v, n, val);
    LCHK();
}
hipError_t vec_fin_beta(const VecCtx &V, const CgScalars &S, const double *prr, const double *prz, hipStream_t st) {
    hipLaunchKernelGGL(k_fin_beta, dim3(V.nprob), dim3(VB), 0, st, V, S, prr, prz);
    LCHK();
}
hipError_t vec_fin_start(const VecCtx &V, const CgScalars &S, const double *prr, const double *prz,
                         const double *bnorm_src, const int *preconv, double tol, hipStream_t st) {
    hipLaunchKernelGGL(k_fin_start, dim3(V.nprob), dim3(VB), 0, st, V, S, prr, prz, bnorm_src, preconv, tol);
    LCHK();
}
hipError_t vec_fin_cont(const VecCtx &V, const CgScalars &S, const double *prr, const double *prz,
                        const int *preconv, const double *ratio, double tol, hipStream_t st) {
    hipLaunchKernelGGL(k_fin_cont, dim3(V.nprob), dim3(VB), 0, st, V, S, prr, prz, preconv, ratio, tol);
    LCHK();
}
hipError_t vec_fin_norm(const VecCtx &V, const double *part, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_fin_norm, dim3(V.nprob), dim3(VB), 0, st, V, part, out);
    LCHK();
}
hipError_t vec_resid(const VecCtx &V, const double *b, const double *q, double *r, double *prr,
                     hipStream_t st) {
    if (V.nblk == 0) return hipSuccess;   // no DOFs
    hipLaunchKernelGGL(k_resid, dim3(V.nblk), dim3(VB), 0, st, V, b, q, r, prr);
    LCHK();
}
hipError_t vec_scale32(const VecCtx &V, const double *r, const double *nrm, float *r32, hipStream_t st) {
    if (V.nblk == 0) return hipSuccess;   // no DOFs
    hipLaunchKernelGGL(k_scale32, dim3(V.nblk), dim3(VB), 0, st, V, r, nrm, r32);
    LCHK();
}
hipError_t vec_correct(const VecCtx &V, const float *d32, const double *nrm, double *x, hipStream_t st) {
    if (V.nblk == 0) return hipSuccess;   // no DOFs
    hipLaunchKernelGGL(k_correct, dim3(V.nblk), dim3(VB), 0, st, V, d32, nrm, x);
    LCHK();
}

#define INST(R)                                                                                       \
    template hipError_t vec_dot<R>(const VecCtx &, const R *, const R *, double *, hipStream_t);     \
    template hipError_t vec_update<R>(const VecCtx &, const CgScalars &, R *, R *, const R *,         \
                                      const R *, const R *, R *, const double *, double *, double *,  \
                                      hipStream_t);                                                   \
    template hipError_t vec_pupdate<R>(const VecCtx &, const CgScalars &, const R *, R *, hipStream_t); \
    template hipError_t vec_update_fold<R>(const VecCtx &, const CgScalars &, R *, const R *, const R *,        \
                                           const double *, double *, double *, hipStream_t);                    \
    template hipError_t vec_flush<R>(const VecCtx &, const CgScalars &, R *, const R *, hipStream_t);            \
    template hipError_t vec_start<R>(const VecCtx &, const R *, const R *, R *, R *, R *, double *,   \
                                     double *, hipStream_t);                                          \
    template hipError_t vec_fill<R>(R *, int64_t, R, hipStream_t);
INST(double)
INST(float)
template hipError_t vec_fill<int>(int *, int64_t, int, hipStream_t);

}  // namespace sipdg
