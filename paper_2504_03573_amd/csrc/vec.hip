// Vector kernels of the Krylov solver.  Every reduction is two-stage with a
// fixed block-to-range assignment and a fixed tree order, so results are
// bitwise reproducible.  Scalars of the recurrences live on the device, one
// per problem, so a CG iteration needs no host round trip.
#include "solver.hpp"

namespace sipdg {

constexpr int VB = 256;   // threads per vector block

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
    for (int64_t i = s + threadIdx.x; i < e; i += VB) acc += (double)a[i] * (double)b[i];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// x += alpha p, r -= alpha q, z = dinv r; partials of r.r and r.z
template <class R>
__global__ __launch_bounds__(VB) void k_update(VecCtx V, const CgScalars S, R *x, R *r, const R *p,
                                               const R *q, const R *dinv, R *z, double *prr,
                                               double *prz) {
    if (V.done && *V.done) return;
    __shared__ double red[VB];
    const int prob = V.blk_prob[blockIdx.x];
    const int64_t s = V.blk_start[blockIdx.x], e = V.blk_start[blockIdx.x + 1];
    const double alpha = S.alpha[prob];
    double rr = 0.0, rz = 0.0;
    for (int64_t i = s + threadIdx.x; i < e; i += VB) {
        const R xi = (R)((double)x[i] + alpha * (double)p[i]);
        const R ri = (R)((double)r[i] - alpha * (double)q[i]);
        const R zi = dinv ? (R)((double)dinv[i] * (double)ri) : ri;
        x[i] = xi;
        r[i] = ri;
        z[i] = zi;
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

// p = z + beta p
template <class R>
__global__ __launch_bounds__(VB) void k_pupdate(VecCtx V, const CgScalars S, const R *z, R *p) {
    if (V.done && *V.done) return;
    const int prob = V.blk_prob[blockIdx.x];
    const int64_t s = V.blk_start[blockIdx.x], e = V.blk_start[blockIdx.x + 1];
    const double beta = S.beta[prob];
    for (int64_t i = s + threadIdx.x; i < e; i += VB) p[i] = (R)((double)z[i] + beta * (double)p[i]);
}

// alpha = rho / p.q per problem (0 once converged); breakdown if p.q <= 0.
__global__ void k_fin_alpha(VecCtx V, CgScalars S, const double *ppq) {
    if (V.done && *V.done) return;
    for (int p = threadIdx.x; p < V.nprob; p += blockDim.x) {
        double pq = 0.0;
        for (int b = V.prob_blk[p]; b < V.prob_blk[p + 1]; ++b) pq += ppq[b];
        if (S.conv[p]) {
            S.alpha[p] = 0.0;
        } else if (!(pq > 0.0)) {
            S.alpha[p] = 0.0;
            S.conv[p] = 2;   // breakdown
            atomicOr(S.flags, 2);
        } else {
            S.alpha[p] = S.rho[p] / pq;
        }
    }
}

// residual test and beta per problem; sets *done when every problem stopped.
__global__ void k_fin_beta(VecCtx V, CgScalars S, const double *prr, const double *prz) {
    if (V.done && *V.done) return;
    const double tol = S.tol[0];
    __shared__ int active;
    if (threadIdx.x == 0) active = 0;
    __syncthreads();
    for (int p = threadIdx.x; p < V.nprob; p += blockDim.x) {
        if (S.conv[p]) {
            S.beta[p] = 0.0;
            continue;
        }
        double rr = 0.0, rz = 0.0;
        for (int b = V.prob_blk[p]; b < V.prob_blk[p + 1]; ++b) {
            rr += prr[b];
            rz += prz[b];
        }
        S.iters[p] += 1;
        const double rel = sqrt(rr) / S.bnorm[p];
        S.rel[p] = rel;
        if (rel <= tol || !(S.bnorm[p] > 0.0)) {
            S.conv[p] = 1;
            S.beta[p] = 0.0;
        } else {
            S.beta[p] = rz / S.rho[p];
            S.rho[p] = rz;
            atomicAdd(&active, 1);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        S.counter[0] += 1;
        if (active == 0) *V.done = 1;
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
        p[i] = zi;
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

// rho = r.z, bnorm given by bnorm_src (or ||r|| when null), conv = (||r|| <= tol bnorm)
__global__ void k_fin_start(VecCtx V, CgScalars S, const double *prr, const double *prz,
                            const double *bnorm_src, const int *preconv, double tol) {
    __shared__ int active;
    if (threadIdx.x == 0) active = 0;
    __syncthreads();
    for (int p = threadIdx.x; p < V.nprob; p += blockDim.x) {
        double rr = 0.0, rz = 0.0;
        for (int b = V.prob_blk[p]; b < V.prob_blk[p + 1]; ++b) {
            rr += prr[b];
            rz += prz[b];
        }
        const double bn = bnorm_src ? bnorm_src[p] : sqrt(rr);
        S.bnorm[p] = bn;
        S.rho[p] = rz;
        S.alpha[p] = 0.0;
        S.beta[p] = 0.0;
        S.iters[p] = 0;
        S.rel[p] = bn > 0.0 ? sqrt(rr) / bn : 0.0;
        const bool c = (preconv && preconv[p]) || !(bn > 0.0) || sqrt(rr) <= tol * bn;
        S.conv[p] = c ? 1 : 0;
        if (!c) atomicAdd(&active, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        *V.done = active == 0 ? 1 : 0;
        S.counter[0] = 0;
        S.flags[0] = 0;
        S.tol[0] = tol;
    }
}

// out_p = sqrt(sum of partials) per problem
__global__ void k_fin_norm(VecCtx V, const double *part, double *out) {
    for (int p = threadIdx.x; p < V.nprob; p += blockDim.x) {
        double s = 0.0;
        for (int b = V.prob_blk[p]; b < V.prob_blk[p + 1]; ++b) s += part[b];
        out[p] = sqrt(s);
    }
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
    hipLaunchKernelGGL(k_dot<R>, dim3(V.nblk), dim3(VB), 0, st, V, a, b, partial);
    LCHK();
}
template <class R>
hipError_t vec_update(const VecCtx &V, const CgScalars &S, R *x, R *r, const R *p, const R *q,
                      const R *dinv, R *z, double *prr, double *prz, hipStream_t st) {
    hipLaunchKernelGGL(k_update<R>, dim3(V.nblk), dim3(VB), 0, st, V, S, x, r, p, q, dinv, z, prr, prz);
    LCHK();
}
template <class R>
hipError_t vec_pupdate(const VecCtx &V, const CgScalars &S, const R *z, R *p, hipStream_t st) {
    hipLaunchKernelGGL(k_pupdate<R>, dim3(V.nblk), dim3(VB), 0, st, V, S, z, p);
    LCHK();
}
template <class R>
hipError_t vec_start(const VecCtx &V, const R *r, const R *dinv, R *z, R *p, R *x, double *prr,
                     double *prz, hipStream_t st) {
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
hipError_t vec_fin_alpha(const VecCtx &V, const CgScalars &S, const double *ppq, hipStream_t st) {
    hipLaunchKernelGGL(k_fin_alpha, dim3(1), dim3(64), 0, st, V, S, ppq);
    LCHK();
}
hipError_t vec_fin_beta(const VecCtx &V, const CgScalars &S, const double *prr, const double *prz, hipStream_t st) {
    hipLaunchKernelGGL(k_fin_beta, dim3(1), dim3(64), 0, st, V, S, prr, prz);
    LCHK();
}
hipError_t vec_fin_start(const VecCtx &V, const CgScalars &S, const double *prr, const double *prz,
                         const double *bnorm_src, const int *preconv, double tol, hipStream_t st) {
    hipLaunchKernelGGL(k_fin_start, dim3(1), dim3(64), 0, st, V, S, prr, prz, bnorm_src, preconv, tol);
    LCHK();
}
hipError_t vec_fin_norm(const VecCtx &V, const double *part, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_fin_norm, dim3(1), dim3(64), 0, st, V, part, out);
    LCHK();
}
hipError_t vec_resid(const VecCtx &V, const double *b, const double *q, double *r, double *prr,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_resid, dim3(V.nblk), dim3(VB), 0, st, V, b, q, r, prr);
    LCHK();
}
hipError_t vec_scale32(const VecCtx &V, const double *r, const double *nrm, float *r32, hipStream_t st) {
    hipLaunchKernelGGL(k_scale32, dim3(V.nblk), dim3(VB), 0, st, V, r, nrm, r32);
    LCHK();
}
hipError_t vec_correct(const VecCtx &V, const float *d32, const double *nrm, double *x, hipStream_t st) {
    hipLaunchKernelGGL(k_correct, dim3(V.nblk), dim3(VB), 0, st, V, d32, nrm, x);
    LCHK();
}

#define INST(R)                                                                                       \
    template hipError_t vec_dot<R>(const VecCtx &, const R *, const R *, double *, hipStream_t);     \
    template hipError_t vec_update<R>(const VecCtx &, const CgScalars &, R *, R *, const R *,         \
                                      const R *, const R *, R *, double *, double *, hipStream_t);    \
    template hipError_t vec_pupdate<R>(const VecCtx &, const CgScalars &, const R *, R *, hipStream_t); \
    template hipError_t vec_start<R>(const VecCtx &, const R *, const R *, R *, R *, R *, double *,   \
                                     double *, hipStream_t);                                          \
    template hipError_t vec_fill<R>(R *, int64_t, R, hipStream_t);
INST(double)
INST(float)
template hipError_t vec_fill<int>(int *, int64_t, int, hipStream_t);

}  // namespace sipdg
