// Restarted GMRES for the operator of a handle (either interface flux; the
// point-to-point flux is nonsymmetric, which is why the paper solves those
// systems with GMRES, Table 2).  Right Jacobi preconditioning with the
// shared-trace diagonal, Arnoldi by classical Gram-Schmidt applied twice
// (one batched dot launch and one batched update launch per pass), Givens
// rotations on the host.  Reductions are two-stage with fixed chunks and a
// fixed tree order, so a solve is bitwise reproducible.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "api_common.hpp"
#include "sipdg.h"

namespace sipdg {

namespace {

constexpr int GB = 256;          // threads per block
constexpr int64_t GCH = 8192;    // vector entries per reduction chunk

__device__ inline double gm_block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = GB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

// partial[j][b] = sum over chunk b of V_j . w, j < k (grid: chunks x k)
__global__ __launch_bounds__(GB) void k_gm_mdot(const double *V, int64_t ldv, const double *w, int64_t n,
                                                double *partial, int nblk) {
    __shared__ double red[GB];
    const int b = blockIdx.x, j = blockIdx.y;
    const int64_t s = (int64_t)b * GCH, e = std::min(n, s + GCH);
    const double *v = V + (int64_t)j * ldv;
    double acc = 0.0;
    for (int64_t i = s + threadIdx.x; i < e; i += GB) acc += v[i] * w[i];
    acc = gm_block_sum(acc, red);
    if (threadIdx.x == 0) partial[(int64_t)j * nblk + b] = acc;
}

// out[j] = sum_b partial[j][b] in a fixed order (one block per j)
__global__ __launch_bounds__(GB) void k_gm_sum(const double *partial, int nblk, double *out) {
    __shared__ double red[GB];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += GB) acc += partial[(int64_t)j * nblk + b];
    acc = gm_block_sum(acc, red);
    if (threadIdx.x == 0) out[j] = acc;
}

// w -= sum_{j<k} h[j] V_j
__global__ __launch_bounds__(GB) void k_gm_maxpy(double *w, const double *V, int64_t ldv, int k, const double *h,
                                                 int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * GB + threadIdx.x; i < n; i += (int64_t)gridDim.x * GB) {
        double acc = w[i];
        for (int j = 0; j < k; ++j) acc -= h[j] * V[(int64_t)j * ldv + i];
        w[i] = acc;
    }
}

// v = s w
__global__ __launch_bounds__(GB) void k_gm_scale(double *v, const double *w, double s, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * GB + threadIdx.x; i < n; i += (int64_t)gridDim.x * GB) v[i] = s * w[i];
}

// z = dinv .* v (dinv null: copy)
__global__ __launch_bounds__(GB) void k_gm_prec(double *z, const double *v, const double *dinv, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * GB + threadIdx.x; i < n; i += (int64_t)gridDim.x * GB)
        z[i] = dinv ? dinv[i] * v[i] : v[i];
}

// r = b - q
__global__ __launch_bounds__(GB) void k_gm_sub(double *r, const double *b, const double *q, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * GB + threadIdx.x; i < n; i += (int64_t)gridDim.x * GB) r[i] = b[i] - q[i];
}

// x += dinv .* (sum_{j<k} y[j] V_j)
__global__ __launch_bounds__(GB) void k_gm_update(double *x, const double *V, int64_t ldv, int k, const double *y,
                                                  const double *dinv, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * GB + threadIdx.x; i < n; i += (int64_t)gridDim.x * GB) {
        double acc = 0.0;
        for (int j = 0; j < k; ++j) acc += y[j] * V[(int64_t)j * ldv + i];
        x[i] += dinv ? dinv[i] * acc : acc;
    }
}

struct GmWork {
    double *V = nullptr, *w = nullptr, *z = nullptr, *part = nullptr, *dh = nullptr;
    ~GmWork() {
        for (double *p : {V, w, z, part, dh})
            if (p) (void)hipFree(p);
    }
};

}  // namespace

}  // namespace sipdg

using namespace sipdg;

void sipdg_gmres_default_opts(sipdg_gmres_opts *o) {
    if (!o) return;
    o->tol = 1e-10;
    o->restart = 30;
    o->maxit = 100000;
    o->precond = 1;
}

int sipdg_gmres_solve(sipdg_handle h, const double *b, double *x, const sipdg_gmres_opts *opts,
                      sipdg_gmres_info *info, void *stream) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    sipdg_gmres_opts o;
    if (opts) o = *opts;
    else sipdg_gmres_default_opts(&o);
    if (!(o.tol > 0.0) || o.maxit <= 0 || o.restart < 1 || o.restart > 1000)
        return fail(SIPDG_EINVAL, "invalid GMRES options (tol > 0, maxit > 0, 1 <= restart <= 1000)");
    const auto t0 = std::chrono::steady_clock::now();
    sipdg_gmres_info inf{};
    const int64_t n = h->ndof;
    if (n == 0) {
        inf.converged = 1;
        if (info) *info = inf;
        return SIPDG_OK;
    }
    if (!b || !x) return fail(SIPDG_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream;
    const int m = o.restart;
    const int nblk = (int)((n + GCH - 1) / GCH);
    const int grid = (int)std::min<int64_t>((n + GB - 1) / GB, 4096);
    const double *dinv = o.precond ? h->d_dinv64 : nullptr;
    GmWork W;
    HIPCHK(hipMalloc((void **)&W.V, sizeof(double) * n * (m + 1)));
    HIPCHK(hipMalloc((void **)&W.w, sizeof(double) * n));
    HIPCHK(hipMalloc((void **)&W.z, sizeof(double) * n));
    HIPCHK(hipMalloc((void **)&W.part, sizeof(double) * (int64_t)nblk * (m + 1)));
    HIPCHK(hipMalloc((void **)&W.dh, sizeof(double) * (m + 2)));
    // dot products of V_0..V_{k-1} with w, to the host
    auto mdot = [&](const double *Vb, int k, const double *w, double *out) -> int {
        hipLaunchKernelGGL(k_gm_mdot, dim3(nblk, k), dim3(GB), 0, st, Vb, n, w, n, W.part, nblk);
        hipLaunchKernelGGL(k_gm_sum, dim3(k), dim3(GB), 0, st, W.part, nblk, W.dh);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(out, W.dh, sizeof(double) * k, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return SIPDG_OK;
    };
    double bn2 = 0.0;
    int rc = mdot(b, 1, b, &bn2);
    if (rc) return rc;
    const double bnorm = std::sqrt(bn2);
    HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * n, st));
    if (bnorm == 0.0) {
        inf.converged = 1;
        HIPCHK(hipStreamSynchronize(st));
        if (info) *info = inf;
        return SIPDG_OK;
    }
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), h1(m + 1), h2(m + 1);
    int total = 0;
    double rel = 1.0;
    for (;;) {
        // r = b - A x into V_0
        rc = apply_impl<double>(h, x, W.w, h->d_tbuf, nullptr, st);
        if (rc) return rc;
        hipLaunchKernelGGL(k_gm_sub, dim3(grid), dim3(GB), 0, st, W.V, b, W.w, n);
        double r2 = 0.0;
        rc = mdot(W.V, 1, W.V, &r2);
        if (rc) return rc;
        const double beta = std::sqrt(r2);
        rel = beta / bnorm;
        if (rel <= o.tol || total >= o.maxit) break;
        hipLaunchKernelGGL(k_gm_scale, dim3(grid), dim3(GB), 0, st, W.V, W.V, 1.0 / beta, n);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int kend = 0;
        for (int j = 0; j < m && total < o.maxit; ++j) {
            double *vj = W.V + (int64_t)j * n, *vn = W.V + (int64_t)(j + 1) * n;
            hipLaunchKernelGGL(k_gm_prec, dim3(grid), dim3(GB), 0, st, W.z, vj, dinv, n);
            rc = apply_impl<double>(h, W.z, W.w, h->d_tbuf, nullptr, st);
            if (rc) return rc;
            // classical Gram-Schmidt, twice
            for (int pass = 0; pass < 2; ++pass) {
                double *hp = pass == 0 ? h1.data() : h2.data();
                rc = mdot(W.V, j + 1, W.w, hp);
                if (rc) return rc;
                HIPCHK(hipMemcpyAsync(W.dh, hp, sizeof(double) * (j + 1), hipMemcpyHostToDevice, st));
                hipLaunchKernelGGL(k_gm_maxpy, dim3(grid), dim3(GB), 0, st, W.w, W.V, n, j + 1, W.dh, n);
            }
            double w2 = 0.0;
            rc = mdot(W.w, 1, W.w, &w2);
            if (rc) return rc;
            const double hn = std::sqrt(w2);
            double *col = &H[(size_t)j * (m + 1)];
            for (int i = 0; i <= j; ++i) col[i] = h1[i] + h2[i];
            col[j + 1] = hn;
            for (int i = 0; i < j; ++i) {   // earlier rotations
                const double t = cs[i] * col[i] + sn[i] * col[i + 1];
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
                col[i] = t;
            }
            const double den = std::hypot(col[j], col[j + 1]);
            cs[j] = den > 0.0 ? col[j] / den : 1.0;
            sn[j] = den > 0.0 ? col[j + 1] / den : 0.0;
            col[j] = den;
            col[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++total;
            kend = j + 1;
            if (hn > 0.0) hipLaunchKernelGGL(k_gm_scale, dim3(grid), dim3(GB), 0, st, vn, W.w, 1.0 / hn, n);
            if (std::fabs(g[j + 1]) / bnorm <= o.tol || hn == 0.0) break;
        }
        // y = R^{-1} g, x += M^{-1} V y
        for (int i = kend - 1; i >= 0; --i) {
            double s = g[i];
            for (int l = i + 1; l < kend; ++l) s -= H[(size_t)l * (m + 1) + i] * y[l];
            y[i] = s / H[(size_t)i * (m + 1) + i];
        }
        HIPCHK(hipMemcpyAsync(W.dh, y.data(), sizeof(double) * kend, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_gm_update, dim3(grid), dim3(GB), 0, st, x, W.V, n, kend, W.dh, dinv, n);
        HIPCHK(hipGetLastError());
        ++inf.restarts;
    }
    HIPCHK(hipStreamSynchronize(st));
    inf.iters = total;
    inf.rel_resid = rel;
    inf.converged = rel <= o.tol;
    inf.time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    if (!inf.converged) return fail(SIPDG_ENOCONV, "GMRES did not reach the tolerance within maxit");
    return SIPDG_OK;
}
