// Jacobi-preconditioned conjugate gradients on the device (the Krylov
// method the symmetric SIPG operator is built for, Xia & Moxey Sec. 2.2),
// in FP64 or as an FP32 inner solve inside FP64 iterative refinement.
//
// One iteration = one operator application + one dot product + a fused
// update with two dot products; all scalars stay on the device, one per
// problem, so batched problems keep separate recurrences and stopping tests.
// graph_k iterations are captured once into a HIP graph and replayed; the
// host reads the stop flag after every replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "api_common.hpp"
#include "sipdg.h"
#include "solver.hpp"

namespace sipdg {

constexpr int64_t CHUNK = 4096;  // vector entries per reduction block

struct CgWork {
    hipStream_t stream = nullptr;
    VecCtx V{};
    int64_t *d_blk_start = nullptr;
    int *d_blk_prob = nullptr, *d_prob_blk = nullptr, *d_done = nullptr;
    CgScalars S{};
    double *d_sc = nullptr;   // backing store of the double scalars
    int *d_si = nullptr;      // backing store of the int scalars
    double *p1 = nullptr, *p2 = nullptr, *p3 = nullptr;   // reduction partials (p3: p.q)
    double *x64 = nullptr, *r64 = nullptr, *z64 = nullptr, *pp64 = nullptr, *q64 = nullptr;
    float *x32 = nullptr, *r32 = nullptr, *z32 = nullptr, *pp32 = nullptr, *q32 = nullptr;
    double *d_norm = nullptr, *d_bnorm = nullptr;
    double *d_ratio = nullptr;   // [nprob] residual-norm ratio of a reliable update
    int *d_preconv = nullptr;
    hipGraphExec_t g64 = nullptr, g32 = nullptr;
    int gk64 = 0, gk32 = 0;
    int gpre64 = -1, gpre32 = -1;   // preconditioner flag the graph was captured with
    int gop64 = -1, gop32 = -1;     // kernel structure, basis and geometry source it was captured with
};

void free_cg(sipdg_ctx *c) {
    CgWork *w = c->cg;
    if (!w) return;
    if (w->g64) (void)hipGraphExecDestroy(w->g64);
    if (w->g32) (void)hipGraphExecDestroy(w->g32);
    void *ptrs[] = {w->d_blk_start, w->d_blk_prob, w->d_prob_blk, w->d_done, w->d_sc, w->d_si,
                    w->p1, w->p2, w->p3, w->x64, w->r64, w->z64, w->pp64, w->q64, w->x32, w->r32,
                    w->z32, w->pp32, w->q32, w->d_norm, w->d_bnorm, w->d_preconv, w->d_ratio};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (w->stream) (void)hipStreamDestroy(w->stream);
    delete w;
    c->cg = nullptr;
}

#define ALLOC(ptr, n) HIPCHK(hipMalloc((void **)&(ptr), sizeof(*(ptr)) * (size_t)std::max<int64_t>(1, (n))))

static int ensure_cg32(sipdg_ctx *c);

static int ensure_cg(sipdg_ctx *c) {
    if (c->cg) return SIPDG_OK;
    CgWork *w = new CgWork();
    c->cg = w;
    HIPCHK(hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking));
    std::vector<int64_t> bs;
    std::vector<int> bp, pb(c->nprob + 1, 0);
    for (int p = 0; p < c->nprob; ++p) {
        pb[p] = (int)bp.size();
        for (int64_t s = c->prob_dof_off[p]; s < c->prob_dof_off[p + 1]; s += CHUNK) {
            bs.push_back(s);
            bp.push_back(p);
        }
    }
    pb[c->nprob] = (int)bp.size();
    const int nblk = (int)bp.size();
    // block b covers [bounds[b], bounds[b+1]); a block never crosses the end
    // of its problem because the next problem starts where it ends
    std::vector<int64_t> bounds(bs);
    bounds.push_back(c->ndof);
    for (int b = 0; b < nblk; ++b)
        if (bounds[b + 1] != std::min(bounds[b] + CHUNK, c->prob_dof_off[bp[b] + 1]))
            return fail(SIPDG_EINVAL, "internal: block layout");
    ALLOC(w->d_blk_start, nblk + 1);
    ALLOC(w->d_blk_prob, nblk);
    ALLOC(w->d_prob_blk, c->nprob + 1);
    HIPCHK(hipMemcpy(w->d_blk_start, bounds.data(), sizeof(int64_t) * (nblk + 1), hipMemcpyHostToDevice));
    if (nblk) HIPCHK(hipMemcpy(w->d_blk_prob, bp.data(), sizeof(int) * nblk, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(w->d_prob_blk, pb.data(), sizeof(int) * (c->nprob + 1), hipMemcpyHostToDevice));
    ALLOC(w->d_done, 1);
    w->V.nblk = nblk;
    w->V.nprob = c->nprob;
    w->V.blk_start = w->d_blk_start;
    w->V.blk_prob = w->d_blk_prob;
    w->V.prob_blk = w->d_prob_blk;
    w->V.done = w->d_done;
    const int np = c->nprob;
    ALLOC(w->d_sc, 5 * np + 1);
    ALLOC(w->d_si, 2 * np + 4);
    HIPCHK(hipMemset(w->d_si, 0, sizeof(int) * (2 * np + 4)));
    w->S.rho = w->d_sc;
    w->S.alpha = w->d_sc + np;
    w->S.beta = w->d_sc + 2 * np;
    w->S.bnorm = w->d_sc + 3 * np;
    w->S.rel = w->d_sc + 4 * np;
    w->S.tol = w->d_sc + 5 * np;
    w->S.conv = w->d_si;
    w->S.iters = w->d_si + np;
    w->S.counter = w->d_si + 2 * np;
    w->S.flags = w->d_si + 2 * np + 1;
    w->S.nact = w->d_si + 2 * np + 2;
    w->S.nfin = w->d_si + 2 * np + 3;
    ALLOC(w->p1, nblk);
    ALLOC(w->p2, nblk);
    ALLOC(w->p3, nblk);
    const int64_t n = c->ndof;
    ALLOC(w->x64, n);
    ALLOC(w->r64, n);
    ALLOC(w->z64, n);
    ALLOC(w->pp64, n);
    ALLOC(w->q64, n);
    ALLOC(w->d_norm, np);
    ALLOC(w->d_bnorm, np);
    ALLOC(w->d_preconv, np);
    ALLOC(w->d_ratio, np);
    return SIPDG_OK;
}

int alloc_cg(sipdg_ctx *c) {
    int rc = ensure_cg(c);
    if (rc) return rc;
    return ensure_cg32(c);
}

void cg_scratch(sipdg_ctx *c, double **a, double **b) {
    *a = c->cg ? c->cg->x64 : nullptr;
    *b = c->cg ? c->cg->q64 : nullptr;
}

static int ensure_cg32(sipdg_ctx *c) {
    CgWork *w = c->cg;
    if (w->x32) return SIPDG_OK;
    const int64_t n = c->ndof;
    ALLOC(w->x32, n);
    ALLOC(w->r32, n);
    ALLOC(w->z32, n);
    ALLOC(w->pp32, n);
    ALLOC(w->q32, n);
    return SIPDG_OK;
}

// The folded CG step (x and p updated inside the next application's trace
// stage, see apply_impl) when the handle's apply can take it; the
// environment variable SIPDG_NO_FOLD=1 keeps the separate vector kernels.
static bool use_fold(const sipdg_ctx *c) {
    const char *env = std::getenv("SIPDG_NO_FOLD");
    return fold_ok(c) && !(env && env[0] == '1');
}

// One CG iteration in precision R on the work vectors.
//   separate: q = A p; p.q; [alpha, formed by every block of] x += alpha p,
//             r -= alpha q, z = M r (with r.r, r.z); beta; p = z + beta p.
//   folded:   [x += alpha p, p = M r + beta p, in the trace stage] q = A p;
//             p.q; [alpha] r -= alpha q (with r.r, r.z); beta.  Same values
//             bit for bit; the last x update is applied by vec_flush.
template <class R>
static int cg_body(sipdg_ctx *c, bool precond, bool fold) {
    CgWork *w = c->cg;
    hipStream_t st = w->stream;
    R *x, *r, *z, *p, *q;
    const R *dinv;
    if constexpr (sizeof(R) == 8) {
        x = w->x64; r = w->r64; z = w->z64; p = w->pp64; q = w->q64;
        dinv = precond ? c->d_dinv64 : nullptr;
    } else {
        x = w->x32; r = w->r32; z = w->z32; p = w->pp32; q = w->q32;
        dinv = precond ? c->d_dinv32 : nullptr;
    }
    if (fold) {
        const CgFold<R> f{p, x, r, dinv, w->S.alpha, w->S.beta, w->S.conv};
        int rc = apply_impl<R>(c, p, q, (R *)c->d_tbuf, w->d_done, st, 3, nullptr, &f);
        if (rc) return rc;
        HIPCHK(vec_dot<R>(w->V, p, q, w->p3, st));
        HIPCHK(vec_update_fold<R>(w->V, w->S, r, q, dinv, w->p3, w->p1, w->p2, st));
        HIPCHK(vec_fin_beta(w->V, w->S, w->p1, w->p2, st));
        return SIPDG_OK;
    }
    int rc = apply_impl<R>(c, p, q, (R *)c->d_tbuf, w->d_done, st);
    if (rc) return rc;
    HIPCHK(vec_dot<R>(w->V, p, q, w->p3, st));
    HIPCHK(vec_update<R>(w->V, w->S, x, r, p, q, dinv, z, w->p3, w->p1, w->p2, st));
    HIPCHK(vec_fin_beta(w->V, w->S, w->p1, w->p2, st));
    HIPCHK(vec_pupdate<R>(w->V, w->S, z, p, st));
    return SIPDG_OK;
}

// Apply the folded step's pending x update (x += alpha p, then alpha = 0).
template <class R>
static int cg_flush(sipdg_ctx *c) {
    CgWork *w = c->cg;
    VecCtx Vall = w->V;
    Vall.done = nullptr;
    if constexpr (sizeof(R) == 8) HIPCHK(vec_flush<double>(Vall, w->S, w->x64, w->pp64, w->stream));
    else HIPCHK(vec_flush<float>(Vall, w->S, w->x32, w->pp32, w->stream));
    return SIPDG_OK;
}

// Run iterations until the batch stops or maxit; graph_k per host check.
template <class R>
static int cg_loop(sipdg_ctx *c, const sipdg_cg_opts &o, double tol, int maxit, int &iters_done,
                   int &flags, int &all_done, bool allow_ckpt, int iter_base) {
    CgWork *w = c->cg;
    hipStream_t st = w->stream;
    const int k = std::max(1, o.graph_k);
    iters_done = 0;
    flags = 0;
    all_done = 0;
    hipGraphExec_t *gexec = sizeof(R) == 8 ? &w->g64 : &w->g32;
    int *gk = sizeof(R) == 8 ? &w->gk64 : &w->gk32;
    int *gpre = sizeof(R) == 8 ? &w->gpre64 : &w->gpre32;
    int *gop = sizeof(R) == 8 ? &w->gop64 : &w->gop32;
    const int pre = o.precond != 0;
    const bool fold = use_fold(c);
    const int opk = 64 * (fold ? 1 : 0) + 32 * c->points + 4 * c->variant + 2 * c->basis + (c->geo_map ? 1 : 0);
    if (o.graph_k > 0 && maxit >= k && (*gexec == nullptr || *gk != k || *gpre != pre || *gop != opk)) {
        if (*gexec) {
            (void)hipGraphExecDestroy(*gexec);
            *gexec = nullptr;
        }
        hipGraph_t graph;
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        int rc = SIPDG_OK;
        for (int i = 0; i < k && rc == SIPDG_OK; ++i) rc = cg_body<R>(c, o.precond != 0, fold);
        hipError_t ec = hipStreamEndCapture(st, &graph);
        if (rc) {
            if (ec == hipSuccess) (void)hipGraphDestroy(graph);
            return rc;
        }
        HIPCHK(ec);
        hipError_t ei = hipGraphInstantiate(gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(ei);
        *gk = k;
        *gpre = pre;
        *gop = opk;
    }
    int last_ckpt = 0;
    while (true) {
        // a replay of the captured graph runs k iterations; near maxit the
        // remaining ones are enqueued one by one so maxit is never exceeded
        const int remaining = maxit - iters_done;
        if (o.graph_k > 0 && remaining >= k) {
            HIPCHK(hipGraphLaunch(*gexec, st));
        } else {
            for (int i = 0; i < std::min(k, remaining); ++i) {
                int rc = cg_body<R>(c, o.precond != 0, fold);
                if (rc) return rc;
            }
        }
        int host[2];
        int done = 0;
        HIPCHK(hipMemcpyAsync(host, w->S.counter, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(&done, w->d_done, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        iters_done = host[0];
        flags = host[1];
        all_done = done;
        const bool stop = done || (flags & 2) || iters_done >= maxit;
        const bool ckpt = allow_ckpt && o.checkpoint && o.checkpoint_every > 0 &&
                          iters_done - last_ckpt >= o.checkpoint_every;
        if (fold && (stop || ckpt)) {
            // x is one step behind in the folded iteration: bring it up to date
            int rc = cg_flush<R>(c);
            if (rc) return rc;
            if (ckpt) HIPCHK(hipStreamSynchronize(st));
        }
        if (ckpt) {
            o.checkpoint(o.checkpoint_user, w->x64, w->r64, iter_base + iters_done);
            last_ckpt = iters_done;
        }
        if (stop) break;
    }
    return SIPDG_OK;
}

// ||b - A x|| / ||b|| per problem into host vector rel (FP64 apply).
static int true_residual(sipdg_ctx *c, const double *b, std::vector<double> &rel,
                         std::vector<double> &bn) {
    CgWork *w = c->cg;
    hipStream_t st = w->stream;
    int rc = apply_impl<double>(c, w->x64, w->q64, c->d_tbuf, nullptr, st);
    if (rc) return rc;
    HIPCHK(vec_resid(w->V, b, w->q64, w->r64, w->p1, st));
    HIPCHK(vec_fin_norm(w->V, w->p1, w->d_norm, st));
    std::vector<double> nr(c->nprob);
    HIPCHK(hipMemcpyAsync(nr.data(), w->d_norm, sizeof(double) * c->nprob, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    rel.resize(c->nprob);
    for (int p = 0; p < c->nprob; ++p) rel[p] = bn[p] > 0 ? nr[p] / bn[p] : 0.0;
    return SIPDG_OK;
}

}  // namespace sipdg

using namespace sipdg;

extern "C" {

void sipdg_cg_default_opts(sipdg_cg_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-10;
    o->maxit = 20000;
    o->mode = SIPDG_CG_F64;
    o->inner_tol = 1e-4;
    o->precond = 1;
    o->graph_k = 10;
    o->max_outer = 50;
    o->ru_delta = 0.1;
}

int sipdg_cg_solve(sipdg_handle h, const double *b, double *x, const sipdg_cg_opts *opts,
                   sipdg_cg_info *info, void *stream) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (h->flux == SIPDG_FLUX_P2P)
        return fail(SIPDG_EINVAL, "CG needs the symmetric shared-trace operator (the point-to-point flux is set)");
    sipdg_cg_opts o;
    if (opts) o = *opts;
    else sipdg_cg_default_opts(&o);
    if (!(o.tol > 0.0) || o.maxit <= 0 ||
        (o.mode != SIPDG_CG_F64 && o.mode != SIPDG_CG_F32_IR && o.mode != SIPDG_CG_F32_RU))
        return fail(SIPDG_EINVAL, "invalid CG options");
    if (o.mode == SIPDG_CG_F32_RU && !(o.ru_delta > 0.0 && o.ru_delta < 1.0))
        return fail(SIPDG_EINVAL, "ru_delta must be in (0, 1)");
    if (o.mode != SIPDG_CG_F64 && !(o.inner_tol > 0.0 && o.inner_tol < 1.0))
        return fail(SIPDG_EINVAL, "inner_tol must be in (0, 1)");
    if (h->ndof == 0) {   // empty mesh: the (empty) zero vector solves it
        if (info) {
            info->iters = 0;
            info->outer_iters = 0;
            info->converged = 1;
            info->rel_resid = 0.0;
            info->time_ms = 0.0;
        }
        return SIPDG_OK;
    }
    if (!b || !x) return fail(SIPDG_EINVAL, "null argument");
    auto t0 = std::chrono::steady_clock::now();
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    int rc = ensure_cg(h);
    if (rc) return rc;
    CgWork *w = h->cg;
    hipStream_t st = w->stream;
    const int64_t n = h->ndof;
    // a previous solve leaves the stop flag set: clear it, and take ||b||
    // with a context that never skips
    HIPCHK(vec_fill<int>(w->d_done, 1, 0, st));
    VecCtx Vall = w->V;
    Vall.done = nullptr;
    HIPCHK(vec_dot<double>(Vall, b, b, w->p1, st));
    HIPCHK(vec_fin_norm(w->V, w->p1, w->d_bnorm, st));
    std::vector<double> bn(h->nprob);
    HIPCHK(hipMemcpyAsync(bn.data(), w->d_bnorm, sizeof(double) * h->nprob, hipMemcpyDeviceToHost, st));
    // x0
    if (o.x0_given) HIPCHK(hipMemcpyAsync(w->x64, x, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    else HIPCHK(vec_fill<double>(w->x64, n, 0.0, st));
    HIPCHK(hipStreamSynchronize(st));

    int total_iters = 0, outer = 0, flags = 0;
    bool breakdown = false, f64_done = false;
    std::vector<double> rel;
    if (o.mode == SIPDG_CG_F64) {
        if (o.x0_given) {
            rc = apply_impl<double>(h, w->x64, w->q64, h->d_tbuf, nullptr, st);
            if (rc) return rc;
            HIPCHK(vec_resid(w->V, b, w->q64, w->r64, w->p1, st));
        } else {
            HIPCHK(hipMemcpyAsync(w->r64, b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        }
        HIPCHK(vec_start<double>(w->V, w->r64, o.precond ? h->d_dinv64 : nullptr, w->z64, w->pp64,
                                 nullptr, w->p1, w->p2, st));
        HIPCHK(vec_fin_start(w->V, w->S, w->p1, w->p2, w->d_bnorm, nullptr, o.tol, st));
        int done = 0;
        rc = cg_loop<double>(h, o, o.tol, o.maxit, total_iters, flags, done, true, 0);
        if (rc) return rc;
        breakdown = (flags & 2) != 0;
        f64_done = done != 0;
        outer = 1;
        // The recursive residual drifts from the true one over many iterations:
        // restart from the true residual r = b - A x (problems that meet the
        // tolerance stay frozen) until every problem's true residual does.
        while (f64_done && !breakdown && total_iters < o.maxit && outer < o.max_outer) {
            rc = true_residual(h, b, rel, bn);
            if (rc) return rc;
            std::vector<int> preconv(h->nprob);
            bool all = true;
            for (int p = 0; p < h->nprob; ++p) {
                preconv[p] = rel[p] <= o.tol ? 1 : 0;
                all = all && preconv[p];
            }
            if (all) break;
            HIPCHK(hipMemcpyAsync(w->d_preconv, preconv.data(), sizeof(int) * h->nprob, hipMemcpyHostToDevice, st));
            HIPCHK(vec_start<double>(w->V, w->r64, o.precond ? h->d_dinv64 : nullptr, w->z64, w->pp64, nullptr,
                                     w->p1, w->p2, st));
            HIPCHK(vec_fin_start(w->V, w->S, w->p1, w->p2, w->d_bnorm, w->d_preconv, o.tol, st));
            int it = 0;
            rc = cg_loop<double>(h, o, o.tol, o.maxit - total_iters, it, flags, done, true, total_iters);
            if (rc) return rc;
            total_iters += it;
            breakdown = (flags & 2) != 0;
            f64_done = done != 0;
            ++outer;
        }
    } else {
        rc = ensure_cg32(h);
        if (rc) return rc;
        std::vector<int> preconv(h->nprob);
        std::vector<double> nr_prev(h->nprob, 0.0);   // residual norms of the previous cycle
        while (true) {
            rc = apply_impl<double>(h, w->x64, w->q64, h->d_tbuf, nullptr, st);
            if (rc) return rc;
            HIPCHK(vec_resid(w->V, b, w->q64, w->r64, w->p1, st));
            HIPCHK(vec_fin_norm(w->V, w->p1, w->d_norm, st));
            std::vector<double> nr(h->nprob);
            HIPCHK(hipMemcpyAsync(nr.data(), w->d_norm, sizeof(double) * h->nprob, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            bool all = true;
            for (int p = 0; p < h->nprob; ++p) {
                preconv[p] = !(bn[p] > 0.0) || nr[p] <= o.tol * bn[p];
                all = all && preconv[p];
            }
            if (o.checkpoint && o.checkpoint_every > 0) o.checkpoint(o.checkpoint_user, w->x64, w->r64, total_iters);
            if (all || outer >= o.max_outer || total_iters >= o.maxit || breakdown) break;
            // the inner solve asks for the reduction the outer residual still
            // needs (half of it, for the FP32 solve's own error), but never for
            // less than inner_tol: the last refinement does no more work than
            // required
            double itol = 1.0;
            for (int p = 0; p < h->nprob; ++p)
                if (!preconv[p] && nr[p] > 0.0) itol = std::min(itol, 0.5 * o.tol * bn[p] / nr[p]);
            itol = std::min(std::max(itol, o.mode == SIPDG_CG_F32_RU ? o.ru_delta : o.inner_tol), 0.5);
            HIPCHK(hipMemcpyAsync(w->d_preconv, preconv.data(), sizeof(int) * h->nprob, hipMemcpyHostToDevice, st));
            HIPCHK(vec_scale32(w->V, w->r64, w->d_norm, w->r32, st));
            if (o.mode == SIPDG_CG_F32_IR || outer == 0) {
                // refinement: a fresh FP32 PCG on the normalised residual
                HIPCHK(vec_start<float>(w->V, w->r32, o.precond ? h->d_dinv32 : nullptr, w->z32, w->pp32,
                                        w->x32, w->p1, w->p2, st));
                HIPCHK(vec_fin_start(w->V, w->S, w->p1, w->p2, nullptr, w->d_preconv, itol, st));
            } else {
                // reliable update: the true residual replaces the recursive one,
                // the search direction is kept (renormalised) and the recursion goes on
                // continue a problem only if its true residual agrees with the
                // FP32 recursion's estimate (rel: reduction reached in the cycle);
                // else restart it (ratio 0 gives p = z)
                std::vector<double> rel_rec(h->nprob), ratio(h->nprob, 0.0);
                HIPCHK(hipMemcpyAsync(rel_rec.data(), w->S.rel, sizeof(double) * h->nprob, hipMemcpyDeviceToHost,
                                      st));
                HIPCHK(hipStreamSynchronize(st));
                for (int p = 0; p < h->nprob; ++p)
                    if (nr_prev[p] > 0.0 && nr[p] <= 1.5 * rel_rec[p] * nr_prev[p]) ratio[p] = nr[p] / nr_prev[p];
                HIPCHK(hipMemcpyAsync(w->d_ratio, ratio.data(), sizeof(double) * h->nprob, hipMemcpyHostToDevice,
                                      st));
                HIPCHK(vec_start<float>(w->V, w->r32, o.precond ? h->d_dinv32 : nullptr, w->z32, nullptr, w->x32,
                                        w->p1, w->p2, st));
                HIPCHK(vec_fin_cont(w->V, w->S, w->p1, w->p2, w->d_preconv, w->d_ratio, itol, st));
                // the folded iteration forms p = M r + beta p itself (alpha is 0)
                if (!use_fold(h)) HIPCHK(vec_pupdate<float>(w->V, w->S, w->z32, w->pp32, st));
            }
            nr_prev = nr;
            int it = 0, idone = 0;
            rc = cg_loop<float>(h, o, itol, o.maxit - total_iters, it, flags, idone, false, total_iters);
            if (rc) return rc;
            total_iters += it;
            breakdown = (flags & 2) != 0;
            HIPCHK(vec_correct(w->V, w->x32, w->d_norm, w->x64, st));
            ++outer;
        }
    }
    rc = true_residual(h, b, rel, bn);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(x, w->x64, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    double worst = 0.0;
    for (double r : rel) worst = std::max(worst, r);
    // both modes: the FP64 true residual of every problem meets the tolerance
    bool conv = worst <= o.tol;
    auto t1 = std::chrono::steady_clock::now();
    if (info) {
        info->iters = total_iters;
        info->outer_iters = outer;
        info->converged = conv && !breakdown;
        info->rel_resid = worst;
        info->time_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    if (breakdown) return fail(SIPDG_EBREAKDOWN, "CG breakdown: p^T A p <= 0 (operator not SPD)");
    if (!conv) return fail(SIPDG_ENOCONV, "CG did not reach the tolerance within maxit");
    return SIPDG_OK;
}

}  // extern "C"
