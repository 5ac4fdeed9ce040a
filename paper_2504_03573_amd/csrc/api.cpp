// C ABI: handle lifetime, operator application, setup products.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "api_common.hpp"
#include "sipdg.h"
#include "solver.hpp"
#include "topology.hpp"
#include "fast3d.hpp"
#include "gfold3d.hpp"
#include "k_tile.hpp"
#include <cstdlib>

using namespace sipdg;

namespace sipdg {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

template <class T>
static int dalloc(T **p, int64_t n) {
    *p = nullptr;
    if (n <= 0) n = 1;
    hipError_t e = hipMalloc((void **)p, sizeof(T) * (size_t)n);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(SIPDG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return SIPDG_OK;
}

template <class T>
static int upload(T **p, const std::vector<T> &v) {
    int rc = dalloc(p, (int64_t)v.size());
    if (rc) return rc;
    if (!v.empty()) HIPCHK(hipMemcpy(*p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return SIPDG_OK;
}

template <class R>
OpArgs<R> make_args(const sipdg_ctx *c, const Group &g, const R *x, R *y, R *tbuf, const int *skip) {
    OpArgs<R> A;
    A.elems = g.d_elems;
    A.count = g.count;
    A.tsz = work_size_for(c->dim, g.P, g.nfmax);
    A.xoff = c->d_xoff;
    A.voff = c->d_voff;
    A.eface = c->d_eface;
    A.foff = c->d_foff;
    A.toff = c->d_toff;
    if constexpr (sizeof(R) == 8) {
        A.vgeo = (const R *)c->d_vgeo64;
        A.fgeo = (const R *)c->d_fgeo64;
        A.lam = (const R *)c->d_lam64;
        A.tau = (const R *)c->d_tau64;
        A.tab = (const R *)c->d_tab64;
    } else {
        A.vgeo = (const R *)c->d_vgeo32;
        A.fgeo = (const R *)c->d_fgeo32;
        A.lam = (const R *)c->d_lam32;
        A.tau = (const R *)c->d_tau32;
        A.tab = (const R *)c->d_tab32;
    }
    A.x = x;
    A.y = y;
    A.tbuf = tbuf;
    A.skip = skip;
    A.order = c->d_order;
    A.faces = c->d_faces;
    if constexpr (sizeof(R) == 8) A.emap = (const R *)c->d_emap64;
    else A.emap = (const R *)c->d_emap32;
    return A;
}
template OpArgs<double> make_args<double>(const sipdg_ctx *, const Group &, const double *, double *, double *, const int *);
template OpArgs<float> make_args<float>(const sipdg_ctx *, const Group &, const float *, float *, float *, const int *);

template <class R>
hipError_t launch_fast3d(int P, int kind, const f3::Args3 &A, const f3::Data3<R> &D, hipStream_t st);

template <class R>
static void fast_args(const sipdg_ctx *c, const Group &g, const R *x, R *y, R *tbuf, const int *skip,
                      bool fused, f3::Args3 &A, f3::Data3<R> &D) {
    A.elems = g.d_elems;
    A.count = g.count;
    A.region = 0;
    A.xoff = c->d_xoff;
    A.voff = c->d_voff;
    A.eface = c->d_eface;
    A.faces = c->d_faces;
    A.order = c->d_order;
    A.foff = c->d_foff;
    A.toff = c->d_toff;
    A.skip = skip;
    if constexpr (sizeof(R) == 8) {
        D.vgeo = (const R *)c->d_vgeo64;
        D.fgeo = (const R *)c->d_fgeo64;
        D.lam = (const R *)c->d_lam64;
        D.tau = (const R *)c->d_tau64;
        D.tab = (const R *)c->d_tab64;
    } else {
        D.vgeo = (const R *)c->d_vgeo32;
        D.fgeo = (const R *)c->d_fgeo32;
        D.lam = (const R *)c->d_lam32;
        D.tau = (const R *)c->d_tau32;
        D.tab = (const R *)c->d_tab32;
    }
    D.x = x;
    D.y = y;
    D.tbuf = tbuf;
}

template <class R>
hipError_t launch_gfold3d(int P, int mode, int nfmax, const g3::Args &A, const g3::Data<R> &D, hipStream_t st);

static inline void rec_mark(LaunchRec *rec, int stage, int gi, bool after, hipStream_t st) {
    if (!rec || rec->n >= rec->cap) return;
    (void)hipEventRecord(rec->ev[2 * rec->n + (after ? 1 : 0)], st);
    if (after) {
        rec->stage[rec->n] = stage;
        rec->group[rec->n] = gi;
        rec->n++;
    }
}

template <class R>
hipError_t launch_gfold3d_persistent(int mode, int grid, const g3::Args &A, const g3::Data<R> &D, hipStream_t st);
template <class R>
hipError_t launch_gfold3d_trace_all(const g3::Args &A, const g3::Data<R> &D, hipStream_t st);

// Can the gather-fold kernels take this order group?  One wavefront per
// element up to order 6 with traces up to 8 x 8; two wavefronts for orders 7
// and 8 (traces up to 10 x 10; not the fused kernel).
static bool gfold_group(const Group &g, bool fused) {
    if (g.P <= 6 && g.nfmax <= 8) return true;
    return !fused && g.P >= 7 && g.P <= 8 && g.nfmax <= 10;
}

// Kernel structures of a 2-D handle: the general kernels, the wavefront
// kernels (an element of order <= 6 with traces <= 8 points needed), and the
// fused wavefront kernel (every element in the wavefront list).
static bool variant_allowed_2d(const sipdg_ctx *c, int v) {
    if (v == SIPDG_VARIANT_GATHER) return true;
    if (v == SIPDG_VARIANT_GATHER_FOLD) return c->w2count > 0;
    if (v == SIPDG_VARIANT_GATHER_FOLD_FUSED) return c->w2count > 0 && c->w2count == c->ne;
    return false;
}

// Default kernel structure: gather-fold in 3-D and, in 2-D, the wavefront
// kernels when an element can take them; the general kernels otherwise.
static int default_variant(const sipdg_ctx *c) {
    if (c->dim == 3) return c->gfold_ok ? SIPDG_VARIANT_GATHER_FOLD : SIPDG_VARIANT_GATHER;
    return c->w2count > 0 ? SIPDG_VARIANT_GATHER_FOLD : SIPDG_VARIANT_GATHER;
}

// per-element constants of affine elements (G~, |J|), in the apply's precision
template <class R>
static const R *egeo_of(const sipdg_ctx *c) {
    if constexpr (sizeof(R) == 8) return (const R *)c->d_egeo64;
    else return (const R *)c->d_egeo32;
}
template <class R>
static const R *emap_of(const sipdg_ctx *c) {
    if constexpr (sizeof(R) == 8) return (const R *)c->d_emap64;
    else return (const R *)c->d_emap32;
}
// the Gauss table set, in the apply's precision
template <class R>
static const R *tabgl_of(const sipdg_ctx *c) {
    if constexpr (sizeof(R) == 8) return (const R *)c->d_tabgl64;
    else return (const R *)c->d_tabgl32;
}

// The gather-fold apply launch of one order group (shared-trace flux): the
// multi-element tile the handle is tuned to for stored-factor (mode 1) and
// map-geometry (mode 4) launches of orders <= 5, else the one-element kernel.
template <class R>
static hipError_t launch_apply_group(const sipdg_ctx *c, int P, int mode, int nfmax, const g3::Args &A,
                                     const g3::Data<R> &D, hipStream_t st) {
    if ((mode == 1 || mode == 4) && P <= 5 && nfmax <= 8 && (c->tile[P] != 1 || c->budget[P] != 2))
        return launch_gfold3d_tile<R>(P, mode == 4 ? g3::GEO_MAP : g3::GEO_POINT, c->tile[P], c->budget[P], A, D,
                                      st);
    return launch_gfold3d<R>(P, mode, nfmax, A, D, st);
}

bool fold_ok(const sipdg_ctx *c) {
    return c->dim == 3 && c->variant == SIPDG_VARIANT_GATHER_FOLD && c->flux == SIPDG_FLUX_SHARED &&
           c->pcount == c->ne && c->ne > 0 && c->d_eprob != nullptr;
}

template <class R>
int apply_impl(sipdg_ctx *c, const R *x, R *y, R *tbuf, const int *skip, hipStream_t st, int stages,
               LaunchRec *rec, const CgFold<R> *fold) {
    if (fold && (!fold_ok(c) || fold->p != x))
        return fail(SIPDG_EINVAL, "internal: folded CG step on an apply that cannot take it");
    const bool gauss = c->points == SIPDG_POINTS_GAUSS;
    if (gauss && (c->variant != SIPDG_VARIANT_GATHER_FOLD || c->flux != SIPDG_FLUX_SHARED))
        return fail(SIPDG_EINVAL, "Gauss points run on the gather_fold structure with the shared-trace flux");
    if (c->dim == 2 && (c->variant == SIPDG_VARIANT_GATHER_FOLD || c->variant == SIPDG_VARIANT_GATHER_FOLD_FUSED)) {
        // 2-D wavefront kernels: one launch per stage for every element of
        // order <= 6 with traces <= 8 points; the general kernels for the
        // groups around orders 7 and 8 (same trace-buffer layout).  The fused
        // structure (one launch) is allowed only when the wavefront list
        // holds every element.
        if (c->groups.empty()) return SIPDG_OK;
        const bool fused = c->variant == SIPDG_VARIANT_GATHER_FOLD_FUSED;
        Data2<R> D2;
        {
            f3::Args3 A3;
            f3::Data3<R> D3;
            fast_args<R>(c, c->groups[0], x, y, tbuf, skip, false, A3, D3);
            D2 = Data2<R>{D3.vgeo, D3.fgeo, D3.lam, D3.tau, D3.tab, x, y, tbuf};
        }
        const Args2 A2{c->d_w2desc, c->d_w2fdesc, c->d_w2nb, c->w2count, skip};
        for (int stage = 1; stage <= 2; ++stage) {
            if (!(stages & stage) || (fused && stage == 1)) continue;
            if (c->w2count > 0) {
                rec_mark(rec, stage, -1, false, st);
                hipError_t e = launch_wave2d<R>(stage == 1 ? 0 : (fused ? 2 : 1), A2, D2, st);
                rec_mark(rec, stage, -1, true, st);
                if (e != hipSuccess)
                    return fail(SIPDG_EHIP, std::string("2-D wavefront kernel: ") + hipGetErrorString(e));
            }
            for (size_t gi = 0; gi < c->groups.size(); ++gi) {
                const Group &g = c->groups[gi];
                if (g.P <= 6 && g.nfmax <= 8) continue;
                OpArgs<R> A = make_args<R>(c, g, x, y, tbuf, skip);
                rec_mark(rec, stage, (int)gi, false, st);
                hipError_t e = launch_op<R>(c->dim, g.P, stage == 1 ? OP_TRACE : OP_APPLY, A, g.nfmax, st);
                rec_mark(rec, stage, (int)gi, true, st);
                if (e != hipSuccess)
                    return fail(SIPDG_EHIP, std::string(stage == 1 ? "trace kernel: " : "apply kernel: ") +
                                                hipGetErrorString(e));
            }
        }
        return SIPDG_OK;
    }
    if (c->flux == SIPDG_FLUX_P2P && c->variant != SIPDG_VARIANT_GATHER) {
        // point-to-point flux through the gather-fold apply: per order group a
        // trace launch (own pair, and the trace interpolated to each
        // neighbour's points), then the apply with every face side on its own
        // point set (nf = n: no lift)
        R *pb = (R *)c->d_tbuf_p2p;
        const R *fgp = sizeof(R) == 8 ? (const R *)c->d_fgeo_p2p64 : (const R *)c->d_fgeo_p2p32;
        for (int stage = 1; stage <= 2; ++stage) {
            if (!(stages & stage)) continue;
            // trace stage: one wavefront launch for the orders <= 6 of the
            // persistent list, one per remaining group
            if (stage == 1 && c->pcount > 0) {
                f3::Args3 A3;
                f3::Data3<R> D3;
                fast_args<R>(c, c->groups[0], x, y, pb, skip, false, A3, D3);
                g3::Args A{A3.elems, c->pcount, A3.xoff, A3.voff, A3.eface, A3.faces, A3.order, A3.foff, A3.toff,
                           A3.skip, c->d_pdesc, c->d_pfdesc_p2p, c->basis, c->d_p2p_side};
                g3::Data<R> D{D3.vgeo, fgp, D3.lam, D3.tau, D3.tab, D3.x, D3.y, pb, egeo_of<R>(c), emap_of<R>(c)};
                rec_mark(rec, 1, -1, false, st);
                hipError_t e = launch_gfold3d_trace_all<R>(A, D, st);
                rec_mark(rec, 1, -1, true, st);
                if (e != hipSuccess)
                    return fail(SIPDG_EHIP, std::string("point-to-point trace: ") + hipGetErrorString(e));
            }
            for (size_t gi = 0; gi < c->groups.size(); ++gi) {
                const Group &g = c->groups[gi];
                if (stage == 1 && c->pcount > 0 && g.P <= 6 && g.nfmax <= 8) continue;
                rec_mark(rec, stage, (int)gi, false, st);
                hipError_t e = hipSuccess;
                f3::Args3 A3;
                f3::Data3<R> D3;
                fast_args<R>(c, g, x, y, pb, skip, false, A3, D3);
                g3::Args A{A3.elems, A3.count, A3.xoff, A3.voff, A3.eface, A3.faces, A3.order, A3.foff,
                           A3.toff, A3.skip, g.d_desc, g.d_fdesc_p2p, c->basis, c->d_p2p_side};
                g3::Data<R> D{D3.vgeo, fgp, D3.lam, D3.tau, D3.tab, D3.x, D3.y, pb, egeo_of<R>(c), emap_of<R>(c)};
                if (stage == 1) {
                    e = launch_gfold3d<R>(g.P, 0, g.P + 2, A, D, st);
                } else {
                    const int mode = c->geo_map ? 4 : 1;
                    if (g.split) {
                        g3::Args Aa = A, Ad = A;
                        Aa.count = g.naff;
                        Ad.count = g.count - g.naff;
                        Ad.desc = g.d_desc + g.naff;
                        Ad.fdesc = g.d_fdesc_p2p + (int64_t)6 * g.naff;
                        e = launch_gfold3d<R>(g.P, 3, g.P + 2, Aa, D, st);
                        if (e == hipSuccess) e = launch_gfold3d<R>(g.P, mode, g.P + 2, Ad, D, st);
                    } else {
                        e = launch_gfold3d<R>(g.P, mode, g.P + 2, A, D, st);
                    }
                }
                rec_mark(rec, stage, (int)gi, true, st);
                if (e != hipSuccess)
                    return fail(SIPDG_EHIP, std::string("point-to-point kernel: ") + hipGetErrorString(e));
            }
        }
        return SIPDG_OK;
    }
    if (c->flux == SIPDG_FLUX_P2P) {
        // point-to-point flux, general kernels (the gather structure): per
        // order group, a trace launch (own face points) then an apply launch
        R *pb = (R *)c->d_tbuf_p2p;
        for (int stage = 1; stage <= 2; ++stage) {
            if (!(stages & stage)) continue;
            for (size_t gi = 0; gi < c->groups.size(); ++gi) {
                const Group &g = c->groups[gi];
                OpArgs<R> A = make_args<R>(c, g, x, y, pb, skip);
                rec_mark(rec, stage, (int)gi, false, st);
                hipError_t e = launch_p2p<R>(g.P, stage, A, g.nfmax, st);
                rec_mark(rec, stage, (int)gi, true, st);
                if (e != hipSuccess)
                    return fail(SIPDG_EHIP, std::string("point-to-point kernel: ") + hipGetErrorString(e));
            }
        }
        return SIPDG_OK;
    }
    if (c->variant == SIPDG_VARIANT_GATHER_FOLD_PERSISTENT) {
        for (int stage = 1; stage <= 2; ++stage) {
            if (!(stages & stage)) continue;
            // orders <= 6: one persistent launch over all of them
            if (c->pcount > 0) {
                f3::Args3 A3;
                f3::Data3<R> D3;
                fast_args<R>(c, c->groups[0], x, y, tbuf, skip, false, A3, D3);
                g3::Args A{A3.elems, c->pcount, A3.xoff, A3.voff, A3.eface, A3.faces, A3.order, A3.foff, A3.toff,
                           A3.skip, c->d_pdesc, c->d_pfdesc, c->basis};
                g3::Data<R> D{D3.vgeo, D3.fgeo, D3.lam, D3.tau, D3.tab, D3.x, D3.y, D3.tbuf, egeo_of<R>(c), emap_of<R>(c)};
                rec_mark(rec, stage, -1, false, st);
                hipError_t e = launch_gfold3d_persistent<R>(stage == 1 ? 0 : 1, c->num_cu * c->blocks_per_cu, A, D, st);
                rec_mark(rec, stage, -1, true, st);
                if (e != hipSuccess)
                    return fail(SIPDG_EHIP, std::string("persistent kernel: ") + hipGetErrorString(e));
            }
            // the rest: per group, gather-fold (orders 7, 8) or the general kernels
            for (size_t gi = 0; gi < c->groups.size(); ++gi) {
                const Group &g = c->groups[gi];
                if (g.P <= 6 && g.nfmax <= 8) continue;
                rec_mark(rec, stage, (int)gi, false, st);
                hipError_t e;
                if (gfold_group(g, false)) {
                    f3::Args3 A3;
                    f3::Data3<R> D3;
                    fast_args<R>(c, g, x, y, tbuf, skip, false, A3, D3);
                    g3::Args A{A3.elems, A3.count, A3.xoff, A3.voff, A3.eface, A3.faces, A3.order, A3.foff,
                               A3.toff, A3.skip, g.d_desc, g.d_fdesc, c->basis};
                    g3::Data<R> D{D3.vgeo, D3.fgeo, D3.lam, D3.tau, D3.tab, D3.x, D3.y, D3.tbuf, egeo_of<R>(c), emap_of<R>(c)};
                    e = launch_gfold3d<R>(g.P, stage == 1 ? 0 : 1, g.nfmax, A, D, st);
                } else {
                    OpArgs<R> A = make_args<R>(c, g, x, y, tbuf, skip);
                    e = launch_op<R>(c->dim, g.P, stage == 1 ? OP_TRACE : OP_APPLY, A, g.nfmax, st);
                }
                rec_mark(rec, stage, (int)gi, true, st);
                if (e != hipSuccess)
                    return fail(SIPDG_EHIP, std::string(stage == 1 ? "trace kernel: " : "apply kernel: ") +
                                                hipGetErrorString(e));
            }
        }
        return SIPDG_OK;
    }
    if (c->variant == SIPDG_VARIANT_GATHER_FOLD || c->variant == SIPDG_VARIANT_GATHER_FOLD_FUSED) {
        const bool fused = c->variant == SIPDG_VARIANT_GATHER_FOLD_FUSED;
        // the groups of a stage are independent: side streams, joined at the end
        // (launches recorded for timing stay on the caller's stream).  Measured
        // on the 32^3 mixed-order mesh: FP64 (2-3 waves per SIMD) gains from
        // groups sharing the CUs, FP32 (4-5 waves) loses, so FP64 only.
        const bool par = c->concurrent && sizeof(R) == 8 && !rec && !c->gstreams.empty();
        hipStream_t main_st = st;
        for (int stage = 1; stage <= 2; ++stage) {
            if (!(stages & stage) || (fused && stage == 1)) continue;
            const int mode = stage == 1 ? 0 : (fused ? 2 : 1);
            // trace stage of the order <= 6 groups (traces <= 8 x 8): one launch
            const bool merged = stage == 1 && c->pcount > 0;
            if (merged) {
                f3::Args3 A3;
                f3::Data3<R> D3;
                fast_args<R>(c, c->groups[0], x, y, tbuf, skip, false, A3, D3);
                g3::Args A{A3.elems, c->pcount, A3.xoff, A3.voff, A3.eface, A3.faces, A3.order, A3.foff, A3.toff,
                           A3.skip, c->d_pdesc, c->d_pfdesc, c->basis};
                g3::Data<R> D{D3.vgeo, D3.fgeo, D3.lam, D3.tau, D3.tab, D3.x, D3.y, D3.tbuf, egeo_of<R>(c), emap_of<R>(c)};
                if (fold) {
                    D.fold_p = fold->p;
                    D.fold_x = fold->x;
                    D.fold_r = fold->r;
                    D.fold_dinv = fold->dinv;
                    D.fold_alpha = fold->alpha;
                    D.fold_beta = fold->beta;
                    D.fold_conv = fold->conv;
                    D.eprob = c->d_eprob;
                }
                rec_mark(rec, stage, -1, false, main_st);
                hipError_t e = launch_gfold3d_trace_all<R>(A, D, main_st);
                rec_mark(rec, stage, -1, true, main_st);
                if (e != hipSuccess) return fail(SIPDG_EHIP, std::string("trace kernel: ") + hipGetErrorString(e));
            }
            if (par && hipEventRecord(c->gevents[0], main_st) != hipSuccess)
                return fail(SIPDG_EHIP, "event record (fork)");
            for (size_t gi = 0; gi < c->groups.size(); ++gi) {
                const Group &g = c->groups[gi];
                if (merged && g.P <= 6 && g.nfmax <= 8) continue;
                hipStream_t st = par ? c->gstreams[gi] : main_st;
                if (par && hipStreamWaitEvent(st, c->gevents[0], 0) != hipSuccess)
                    return fail(SIPDG_EHIP, "stream wait (fork)");
                struct Join {
                    bool on;
                    hipEvent_t ev;
                    hipStream_t s;
                    ~Join() {
                        if (on) (void)hipEventRecord(ev, s);
                    }
                } join{par, par ? c->gevents[1 + gi] : nullptr, st};
                if (!gfold_group(g, fused)) {
                    // orders <= 6 next to orders above 6 (traces finer than the
                    // 8 x 8 lane grid): the general kernels, same trace-buffer layout
                    OpArgs<R> A = make_args<R>(c, g, x, y, tbuf, skip);
                    rec_mark(rec, stage, (int)gi, false, st);
                    hipError_t e = launch_op<R>(c->dim, g.P, stage == 1 ? OP_TRACE : OP_APPLY, A, g.nfmax, st);
                    rec_mark(rec, stage, (int)gi, true, st);
                    if (e != hipSuccess)
                        return fail(SIPDG_EHIP, std::string(stage == 1 ? "trace kernel: " : "apply kernel: ") +
                                                    hipGetErrorString(e));
                    continue;
                }
                f3::Args3 A3;
                f3::Data3<R> D3;
                fast_args<R>(c, g, x, y, tbuf, skip, fused, A3, D3);
                g3::Args A{A3.elems, A3.count, A3.xoff, A3.voff, A3.eface, A3.faces, A3.order, A3.foff, A3.toff,
                           A3.skip, g.d_desc, g.d_fdesc, c->basis};
                g3::Data<R> D{D3.vgeo, D3.fgeo, D3.lam, D3.tau, D3.tab, D3.x, D3.y, D3.tbuf, egeo_of<R>(c), emap_of<R>(c)};
                // Gauss volume points: that table set (its trace tables are
                // the GLL set's) and geometry from the maps or affine constants
                if (gauss) D.tab = tabgl_of<R>(c);
                const int def_mode = gauss ? 5 : (c->geo_map ? 4 : 1), aff_mode = gauss ? 6 : 3;
                rec_mark(rec, stage, (int)gi, false, st);
                hipError_t e = hipSuccess;
                if (mode == 1 && g.split) {
                    // the group's affine elements (first in its descriptors) and
                    // the deformed rest.  Under graph capture side by side (the
                    // fork and join are graph edges); eagerly one after the
                    // other, since an event fork and join per group costs more
                    // than the overlap of the two launches' tails gains
                    g3::Args Aa = A, Ad = A;
                    Aa.count = g.naff;
                    Ad.count = g.count - g.naff;
                    Ad.desc = g.d_desc + g.naff;
                    Ad.fdesc = g.d_fdesc + (int64_t)6 * g.naff;
                    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
                    if (Ad.count > 0 && c->aff_stream && !rec && hipStreamIsCapturing(st, &cap) != hipSuccess)
                        return fail(SIPDG_EHIP, "stream capture query");
                    const bool side = cap == hipStreamCaptureStatusActive;
                    if (side) {
                        if (hipEventRecord(c->aff_ev[0], st) != hipSuccess ||
                            hipStreamWaitEvent(c->aff_stream, c->aff_ev[0], 0) != hipSuccess)
                            return fail(SIPDG_EHIP, "event record / wait (affine fork)");
                    }
                    e = launch_gfold3d<R>(g.P, aff_mode, g.nfmax, Aa, D, side ? c->aff_stream : st);
                    if (e == hipSuccess) e = launch_apply_group<R>(c, g.P, def_mode, g.nfmax, Ad, D, st);
                    if (side) {
                        if (hipEventRecord(c->aff_ev[1], c->aff_stream) != hipSuccess ||
                            hipStreamWaitEvent(st, c->aff_ev[1], 0) != hipSuccess)
                            return fail(SIPDG_EHIP, "event record / wait (affine join)");
                    }
                } else if (mode == 1) {
                    e = launch_apply_group<R>(c, g.P, def_mode, g.nfmax, A, D, st);
                } else {
                    e = launch_gfold3d<R>(g.P, mode, g.nfmax, A, D, st);
                }
                rec_mark(rec, stage, (int)gi, true, st);
                if (e != hipSuccess)
                    return fail(SIPDG_EHIP, std::string(stage == 1 ? "trace kernel: " : "apply kernel: ") +
                                                hipGetErrorString(e));
            }
            if (par)
                for (size_t gi = 0; gi < c->groups.size(); ++gi)
                    if (hipStreamWaitEvent(main_st, c->gevents[1 + gi], 0) != hipSuccess)
                        return fail(SIPDG_EHIP, "stream wait (join)");
        }
        return SIPDG_OK;
    }
    if (c->variant != SIPDG_VARIANT_GATHER) {
        const bool fused = c->variant == SIPDG_VARIANT_FUSED;
        if ((stages & 1) && !fused) {
            for (size_t gi = 0; gi < c->groups.size(); ++gi) {
                const Group &g = c->groups[gi];
                f3::Args3 A;
                f3::Data3<R> D;
                fast_args<R>(c, g, x, y, tbuf, skip, false, A, D);
                rec_mark(rec, 1, (int)gi, false, st);
                hipError_t e = launch_fast3d<R>(g.P, 0, A, D, st);
                rec_mark(rec, 1, (int)gi, true, st);
                if (e != hipSuccess) return fail(SIPDG_EHIP, std::string("trace kernel: ") + hipGetErrorString(e));
            }
        }
        if (stages & 2) {
            for (size_t gi = 0; gi < c->groups.size(); ++gi) {
                const Group &g = c->groups[gi];
                f3::Args3 A;
                f3::Data3<R> D;
                fast_args<R>(c, g, x, y, tbuf, skip, fused, A, D);
                rec_mark(rec, 2, (int)gi, false, st);
                hipError_t e = launch_fast3d<R>(g.P, fused ? 2 : 1, A, D, st);
                rec_mark(rec, 2, (int)gi, true, st);
                if (e != hipSuccess) return fail(SIPDG_EHIP, std::string("apply kernel: ") + hipGetErrorString(e));
            }
        }
        return SIPDG_OK;
    }
    if (stages & 1) {
        for (size_t gi = 0; gi < c->groups.size(); ++gi) {
            const Group &g = c->groups[gi];
            OpArgs<R> A = make_args<R>(c, g, x, y, tbuf, skip);
            rec_mark(rec, 1, (int)gi, false, st);
            hipError_t e = launch_op<R>(c->dim, g.P, OP_TRACE, A, g.nfmax, st);
            rec_mark(rec, 1, (int)gi, true, st);
            if (e != hipSuccess) return fail(SIPDG_EHIP, std::string("trace kernel: ") + hipGetErrorString(e));
        }
    }
    if (stages & 2) {
        for (size_t gi = 0; gi < c->groups.size(); ++gi) {
            const Group &g = c->groups[gi];
            OpArgs<R> A = make_args<R>(c, g, x, y, tbuf, skip);
            rec_mark(rec, 2, (int)gi, false, st);
            hipError_t e = launch_op<R>(c->dim, g.P, OP_APPLY, A, g.nfmax, st);
            rec_mark(rec, 2, (int)gi, true, st);
            if (e != hipSuccess) return fail(SIPDG_EHIP, std::string("apply kernel: ") + hipGetErrorString(e));
        }
    }
    return SIPDG_OK;
}
template int apply_impl<double>(sipdg_ctx *, const double *, double *, double *, const int *, hipStream_t, int,
                                LaunchRec *, const CgFold<double> *);
template int apply_impl<float>(sipdg_ctx *, const float *, float *, float *, const int *, hipStream_t, int,
                               LaunchRec *, const CgFold<float> *);

int refresh_diag(sipdg_ctx *c, hipStream_t st) {
    for (const Group &g : c->groups) {
        hipError_t e = launch_diag(c->dim, g.P, g.count, g.d_elems, c->d_xoff, c->d_voff, c->d_eface, c->d_foff,
                                   c->d_vgeo64, c->d_fgeo64, c->d_lam64, c->d_tau64, c->d_tab64, c->d_diag64, st);
        if (e != hipSuccess) return fail(SIPDG_EHIP, std::string("diag kernel: ") + hipGetErrorString(e));
    }
    hipError_t e = launch_recip(c->d_diag64, c->d_dinv64, c->d_dinv32, c->ndof, st);
    if (e != hipSuccess) return fail(SIPDG_EHIP, std::string("recip kernel: ") + hipGetErrorString(e));
    return SIPDG_OK;
}

static int upload_tau(sipdg_ctx *c) {
    std::vector<double> tau(c->nfaces);
    for (int64_t F = 0; F < c->nfaces; ++F) tau[F] = c->sigma[c->face_prob[F]] * c->tau0[F];
    if (c->nfaces) HIPCHK(hipMemcpy(c->d_tau64, tau.data(), sizeof(double) * c->nfaces, hipMemcpyHostToDevice));
    hipError_t e = launch_cast_f32(c->d_tau64, c->d_tau32, c->nfaces, 0);
    if (e != hipSuccess) return fail(SIPDG_EHIP, hipGetErrorString(e));
    return SIPDG_OK;
}

}  // namespace sipdg

static void free_ctx(sipdg_ctx *c) {
    if (!c) return;
    void *ptrs[] = {c->d_xoff, c->d_voff, c->d_foff, c->d_toff, c->d_qoff, c->d_boff,
                    c->d_prob_elem_off, c->d_prob_face_off, c->d_prob_dof_off, c->d_eface,
                    c->d_faces, c->d_order, c->d_is_interior, c->d_face_nf, c->d_flag,
                    c->d_corners, c->d_tab64, c->d_tab32, c->d_vgeo64, c->d_fgeo64, c->d_lam64,
                    c->d_tau64, c->d_vgeo32, c->d_fgeo32, c->d_lam32, c->d_tau32, c->d_tau0,
                    c->d_tbuf, c->d_tbuf2, c->d_face_tmp, c->d_elem_tmp, c->d_diag64,
                    c->d_dinv64, c->d_dinv32, c->d_egeo64, c->d_egeo32, c->d_emap64, c->d_emap32,
                    c->d_tbuf_p2p, c->d_p2p_side, c->d_fgeo_p2p64, c->d_fgeo_p2p32, c->d_w2desc, c->d_w2fdesc, c->d_w2nb, c->d_eprob,
                    c->d_pfdesc_p2p, c->d_tabgl64, c->d_tabgl32};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (c->d_pdesc) (void)hipFree(c->d_pdesc);
    if (c->d_pfdesc) (void)hipFree(c->d_pfdesc);
    if (c->aff_stream) (void)hipStreamDestroy(c->aff_stream);
    for (hipEvent_t ev : c->aff_ev)
        if (ev) (void)hipEventDestroy(ev);
    for (hipStream_t sg : c->gstreams)
        if (sg) (void)hipStreamDestroy(sg);
    for (hipEvent_t ev : c->gevents)
        if (ev) (void)hipEventDestroy(ev);
    for (Group &g : c->groups) {
        if (g.d_elems) (void)hipFree(g.d_elems);
        if (g.d_desc) (void)hipFree(g.d_desc);
        if (g.d_fdesc) (void)hipFree(g.d_fdesc);
        if (g.d_fdesc_p2p) (void)hipFree(g.d_fdesc_p2p);
    }
    free_cg(c);
    delete c;
}

// FNV-1a over the mesh: dimension, problem count, element counts, orders,
// corner coordinates (bit patterns) and face count.  Keys the autotuner's
// cache: the same meshes give the same signature.
static uint64_t mesh_signature(const Topology &T) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](const void *p, size_t n) {
        const unsigned char *b = (const unsigned char *)p;
        for (size_t i = 0; i < n; ++i) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    };
    mix(&T.dim, sizeof(T.dim));
    mix(&T.nprob, sizeof(T.nprob));
    mix(T.prob_elem_off.data(), sizeof(int64_t) * T.prob_elem_off.size());
    mix(T.order.data(), sizeof(int) * T.order.size());
    mix(T.corners.data(), sizeof(double) * T.corners.size());
    mix(&T.nfaces, sizeof(T.nfaces));
    return h;
}

static int create_impl(int nprob, const sipdg_mesh_desc *descs, sipdg_handle *out) {
    if (!out) return fail(SIPDG_EINVAL, "null output handle");
    *out = nullptr;
    Topology T;
    std::string err;
    int rc = build_topology(nprob, descs, T, err);
    if (rc) return fail(rc, err);

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return fail(SIPDG_EHIP, "no HIP device available");
    }
    sipdg_ctx *c = new sipdg_ctx();
    (void)hipGetDevice(&c->device);
    c->dim = T.dim;
    c->nprob = T.nprob;
    c->ne = T.ne;
    c->ndof = T.ndof;
    c->nfaces = T.nfaces;
    c->nvq = T.qoff[T.ne];
    c->nbq = T.boff[T.ne];
    c->vgeo_len = T.vgeo_len;
    c->fgeo_len = T.fgeo_len;
    c->tbuf_len = T.tbuf_len;
    c->order = T.order;
    c->xoff = T.xoff;
    c->prob_dof_off = T.prob_dof_off;
    c->prob_elem_off = T.prob_elem_off;
    c->prob_face_off = T.prob_face_off;
    c->tau0 = T.tau0;
    c->sigma = T.sigma;
    c->face_prob = T.face_prob;

#define TRY(x)                 \
    do {                       \
        int _r = (x);          \
        if (_r) {              \
            free_ctx(c);       \
            return _r;         \
        }                      \
    } while (0)
#define TRYHIP(x)                                                                        \
    do {                                                                                 \
        hipError_t _e = (x);                                                             \
        if (_e != hipSuccess) {                                                          \
            free_ctx(c);                                                                 \
            return fail(SIPDG_EHIP, std::string(#x) + ": " + hipGetErrorString(_e));     \
        }                                                                                \
    } while (0)

    TRY(upload(&c->d_xoff, T.xoff));
    TRY(upload(&c->d_voff, T.voff));
    TRY(upload(&c->d_foff, T.foff));
    TRY(upload(&c->d_toff, T.toff));
    TRY(upload(&c->d_qoff, T.qoff));
    TRY(upload(&c->d_boff, T.boff));
    TRY(upload(&c->d_prob_elem_off, T.prob_elem_off));
    TRY(upload(&c->d_prob_face_off, T.prob_face_off));
    TRY(upload(&c->d_prob_dof_off, T.prob_dof_off));
    TRY(upload(&c->d_eface, T.eface));
    TRY(upload(&c->d_faces, T.faces));
    TRY(upload(&c->d_order, T.order));
    TRY(upload(&c->d_corners, T.corners));
    // affine (parallelepiped) elements: G~ and |J| are constant over the element
    // (the paper's regular-element specialisation); the gather-fold apply then
    // reads 7 values per element instead of 7 per point
    std::vector<int> affine(T.ne, 0);
    {
        std::vector<double> eg((size_t)std::max<int64_t>(T.ne, 1) * 8, 0.0);
        const char *off = std::getenv("SIPDG_NO_AFFINE");
        if (T.dim == 3 && !(off && off[0] == '1')) {
            for (int64_t e = 0; e < T.ne; ++e) {
                const double *X = &T.corners[(size_t)e * 24];
                double E[3][3], diam = 0.0, xmax = 0.0;
                for (int k = 0; k < 3; ++k) {
                    double n2 = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        E[k][a] = X[(1 << k) * 3 + a] - X[a];
                        n2 += E[k][a] * E[k][a];
                    }
                    diam = std::max(diam, std::sqrt(n2));
                }
                for (int i = 0; i < 24; ++i) xmax = std::max(xmax, std::fabs(X[i]));
                // a parallelepiped up to the rounding of the corner coordinates:
                // the constant Jacobian then differs from the per-point one by
                // about tol / edge, far below the FP64 parity bar
                const double tol = 1e-14 * diam + 16.0 * DBL_EPSILON * xmax;
                bool ok = diam > 0.0;
                for (int v = 0; v < 8 && ok; ++v)
                    for (int a = 0; a < 3; ++a) {
                        double pred = X[a];
                        for (int k = 0; k < 3; ++k)
                            if ((v >> k) & 1) pred += E[k][a];
                        if (std::fabs(X[v * 3 + a] - pred) > tol) ok = false;
                    }
                if (!ok) continue;
                double J[3][3], A[3][3];
                for (int a = 0; a < 3; ++a)
                    for (int k = 0; k < 3; ++k) J[a][k] = 0.5 * E[k][a];
                A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
                A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
                A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
                A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
                A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
                A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
                A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
                A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
                A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
                const double det = J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
                if (!(det > 0.0)) continue;
                int cidx = 0;
                for (int a = 0; a < 3; ++a)
                    for (int b = a; b < 3; ++b) {
                        double t = 0.0;
                        for (int cc = 0; cc < 3; ++cc) t += A[a][cc] * A[b][cc];
                        eg[(size_t)e * 8 + cidx++] = t / det;
                    }
                eg[(size_t)e * 8 + 6] = det;
                affine[e] = 1;
            }
        }
        TRY(upload(&c->d_egeo64, eg));
        TRY(dalloc(&c->d_egeo32, (int64_t)eg.size()));
        TRYHIP(launch_cast_f32(c->d_egeo64, c->d_egeo32, (int64_t)eg.size(), 0));
    }
    // trilinear map per element: x(xi) = sum_S c_S prod_{k in S} xi_k with
    // c_S = 1/8 sum_v X_v prod_{k in S} s_k(v), s_k(v) = +1 if bit k of v else -1;
    // stored c1..c7 = S {0}, {1}, {2}, {0,1}, {0,2}, {1,2}, {0,1,2}
    if (T.dim == 3) {
        static const int SUB[7] = {1, 2, 4, 3, 5, 6, 7};   // bit masks of S
        std::vector<double> cm((size_t)std::max<int64_t>(T.ne, 1) * 24, 0.0);
        for (int64_t e = 0; e < T.ne; ++e) {
            const double *X = &T.corners[(size_t)e * 24];
            for (int i = 0; i < 7; ++i)
                for (int a = 0; a < 3; ++a) {
                    double t = 0.0;
                    for (int v = 0; v < 8; ++v) {
                        const int neg = __builtin_popcount(SUB[i] & ~v & 7) & 1;
                        t += neg ? -X[v * 3 + a] : X[v * 3 + a];
                    }
                    cm[(size_t)e * 24 + 3 * i + a] = 0.125 * t;
                }
        }
        TRY(upload(&c->d_emap64, cm));
        TRY(dalloc(&c->d_emap32, (int64_t)cm.size()));
        TRYHIP(launch_cast_f32(c->d_emap64, c->d_emap32, (int64_t)cm.size(), 0));
    }
    TRY(upload(&c->d_tau0, T.tau0));
    {
        std::vector<int> interior(T.nfaces), nf(T.nfaces);
        for (int64_t F = 0; F < T.nfaces; ++F) {
            interior[F] = T.faces[F].eR >= 0;
            nf[F] = T.faces[F].nf;
        }
        TRY(upload(&c->d_is_interior, interior));
        TRY(upload(&c->d_face_nf, nf));
    }
    {
        std::vector<double> tab(TAB_SIZE);
        build_tables(tab.data());
        TRY(upload(&c->d_tab64, tab));
        TRY(dalloc(&c->d_tab32, TAB_SIZE));
        TRYHIP(launch_cast_f32(c->d_tab64, c->d_tab32, TAB_SIZE, 0));
        build_tables(tab.data(), 0, true);
        TRY(upload(&c->d_tabgl64, tab));
        TRY(dalloc(&c->d_tabgl32, TAB_SIZE));
        TRYHIP(launch_cast_f32(c->d_tabgl64, c->d_tabgl32, TAB_SIZE, 0));
    }
    TRY(dalloc(&c->d_flag, 1));
    TRYHIP(hipMemset(c->d_flag, 0, sizeof(int)));
    TRY(dalloc(&c->d_vgeo64, T.vgeo_len));
    TRY(dalloc(&c->d_fgeo64, T.fgeo_len));
    TRY(dalloc(&c->d_vgeo32, T.vgeo_len));
    TRY(dalloc(&c->d_fgeo32, T.fgeo_len));
    TRYHIP(launch_geo_volume(c->dim, c->ne, c->d_corners, c->d_order, c->d_voff, c->d_tab64, c->d_vgeo64, c->d_flag, 0));
    TRYHIP(launch_geo_faces(c->dim, c->nfaces, c->d_corners, c->d_faces, c->d_foff, c->d_tab64, c->d_fgeo64, c->d_flag, 0));
    TRYHIP(launch_cast_f32(c->d_vgeo64, c->d_vgeo32, T.vgeo_len, 0));
    TRYHIP(launch_cast_f32(c->d_fgeo64, c->d_fgeo32, T.fgeo_len, 0));
    int flag = 0;
    TRYHIP(hipMemcpy(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost));
    if (flag) {
        free_ctx(c);
        return fail(SIPDG_EMESH, "non-positive Jacobian at a quadrature point");
    }
    TRY(upload(&c->d_lam64, T.lambda));
    TRY(dalloc(&c->d_lam32, T.ne));
    TRYHIP(launch_cast_f32(c->d_lam64, c->d_lam32, T.ne, 0));
    TRY(dalloc(&c->d_tau64, T.nfaces));
    TRY(dalloc(&c->d_tau32, T.nfaces));
    TRY(upload_tau(c));
    TRY(dalloc(&c->d_tbuf, T.tbuf_len));

    // order groups, each with the largest trace that touches it
    for (int P = 1; P <= PMAX; ++P) {
        std::vector<int> ids;
        int nfmax = P + 2;
        for (int64_t e = 0; e < T.ne; ++e) {
            if (T.order[e] != P) continue;
            ids.push_back((int)e);
            for (int f = 0; f < 2 * T.dim; ++f) nfmax = std::max(nfmax, face_nf(T.eface[(size_t)e * 2 * T.dim + f].info));
        }
        if (ids.empty()) continue;
        Group g;
        g.P = P;
        g.count = (int)ids.size();
        g.nfmax = nfmax;
        g.d_elems = nullptr;
        TRY(upload(&g.d_elems, ids));
        {
            const int d = T.dim, nlf = 2 * d;
            const int npts = d == 3 ? (P + 2) * (P + 2) * (P + 2) : (P + 2) * (P + 2);
            const int nm = d == 3 ? (P + 1) * (P + 1) * (P + 1) : (P + 1) * (P + 1);
            for (int w = 0; w < 2; ++w) {
                const double wb = w == 0 ? 8.0 : 4.0;
                double sum = 0;
                for (int e : ids) {
                    // geometry: per-point factors, or 7 constants of an affine element
                    const double ng = affine[e] ? 7.0 : (double)npts * (d * (d + 1) / 2 + 1);
                    sum += wb * (2.0 * nm + ng + 1);
                    for (int f = 0; f < nlf; ++f) {
                        const FaceRef fr = T.eface[(size_t)e * nlf + f];
                        const int nf = face_nf(fr.info);
                        const double npf = d == 3 ? nf * nf : nf;
                        if (face_slot(fr.info) == 2) sum += wb * (d + 1) * npf + 32.0;
                        else sum += 0.5 * (wb * (2 * d + 1) * npf + 32.0);
                    }
                }
                g.alg_bytes[w] = sum;
            }
        }
        c->groups.push_back(g);
        if (T.dim == 3) {
            // groups at least half affine: affine elements first in the
            // descriptors (an apply launch of their own).  Below half, two
            // half-filled launches cost more than the affine part saves
            // (measured on 32^3 meshes, orders 3-6): the group keeps element
            // order and reads per-point factors.
            int naff = 0;
            for (int e : ids) naff += affine[e];
            const bool split = naff > 0 && 2 * naff >= (int)ids.size();
            std::vector<int> ord(ids);
            if (split) std::stable_partition(ord.begin(), ord.end(), [&](int e) { return affine[e] != 0; });
            c->groups.back().naff = naff;
            c->groups.back().split = split;
            std::vector<ElemDesc> desc(ids.size());
            std::vector<FaceDesc> fdesc(ids.size() * 6);
            for (size_t i = 0; i < ord.size(); ++i) {
                const int64_t e = ord[i];
                desc[i] = ElemDesc{T.xoff[e], T.voff[e], (int)e, affine[e] ? ELEM_AFFINE : 0};
                for (int f = 0; f < 6; ++f) {
                    const FaceRef fr = T.eface[(size_t)e * 6 + f];
                    fdesc[i * 6 + f] = FaceDesc{T.foff[fr.F], T.toff[fr.F], fr.F, fr.info};
                }
            }
            TRY(upload(&c->groups.back().d_desc, desc));
            TRY(upload(&c->groups.back().d_fdesc, fdesc));
        }
        // check the block fits in LDS
        hipDeviceProp_t prop;
        TRYHIP(hipGetDeviceProperties(&prop, c->device));
        size_t need = lds_for(T.dim, P, work_size_for(T.dim, P, nfmax), true, sizeof(double));
        size_t limit = prop.sharedMemPerBlock;
        if (prop.maxSharedMemoryPerMultiProcessor > limit) limit = prop.maxSharedMemoryPerMultiProcessor;
        if (need > limit) {
            free_ctx(c);
            return fail(SIPDG_EINVAL, "order " + std::to_string(P) + " needs " + std::to_string(need) +
                                          " bytes of LDS per block, device allows " + std::to_string(limit));
        }
    }
    {
        int pmax = 0;
        for (int o : T.order) pmax = std::max(pmax, o);
        if (T.dim == 2) {
            // the 2-D wavefront list: elements of order <= 6 whose faces have
            // at most 8 trace points, by decreasing order
            std::vector<ElemDesc> wd;
            std::vector<FaceDesc> wf;
            std::vector<NbDesc2> wn;
            for (int P = 6; P >= 1; --P) {
                for (int64_t e = 0; e < T.ne; ++e) {
                    if (T.order[e] != P) continue;
                    int nfm = 0;
                    for (int f = 0; f < 4; ++f) nfm = std::max(nfm, face_nf(T.eface[(size_t)e * 4 + f].info));
                    if (nfm > 8) continue;
                    wd.push_back(ElemDesc{T.xoff[e], T.voff[e], (int)e, P});
                    for (int f = 0; f < 4; ++f) {
                        const FaceRef fr = T.eface[(size_t)e * 4 + f];
                        wf.push_back(FaceDesc{T.foff[fr.F], T.toff[fr.F], fr.F, fr.info});
                        NbDesc2 nd{0, 0, 0};
                        const int slot = face_slot(fr.info);
                        if (slot != 2) {
                            const FaceTopo &ft = T.faces[fr.F];
                            const int nb = slot == 0 ? ft.eR : ft.eL;
                            const int fn = slot == 0 ? ft.fR : ft.fL;
                            const int on = slot == 0 ? ft.orient : 0;
                            nd.xn = T.xoff[nb];
                            nd.code = (T.order[nb] + 1) | (fn << 4) | (on << 6);
                        }
                        wn.push_back(nd);
                    }
                }
            }
            c->w2count = (int)wd.size();
            if (!wd.empty()) {
                TRY(upload(&c->d_w2desc, wd));
                TRY(upload(&c->d_w2fdesc, wf));
                TRY(upload(&c->d_w2nb, wn));
            }
        }
        if (T.dim == 3) {
            std::vector<ElemDesc> pd;
            std::vector<FaceDesc> pf;
            for (int P = 6; P >= 1; --P) {
                for (const Group &g : c->groups) {
                    if (g.P != P || g.nfmax > 8) continue;
                    const size_t base = pd.size();
                    pd.resize(base + g.count);
                    pf.resize((base + g.count) * 6);
                    TRYHIP(hipMemcpy(pd.data() + base, g.d_desc, sizeof(ElemDesc) * g.count, hipMemcpyDeviceToHost));
                    TRYHIP(hipMemcpy(pf.data() + base * 6, g.d_fdesc, sizeof(FaceDesc) * 6 * g.count,
                                     hipMemcpyDeviceToHost));
                    for (int i = 0; i < g.count; ++i) pd[base + i].pad |= P;   // keeps ELEM_AFFINE
                }
            }
            c->pcount = (int)pd.size();
            if (!pd.empty()) {
                TRY(upload(&c->d_pdesc, pd));
                TRY(upload(&c->d_pfdesc, pf));
            }
            hipDeviceProp_t prop;
            TRYHIP(hipGetDeviceProperties(&prop, c->device));
            c->num_cu = prop.multiProcessorCount;
        }
        bool part_affine = false;
        for (const Group &g : c->groups) part_affine |= g.split && g.naff < g.count;
        if (part_affine) {
            TRYHIP(hipStreamCreateWithFlags(&c->aff_stream, hipStreamNonBlocking));
            for (auto &ev : c->aff_ev) TRYHIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        }
        if (c->groups.size() > 1) {
            c->gstreams.assign(c->groups.size(), nullptr);
            c->gevents.assign(c->groups.size() + 1, nullptr);
            for (auto &sg : c->gstreams) TRYHIP(hipStreamCreateWithFlags(&sg, hipStreamNonBlocking));
            for (auto &ev : c->gevents) TRYHIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        }
        // opt-in: concurrent order groups (FP64 only) shorten an application
        // by a few per cent, but make the launches share the GPU, so that one
        // launch's duration is no longer its own
        const char *conc = std::getenv("SIPDG_CONCURRENT");
        if (conc && conc[0] == '1') c->concurrent = true;
        c->fast_ok = T.dim == 3 && pmax <= 6;
        c->gfold_ok = T.dim == 3;
        c->fast_ok0 = c->fast_ok;
        c->gfold_ok0 = c->gfold_ok;
        c->variant = default_variant(c);
        const char *env = std::getenv("SIPDG_VARIANT");
        if (env && c->gfold_ok) {
            std::string v(env);
            if (v == "gather") c->variant = SIPDG_VARIANT_GATHER;
            else if (v == "two_stage") c->variant = SIPDG_VARIANT_TWO_STAGE;
            else if (v == "fused") c->variant = SIPDG_VARIANT_FUSED;
            else if (v == "gather_fold") c->variant = SIPDG_VARIANT_GATHER_FOLD;
            else if (v == "gather_fold_fused") c->variant = SIPDG_VARIANT_GATHER_FOLD_FUSED;
            if (!c->fast_ok && c->variant != SIPDG_VARIANT_GATHER_FOLD) c->variant = SIPDG_VARIANT_GATHER;
        }
    }
    TRY(dalloc(&c->d_diag64, T.ndof));
    TRY(dalloc(&c->d_dinv64, T.ndof));
    TRY(dalloc(&c->d_dinv32, T.ndof));
    // every buffer a later call uses, now: the parameter gradients' second
    // trace buffer and per-face / per-element partial sums, and the CG work
    // vectors (also the autotuner's timing vectors)
    TRY(dalloc(&c->d_tbuf2, std::max<int64_t>(1, c->tbuf_len)));
    TRY(dalloc(&c->d_face_tmp, std::max<int64_t>(1, c->nfaces)));
    TRY(dalloc(&c->d_elem_tmp, std::max<int64_t>(1, c->ne)));
    TRY(alloc_cg(c));
    {
        // element -> problem (the folded CG step reads its problem's scalars)
        std::vector<int> ep(std::max<int64_t>(1, c->ne), 0);
        for (int p = 0; p < c->nprob; ++p)
            for (int64_t e = c->prob_elem_off[p]; e < c->prob_elem_off[p + 1]; ++e) ep[e] = p;
        TRY(upload(&c->d_eprob, ep));
    }
    // the allocation-free apply's scratch address on this device
    TRY(noalloc_setup(c->device));
    c->signature = mesh_signature(T);
    TRY(refresh_diag(c, 0));
    TRYHIP(hipDeviceSynchronize());
    if (descs[0].basis == SIPDG_BASIS_MODAL) TRY(sipdg_set_basis(c, SIPDG_BASIS_MODAL));
#undef TRY
#undef TRYHIP
    *out = c;
    return SIPDG_OK;
}

namespace {

// ---------------------------------------------------------------- autotuner cache

#ifndef SIPDG_SOURCE_HASH
#define SIPDG_SOURCE_HASH "unversioned"
#endif

struct TuneRec {
    int variant = 0, blocks_per_cu = 8;
    int tile[SIPDG_MAX_ORDER + 1] = {1, 1, 1, 1, 1, 1, 1, 1, 1};
    int budget[SIPDG_MAX_ORDER + 1] = {2, 2, 2, 2, 2, 2, 2, 2, 2};
    double ms[SIPDG_NUM_VARIANTS] = {0, 0, 0, 0, 0, 0};
};

std::string tune_key(const sipdg_ctx *h) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch.resize(colon);
        cus = prop.multiProcessorCount;
    }
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%016llx-%s-%s-%d", (unsigned long long)h->signature, SIPDG_SOURCE_HASH,
                  arch.c_str(), cus);
    return buf;
}

// integers / doubles of the JSON array after `name` on one record line
template <class T>
bool json_array(const std::string &line, const char *name, T *vals, int n) {
    size_t p = line.find(name);
    if (p == std::string::npos) return false;
    p = line.find('[', p);
    if (p == std::string::npos) return false;
    const char *c = line.c_str() + p + 1;
    for (int i = 0; i < n; ++i) {
        char *end = nullptr;
        const double v = std::strtod(c, &end);
        if (end == c) return false;
        vals[i] = (T)v;
        c = end;
        while (*c == ' ' || *c == ',') ++c;
    }
    return true;
}

bool json_int(const std::string &line, const char *name, int &v) {
    size_t p = line.find(name);
    if (p == std::string::npos) return false;
    p = line.find(':', p);
    if (p == std::string::npos) return false;
    char *end = nullptr;
    const long x = std::strtol(line.c_str() + p + 1, &end, 10);
    if (end == line.c_str() + p + 1) return false;
    v = (int)x;
    return true;
}

// the cache file: a JSON object, one record per line
//   "<key>": {"variant": V, "blocks_per_cu": B, "tile": [9], "budget": [9], "ms": [6]}
std::vector<std::pair<std::string, std::string>> cache_records(const char *path) {
    std::vector<std::pair<std::string, std::string>> out;
    std::FILE *f = std::fopen(path, "r");
    if (!f) return out;
    std::string line;
    int ch;
    auto flush = [&]() {
        size_t a = line.find('"');
        if (a != std::string::npos && line.find("\"variant\"") != std::string::npos) {
            const size_t b = line.find('"', a + 1);
            if (b != std::string::npos) {
                std::string rec = line;
                while (!rec.empty() && (rec.back() == ',' || rec.back() == ' ' || rec.back() == '\r')) rec.pop_back();
                out.emplace_back(line.substr(a + 1, b - a - 1), rec);
            }
        }
        line.clear();
    };
    while ((ch = std::fgetc(f)) != EOF) {
        if (ch == '\n') flush();
        else line.push_back((char)ch);
    }
    flush();
    std::fclose(f);
    return out;
}

bool cache_lookup(const char *path, const std::string &key, TuneRec &r) {
    for (const auto &kv : cache_records(path)) {
        if (kv.first != key) continue;
        const std::string &l = kv.second;
        TuneRec t;
        if (!json_int(l, "\"variant\"", t.variant) || !json_int(l, "\"blocks_per_cu\"", t.blocks_per_cu) ||
            !json_array(l, "\"tile\"", t.tile, SIPDG_MAX_ORDER + 1) ||
            !json_array(l, "\"budget\"", t.budget, SIPDG_MAX_ORDER + 1) ||
            !json_array(l, "\"ms\"", t.ms, SIPDG_NUM_VARIANTS))
            return false;
        r = t;
        return true;
    }
    return false;
}

void cache_store(const char *path, const std::string &key, const TuneRec &r) {
    auto recs = cache_records(path);
    std::string line = "\"" + key + "\": {\"variant\": " + std::to_string(r.variant) +
                       ", \"blocks_per_cu\": " + std::to_string(r.blocks_per_cu) + ", \"tile\": [";
    for (int P = 0; P <= SIPDG_MAX_ORDER; ++P) line += (P ? ", " : "") + std::to_string(r.tile[P]);
    line += "], \"budget\": [";
    for (int P = 0; P <= SIPDG_MAX_ORDER; ++P) line += (P ? ", " : "") + std::to_string(r.budget[P]);
    line += "], \"ms\": [";
    for (int v = 0; v < SIPDG_NUM_VARIANTS; ++v) {
        char b[64];
        std::snprintf(b, sizeof(b), "%s%.6g", v ? ", " : "", r.ms[v]);
        line += b;
    }
    line += "]}";
    bool found = false;
    for (auto &kv : recs)
        if (kv.first == key) {
            kv.second = line;
            found = true;
        }
    if (!found) recs.emplace_back(key, line);
    const std::string tmp = std::string(path) + ".tmp";
    std::FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fputs("{\n", f);
    for (size_t i = 0; i < recs.size(); ++i) {
        std::fputs(recs[i].second.c_str(), f);
        std::fputs(i + 1 < recs.size() ? ",\n" : "\n", f);
    }
    std::fputs("}\n", f);
    const bool ok = std::fclose(f) == 0;
    if (ok) (void)std::rename(tmp.c_str(), path);
    else (void)std::remove(tmp.c_str());
}

// a cached tuning, if this build and mesh allow every part of it
int apply_tuning(sipdg_ctx *h, const TuneRec &r) {
    for (int P = 1; P <= SIPDG_MAX_ORDER; ++P) {
        bool ok = false;
        for (const TileShape &ts : tile_shapes(P)) ok |= ts.tile == r.tile[P] && ts.budget == r.budget[P];
        if (!ok) return SIPDG_EINVAL;
    }
    if (r.blocks_per_cu < 1 || r.blocks_per_cu > 64) return SIPDG_EINVAL;
    const int keep = h->variant;
    if (sipdg_set_variant(h, r.variant) != SIPDG_OK) {
        h->variant = keep;
        return SIPDG_EINVAL;
    }
    h->blocks_per_cu = r.blocks_per_cu;
    for (int P = 0; P <= SIPDG_MAX_ORDER; ++P) {
        h->tile[P] = r.tile[P];
        h->budget[P] = r.budget[P];
    }
    return SIPDG_OK;
}

}  // namespace

extern "C" {

int sipdg_create(const sipdg_mesh_desc *desc, sipdg_handle *out) {
    if (!desc) return fail(SIPDG_EINVAL, "null mesh description");
    return create_impl(1, desc, out);
}

int sipdg_create_batch(int n_problems, const sipdg_mesh_desc *descs, sipdg_handle *out) {
    if (n_problems <= 0 || !descs) return fail(SIPDG_EINVAL, "need at least one problem");
    return create_impl(n_problems, descs, out);
}

void sipdg_destroy(sipdg_handle h) {
    if (h) {
        (void)hipDeviceSynchronize();
        free_ctx(h);
    }
}

int sipdg_mesh_inspect(const sipdg_mesh_desc *desc, sipdg_mesh_stats *st) {
    if (!desc || !st) return fail(SIPDG_EINVAL, "null argument");
    Topology T;
    std::string err;
    int rc = build_topology(1, desc, T, err);
    if (rc) return fail(rc, err);
    std::memset(st, 0, sizeof(*st));
    st->n_elems = T.ne;
    st->n_dofs = T.ndof;
    st->n_interior_faces = T.n_interior;
    st->n_boundary_faces = T.n_boundary;
    st->n_nonconforming_faces = T.n_nonconf;
    for (int o = 0; o < 8; ++o) st->orientation_count[o] = T.orient_count[o];
    st->n_volume_points = T.qoff[T.ne];
    st->n_trace_points = T.n_trace_points;
    st->n_interior_trace_points = T.n_int_trace_points;
    st->n_boundary_trace_points = T.n_bnd_trace_points;
    for (int64_t e = 0; e < T.ne; ++e) st->elems_per_order[T.order[e]]++;
    return SIPDG_OK;
}

int sipdg_num_dofs(sipdg_handle h, int64_t *n) {
    if (!h || !n) return fail(SIPDG_EINVAL, "null argument");
    *n = h->ndof;
    return SIPDG_OK;
}

int sipdg_num_elems(sipdg_handle h, int64_t *n) {
    if (!h || !n) return fail(SIPDG_EINVAL, "null argument");
    *n = h->ne;
    return SIPDG_OK;
}

int sipdg_num_problems(sipdg_handle h, int *n) {
    if (!h || !n) return fail(SIPDG_EINVAL, "null argument");
    *n = h->nprob;
    return SIPDG_OK;
}

int sipdg_elem_offsets(sipdg_handle h, int64_t *off) {
    if (!h || !off) return fail(SIPDG_EINVAL, "null argument");
    std::memcpy(off, h->xoff.data(), sizeof(int64_t) * (h->ne + 1));
    return SIPDG_OK;
}

int sipdg_problem_offsets(sipdg_handle h, int64_t *dof_off, int64_t *elem_off) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (dof_off) std::memcpy(dof_off, h->prob_dof_off.data(), sizeof(int64_t) * (h->nprob + 1));
    if (elem_off) std::memcpy(elem_off, h->prob_elem_off.data(), sizeof(int64_t) * (h->nprob + 1));
    return SIPDG_OK;
}

int sipdg_apply(sipdg_handle h, const void *x, void *y, int precision, void *stream) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (h->ndof == 0) return SIPDG_OK;   // empty mesh: nothing to do
    if (!x || !y) return fail(SIPDG_EINVAL, "null argument");
    if (x == y) return fail(SIPDG_EINVAL, "x and y must not alias");
    hipStream_t st = (hipStream_t)stream;
    if (precision == SIPDG_F64)
        return apply_impl<double>(h, (const double *)x, (double *)y, h->d_tbuf, nullptr, st);
    if (precision == SIPDG_F32)
        return apply_impl<float>(h, (const float *)x, (float *)y, (float *)h->d_tbuf, nullptr, st);
    return fail(SIPDG_EINVAL, "precision must be SIPDG_F64 or SIPDG_F32");
}

int sipdg_apply_stage(sipdg_handle h, const void *x, void *y, int precision, int stage, void *stream) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (stage != 1 && stage != 2) return fail(SIPDG_EINVAL, "stage must be 1 or 2");
    if (h->ndof == 0) return SIPDG_OK;
    if (!x || (stage == 2 && !y)) return fail(SIPDG_EINVAL, "null argument");
    if (x == y) return fail(SIPDG_EINVAL, "x and y must not alias");
    hipStream_t st = (hipStream_t)stream;
    if (precision == SIPDG_F64)
        return apply_impl<double>(h, (const double *)x, (double *)y, h->d_tbuf, nullptr, st, stage);
    if (precision == SIPDG_F32)
        return apply_impl<float>(h, (const float *)x, (float *)y, (float *)h->d_tbuf, nullptr, st, stage);
    return fail(SIPDG_EINVAL, "precision must be SIPDG_F64 or SIPDG_F32");
}

int sipdg_apply_timed(sipdg_handle h, const void *x, void *y, int precision, int reps,
                      sipdg_launch_info *info, int max_launches, int *n_launches, void *stream) {
    if (!h || !info || !n_launches) return fail(SIPDG_EINVAL, "null argument");
    if (precision != SIPDG_F64 && precision != SIPDG_F32)
        return fail(SIPDG_EINVAL, "precision must be SIPDG_F64 or SIPDG_F32");
    if (h->ndof == 0) {   // empty mesh: no launches
        *n_launches = 0;
        return SIPDG_OK;
    }
    if (!x || !y) return fail(SIPDG_EINVAL, "null argument");
    if (x == y) return fail(SIPDG_EINVAL, "x and y must not alias");
    if (reps <= 0) reps = 1;
    hipStream_t st = (hipStream_t)stream;
    const int per = 2 * (int)h->groups.size() + 1;   // launches of one application, at most
    if (per > 64) return fail(SIPDG_EINVAL, "too many order groups");
    std::vector<hipEvent_t> ev((size_t)2 * per * reps, nullptr);
    int rc = SIPDG_OK;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) rc = fail(SIPDG_EHIP, "event create");
    std::vector<LaunchRec> recs(reps);
    for (int r = 0; r < reps && rc == SIPDG_OK; ++r) {
        recs[r].ev = ev.data() + (size_t)2 * per * r;
        recs[r].cap = per;
        rc = precision == SIPDG_F64
                 ? apply_impl<double>(h, (const double *)x, (double *)y, h->d_tbuf, nullptr, st, 3, &recs[r])
                 : apply_impl<float>(h, (const float *)x, (float *)y, (float *)h->d_tbuf, nullptr, st, 3,
                                     &recs[r]);
    }
    if (rc == SIPDG_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(SIPDG_EHIP, "stream sync");
    int n = 0;
    if (rc == SIPDG_OK) {
        n = std::min(recs[0].n, max_launches);
        for (int i = 0; i < n; ++i) {
            double sum = 0;
            for (int r = 0; r < reps; ++r) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, recs[r].ev[2 * i], recs[r].ev[2 * i + 1]) != hipSuccess) {
                    rc = fail(SIPDG_EHIP, "event elapsed time");
                    break;
                }
                sum += ms;
            }
            info[i].ms = sum / reps;
            info[i].stage = recs[0].stage[i];
            const int gi = recs[0].group[i];
            const int w = precision == SIPDG_F64 ? 0 : 1;
            if (gi >= 0) {
                const Group &g = h->groups[gi];
                info[i].order = g.P;
                info[i].elements = g.count;
                info[i].alg_bytes = info[i].stage == 2 && h->flux == SIPDG_FLUX_SHARED && h->points == SIPDG_POINTS_GLL
                                        ? g.alg_bytes[w]
                                        : 0.0;
            } else {
                // the persistent launch: every group of order <= 6 with traces <= 8 x 8
                info[i].order = 0;
                info[i].elements = h->pcount;
                double ab = 0.0;
                for (const Group &g : h->groups)
                    if (g.P <= 6 && g.nfmax <= 8) ab += g.alg_bytes[w];
                info[i].alg_bytes = info[i].stage == 2 ? ab : 0.0;
            }
        }
    }
    *n_launches = n;
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

static const char *P2P_ONLY_APPLY =
    "the point-to-point flux gives a nonsymmetric operator: only the apply calls and GMRES use it "
    "(set SIPDG_FLUX_SHARED for this call)";
static const char *GAUSS_ONLY =
    "Gauss volume points: only the apply calls (transpose included), CG and GMRES use them "
    "(set SIPDG_POINTS_GLL for this call)";

int sipdg_apply_transpose(sipdg_handle h, const void *g, void *xbar, int precision, void *stream) {
    // the shared-trace operator is symmetric on either point set
    if (h && h->flux == SIPDG_FLUX_P2P) return fail(SIPDG_EINVAL, P2P_ONLY_APPLY);
    return sipdg_apply(h, g, xbar, precision, stream);
}

// Point-to-point flux structures (first switch): the buffer, and for the
// gather-fold apply each face side's own point set: offsets, factors from the
// element maps, and per order group the face descriptors in launch order.
static int build_p2p(sipdg_ctx *h) {
    const int64_t nf = h->nfaces, ne = h->ne;
    std::vector<FaceTopo> faces(std::max<int64_t>(nf, 1));
    std::vector<int> order(std::max<int64_t>(ne, 1));
    std::vector<FaceRef> eface(std::max<int64_t>(ne * 6, 1));
    if (nf > 0) HIPCHK(hipMemcpy(faces.data(), h->d_faces, sizeof(FaceTopo) * nf, hipMemcpyDeviceToHost));
    if (ne > 0) {
        HIPCHK(hipMemcpy(order.data(), h->d_order, sizeof(int) * ne, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(eface.data(), h->d_eface, sizeof(FaceRef) * ne * 6, hipMemcpyDeviceToHost));
    }
    std::vector<int64_t> side((size_t)std::max<int64_t>(nf, 1) * 4, 0);
    int64_t fo = 0, to = 0;
    for (int64_t F = 0; F < nf; ++F) {
        const FaceTopo &ft = faces[F];
        for (int s = 0; s < (ft.eR >= 0 ? 2 : 1); ++s) {
            const int n = order[s ? ft.eR : ft.eL] + 2;
            side[F * 4 + 2 * s] = fo;
            side[F * 4 + 2 * s + 1] = to;
            fo += 7 * (int64_t)n * n;
            to += (ft.eR >= 0 ? 4 : 2) * (int64_t)n * n;
        }
    }
    // one buffer for both p2p structures: the general kernels use 2 x toff
    HIPCHK(hipMalloc(&h->d_tbuf_p2p, sizeof(double) * std::max<int64_t>(1, std::max(2 * h->tbuf_len, to))));
    int rc = upload(&h->d_p2p_side, side);
    if (!rc) rc = dalloc(&h->d_fgeo_p2p64, std::max<int64_t>(fo, 1));
    if (!rc) rc = dalloc(&h->d_fgeo_p2p32, std::max<int64_t>(fo, 1));
    if (rc) return rc;
    HIPCHK(launch_p2p_factors(nf, h->d_faces, h->d_order, h->d_p2p_side, h->d_emap64, h->d_tab64, h->d_fgeo_p2p64, 0));
    HIPCHK(launch_cast_f32(h->d_fgeo_p2p64, h->d_fgeo_p2p32, std::max<int64_t>(fo, 1), 0));
    // face descriptors in the launch order of a descriptor list
    auto p2p_fdesc = [&](const ElemDesc *d_desc, int count, FaceDesc **out) -> int {
        std::vector<ElemDesc> desc(count);
        HIPCHK(hipMemcpy(desc.data(), d_desc, sizeof(ElemDesc) * count, hipMemcpyDeviceToHost));
        std::vector<FaceDesc> fd((size_t)count * 6);
        for (int i = 0; i < count; ++i) {
            const int e = desc[i].e, n = order[e] + 2;
            for (int f = 0; f < 6; ++f) {
                const FaceRef fr = eface[(size_t)e * 6 + f];
                const int slot = face_slot(fr.info), si = slot == 1 ? 1 : 0;
                const int info = slot | (face_orient(fr.info) << 2) | (n << 5);
                fd[(size_t)i * 6 + f] = FaceDesc{side[(size_t)fr.F * 4 + 2 * si], side[(size_t)fr.F * 4 + 2 * si + 1],
                                                 fr.F, info};
            }
        }
        return upload(out, fd);
    };
    for (Group &g : h->groups) {
        rc = p2p_fdesc(g.d_desc, g.count, &g.d_fdesc_p2p);
        if (rc) return rc;
    }
    if (h->pcount > 0) {
        rc = p2p_fdesc(h->d_pdesc, h->pcount, &h->d_pfdesc_p2p);
        if (rc) return rc;
    }
    HIPCHK(hipDeviceSynchronize());
    return SIPDG_OK;
}

int sipdg_set_flux(sipdg_handle h, int flux) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (flux != SIPDG_FLUX_SHARED && flux != SIPDG_FLUX_P2P) return fail(SIPDG_EINVAL, "unknown flux");
    if (flux == SIPDG_FLUX_P2P) {
        if (h->dim != 3) return fail(SIPDG_EINVAL, "the point-to-point flux needs a 3-D mesh");
        if (h->points == SIPDG_POINTS_GAUSS)
            return fail(SIPDG_EINVAL, "the point-to-point flux takes GLL volume points (each side's own face points)");
        if (!h->d_tbuf_p2p) {
            int rc = build_p2p(h);
            if (rc) return rc;
        }
    }
    h->flux = flux;
    return SIPDG_OK;
}

int sipdg_get_flux(sipdg_handle h, int *flux) {
    if (!h || !flux) return fail(SIPDG_EINVAL, "null argument");
    *flux = h->flux;
    return SIPDG_OK;
}

int sipdg_set_basis(sipdg_handle h, int basis) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (basis != SIPDG_BASIS_LEGENDRE && basis != SIPDG_BASIS_MODAL) return fail(SIPDG_EINVAL, "unknown basis");
    if (basis == h->basis) return SIPDG_OK;
    HIPCHK(hipDeviceSynchronize());
    std::vector<double> tab(TAB_SIZE);
    build_tables(tab.data(), basis);
    HIPCHK(hipMemcpy(h->d_tab64, tab.data(), sizeof(double) * TAB_SIZE, hipMemcpyHostToDevice));
    HIPCHK(launch_cast_f32(h->d_tab64, h->d_tab32, TAB_SIZE, 0));
    build_tables(tab.data(), basis, true);
    HIPCHK(hipMemcpy(h->d_tabgl64, tab.data(), sizeof(double) * TAB_SIZE, hipMemcpyHostToDevice));
    HIPCHK(launch_cast_f32(h->d_tabgl64, h->d_tabgl32, TAB_SIZE, 0));
    h->basis = basis;
    // the two-stage, fused and persistent structures evaluate Legendre
    // endpoint values in closed form; gather and gather-fold take either basis
    h->fast_ok = basis == SIPDG_BASIS_LEGENDRE && h->fast_ok0;
    h->gfold_ok = h->gfold_ok0;
    h->variant = default_variant(h);
    if (h->ne > 0) {
        int rc = refresh_diag(h, 0);
        if (rc) return rc;
    }
    HIPCHK(hipDeviceSynchronize());
    return SIPDG_OK;
}

int sipdg_set_points(sipdg_handle h, int points) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (points != SIPDG_POINTS_GLL && points != SIPDG_POINTS_GAUSS) return fail(SIPDG_EINVAL, "unknown point set");
    if (points == SIPDG_POINTS_GAUSS) {
        if (!h->gfold_ok) return fail(SIPDG_EINVAL, "Gauss volume points need a 3-D mesh");
        if (h->flux != SIPDG_FLUX_SHARED)
            return fail(SIPDG_EINVAL, "Gauss volume points take the shared-trace flux");
        for (const Group &g : h->groups)
            if (!gfold_group(g, false))
                return fail(SIPDG_EINVAL, "Gauss volume points need every order group on the gather-fold kernels "
                                          "(orders <= 6 with traces <= 8 x 8, orders 7 and 8 with traces <= 10 x 10)");
        h->variant = SIPDG_VARIANT_GATHER_FOLD;
    }
    h->points = points;
    return SIPDG_OK;
}

int sipdg_get_points(sipdg_handle h, int *points) {
    if (!h || !points) return fail(SIPDG_EINVAL, "null argument");
    *points = h->points;
    return SIPDG_OK;
}

int sipdg_get_basis(sipdg_handle h, int *basis) {
    if (!h || !basis) return fail(SIPDG_EINVAL, "null argument");
    *basis = h->basis;
    return SIPDG_OK;
}

int sipdg_diagonal(sipdg_handle h, double *d, void *stream) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (h->flux == SIPDG_FLUX_P2P) return fail(SIPDG_EINVAL, P2P_ONLY_APPLY);
    if (h->points == SIPDG_POINTS_GAUSS) return fail(SIPDG_EINVAL, GAUSS_ONLY);
    if (h->ndof == 0) return SIPDG_OK;
    if (!d) return fail(SIPDG_EINVAL, "null argument");
    HIPCHK(hipMemcpyAsync(d, h->d_diag64, sizeof(double) * h->ndof, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return SIPDG_OK;
}

int sipdg_set_lambda(sipdg_handle h, const double *lam, void *stream) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (h->ne == 0) return SIPDG_OK;
    if (!lam) return fail(SIPDG_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipMemcpyAsync(h->d_lam64, lam, sizeof(double) * h->ne, hipMemcpyDeviceToDevice, st));
    HIPCHK(launch_cast_f32(h->d_lam64, h->d_lam32, h->ne, st));
    int rc = refresh_diag(h, st);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(st));
    return SIPDG_OK;
}

int sipdg_set_penalty_scale(sipdg_handle h, int problem, double sigma) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (!(sigma > 0.0)) return fail(SIPDG_EINVAL, "penalty scale must be positive");
    if (problem >= h->nprob) return fail(SIPDG_EINVAL, "problem index out of range");
    for (int p = 0; p < h->nprob; ++p)
        if (problem < 0 || p == problem) h->sigma[p] = sigma;
    HIPCHK(hipDeviceSynchronize());
    int rc = upload_tau(h);
    if (rc) return rc;
    rc = refresh_diag(h, 0);
    if (rc) return rc;
    HIPCHK(hipDeviceSynchronize());
    return SIPDG_OK;
}

int sipdg_num_points(sipdg_handle h, int64_t *nv, int64_t *nb) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (nv) *nv = h->nvq;
    if (nb) *nb = h->nbq;
    return SIPDG_OK;
}

int sipdg_num_affine(sipdg_handle h, int64_t *n_affine) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (!n_affine) return fail(SIPDG_EINVAL, "null argument");
    int64_t n = 0;
    for (const Group &g : h->groups) n += g.naff;
    *n_affine = n;
    return SIPDG_OK;
}

int sipdg_quad_points(sipdg_handle h, double *xq, double *xb, void *stream) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (h->points == SIPDG_POINTS_GAUSS) return fail(SIPDG_EINVAL, GAUSS_ONLY);
    if (h->ne == 0) return SIPDG_OK;
    if (!xq || (!xb && h->nbq)) return fail(SIPDG_EINVAL, "null argument");
    HIPCHK(launch_points(h->dim, h->ne, h->d_corners, h->d_order, h->d_eface, h->d_qoff, h->d_boff,
                         h->d_tab64, xq, xb, (hipStream_t)stream));
    return SIPDG_OK;
}

int sipdg_load_vector(sipdg_handle h, const double *s, const double *g, double *b, void *stream) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (h->points == SIPDG_POINTS_GAUSS) return fail(SIPDG_EINVAL, GAUSS_ONLY);
    if (h->ndof == 0) return SIPDG_OK;
    if (!s || !b || (!g && h->nbq)) return fail(SIPDG_EINVAL, "null argument");
    for (const Group &gr : h->groups) {
        OpArgs<double> A = make_args<double>(h, gr, nullptr, b, nullptr, nullptr);
        A.tsz = work_size_for(h->dim, gr.P, gr.P + 2);
        HIPCHK(launch_load(h->dim, gr.P, A, h->d_qoff, h->d_boff, s, g, (hipStream_t)stream));
    }
    return SIPDG_OK;
}

int sipdg_param_grad(sipdg_handle h, const double *a, const double *b, double *dlam, double *dsig,
                     void *stream) {
    if (!h || !dsig) return fail(SIPDG_EINVAL, "null argument");
    if (h->flux == SIPDG_FLUX_P2P) return fail(SIPDG_EINVAL, P2P_ONLY_APPLY);
    if (h->points == SIPDG_POINTS_GAUSS) return fail(SIPDG_EINVAL, GAUSS_ONLY);
    hipStream_t st = (hipStream_t)stream;
    if (h->ne == 0) {   // empty mesh: every problem's penalty gradient is zero
        HIPCHK(hipMemsetAsync(dsig, 0, sizeof(double) * h->nprob, st));
        return SIPDG_OK;
    }
    if (!a || !b || !dlam) return fail(SIPDG_EINVAL, "null argument");
    // traces of a and b: the trace stage of the handle's kernel structure
    // (every structure but the fused ones has one), else the general kernels
    const bool fused = h->variant == SIPDG_VARIANT_FUSED || h->variant == SIPDG_VARIANT_GATHER_FOLD_FUSED;
    if (!fused) {
        int rc = apply_impl<double>(h, a, nullptr, h->d_tbuf, nullptr, st, 1);
        if (rc) return rc;
        rc = apply_impl<double>(h, b, nullptr, h->d_tbuf2, nullptr, st, 1);
        if (rc) return rc;
    }
    for (const Group &g : h->groups) {
        OpArgs<double> A;
        if (fused) {
            A = make_args<double>(h, g, a, nullptr, h->d_tbuf, nullptr);
            HIPCHK(launch_op<double>(h->dim, g.P, OP_TRACE, A, g.nfmax, st));
            A = make_args<double>(h, g, b, nullptr, h->d_tbuf2, nullptr);
            HIPCHK(launch_op<double>(h->dim, g.P, OP_TRACE, A, g.nfmax, st));
        }
        A = make_args<double>(h, g, nullptr, nullptr, nullptr, nullptr);
        A.tsz = work_size_for(h->dim, g.P, g.P + 2);
        HIPCHK(launch_pgrad_elem(h->dim, g.P, A, a, b, h->d_tau0, dlam, h->d_elem_tmp, st));
    }
    HIPCHK(launch_pgrad_faces(h->dim, h->nfaces, h->d_is_interior, h->d_toff, h->d_foff, h->d_face_nf,
                              h->d_fgeo64, h->d_tau0, h->d_tbuf, h->d_tbuf2, h->d_face_tmp, st));
    HIPCHK(launch_segsum(h->nprob, h->d_prob_face_off, h->d_face_tmp, dsig, 0, st));
    HIPCHK(launch_segsum(h->nprob, h->d_prob_elem_off, h->d_elem_tmp, dsig, 1, st));
    return SIPDG_OK;
}

int sipdg_set_variant(sipdg_handle h, int variant) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (h->points == SIPDG_POINTS_GAUSS && variant != SIPDG_VARIANT_GATHER_FOLD)
        return fail(SIPDG_EINVAL, "Gauss volume points run on the gather_fold structure only");
    if (h->dim == 2) {
        if (!variant_allowed_2d(h, variant))
            return fail(SIPDG_EINVAL, variant == SIPDG_VARIANT_GATHER_FOLD_FUSED
                                          ? "2-D gather_fold_fused needs every element of order <= 6 with traces <= 8 points"
                                          : "2-D meshes take gather, gather_fold (an element of order <= 6) or "
                                            "gather_fold_fused");
        h->variant = variant;
        return SIPDG_OK;
    }
    if (variant == SIPDG_VARIANT_GATHER) {
        h->variant = variant;
        return SIPDG_OK;
    }
    if (variant < 0 || variant >= SIPDG_NUM_VARIANTS)
        return fail(SIPDG_EINVAL, "unknown variant");
    if (variant == SIPDG_VARIANT_GATHER_FOLD || variant == SIPDG_VARIANT_GATHER_FOLD_PERSISTENT) {
        if (!h->gfold_ok) return fail(SIPDG_EINVAL, "gather_fold needs a 3-D mesh");
        if (variant == SIPDG_VARIANT_GATHER_FOLD_PERSISTENT && h->basis != SIPDG_BASIS_LEGENDRE)
            return fail(SIPDG_EINVAL, "the persistent structure needs the Legendre basis");
    } else if (!h->fast_ok) {
        return fail(SIPDG_EINVAL, "variant needs a 3-D mesh with every order <= 6");
    }
    h->variant = variant;
    return SIPDG_OK;
}

int sipdg_set_geometry(sipdg_handle h, int source) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (source != SIPDG_GEOMETRY_STORED && source != SIPDG_GEOMETRY_MAP)
        return fail(SIPDG_EINVAL, "unknown geometry source");
    if (source == SIPDG_GEOMETRY_MAP && h->dim != 3) return fail(SIPDG_EINVAL, "geometry from the map needs a 3-D mesh");
    h->geo_map = source == SIPDG_GEOMETRY_MAP;
    return SIPDG_OK;
}

int sipdg_get_geometry(sipdg_handle h, int *source) {
    if (!h || !source) return fail(SIPDG_EINVAL, "null argument");
    *source = h->geo_map ? SIPDG_GEOMETRY_MAP : SIPDG_GEOMETRY_STORED;
    return SIPDG_OK;
}

int sipdg_get_variant(sipdg_handle h, int *variant) {
    if (!h || !variant) return fail(SIPDG_EINVAL, "null argument");
    *variant = h->variant;
    return SIPDG_OK;
}

int sipdg_autotune(sipdg_handle h, const char *cache_path, int reps, double *ms_out, void *stream) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (h->flux == SIPDG_FLUX_P2P) return fail(SIPDG_EINVAL, P2P_ONLY_APPLY);
    if (h->points == SIPDG_POINTS_GAUSS) return fail(SIPDG_EINVAL, GAUSS_ONLY);
    if (reps <= 0) reps = 20;
    if (ms_out)
        for (int v = 0; v < SIPDG_NUM_VARIANTS; ++v) ms_out[v] = 0.0;
    const std::string key = tune_key(h);
    TuneRec rec;
    if (cache_path && cache_lookup(cache_path, key, rec) && apply_tuning(h, rec) == SIPDG_OK) {
        h->tune_from_cache = true;
        if (ms_out)
            for (int v = 0; v < SIPDG_NUM_VARIANTS; ++v) ms_out[v] = rec.ms[v];
        return SIPDG_OK;
    }
    h->tune_from_cache = false;
    hipStream_t st = (hipStream_t)stream;
    // timing vectors: two of the CG work vectors (allocated at create)
    double *x = nullptr, *y = nullptr;
    cg_scratch(h, &x, &y);
    if (!x || !y) return fail(SIPDG_EHIP, "internal: CG work vectors missing");
    HIPCHK(vec_fill<double>(x, h->ndof, 0.0, st));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto time_apply = [&](double &ms_per) -> int {
        int rc = SIPDG_OK;
        for (int i = 0; i < 3 && rc == SIPDG_OK; ++i) rc = apply_impl<double>(h, x, y, h->d_tbuf, nullptr, st);
        if (rc == SIPDG_OK && hipEventRecord(e0, st) != hipSuccess) rc = fail(SIPDG_EHIP, "event record");
        for (int i = 0; i < reps && rc == SIPDG_OK; ++i) rc = apply_impl<double>(h, x, y, h->d_tbuf, nullptr, st);
        if (rc == SIPDG_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
            rc = fail(SIPDG_EHIP, "event sync");
        float ms = 0.f;
        if (rc == SIPDG_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(SIPDG_EHIP, "event time");
        ms_per = ms / reps;
        return rc;
    };
    const int keep = h->variant;
    double best = 1e300;
    int best_v = keep;
    int rc = SIPDG_OK;
    for (int v = 0; v < SIPDG_NUM_VARIANTS && rc == SIPDG_OK; ++v) {
        rec.ms[v] = 0.0;
        const bool gf = v == SIPDG_VARIANT_GATHER_FOLD || v == SIPDG_VARIANT_GATHER_FOLD_PERSISTENT;
        if (h->dim == 2 ? !variant_allowed_2d(h, v) : (gf ? !h->gfold_ok : (v != SIPDG_VARIANT_GATHER && !h->fast_ok)))
            continue;
        if (v == SIPDG_VARIANT_GATHER_FOLD_PERSISTENT && h->basis != SIPDG_BASIS_LEGENDRE) continue;
        h->variant = v;
        double vbest = 1e300;
        if (v == SIPDG_VARIANT_GATHER_FOLD_PERSISTENT) {
            // the persistent launch's shape: blocks per compute unit
            const int shapes[] = {2, 4, 6, 8, 12, 16};
            int vshape = h->blocks_per_cu;
            for (int si = 0; si < 6 && rc == SIPDG_OK; ++si) {
                h->blocks_per_cu = shapes[si];
                double t = 0.0;
                rc = time_apply(t);
                if (rc == SIPDG_OK && t < vbest) {
                    vbest = t;
                    vshape = shapes[si];
                }
            }
            h->blocks_per_cu = vshape;
        } else if (v == SIPDG_VARIANT_GATHER_FOLD && h->dim == 3) {
            // tile shape of each order group's apply launch, one order at a
            // time (the others fixed at their best so far).  Each candidate
            // is timed in alternation with the incumbent shape, twice each,
            // and the faster run of each kept, so that a slow early run or a
            // drifting clock does not favour the shape timed later; it must
            // win by more than the timing noise (2 %), so that runs of the
            // same build keep the same shapes unless one clearly wins.
            rc = time_apply(vbest);
            for (int P = 1; P <= SIPDG_MAX_ORDER && rc == SIPDG_OK; ++P) {
                bool present = false;
                for (const Group &g : h->groups) present |= g.P == P && g.count > 0;
                if (!present) continue;
                int bt = h->tile[P], bb = h->budget[P];
                for (const TileShape &ts : tile_shapes(P)) {
                    if (ts.tile == bt && ts.budget == bb) continue;
                    double ti = 1e300, tc = 1e300;
                    for (int k = 0; k < 2 && rc == SIPDG_OK; ++k) {
                        double t = 0.0;
                        h->tile[P] = bt;
                        h->budget[P] = bb;
                        rc = time_apply(t);
                        ti = std::min(ti, t);
                        if (rc != SIPDG_OK) break;
                        h->tile[P] = ts.tile;
                        h->budget[P] = ts.budget;
                        rc = time_apply(t);
                        tc = std::min(tc, t);
                    }
                    if (rc != SIPDG_OK) break;
                    if (tc < 0.98 * ti) {
                        bt = ts.tile;
                        bb = ts.budget;
                        vbest = tc;
                    } else {
                        vbest = std::min(vbest, ti);
                    }
                }
                h->tile[P] = bt;
                h->budget[P] = bb;
            }
        } else {
            rc = time_apply(vbest);
        }
        if (rc == SIPDG_OK && vbest < 1e300) {
            rec.ms[v] = vbest;
            if (vbest < best) {
                best = vbest;
                best_v = v;
            }
        }
    }
    h->variant = rc == SIPDG_OK ? best_v : keep;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (ms_out)
        for (int v = 0; v < SIPDG_NUM_VARIANTS; ++v) ms_out[v] = rec.ms[v];
    if (cache_path) {
        rec.variant = h->variant;
        rec.blocks_per_cu = h->blocks_per_cu;
        for (int P = 0; P <= SIPDG_MAX_ORDER; ++P) {
            rec.tile[P] = h->tile[P];
            rec.budget[P] = h->budget[P];
        }
        cache_store(cache_path, key, rec);
    }
    return SIPDG_OK;
}

int sipdg_set_tile(sipdg_handle h, int order, int tile, int budget) {
    if (!h) return fail(SIPDG_EINVAL, "null handle");
    if (order < 1 || order > SIPDG_MAX_ORDER) return fail(SIPDG_EINVAL, "order outside [1, 8]");
    for (const TileShape &ts : tile_shapes(order))
        if (ts.tile == tile && ts.budget == budget) {
            h->tile[order] = tile;
            h->budget[order] = budget;
            return SIPDG_OK;
        }
    return fail(SIPDG_EINVAL, "tile shape not built for this order");
}

int sipdg_get_tuning(sipdg_handle h, sipdg_tuning *t) {
    if (!h || !t) return fail(SIPDG_EINVAL, "null argument");
    t->variant = h->variant;
    t->blocks_per_cu = h->blocks_per_cu;
    t->from_cache = h->tune_from_cache ? 1 : 0;
    t->signature = h->signature;
    for (int P = 0; P <= SIPDG_MAX_ORDER; ++P) {
        t->tile[P] = h->tile[P];
        t->budget[P] = h->budget[P];
    }
    return SIPDG_OK;
}

const char *sipdg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
