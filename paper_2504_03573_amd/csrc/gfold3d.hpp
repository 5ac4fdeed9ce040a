// Gather-fold hexahedron kernel, one launch per order group: orders 1..6
// (n = p+2 <= 8 GLL points per direction) whose faces all have traces of at
// most 8 x 8 points (every neighbour of order <= 6), one 64-lane wavefront
// per element; orders 7 and 8 (traces up to 10 x 10), two wavefronts per
// element.
//
// Volume terms (Xia & Moxey, Sec. 3.1 basic operators): lane (q0, q1) keeps
// the xi_2 column of its n points in registers ("column layout").  BwdTrans,
// the collocation derivative and their transposes are line contractions
// whose 1-D table entries are wave-uniform, so they come through the scalar
// cache; LDS is used only to move lines between the three layouts
//   column  lane (q0, q1) holds (q0, q1, .)
//   line-0  lane (q1, q2) holds (., q1, q2)
//   line-1  lane (q0, q2) holds (q0, ., q2)
// through two padded point arrays whose strides (9 along q1 (11 for n = 10),
// and 24..120 along q2, odd multiples of 8) spread the three access patterns
// over the LDS banks.
//
// Faces (Sec. 3.2 GathrInterp, Sec. 3.3 shared trace space): GLL points
// include the element's faces, so u and grad_xi u at an element's own face
// points fall out of the volume evaluation: a column's ends for the faces
// normal to xi_2, a line-0 or line-1 lane's ends for the faces normal to xi_0
// and xi_1.  In every face phase lane (t1, t2) holds trace point (t1, t2) in
// the element's own face coordinates.  When the shared trace is finer than the
// element (n_F > n), the four fields are interpolated to the trace with the
// Lagrange matrix I (n_F x n) and the flux is brought back with I^T, which is
// exact because everything interpolated is a polynomial of degree <= p on the
// face (the transposed evaluation of Sec. 3.3, TraceIProduct).  The
// neighbour's u and grad_xi u at the same trace points are evaluated from its
// coefficients (TracePhysEval: a reduction along its face normal with
// P_i(+-1), P'_i(+-1) and two contractions with the Legendre tables at the
// trace's GLL points), directly at the points given by the orientation map.
// The flux of eq. IP is formed at every trace point and its lift -- a value
// for the phi test term and a vector for the grad phi test term -- is added to
// the volume's pointwise terms at the face points, so the inner product with
// the basis (IProduct) lifts faces and volume at once and y is written once.
//
// Trace stage of the two-stage structure (k3t_elem): no volume work; the
// element's own u and grad_xi u at its trace points come from the same face
// reduction and two contractions as the neighbour's evaluation above.
#pragma once

#include "context.hpp"
#include "launch.hpp"

namespace sipdg {
namespace g3 {

constexpr int W = 64;           // lanes per element, orders <= 6
constexpr int S9 = PMAX + 1;    // row stride of the BF/DBF tables

// Lane geometry.  Orders <= 6: one 64-lane wavefront per element; lane l
// holds point column / trace point (l % 8, l / 8); traces up to 8 x 8.
// Orders 7 and 8 (9 x 9 and 10 x 10 columns, traces up to 10 x 10): two
// wavefronts per element, lane l at (l % 10, l / 10).
template <int P>
struct Geo {
    static constexpr int W = P <= 6 ? 64 : 128;     // threads per element
    static constexpr int S = P <= 6 ? 8 : 10;       // lane stride of the 2-D grids
    static constexpr int NFMAX = P <= 6 ? 8 : 10;   // largest trace per direction
};
// Thread index in the lane grid of one element's face phase: the block's
// thread in the one-element kernels, the lane in its wavefront in the
// multi-element tiles (there each wavefront runs one element's faces at a
// time).
template <int P>
__device__ __forceinline__ int flane() {
    return Geo<P>::W == 64 ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
}
template <int P>
__device__ __forceinline__ int gx(int l) { return l % Geo<P>::S; }
template <int P>
__device__ __forceinline__ int gy(int l) { return l / Geo<P>::S; }

template <int P>
struct Sz {
    static constexpr int N = P + 2, NP = P + 1;
    static constexpr int NPTS = N * N * N;
    static constexpr int S1 = N <= 9 ? 9 : 11;   // odd and >= N
    static constexpr int S2 = N == 10 ? 120 : (N == 9 ? 88 : (N >= 7 ? 72 : (N >= 5 ? 56 : (N == 4 ? 40 : 24))));
    static_assert(S1 >= N && S2 >= S1 * (N - 1) + N, "point arrays must not overlap");
    static constexpr int ARR = S2 * N;          // one padded point array
    static constexpr int SCR = 24 * Geo<P>::W;  // face scratch, aliases the point arrays
    // Every trace of this order has the element's own n points (n = NFMAX):
    // the apply takes its own (u, g) from its face values instead of the trace
    // buffer, and keeps the fields of the faces normal to xi_1 and xi_2 until
    // their phase in OWN_STASH = [16][W] at 8 W, past the lifted-flux array FB
    // (each lane reads back only its own entries).  The stash takes the place
    // of the face scratch, which no face of this order uses (none
    // interpolates), and of the point arrays, which are dead from the end of
    // the gradient phase until the inner product.
    static constexpr bool OWN = N == Geo<P>::NFMAX;
    static constexpr int STASH_OFF = 8 * Geo<P>::W;
    static_assert(!OWN || STASH_OFF + 16 * Geo<P>::W <= SCR, "the stash must fit the face scratch");
    static constexpr int TOTAL = 2 * ARR > SCR ? 2 * ARR : SCR;
};

// face scratch (R units from the block's LDS base, W = Geo<P>::W):
//   FB [2 sides][4 fields][W] at 0       lifted flux of the faces normal to xi_0
//                                         or xi_1, for the column lanes
//   [8 W, 24 W)                           interpolation / lift / neighbour work
constexpr int FB_OFF = 0;

struct Args {
    const int *elems;
    int count;
    const int64_t *xoff;
    const int64_t *voff;
    const FaceRef *eface;
    const FaceTopo *faces;
    const int *order;
    const int64_t *foff;
    const int64_t *toff;
    const int *skip;
    const ElemDesc *desc;    // [count]
    const FaceDesc *fdesc;   // [count][6]
    int basis = 0;           // host side: 0 Legendre, 1 modified C0 modal (trace kernels)
    const int64_t *side = nullptr;   // point-to-point trace: [nf][2][factor, buffer offset]
};

template <class R>
struct Data {
    const R *__restrict__ vgeo;
    const R *__restrict__ fgeo;
    const R *__restrict__ lam;
    const R *__restrict__ tau;
    const R *__restrict__ tab;
    const R *__restrict__ x;
    R *__restrict__ y;
    R *__restrict__ tbuf;
    const R *__restrict__ egeo;   // [ne][8]: G~ (00 01 02 11 12 22), |J| of affine elements
    const R *__restrict__ emap;   // [ne][24]: trilinear map coefficients c1..c7 (x, y, z), pad
    // One conjugate-gradient step folded into the trace stage (k3t_all with
    // FOLD only): the coefficients are the search direction p, and before
    // they are used the element's entries get  x += alpha p  (the previous
    // step's update, deferred) and  p = D^-1 r + beta p  (p kept for a
    // stopped problem), with alpha, beta, the stop flag of the element's
    // problem (eprob: element -> problem).  fold_dinv null: no preconditioner.
    R *fold_p = nullptr;
    R *fold_x = nullptr;
    const R *fold_r = nullptr;
    const R *fold_dinv = nullptr;
    const double *fold_alpha = nullptr;
    const double *fold_beta = nullptr;
    const int *fold_conv = nullptr;
    const int *eprob = nullptr;
};

// Rows of adj(J) and det J of the trilinear map with coefficients c1..c7
// (each x, y, z) at xi: the columns of J are dx/dxi_k, the rows of adj(J) the
// cross products of the columns.
template <class R>
__device__ __forceinline__ R map_adjugate3(const R *cm, R x0, R x1, R x2, R r[3][3]) {
    R j0[3], j1[3], j2[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        j0[c] = cm[c] + cm[9 + c] * x1 + cm[12 + c] * x2 + cm[18 + c] * x1 * x2;
        j1[c] = cm[3 + c] + cm[9 + c] * x0 + cm[15 + c] * x2 + cm[18 + c] * x0 * x2;
        j2[c] = cm[6 + c] + cm[12 + c] * x0 + cm[15 + c] * x1 + cm[18 + c] * x0 * x1;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        r[0][c] = j1[c1] * j2[c2] - j1[c2] * j2[c1];
        r[1][c] = j2[c1] * j0[c2] - j2[c2] * j0[c1];
        r[2][c] = j0[c1] * j1[c2] - j0[c2] * j1[c1];
    }
    return j0[0] * r[0][0] + j0[1] * r[0][1] + j0[2] * r[0][2];
}

// Tables are read through the constant address space: the compiler may then
// assume no store of the kernel writes them and reads wave-uniform entries
// with scalar loads (a __restrict__ on a struct member does not tell it that).
template <class R>
using ctab = const __attribute__((address_space(4))) R *;
template <class R>
__device__ __forceinline__ ctab<R> as_const(const R *p) {
    return (ctab<R>)p;
}

// LDS copy of the interpolation matrices I(n, m) [m][n] for m = n+1 .. the
// largest trace, the finer traces an element of order p can meet, by m.
template <int P>
struct ITab {
    static constexpr int N = P + 2, M = Geo<P>::NFMAX;
    static constexpr int SIZE = N < M ? N * ((M * (M + 1)) / 2 - (N * (N + 1)) / 2) : 0;
};
template <int P>
__device__ __forceinline__ int itab_off(int m) {
    constexpr int N = P + 2;
    return N * (((m - 1) * m) / 2 - (N * (N + 1)) / 2);
}
// LDS copy of the trace tables P_i(z_t), P'_i(z_t), i < 7, at the m-point
// GLL traces m = n .. 8 a face of an element of order p can have (fused
// kernel: the neighbour's trace evaluation), [m][7] each, BF then DBF per m.
template <int P>
struct BTab {
    static constexpr int N = P + 2;
    static constexpr int SIZE = N <= 8 ? 14 * ((8 * 9) / 2 - ((N - 1) * N) / 2) : 0;
};
template <int P>
__device__ __forceinline__ int btab_off(int m) {
    constexpr int N = P + 2;
    return 14 * (((m - 1) * m) / 2 - ((N - 1) * N) / 2);
}
// LDS copy of the trace tables for the Gauss apply: per trace size m = n ..
// the largest trace, BF [m][NP] then DBF [m][NP].
template <int P>
struct GTab {
    static constexpr int NP = P + 1, N = P + 2, M = Geo<P>::NFMAX;
    static constexpr int off(int m) { return NP * ((m - 1) * m - (N - 1) * N); }
    static constexpr int SIZE = off(M + 1);
};

// mode 3 (Gauss volume points): the point arrays, then the face terms of
// every mode [NP^3] and the trace tables (no interpolation tables)
template <int P>
__host__ __device__ constexpr int lds_total(int mode) {
    return mode == 3 ? Sz<P>::TOTAL + (((P + 1) * (P + 1) * (P + 1) + 3) & ~3) + GTab<P>::SIZE
                     : Sz<P>::TOTAL + ((ITab<P>::SIZE + 3) & ~3) + (mode == 2 ? ((BTab<P>::SIZE + 3) & ~3) : 0);
}

template <int P>
__device__ __forceinline__ int pa(int i0, int i1, int i2) {
    return i0 + Sz<P>::S1 * i1 + Sz<P>::S2 * i2;
}

// face coordinate directions of the face normal to k (increasing order)
__device__ __forceinline__ int dir_a(int k) { return k == 0 ? 1 : 0; }
__device__ __forceinline__ int dir_b(int k) { return k == 2 ? 1 : 2; }

// P_i(s) and P'_i(s) at s = -1 (side 0) and +1 (side 1)
template <class R>
__device__ __forceinline__ R end_val(int i, int s) { return (s || !(i & 1)) ? R(1) : R(-1); }
template <class R>
__device__ __forceinline__ R end_der(int i, int s) {
    const R v = R(0.5) * R(i) * R(i + 1);
    return (s || (i & 1)) ? v : -v;
}

// mode with face indices (ia, ib) and normal index ik on the face normal to k
__device__ __forceinline__ int mode_rt(int np, int k, int ia, int ib, int ik) {
    if (k == 0) return ik + np * (ia + np * ib);
    if (k == 1) return ia + np * (ik + np * ib);
    return ia + np * (ib + np * ik);
}

// canonical (owner) trace index -> face coordinates of a side with
// orientation code o (inverse of canon_index)
__device__ __forceinline__ void canon_inverse(int o, int nf, int qc, int &r1, int &r2) {
    const int c1 = qc % nf, c2 = qc / nf;
    const int a1 = (o & 4) ? c2 : c1, a2 = (o & 4) ? c1 : c2;
    r1 = (o & 1) ? nf - 1 - a1 : a1;
    r2 = (o & 2) ? nf - 1 - a2 : a2;
}

// Per-face values that are the same on every lane.  Lane f < 6 of the
// wavefront loads those of local face f at kernel start (one round of
// dependent loads for all six faces); face_uniform() broadcasts them.
template <class R>
struct MetaV {
    int F = 0, info = 0, nb = 0, fnon = 0, npn = 0;
    int64_t fo = 0, to = 0, xn = 0;
    R tau = 0;
};

template <class R>
struct FaceU {
    int F, slot, nf, o, npf;
    int nb, kn, sn, on, npn;
    int64_t fo, to, xn;
    R tau;
};

__device__ __forceinline__ int rl32(int v, int f) { return __builtin_amdgcn_readlane(v, f); }
__device__ __forceinline__ int64_t rl64(int64_t v, int f) {
    const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffff), f);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), f);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ double rlR(double v, int f) { return __longlong_as_double(rl64(__double_as_longlong(v), f)); }
__device__ __forceinline__ float rlR(float v, int f) { return __int_as_float(rl32(__float_as_int(v), f)); }

template <class R, int MODE>
__device__ __forceinline__ MetaV<R> load_meta(const Args &A, const Data<R> &D, int blk) {
    MetaV<R> m;
    const int l = threadIdx.x;
    if ((l & 63) < 6) {   // lanes 0..5 of every wavefront of the element
        const FaceDesc fr = A.fdesc[(int64_t)blk * 6 + (l & 63)];
        m.F = fr.F;
        m.info = fr.info;
        m.fo = fr.fo;
        m.to = fr.to;
        m.tau = D.tau[fr.F];
        const int slot = face_slot(fr.info);
        if (slot != 2) {
            if (MODE == 2) {
                const FaceTopo ft = A.faces[fr.F];
                m.nb = slot == 0 ? ft.eR : ft.eL;
                const int fn = slot == 0 ? ft.fR : ft.fL;
                const int on = slot == 0 ? ft.orient : 0;
                m.fnon = fn | (on << 3);
                m.npn = A.order[m.nb] + 1;
                m.xn = A.xoff[m.nb];
            }
        }
    }
    return m;
}

template <class R>
__device__ __forceinline__ FaceU<R> face_uniform(const MetaV<R> &m, int f) {
    FaceU<R> u;
    u.F = rl32(m.F, f);
    const int info = rl32(m.info, f);
    u.slot = face_slot(info);
    u.nf = face_nf(info);
    u.o = face_orient(info);
    u.npf = u.nf * u.nf;
    u.nb = rl32(m.nb, f);
    const int fnon = rl32(m.fnon, f);
    u.kn = (fnon & 7) >> 1;
    u.sn = fnon & 1;
    u.on = fnon >> 3;
    u.npn = rl32(m.npn, f);
    u.fo = rl64(m.fo, f);
    u.to = rl64(m.to, f);
    u.xn = rl64(m.xn, f);
    u.tau = rlR(m.tau, f);
    return u;
}

// Per-lane data of one face at this lane's trace point (t1, t2) in the
// element's own face coordinates: the canonical index, a = w J_s, the
// element's C along its (k, a, b) directions, and
//   MODE 1: the element's own (u, g) = (ou, og) and the neighbour's
//           (n0, n1) from the trace buffer (MODE 3: the same, own values
//           always from the buffer),
//   MODE 2: the neighbour's C along its own (k, a, b) directions.
template <class R>
struct FaceD {
    int qc;
    R aw, Ck, Ca, Cb, n0, n1, n2, ou, og;
};

// Trace-buffer position of a side: interior faces hold [owner][other],
// boundary faces only the element's own.
__device__ __forceinline__ int tb_side(int slot) { return slot == 1 ? 1 : 0; }

template <class R, int P, int MODE>
__device__ __forceinline__ FaceD<R> load_face(const Data<R> &D, const FaceU<R> &u, int k) {
    FaceD<R> d;
    d.qc = 0;
    d.aw = d.Ck = d.Ca = d.Cb = d.n0 = d.n1 = d.n2 = d.ou = d.og = R(0);
    const int l = flane<P>(), t1 = gx<P>(l), t2 = gy<P>(l);
    if (t1 >= u.nf || t2 >= u.nf) return d;
    const int npf = u.npf;
    d.qc = canon_index(u.o, u.nf, t1, t2);
    const R *__restrict__ fg = D.fgeo + u.fo;
    const R *__restrict__ Co = fg + npf * (u.slot == 1 ? 4 : 1) + d.qc;
    d.Ck = Co[k * npf];
    d.Ca = Co[dir_a(k) * npf];
    d.Cb = Co[dir_b(k) * npf];
    if (MODE == 0) return d;
    d.aw = fg[d.qc];
    if (MODE == 1 || MODE == 3) {
        const R *__restrict__ tb = D.tbuf + u.to + d.qc;
        const int so = tb_side(u.slot);
        if constexpr (!Sz<P>::OWN || MODE == 3) {
            d.ou = tb[so * 2 * npf];
            d.og = tb[so * 2 * npf + npf];
        }
        if (u.slot != 2) {
            d.n0 = tb[(1 - so) * 2 * npf];
            d.n1 = tb[(1 - so) * 2 * npf + npf];
        }
        return d;
    }
    if (u.slot == 2) return d;
    {
        const R *__restrict__ Cn = fg + npf * (u.slot == 0 ? 4 : 1) + d.qc;
        d.n0 = Cn[u.kn * npf];
        d.n1 = Cn[dir_a(u.kn) * npf];
        d.n2 = Cn[dir_b(u.kn) * npf];
    }
    return d;
}

// Own u, grad_xi u at trace point (t1, t2): the face point itself when the
// trace has the element's points, else interpolated with I (n_F x n) along
// both face directions through LDS.
// The same for the two faces of one direction at once (scratch: 1024 R at sm).
template <class R, int P>
__device__ __forceinline__ void own_trace2(const R *itl, int nfA, int nfB, R *sm, R vA[4], R vB[4]) {
    constexpr int WG = Geo<P>::W, SG = Geo<P>::S;
    (void)WG;
    (void)SG;
    constexpr int N = P + 2;
    const bool nA = nfA != N, nB = nfB != N;
    if (!nA && !nB) return;
    const int l = flane<P>(), t1 = gx<P>(l), t2 = gy<P>(l);
    R *ISA = sm, *ITA = sm + 4 * WG, *ISB = sm + 8 * WG, *ITB = sm + 12 * WG;
    const R *IA = itl + itab_off<P>(nfA), *IB = itl + itab_off<P>(nfB);
    if (t1 < N && t2 < N) {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            if (nA) ISA[f * WG + l] = vA[f];
            if (nB) ISB[f * WG + l] = vB[f];
        }
    }
    __syncthreads();
    if (nA && t1 < nfA && t2 < N) {
        R c[4] = {0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const R w = IA[t1 * N + j];
#pragma unroll
            for (int f = 0; f < 4; ++f) c[f] += w * ISA[f * WG + j + SG * t2];
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) ITA[f * WG + l] = c[f];
    }
    if (nB && t1 < nfB && t2 < N) {
        R c[4] = {0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const R w = IB[t1 * N + j];
#pragma unroll
            for (int f = 0; f < 4; ++f) c[f] += w * ISB[f * WG + j + SG * t2];
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) ITB[f * WG + l] = c[f];
    }
    __syncthreads();
    if (nA) {
        R c[4] = {0, 0, 0, 0};
        if (t1 < nfA && t2 < nfA) {
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const R w = IA[t2 * N + j];
#pragma unroll
                for (int f = 0; f < 4; ++f) c[f] += w * ITA[f * WG + t1 + SG * j];
            }
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) vA[f] = c[f];
    }
    if (nB) {
        R c[4] = {0, 0, 0, 0};
        if (t1 < nfB && t2 < nfB) {
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const R w = IB[t2 * N + j];
#pragma unroll
                for (int f = 0; f < 4; ++f) c[f] += w * ITB[f * WG + t1 + SG * j];
            }
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) vB[f] = c[f];
    }
    __syncthreads();
}

// Transposed interpolation of the lifted flux of the two faces of one
// direction back to the element's face points (scratch: 1024 R at sm).
// UNI: every thread of the block reaches every barrier (the wavefronts of a
// multi-element tile lift different elements' faces side by side).  FSI: the
// field stride of the half-lifted arrays (rows t2 < n only: S n suffices).
template <class R, int P, bool UNI = false, int FSI = Geo<P>::W>
__device__ __forceinline__ void lift2(const R *itl, int nfA, int nfB, R *sm, R LA[4], R LB[4]) {
    constexpr int WG = Geo<P>::W, SG = Geo<P>::S;
    (void)WG;
    (void)SG;
    constexpr int N = P + 2;
    static_assert(FSI >= SG * N, "half-lifted rows t2 < n must fit the field stride");
    const bool nA = nfA != N, nB = nfB != N;
    if (!UNI && !nA && !nB) return;
    const int l = flane<P>(), t1 = gx<P>(l), t2 = gy<P>(l);
    R *ITA = sm, *ISA = sm + 4 * WG, *ITB = sm + 4 * WG + 4 * FSI, *ISB = sm + 8 * WG + 4 * FSI;
    const R *IA = itl + itab_off<P>(nfA), *IB = itl + itab_off<P>(nfB);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        if (nA) ITA[f * WG + l] = LA[f];
        if (nB) ITB[f * WG + l] = LB[f];
    }
    __syncthreads();
    if (nA && t1 < nfA && t2 < N) {
        R c[4] = {0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < Geo<P>::NFMAX; ++t) {
            if (t < nfA) {
                const R w = IA[t * N + t2];
#pragma unroll
                for (int f = 0; f < 4; ++f) c[f] += w * ITA[f * WG + t1 + SG * t];
            }
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) ISA[f * FSI + l] = c[f];
    }
    if (nB && t1 < nfB && t2 < N) {
        R c[4] = {0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < Geo<P>::NFMAX; ++t) {
            if (t < nfB) {
                const R w = IB[t * N + t2];
#pragma unroll
                for (int f = 0; f < 4; ++f) c[f] += w * ITB[f * WG + t1 + SG * t];
            }
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) ISB[f * FSI + l] = c[f];
    }
    __syncthreads();
    if (nA) {
        R c[4] = {0, 0, 0, 0};
        if (t1 < N && t2 < N) {
#pragma unroll
            for (int t = 0; t < Geo<P>::NFMAX; ++t) {
                if (t < nfA) {
                    const R w = IA[t * N + t1];
#pragma unroll
                    for (int f = 0; f < 4; ++f) c[f] += w * ISA[f * FSI + t + SG * t2];
                }
            }
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) LA[f] = c[f];
    }
    if (nB) {
        R c[4] = {0, 0, 0, 0};
        if (t1 < N && t2 < N) {
#pragma unroll
            for (int t = 0; t < Geo<P>::NFMAX; ++t) {
                if (t < nfB) {
                    const R w = IB[t * N + t1];
#pragma unroll
                    for (int f = 0; f < 4; ++f) c[f] += w * ISB[f * FSI + t + SG * t2];
                }
            }
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) LB[f] = c[f];
    }
    __syncthreads();
}

// Own (u, g) of the two faces of one direction from this lane's stashed
// fields (u, d_k u, d_a u, d_b u of each face, from entry f0 on): g = C . grad_xi u.
template <class R, int P>
__device__ __forceinline__ void own_from_stash(const R *OS, int f0, FaceD<R> &dA, FaceD<R> &dB) {
    constexpr int ws = Geo<P>::W;
    const int l = threadIdx.x;
    const R *o = OS + f0 * ws + l;
    dA.ou = o[0];
    dA.og = dA.Ck * o[ws] + dA.Ca * o[2 * ws] + dA.Cb * o[3 * ws];
    dB.ou = o[4 * ws];
    dB.og = dB.Ck * o[5 * ws] + dB.Ca * o[6 * ws] + dB.Cb * o[7 * ws];
}

// Flux of eq. IP at this lane's trace point from both sides' (u, g) in the
// trace buffer (apply kernel of the two-stage structure): this side's test
// terms L = (F_v, F_g C_k, F_g C_a, F_g C_b), not yet lifted.
template <class R, int P>
__device__ __forceinline__ void flux_tb(const FaceU<R> &fu, const FaceD<R> &fd, R L[4]) {
    const int l = flane<P>(), t1 = gx<P>(l), t2 = gy<P>(l);
    R Fv = 0, Fg = 0;
    if (t1 < fu.nf && t2 < fu.nf) {
        const R un = fu.slot == 2 ? -fd.ou : fd.n0;   // mirrored exterior state on the boundary
        const R gn = fu.slot == 2 ? -fd.og : fd.n1;
        const R jump = fd.ou - un;
        Fv = R(-0.5) * (fd.og - gn) + fu.tau * fd.aw * jump;
        Fg = R(-0.5) * jump;
    }
    L[0] = Fv;
    L[1] = Fg * fd.Ck;
    L[2] = Fg * fd.Ca;
    L[3] = Fg * fd.Cb;
}

// Reduction of the neighbour's coefficients along its face normal with
// P_i(s), P'_i(s) (first step of TracePhysEval), at lane (ia, ib) of its face
// modes; zero elsewhere and on boundary faces.
template <class R, int P>
__device__ __forceinline__ void nbr_reduce(const Data<R> &D, const FaceU<R> &fu, R &v0, R &v1) {
    v0 = v1 = R(0);
    if (fu.slot == 2) return;
    const int l = threadIdx.x, t1 = gx<P>(l), t2 = gy<P>(l);
    if (t1 < fu.npn && t2 < fu.npn) {
        const R *__restrict__ xn = D.x + fu.xn;
#pragma unroll
        for (int ik = 0; ik < 7; ++ik) {
            if (ik < fu.npn) {
                const R xv = xn[mode_rt(fu.npn, fu.kn, t1, t2, ik)];
                v0 += end_val<R>(ik, fu.sn) * xv;
                v1 += end_der<R>(ik, fu.sn) * xv;
            }
        }
    }
}

// The neighbours' u and g = C_n . grad_xi u_n at this lane's trace point for
// the two faces of one direction, from their face-normal reductions: the two
// contractions of TracePhysEval with the LDS trace tables, the second one at
// the neighbour's coordinates of this lane's point (scratch: 640 R at sm).
template <class R, int P>
__device__ __forceinline__ void nbr_pair(const R *btl, const FaceU<R> &fA, const FaceD<R> &dA, R a0, R a1,
                                         const FaceU<R> &fB, const FaceD<R> &dB, R b0, R b1, R *sm, R &unA,
                                         R &gnA, R &unB, R &gnB) {
    constexpr int WG = Geo<P>::W, SG = Geo<P>::S;
    (void)WG;
    (void)SG;
    const int l = threadIdx.x, t1 = gx<P>(l), t2 = gy<P>(l);
    R *NU = sm, *NWA = sm + 4 * WG, *NWB = sm + 7 * WG;
    const bool iA = fA.slot != 2, iB = fB.slot != 2;
    unA = gnA = unB = gnB = R(0);
    if (!iA && !iB) return;
    NU[l] = a0;
    NU[WG + l] = a1;
    NU[2 * WG + l] = b0;
    NU[3 * WG + l] = b1;
    __syncthreads();
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const FaceU<R> &f = side ? fB : fA;
        if (side ? !iB : !iA) continue;
        if (t1 < f.nf && t2 < f.npn) {
            const R *bf = btl + btab_off<P>(f.nf) + 7 * t1, *dbf = bf + 7 * f.nf;
            const R *u0 = NU + 2 * side * WG + SG * t2, *u1 = u0 + WG;
            R w0 = 0, w0d = 0, w1 = 0;
#pragma unroll
            for (int ia = 0; ia < 7; ++ia) {
                if (ia < f.npn) {
                    const R bv = bf[ia], x0 = u0[ia];
                    w0 += bv * x0;
                    w0d += dbf[ia] * x0;
                    w1 += bv * u1[ia];
                }
            }
            R *nw = side ? NWB : NWA;
            nw[l] = w0;
            nw[WG + l] = w0d;
            nw[2 * WG + l] = w1;
        }
    }
    __syncthreads();
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const FaceU<R> &f = side ? fB : fA;
        const FaceD<R> &d = side ? dB : dA;
        if (side ? !iB : !iA) continue;
        if (t1 < f.nf && t2 < f.nf) {
            int r1, r2;
            canon_inverse(f.on, f.nf, d.qc, r1, r2);
            const R *bf = btl + btab_off<P>(f.nf) + 7 * r2, *dbf = bf + 7 * f.nf;
            const R *nw = (side ? NWB : NWA) + r1;
            R vu = 0, vda = 0, vdb = 0, vdk = 0;
#pragma unroll
            for (int ib = 0; ib < 7; ++ib) {
                if (ib < f.npn) {
                    const R bv = bf[ib], w0 = nw[SG * ib];
                    vu += bv * w0;
                    vda += bv * nw[WG + SG * ib];
                    vdb += dbf[ib] * w0;
                    vdk += bv * nw[2 * WG + SG * ib];
                }
            }
            const R un = vu, gn = d.n0 * vdk + d.n1 * vda + d.n2 * vdb;
            if (side) {
                unB = un;
                gnB = gn;
            } else {
                unA = un;
                gnA = gn;
            }
        }
    }
    __syncthreads();
}

// Flux of eq. IP at this lane's trace point from the element's own (u, g) and
// the neighbour's (or the mirrored state on the boundary): this side's test
// terms L = (F_v, F_g C_k, F_g C_a, F_g C_b), not yet lifted.
template <class R, int P>
__device__ __forceinline__ void flux_own(const FaceU<R> &fu, const FaceD<R> &fd, R u, R g, R un, R gn, R L[4]) {
    const int l = threadIdx.x, t1 = gx<P>(l), t2 = gy<P>(l);
    R Fv = 0, Fg = 0;
    if (t1 < fu.nf && t2 < fu.nf) {
        if (fu.slot == 2) {
            un = -u;
            gn = -g;
        }
        const R jump = u - un;
        Fv = R(-0.5) * (g - gn) + fu.tau * fd.aw * jump;
        Fg = R(-0.5) * jump;
    }
    L[0] = Fv;
    L[1] = Fg * fd.Ck;
    L[2] = Fg * fd.Ca;
    L[3] = Fg * fd.Cb;
}

// Fused apply, one direction: own traces (interpolated when finer), the
// neighbours' by TracePhysEval, flux, lift back to the face points.
template <class R, int P>
__device__ __forceinline__ void face_pair_fused(const R *itl, const R *btl, const FaceU<R> &fA, const FaceD<R> &dA,
                                                R vA[4], R a0, R a1, const FaceU<R> &fB, const FaceD<R> &dB,
                                                R vB[4], R b0, R b1, R *sm, R LA[4], R LB[4]) {
    own_trace2<R, P>(itl, fA.nf, fB.nf, sm, vA, vB);
    const R gA = dA.Ck * vA[1] + dA.Ca * vA[2] + dA.Cb * vA[3];
    const R gB = dB.Ck * vB[1] + dB.Ca * vB[2] + dB.Cb * vB[3];
    R unA, gnA, unB, gnB;
    nbr_pair<R, P>(btl, fA, dA, a0, a1, fB, dB, b0, b1, sm, unA, gnA, unB, gnB);
    flux_own<R, P>(fA, dA, vA[0], gA, unA, gnA, LA);
    flux_own<R, P>(fB, dB, vB[0], gB, unB, gnB, LB);
    lift2<R, P>(itl, fA.nf, fB.nf, sm, LA, LB);
}

// 1-D mode i and its derivative at s = -1 (side 0) or +1 (side 1) for the
// basis of the handle: Legendre (P_i(+-1), P'_i(+-1)) or modified C0
// (psi_0 = (1 - x)/2, psi_1 = (1 + x)/2, bubbles zero at both ends with
// psi'_i(-1) = (-1)^i (i-1)/2, psi'_i(+1) = -(i-1)/2).
template <class R>
__device__ __forceinline__ void end_vd(int basis, int i, int s, R &v, R &d) {
    if (basis == 0) {
        v = end_val<R>(i, s);
        d = end_der<R>(i, s);
    } else if (i < 2) {
        v = (i == s) ? R(1) : R(0);
        d = i == 0 ? R(-0.5) : R(0.5);
    } else {
        const R h = R(0.5 * (i - 1));
        v = R(0);
        d = (s || (i & 1)) ? -h : h;
    }
}

// Gauss volume points (apply MODE 3): the element boundary is not among the
// volume points, so the faces' terms go to the modes directly.  For the two
// faces normal to xi_k, lane (t1, t2) forms L = (F_v, F_g C_k, F_g C_a,
// F_g C_b) at its trace point from both sides' (u, g) in the trace buffer;
// the transpose of the trace evaluation (TraceIProduct on the trace's GLL
// points, then the transpose of TracePhysEval's face-normal reduction) adds
//   sum_t L0 phi_i + L1 d_k phi_i + L2 d_a phi_i + L3 d_b phi_i
// to mode i = (i_k, i_a, i_b) of YF [NP^3].  The trace tables go to GT in
// LDS, loaded with the first direction's face data; each direction's face
// data is loaded while the previous one is contracted.  Scratch LS: 14 W.
template <class R, int P>
__device__ __forceinline__ void gauss_faces(const Args &A, const Data<R> &D, const MetaV<R> &meta, R *LS, R *YF,
                                            R *GT) {
    using G = GTab<P>;
    constexpr int NP = P + 1, N = P + 2, WG = Geo<P>::W, SG = Geo<P>::S, NM = NP * NP * NP;
    constexpr int HALF = G::SIZE / 2, BIT = (HALF + WG - 1) / WG;
    const int l = threadIdx.x, a = gx<P>(l), b = gy<P>(l);
    // table entry i of the BF half: set m, row t, mode j (the DBF entry follows the set's BF rows)
    R bv[2 * BIT];
    int bo[BIT];
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
        const int i = l + it * WG;
        int m = N, r = i;
#pragma unroll
        for (int mm = N; mm < G::M; ++mm)
            if (r >= m * NP) {
                r -= m * NP;
                ++m;
            }
        const int t = r / NP, j = r - t * NP;
        const bool ok = i < HALF;
        bv[2 * it] = ok ? D.tab[tab_off_BF(m) + t * S9 + j] : R(0);
        bv[2 * it + 1] = ok ? D.tab[tab_off_DBF(m) + t * S9 + j] : R(0);
        bo[it] = ok ? G::off(m) + r + ((m * NP) << 16) : -1;
    }
    FaceU<R> fu[2];
    FaceD<R> fd[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        fu[s] = face_uniform<R>(meta, s);
        fd[s] = load_face<R, P, 3>(D, fu[s], 0);
    }
    for (int i = l; i < NM; i += WG) YF[i] = R(0);
#pragma unroll
    for (int it = 0; it < BIT; ++it)
        if (bo[it] >= 0) {
            const int o = bo[it] & 0xffff, step = bo[it] >> 16;
            GT[o] = bv[2 * it];
            GT[o + step] = bv[2 * it + 1];
        }
    R *SS = LS + 8 * WG;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        int nfs[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            R L[4];
            flux_tb<R, P>(fu[s], fd[s], L);
#pragma unroll
            for (int f = 0; f < 4; ++f) LS[(4 * s + f) * WG + l] = L[f];
            nfs[s] = fu[s].nf;
        }
        if (k < 2) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                fu[s] = face_uniform<R>(meta, 2 * (k + 1) + s);
                fd[s] = load_face<R, P, 3>(D, fu[s], k + 1);
            }
        }
        __syncthreads();
        // transposed contraction along b: lane (t1, i_b)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int nf = nfs[s];
            if (a < nf && b < NP) {
                const R *bf = GT + G::off(nf) + b, *dbf = bf + nf * NP;
                const R *Lp = LS + 4 * s * WG + a;
                R s0 = 0, s1 = 0, s2 = 0;
                for (int t2 = 0; t2 < nf; ++t2) {
                    const R bt = bf[t2 * NP];
                    s0 += bt * Lp[SG * t2] + dbf[t2 * NP] * Lp[3 * WG + SG * t2];
                    s1 += bt * Lp[WG + SG * t2];
                    s2 += bt * Lp[2 * WG + SG * t2];
                }
                SS[3 * s * WG + l] = s0;
                SS[(3 * s + 1) * WG + l] = s1;
                SS[(3 * s + 2) * WG + l] = s2;
            }
        }
        __syncthreads();
        // transposed contraction along a, then the face-normal expansion:
        // lane (i_a, i_b) owns the modes (*, i_a, i_b) of this direction
        if (a < NP && b < NP) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int nf = nfs[s];
                const R *bf = GT + G::off(nf) + a, *dbf = bf + nf * NP;
                const R *Sp = SS + 3 * s * WG + SG * b;
                R v0 = 0, v1 = 0;
                for (int t1 = 0; t1 < nf; ++t1) {
                    const R bt = bf[t1 * NP];
                    v0 += bt * Sp[t1] + dbf[t1 * NP] * Sp[2 * WG + t1];
                    v1 += bt * Sp[WG + t1];
                }
#pragma unroll
                for (int ik = 0; ik < NP; ++ik) {
                    R ev, ed;
                    end_vd<R>(A.basis, ik, s, ev, ed);
                    YF[mode_rt(NP, k, a, b, ik)] += ev * v0 + ed * v1;
                }
            }
        }
        __syncthreads();
    }
}

// Where the apply takes an element's geometric factors from (a launch of
// one kind covers elements of one kind).
enum : int {
    GEO_POINT = 0,    // stored per-point factors G~ w and |J| w
    GEO_AFFINE = 1,   // affine element: 7 constants per element
    GEO_MAP = 2,      // from the element's trilinear map, at every point
};

// Points per batch of stored-factor loads in the pointwise terms (7 values
// per point), per order: as many as fit the register budget of the launch's
// occupancy (FP64 orders 3, 4 and 6 stay at 3 waves per SIMD with 3, 2 and 2
// points per batch, order 5 only with 1).  FP32 loads a whole column at once.
template <class R, int P>
struct PwBatch {
    static constexpr int N = P + 2;
    static constexpr int V = sizeof(R) == 4 ? N : (P <= 2 ? N : P == 3 ? 3 : P == 4 ? 2 : P == 6 ? 2 : 1);
};

// Pointwise terms of one column (q0, q1) = (a, b), in place:
// u <- lambda w |J| u, d <- (w G~) d with d the reference gradient.
// GEO_POINT reads the stored per-point factors, in chunks, so that the loads
// of one chunk are in flight together.  GEO_AFFINE (the paper's regular
// elements): constant G~ and |J|, 7 wave-uniform values per element, times the
// tensor GLL weight w_a w_b w_q.  GEO_MAP (deformed elements, geometry derived
// on the fly as the paper's design trades data for arithmetic): the
// trilinear map x = c0 + c1 xi0 + c2 xi1 + c3 xi2 + c4 xi0 xi1 + c5 xi0 xi2 +
// c6 xi1 xi2 + c7 xi0 xi1 xi2 gives, along the lane's column (xi0, xi1 fixed),
// dx/dxi0 and dx/dxi1 linear in xi2 and dx/dxi2 constant; the rows of adj(J)
// are the cross products of J's columns, G~ = adj adj^T / |J|.
template <class R, int P, int GEO>
__device__ __forceinline__ void pointwise(const Data<R> &D, const ElemDesc &ed, int a, int b, R *u, R *d0, R *d1,
                                          R *d2) {
    constexpr int N = P + 2, NPTS = N * N * N;
    const int64_t e = ed.e;
    if constexpr (GEO == GEO_MAP) {
        const ctab<R> cm = as_const(D.emap) + 24 * e;   // c1..c7, each (x, y, z)
        const ctab<R> Xq = as_const(D.tab) + tab_off_X(N);
        const ctab<R> W = as_const(D.tab) + tab_off_W(N);
        const R xa = D.tab[tab_off_X(N) + a], xb = D.tab[tab_off_X(N) + b];
        const R wab = D.tab[tab_off_W(N) + a] * D.tab[tab_off_W(N) + b];
        const R lam = D.lam[e];
        R A0[3], B0[3], A1[3], B1[3], J2[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const R c1 = cm[c], c2 = cm[3 + c], c3 = cm[6 + c], c4 = cm[9 + c];
            const R c5 = cm[12 + c], c6 = cm[15 + c], c7 = cm[18 + c];
            A0[c] = c1 + c4 * xb;
            B0[c] = c5 + c7 * xb;
            A1[c] = c2 + c4 * xa;
            B1[c] = c6 + c7 * xa;
            J2[c] = c3 + c5 * xa + (c6 + c7 * xa) * xb;
        }
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const R z = Xq[q];
            R j0[3], j1[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                j0[c] = A0[c] + B0[c] * z;
                j1[c] = A1[c] + B1[c] * z;
            }
            // rows of adj(J): j1 x j2, j2 x j0, j0 x j1
            const R r00 = j1[1] * J2[2] - j1[2] * J2[1], r01 = j1[2] * J2[0] - j1[0] * J2[2],
                    r02 = j1[0] * J2[1] - j1[1] * J2[0];
            const R r10 = J2[1] * j0[2] - J2[2] * j0[1], r11 = J2[2] * j0[0] - J2[0] * j0[2],
                    r12 = J2[0] * j0[1] - J2[1] * j0[0];
            const R r20 = j0[1] * j1[2] - j0[2] * j1[1], r21 = j0[2] * j1[0] - j0[0] * j1[2],
                    r22 = j0[0] * j1[1] - j0[1] * j1[0];
            const R det = j0[0] * r00 + j0[1] * r01 + j0[2] * r02;
            const R w = wab * W[q];
            const R s = w / det;
            const R g00 = s * (r00 * r00 + r01 * r01 + r02 * r02);
            const R g01 = s * (r00 * r10 + r01 * r11 + r02 * r12);
            const R g02 = s * (r00 * r20 + r01 * r21 + r02 * r22);
            const R g11 = s * (r10 * r10 + r11 * r11 + r12 * r12);
            const R g12 = s * (r10 * r20 + r11 * r21 + r12 * r22);
            const R g22 = s * (r20 * r20 + r21 * r21 + r22 * r22);
            const R c0 = d0[q], c1 = d1[q], c2 = d2[q];
            u[q] = lam * (w * det) * u[q];
            d0[q] = g00 * c0 + g01 * c1 + g02 * c2;
            d1[q] = g01 * c0 + g11 * c1 + g12 * c2;
            d2[q] = g02 * c0 + g12 * c1 + g22 * c2;
        }
        return;
    }
    if constexpr (GEO == GEO_AFFINE) {
        const ctab<R> eg = as_const(D.egeo) + 8 * e;
        const ctab<R> W = as_const(D.tab) + tab_off_W(N);
        const R G00 = eg[0], G01 = eg[1], G02 = eg[2], G11 = eg[3], G12 = eg[4], G22 = eg[5];
        const R lamj = D.lam[e] * eg[6];
        const R wab = D.tab[tab_off_W(N) + a] * D.tab[tab_off_W(N) + b];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const R w = wab * W[q];
            const R c0 = w * d0[q], c1 = w * d1[q], c2 = w * d2[q];
            u[q] = lamj * w * u[q];
            d0[q] = G00 * c0 + G01 * c1 + G02 * c2;
            d1[q] = G01 * c0 + G11 * c1 + G12 * c2;
            d2[q] = G02 * c0 + G12 * c1 + G22 * c2;
        }
        return;
    }
    const R *__restrict__ vg = D.vgeo + ed.voff + a + N * b;
    const R lam = D.lam[e];
    // QB points' factors are loaded before any of them is used (one memory
    // round trip per batch instead of one per point); the scheduling barrier
    // keeps the compiler from interleaving loads and uses again.
    constexpr int QB = PwBatch<R, P>::V;
#pragma unroll
    for (int q0 = 0; q0 < N; q0 += QB) {
        R g[QB][7];
#pragma unroll
        for (int j = 0; j < QB; ++j) {
            if (q0 + j < N) {
#pragma unroll
                for (int f = 0; f < 7; ++f) g[j][f] = vg[f * NPTS + N * N * (q0 + j)];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < QB; ++j) {
            const int q = q0 + j;
            if (q < N) {
                const R c0 = d0[q], c1 = d1[q], c2 = d2[q];
                u[q] = lam * g[j][6] * u[q];
                d0[q] = g[j][0] * c0 + g[j][1] * c1 + g[j][2] * c2;
                d1[q] = g[j][1] * c0 + g[j][3] * c1 + g[j][4] * c2;
                d2[q] = g[j][2] * c0 + g[j][4] * c1 + g[j][5] * c2;
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// MODE 1 (apply, two-stage): y = A x with both sides' (u, g) read from the
//   trace buffer written by the trace stage (k3t_elem); orders 6 and 8 take
//   their own (u, g) from their face values instead.
// MODE 2 (apply, fused): y = A x with the neighbours' traces evaluated here.
// MODE 3 (apply, Gauss volume points): the volume terms at the element's
//   Gauss points (tables and factors of that set: D.tab is the Gauss table
//   set, GEO the map or affine constants), the faces' terms from the trace
//   buffer lifted to the modes (gauss_faces), added at the write of y.
// One element: descriptor blk of A.desc / A.fdesc, LDS at smem_raw.
template <class R, int P, int MODE, int GEO = GEO_POINT>
__device__ __forceinline__ void k3g_elem(const Args &A, const Data<R> &D, int blk, unsigned char *smem_raw) {
    constexpr int WG = Geo<P>::W, SG = Geo<P>::S;
    (void)WG;
    (void)SG;
    using S = Sz<P>;
    constexpr int N = S::N, NP = S::NP, NPTS = S::NPTS;
    R *SA = reinterpret_cast<R *>(smem_raw);
    R *SB = SA + S::ARR;
    R *FB = SA + FB_OFF;
    const ElemDesc ed = A.desc[blk];
    const int64_t e = ed.e;
    const int l = threadIdx.x, a = gx<P>(l), b = gy<P>(l);
    const bool col = a < N && b < N;
    const ctab<R> Bt = as_const(D.tab) + tab_off_B(P);   // [N][NP]
    const ctab<R> Dt = as_const(D.tab) + tab_off_D(N);   // [N][N]
    const int64_t xo = ed.xoff;
    // Prologue: the first line contraction's coefficients, the face
    // descriptors and the interpolation tables are all requested before any
    // of them is waited for (one memory round trip instead of a chain).
    constexpr bool XEARLY = MODE != 3;
    R xv[NP];
    if (XEARLY && a < NP && b < NP) {
        const R *__restrict__ xe = D.x + xo + NP * (a + NP * b);
#pragma unroll
        for (int i = 0; i < NP; ++i) xv[i] = xe[i];
    }
    const MetaV<R> meta = load_meta<R, MODE>(A, D, blk);
    // interpolation tables I(n, m) of this order for m = n+1 .. the largest
    // trace: m n <= W entries each, one per lane, stored to LDS after the
    // first contraction (read after several syncs)
    R *itl = SA + S::TOTAL;
    constexpr int NIT = (MODE != 3 && Geo<P>::NFMAX > N) ? Geo<P>::NFMAX - N : 0;
    static_assert(Geo<P>::NFMAX * N <= WG || NIT == 0, "one table entry per lane");
    R itv[NIT > 0 ? NIT : 1];
#pragma unroll
    for (int j = 0; j < NIT; ++j) {
        const int m = N + 1 + j;
        itv[j] = l < m * N ? D.tab[tab_off_I(N, m) + l] : R(0);
    }
    // Gauss volume points: the faces' terms of every mode first (the point
    // arrays serve as scratch), kept after them
    R *YF = SA + S::TOTAL;
    if constexpr (MODE == 3) gauss_faces<R, P>(A, D, meta, SA, YF, YF + ((NP * NP * NP + 3) & ~3));
    // fused: the trace tables, and every neighbour's face-normal reduction
    // (their coefficient loads in flight together, during the volume work)
    R *btl = itl + ((ITab<P>::SIZE + 3) & ~3);
    R nv0[MODE == 2 ? 6 : 1], nv1[MODE == 2 ? 6 : 1];
    if (MODE == 2) {
#pragma unroll
        for (int m = N; m <= 8; ++m) {
            const R *__restrict__ bf = D.tab + tab_off_BF(m), *__restrict__ dbf = D.tab + tab_off_DBF(m);
            for (int i = l; i < 7 * m; i += WG) {
                btl[btab_off<P>(m) + i] = bf[(i / 7) * S9 + i % 7];
                btl[btab_off<P>(m) + 7 * m + i] = dbf[(i / 7) * S9 + i % 7];
            }
        }
#pragma unroll
        for (int f = 0; f < (MODE == 2 ? 6 : 0); ++f) nbr_reduce<R, P>(D, face_uniform<R>(meta, f), nv0[f], nv1[f]);
    }

    // BwdTrans along xi_0: lane (i1, i2)
    if (a < NP && b < NP) {
        if constexpr (!XEARLY) {
            const R *__restrict__ xe = D.x + xo + NP * (a + NP * b);
#pragma unroll
            for (int i = 0; i < NP; ++i) xv[i] = xe[i];
        }
#pragma unroll
        for (int q = 0; q < N; ++q) {
            R s = 0;
#pragma unroll
            for (int i = 0; i < NP; ++i) s += Bt[q * NP + i] * xv[i];
            SA[pa<P>(q, a, b)] = s;
        }
    }
#pragma unroll
    for (int j = 0; j < NIT; ++j) {
        const int m = N + 1 + j;
        if (l < m * N) itl[itab_off<P>(m) + l] = itv[j];
    }
    __syncthreads();
    // along xi_1: lane (q0, i2)
    if (a < N && b < NP) {
        R v[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) v[i] = SA[pa<P>(a, i, b)];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            R s = 0;
#pragma unroll
            for (int i = 0; i < NP; ++i) s += Bt[q * NP + i] * v[i];
            SB[pa<P>(a, q, b)] = s;
        }
    }
    __syncthreads();
    // along xi_2 into the column, and d_2 u in the column
    R u[N], d0[N], d1[N], d2[N];
    if (col) {
        R v[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) v[i] = SB[pa<P>(a, b, i)];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            R s = 0;
#pragma unroll
            for (int i = 0; i < NP; ++i) s += Bt[q * NP + i] * v[i];
            u[q] = s;
        }
#pragma unroll
        for (int q = 0; q < N; ++q) {
            R s = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) s += Dt[q * N + j] * u[j];
            d2[q] = s;
        }
    }
    __syncthreads();
    if (col) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            SA[pa<P>(a, b, q)] = u[q];
            SB[pa<P>(a, b, q)] = d2[q];
        }
    }
    __syncthreads();
    // apply kernels: the first faces' per-point data in flight during the line
    // phases (orders whose own traces come from registers: after the pointwise
    // terms, which keeps them within the register budget of 3 waves per SIMD)
    FaceU<R> fu0, fu1;
    FaceD<R> fd0, fd1;
    constexpr bool FACE_LATE = MODE == 1 && S::OWN;
    if constexpr (MODE != 3 && !FACE_LATE) {
        fu0 = face_uniform<R>(meta, 0);
        fd0 = load_face<R, P, MODE>(D, fu0, 0);
        fu1 = face_uniform<R>(meta, 1);
        fd1 = load_face<R, P, MODE>(D, fu1, 0);
    }
    // d_0 u on line-0 lanes (q1, q2) = (a, b), d_1 u on line-1 lanes (q0, q2) = (a, b);
    // keep the faces' values at the line ends
    R x_u[2], x_dk[2], x_da[2], x_db[2];   // faces normal to xi_0 at (q1, q2) = (a, b)
    R y_u[2], y_dk[2], y_da[2], y_db[2];   // faces normal to xi_1 at (q0, q2) = (a, b)
    R l0[N], l1[N];
    if (col) {
        R v[N], w[N];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            v[j] = SA[pa<P>(j, a, b)];
            w[j] = SA[pa<P>(a, j, b)];
        }
        x_db[0] = SB[pa<P>(0, a, b)];
        x_db[1] = SB[pa<P>(N - 1, a, b)];
        y_db[0] = SB[pa<P>(a, 0, b)];
        y_db[1] = SB[pa<P>(a, N - 1, b)];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            R s = 0, t = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                s += Dt[q * N + j] * v[j];
                t += Dt[q * N + j] * w[j];
            }
            l0[q] = s;
            l1[q] = t;
        }
        x_u[0] = v[0];
        x_u[1] = v[N - 1];
        x_dk[0] = l0[0];
        x_dk[1] = l0[N - 1];
        y_u[0] = w[0];
        y_u[1] = w[N - 1];
        y_dk[0] = l1[0];
        y_dk[1] = l1[N - 1];
    }
    __syncthreads();
    if (col) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            SA[pa<P>(q, a, b)] = l0[q];
            SB[pa<P>(a, q, b)] = l1[q];
        }
    }
    __syncthreads();
    R z_u[2], z_dk[2], z_da[2], z_db[2];   // faces normal to xi_2 at (q0, q1) = (a, b)
    if (col) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            d0[q] = SA[pa<P>(a, b, q)];
            d1[q] = SB[pa<P>(a, b, q)];
        }
    }
    if (col) {
        x_da[0] = SB[pa<P>(0, a, b)];
        x_da[1] = SB[pa<P>(N - 1, a, b)];
        y_da[0] = SA[pa<P>(a, 0, b)];
        y_da[1] = SA[pa<P>(a, N - 1, b)];
        z_u[0] = u[0];
        z_u[1] = u[N - 1];
        z_dk[0] = d2[0];
        z_dk[1] = d2[N - 1];
        z_da[0] = SA[pa<P>(a, b, 0)];
        z_da[1] = SA[pa<P>(a, b, N - 1)];
        z_db[0] = SB[pa<P>(a, b, 0)];
        z_db[1] = SB[pa<P>(a, b, N - 1)];
    }
    R *OS = SA + S::STASH_OFF;   // own-field stash (S::OWN), over the point arrays
    if constexpr (MODE == 1 && S::OWN) {
        __syncthreads();   // every lane's point-array reads before the stash overwrites them
        // the fields of the faces normal to xi_1 and xi_2 kept in the stash;
        // those normal to xi_0 stay in registers
        if (col) {
            const R st[16] = {y_u[0], y_dk[0], y_da[0], y_db[0], y_u[1], y_dk[1], y_da[1], y_db[1],
                              z_u[0], z_dk[0], z_da[0], z_db[0], z_u[1], z_dk[1], z_da[1], z_db[1]};
#pragma unroll
            for (int f = 0; f < 16; ++f) OS[f * WG + l] = st[f];
        }
    }
    __syncthreads();


    if constexpr (MODE == 3) {
        if (col) pointwise<R, P, GEO>(D, ed, a, b, u, d0, d1, d2);
    } else if constexpr (MODE == 1) {
    // pointwise: m = lambda w|J| u, q = (G w) grad_xi u  (in place: u <- m, d <- q);
    // in chunks, so that the factor loads of one chunk are in flight together
    if (col) pointwise<R, P, GEO>(D, ed, a, b, u, d0, d1, d2);
        if constexpr (FACE_LATE) {
            fu0 = face_uniform<R>(meta, 0);
            fd0 = load_face<R, P, MODE>(D, fu0, 0);
            fu1 = face_uniform<R>(meta, 1);
            fd1 = load_face<R, P, MODE>(D, fu1, 0);
            // own (u, g) of the faces normal to xi_0 from the registers
            fd0.ou = x_u[0];
            fd0.og = fd0.Ck * x_dk[0] + fd0.Ca * x_da[0] + fd0.Cb * x_db[0];
            fd1.ou = x_u[1];
            fd1.og = fd1.Ck * x_dk[1] + fd1.Ca * x_da[1] + fd1.Cb * x_db[1];
        }

        // faces, both of one direction at a time: flux from the trace buffer,
        // lifted back to the face points, added to the pointwise terms.
        // Normal to xi_0: own points (q1, q2) on column lanes q0 = 0, n-1.
        {
            R LA[4], LB[4];
            flux_tb<R, P>(fu0, fd0, LA);
            flux_tb<R, P>(fu1, fd1, LB);
            const FaceU<R> fu2 = face_uniform<R>(meta, 2);
            FaceD<R> fd2 = load_face<R, P, MODE>(D, fu2, 1);
            const FaceU<R> fu3 = face_uniform<R>(meta, 3);
            FaceD<R> fd3 = load_face<R, P, MODE>(D, fu3, 1);
            lift2<R, P>(itl, fu0.nf, fu1.nf, SA + 8 * WG, LA, LB);
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                FB[f * WG + l] = LA[f];
                FB[4 * WG + f * WG + l] = LB[f];
            }
            __syncthreads();
            if (col && (a == 0 || a == N - 1)) {
                const R *fb = FB + (a == 0 ? 0 : 4 * WG) + b;
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    u[q] += fb[SG * q];
                    d0[q] += fb[WG + SG * q];
                    d1[q] += fb[2 * WG + SG * q];
                    d2[q] += fb[3 * WG + SG * q];
                }
            }
            __syncthreads();
            // normal to xi_1: own points (q0, q2) on column lanes q1 = 0, n-1
            if constexpr (S::OWN) own_from_stash<R, P>(OS, 0, fd2, fd3);
            flux_tb<R, P>(fu2, fd2, LA);
            flux_tb<R, P>(fu3, fd3, LB);
            fu0 = face_uniform<R>(meta, 4);
            fd0 = load_face<R, P, MODE>(D, fu0, 2);
            fu1 = face_uniform<R>(meta, 5);
            fd1 = load_face<R, P, MODE>(D, fu1, 2);
            lift2<R, P>(itl, fu2.nf, fu3.nf, SA + 8 * WG, LA, LB);
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                FB[f * WG + l] = LA[f];
                FB[4 * WG + f * WG + l] = LB[f];
            }
            __syncthreads();
            if (col && (b == 0 || b == N - 1)) {
                const R *fb = FB + (b == 0 ? 0 : 4 * WG) + a;
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    u[q] += fb[SG * q];
                    d1[q] += fb[WG + SG * q];
                    d0[q] += fb[2 * WG + SG * q];
                    d2[q] += fb[3 * WG + SG * q];
                }
            }
            __syncthreads();
            // normal to xi_2: own points (q0, q1) are the column ends
            if constexpr (S::OWN) own_from_stash<R, P>(OS, 8, fd0, fd1);
            flux_tb<R, P>(fu0, fd0, LA);
            flux_tb<R, P>(fu1, fd1, LB);
            lift2<R, P>(itl, fu0.nf, fu1.nf, SA + 8 * WG, LA, LB);
            if (col) {
                u[0] += LA[0];
                d2[0] += LA[1];
                d0[0] += LA[2];
                d1[0] += LA[3];
                u[N - 1] += LB[0];
                d2[N - 1] += LB[1];
                d0[N - 1] += LB[2];
                d1[N - 1] += LB[3];
            }
        }
    } else {
        // fused: as the two-stage apply, with the element's own traces from its
        // face values and the neighbours' evaluated here
        if (col) pointwise<R, P, GEO_POINT>(D, ed, a, b, u, d0, d1, d2);
        R LA[4], LB[4];
        {
            const FaceU<R> fu2 = face_uniform<R>(meta, 2);
            const FaceD<R> fd2 = load_face<R, P, MODE>(D, fu2, 1);
            const FaceU<R> fu3 = face_uniform<R>(meta, 3);
            const FaceD<R> fd3 = load_face<R, P, MODE>(D, fu3, 1);
            R vA[4] = {x_u[0], x_dk[0], x_da[0], x_db[0]}, vB[4] = {x_u[1], x_dk[1], x_da[1], x_db[1]};
            face_pair_fused<R, P>(itl, btl, fu0, fd0, vA, nv0[0], nv1[0], fu1, fd1, vB, nv0[1], nv1[1], SA + 8 * WG,
                                  LA, LB);
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                FB[f * WG + l] = LA[f];
                FB[4 * WG + f * WG + l] = LB[f];
            }
            __syncthreads();
            if (col && (a == 0 || a == N - 1)) {
                const R *fb = FB + (a == 0 ? 0 : 4 * WG) + b;
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    u[q] += fb[SG * q];
                    d0[q] += fb[WG + SG * q];
                    d1[q] += fb[2 * WG + SG * q];
                    d2[q] += fb[3 * WG + SG * q];
                }
            }
            __syncthreads();
            fu0 = face_uniform<R>(meta, 4);
            fd0 = load_face<R, P, MODE>(D, fu0, 2);
            fu1 = face_uniform<R>(meta, 5);
            fd1 = load_face<R, P, MODE>(D, fu1, 2);
            R wA[4] = {y_u[0], y_dk[0], y_da[0], y_db[0]}, wB[4] = {y_u[1], y_dk[1], y_da[1], y_db[1]};
            face_pair_fused<R, P>(itl, btl, fu2, fd2, wA, nv0[2], nv1[2], fu3, fd3, wB, nv0[3], nv1[3], SA + 8 * WG,
                                  LA, LB);
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                FB[f * WG + l] = LA[f];
                FB[4 * WG + f * WG + l] = LB[f];
            }
            __syncthreads();
            if (col && (b == 0 || b == N - 1)) {
                const R *fb = FB + (b == 0 ? 0 : 4 * WG) + a;
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    u[q] += fb[SG * q];
                    d1[q] += fb[WG + SG * q];
                    d0[q] += fb[2 * WG + SG * q];
                    d2[q] += fb[3 * WG + SG * q];
                }
            }
            __syncthreads();
        }
        {
            R vA[4] = {z_u[0], z_dk[0], z_da[0], z_db[0]}, vB[4] = {z_u[1], z_dk[1], z_da[1], z_db[1]};
            face_pair_fused<R, P>(itl, btl, fu0, fd0, vA, nv0[4], nv1[4], fu1, fd1, vB, nv0[5], nv1[5], SA + 8 * WG,
                                  LA, LB);
            if (col) {
                u[0] += LA[0];
                d2[0] += LA[1];
                d0[0] += LA[2];
                d1[0] += LA[3];
                u[N - 1] += LB[0];
                d2[N - 1] += LB[1];
                d0[N - 1] += LB[2];
                d1[N - 1] += LB[3];
            }
        }
    }

    // IProduct: y = B^T (m + D_0^T q_0 + D_1^T q_1 + D_2^T q_2)
    if constexpr (MODE == 1 && S::OWN) __syncthreads();   // the stash reads before the point arrays return
    R z[N];
    if (col) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            SA[pa<P>(a, b, q)] = d0[q];
            SB[pa<P>(a, b, q)] = d1[q];
        }
#pragma unroll
        for (int j = 0; j < N; ++j) {
            R s = u[j];
#pragma unroll
            for (int q = 0; q < N; ++q) s += Dt[q * N + j] * d2[q];
            z[j] = s;
        }
    }
    __syncthreads();
    if (col) {
        R v[N], w[N];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            v[j] = SA[pa<P>(j, a, b)];
            w[j] = SB[pa<P>(a, j, b)];
        }
#pragma unroll
        for (int j = 0; j < N; ++j) {
            R s = 0, t = 0;
#pragma unroll
            for (int q = 0; q < N; ++q) {
                s += Dt[q * N + j] * v[q];
                t += Dt[q * N + j] * w[q];
            }
            l0[j] = s;
            l1[j] = t;
        }
    }
    __syncthreads();
    if (col) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            SA[pa<P>(q, a, b)] = l0[q];
            SB[pa<P>(a, q, b)] = l1[q];
        }
    }
    __syncthreads();
    R w2[NP];
    if (col) {
#pragma unroll
        for (int q = 0; q < N; ++q) z[q] += SA[pa<P>(a, b, q)] + SB[pa<P>(a, b, q)];
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            R s = 0;
#pragma unroll
            for (int q = 0; q < N; ++q) s += Bt[q * NP + i] * z[q];
            w2[i] = s;
        }
    }
    __syncthreads();
    if (col) {
#pragma unroll
        for (int i = 0; i < NP; ++i) SA[pa<P>(a, b, i)] = w2[i];
    }
    __syncthreads();
    // B^T along xi_1: lane (q0, i2)
    if (a < N && b < NP) {
        R v[N];
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] = SA[pa<P>(a, j, b)];
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            R s = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) s += Bt[j * NP + i] * v[j];
            SB[pa<P>(a, i, b)] = s;
        }
    }
    __syncthreads();
    // B^T along xi_0: lane (i1, i2), y written once
    if (a < NP && b < NP) {
        R v[N];
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] = SB[pa<P>(j, a, b)];
        R *__restrict__ ye = D.y + xo + NP * (a + NP * b);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            R s = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) s += Bt[j * NP + i] * v[j];
            if constexpr (MODE == 3) s += YF[i + NP * (a + NP * b)];
            ye[i] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// Trace kernel by face reductions (the element's own trace evaluation, eq.
// TracePhysEval of Sec. 3.2): for the two faces normal to xi_k, lane (ia, ib)
// reduces the coefficients along xi_k against P_i(+-1) and P'_i(+-1); two 1-D
// contractions with P_i, P'_i at the face's n_F GLL trace points then give u
// and grad_xi u there directly.  u is a polynomial of degree p in each
// direction, so this equals interpolating the face values at the p + 2 GLL
// points to the trace (up to rounding), without the volume transform.
//
// LDS (R units): the coefficients [NP^3], the reductions of one direction
// [4][W], the first contractions of its two faces [2 sides][3][W], and the
// trace tables P_i(z_t), P'_i(z_t), t < m, i < NP for m = n .. NFMAX.
template <int P>
struct TSz {
    static constexpr int NP = P + 1, N = P + 2, W = Geo<P>::W, M = Geo<P>::NFMAX;
    static constexpr int XS = (NP * NP * NP + 1) & ~1;
    static constexpr int NU = 4 * W, NW = 6 * W;
    // table set of m trace points: BF [m][NP] then DBF [m][NP]
    static constexpr int bt_off(int m) { return NP * ((m - 1) * m - (N - 1) * N); }
    static constexpr int BT = bt_off(M + 1);
    static constexpr int TOTAL = XS + NU + NW + BT;
};

template <class R, int P, int BASIS = 0, bool P2P = false, bool FOLD = false>
__device__ __forceinline__ void k3t_elem(const Args &A, const Data<R> &D, int blk, unsigned char *smem_raw) {
    using T = TSz<P>;
    constexpr int NP = T::NP, N = T::N, WG = T::W, SG = Geo<P>::S, NM = NP * NP * NP;
    R *XS = reinterpret_cast<R *>(smem_raw);
    R *NU = XS + T::XS;
    R *NW = NU + T::NU;
    R *BT = NW + T::NW;
    const ElemDesc ed = A.desc[blk];
    const int l = threadIdx.x, a = gx<P>(l), b = gy<P>(l);
    const bool ln = a < NP && b < NP;
    const MetaV<R> meta = load_meta<R, 0>(A, D, blk);
    // point-to-point flux (every face side on its own point set): lane f < 6
    // holds the neighbour's n, slot and factor / buffer offsets of face f
    int nb_no = 0, nb_so = 0;
    int64_t nb_fo = 0, nb_to = 0;
    if constexpr (P2P) {
        if ((l & 63) < 6) {
            const FaceDesc fr = A.fdesc[(int64_t)blk * 6 + (l & 63)];
            const int slot = face_slot(fr.info);
            if (slot != 2) {
                const FaceTopo ft = A.faces[fr.F];
                nb_so = 1 - slot;
                nb_no = A.order[slot == 0 ? ft.eR : ft.eL] + 2;
                nb_fo = A.side[(int64_t)fr.F * 4 + 2 * nb_so];
                nb_to = A.side[(int64_t)fr.F * 4 + 2 * nb_so + 1];
            }
        }
    }
    // the coefficients (coalesced) and the trace tables into LDS: every load
    // issued before the first store
    constexpr int XIT = (NM + WG - 1) / WG, BIT = (T::BT / 2 + WG - 1) / WG;
    R xv[XIT], bv[2 * BIT];
    if constexpr (FOLD) {
        // the CG step on this element's entries (arithmetic as the separate
        // vector kernels: in FP64, rounded to R once per stored value)
        const int pr = D.eprob[ed.e];
        const double al = D.fold_alpha[pr], be = D.fold_beta[pr];
        const bool stop = D.fold_conv[pr] != 0;
        R *__restrict__ pe = D.fold_p + ed.xoff;
        R *__restrict__ xe = D.fold_x + ed.xoff;
        const R *__restrict__ re = D.fold_r + ed.xoff;
        const R *__restrict__ de = D.fold_dinv ? D.fold_dinv + ed.xoff : nullptr;
        R po[XIT], xo[XIT], ro[XIT], dv[XIT];
#pragma unroll
        for (int it = 0; it < XIT; ++it) {
            const int i = l + it * WG;
            const int j = (it + 1) * WG <= NM || i < NM ? i : 0;
            po[it] = pe[j];
            xo[it] = xe[j];
            ro[it] = re[j];
            dv[it] = de ? de[j] : R(1);
        }
#pragma unroll
        for (int it = 0; it < XIT; ++it) {
            const int i = l + it * WG;
            const R z = de ? (R)((double)dv[it] * (double)ro[it]) : ro[it];
            const R pn = stop ? po[it] : (R)((double)z + be * (double)po[it]);
            xv[it] = (it + 1) * WG <= NM || i < NM ? pn : R(0);
            if ((it + 1) * WG <= NM || i < NM) {
                xe[i] = (R)((double)xo[it] + al * (double)po[it]);
                pe[i] = pn;
            }
        }
    } else {
        const R *__restrict__ xe = D.x + ed.xoff;
#pragma unroll
        for (int it = 0; it < XIT; ++it) {
            const int i = l + it * WG;
            xv[it] = (it + 1) * WG <= NM || i < NM ? xe[i < NM ? i : 0] : R(0);
        }
    }
    // table entry i of the BF half: set m, row t, mode j (the DBF entry follows the row set)
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
        const int i = l + it * WG;
        int m = N, r = i;
#pragma unroll
        for (int mm = N; mm < T::M; ++mm)
            if (r >= m * NP) {
                r -= m * NP;
                ++m;
            }
        const int t = r / NP, j = r - t * NP;
        const bool ok = i < T::BT / 2;
        bv[2 * it] = ok ? D.tab[tab_off_BF(m) + t * S9 + j] : R(0);
        bv[2 * it + 1] = ok ? D.tab[tab_off_DBF(m) + t * S9 + j] : R(0);
    }
    // every face's per-point data in flight meanwhile
    FaceU<R> tu[6];
    FaceD<R> td[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        tu[f] = face_uniform<R>(meta, f);
        td[f] = load_face<R, P, 0>(D, tu[f], f >> 1);
    }
#pragma unroll
    for (int it = 0; it < XIT; ++it)
        if ((it + 1) * WG <= NM || l + it * WG < NM) XS[l + it * WG] = xv[it];
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
        const int i = l + it * WG;
        if (i < T::BT / 2) {
            int m = N, r = i;
#pragma unroll
            for (int mm = N; mm < T::M; ++mm)
                if (r >= m * NP) {
                    r -= m * NP;
                    ++m;
                }
            BT[T::bt_off(m) + r] = bv[2 * it];
            BT[T::bt_off(m) + m * NP + r] = bv[2 * it + 1];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        // reductions along xi_k at xi_k = -1 (r0: u, r1: d_k u) and +1 (r2, r3)
        R r0 = 0, r1 = 0, r2 = 0, r3 = 0;
        if (ln) {
#pragma unroll
            for (int ik = 0; ik < NP; ++ik) {
                const int idx = k == 0 ? ik + NP * (a + NP * b) : (k == 1 ? a + NP * (ik + NP * b) : a + NP * (b + NP * ik));
                const R xv = XS[idx];
                if constexpr (BASIS == 0) {
                    // Legendre: P_i(+-1) = (+-1)^i, P'_i(+-1) = (+-1)^(i+1) i(i+1)/2
                    const R dv = R(0.5 * ik * (ik + 1));
                    const R sx = (ik & 1) ? -xv : xv;
                    r0 += sx;
                    r1 -= dv * sx;
                    r2 += xv;
                    r3 += dv * xv;
                } else {
                    // modified C0: psi_0(-1) = psi_1(+1) = 1, bubbles vanish at
                    // the ends; psi'_0 = -1/2, psi'_1 = 1/2, and for i >= 2
                    // psi'_i(-1) = (-1)^i (i-1)/2, psi'_i(+1) = -(i-1)/2
                    if (ik == 0) {
                        r0 += xv;
                        r1 -= R(0.5) * xv;
                        r3 -= R(0.5) * xv;
                    } else if (ik == 1) {
                        r2 += xv;
                        r1 += R(0.5) * xv;
                        r3 += R(0.5) * xv;
                    } else {
                        const R dv = R(0.5 * (ik - 1));
                        r1 += (ik & 1) ? -dv * xv : dv * xv;
                        r3 -= dv * xv;
                    }
                }
            }
        }
        NU[l] = r0;
        NU[WG + l] = r1;
        NU[2 * WG + l] = r2;
        NU[3 * WG + l] = r3;
        __syncthreads();
        // first contraction, along the face direction a: lane (t1, ib)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const FaceU<R> &fu = tu[2 * k + s];
            if (a < fu.nf && b < NP) {
                const R *bf = BT + T::bt_off(fu.nf) + NP * a, *dbf = bf + fu.nf * NP;
                const R *u0 = NU + 2 * s * WG + SG * b, *u1 = u0 + WG;
                R w0 = 0, w0d = 0, w1 = 0;
#pragma unroll
                for (int ia = 0; ia < NP; ++ia) {
                    const R x0 = u0[ia];
                    w0 += bf[ia] * x0;
                    w0d += dbf[ia] * x0;
                    w1 += bf[ia] * u1[ia];
                }
                NW[3 * s * WG + l] = w0;
                NW[(3 * s + 1) * WG + l] = w0d;
                NW[(3 * s + 2) * WG + l] = w1;
            }
        }
        __syncthreads();
        // second contraction, along b: lane (t1, t2); g = C . grad_xi u; store
        R pv[2][4];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const FaceU<R> &fu = tu[2 * k + s];
            const FaceD<R> &fd = td[2 * k + s];
            pv[s][0] = pv[s][1] = pv[s][2] = pv[s][3] = R(0);
            if (a < fu.nf && b < fu.nf) {
                const R *bf = BT + T::bt_off(fu.nf) + NP * b, *dbf = bf + fu.nf * NP;
                const R *w0 = NW + 3 * s * WG + a, *w0d = w0 + WG, *w1 = w0 + 2 * WG;
                R vu = 0, vda = 0, vdb = 0, vdk = 0;
#pragma unroll
                for (int ib = 0; ib < NP; ++ib) {
                    const R bv = bf[ib], x0 = w0[SG * ib];
                    vu += bv * x0;
                    vda += bv * w0d[SG * ib];
                    vdb += dbf[ib] * x0;
                    vdk += bv * w1[SG * ib];
                }
                R *__restrict__ tb = D.tbuf + fu.to + tb_side(fu.slot) * 2 * fu.npf + fd.qc;
                tb[0] = vu;
                tb[fu.npf] = fd.Ck * vdk + fd.Ca * vda + fd.Cb * vdb;
                pv[s][0] = vu;
                pv[s][1] = vda;
                pv[s][2] = vdb;
                pv[s][3] = vdk;
            }
        }
        if constexpr (P2P) {
            // this side's u and grad_x u (own points, canonical order) to the
            // neighbour's points: two passes through LDS (I(n -> n_o)); then
            // (I u, -an_o . I grad u) into the neighbour's slot
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int f = 2 * k + s;
                const int no = rl32(nb_no, f);
                if (no == 0) continue;   // boundary face (uniform)
                __syncthreads();
                if (a < N && b < N) {
                    const R *X = D.tab + tab_off_X(N);
                    R xi[3], d[3];
                    xi[k] = s ? R(1) : R(-1);
                    xi[dir_a(k)] = X[a];
                    xi[dir_b(k)] = X[b];
                    d[k] = pv[s][3];
                    d[dir_a(k)] = pv[s][1];
                    d[dir_b(k)] = pv[s][2];
                    R r[3][3];
                    const R inv = R(1) / map_adjugate3<R>(D.emap + (int64_t)24 * ed.e, xi[0], xi[1], xi[2], r);
                    const int qc = td[f].qc;
                    NU[qc] = pv[s][0];
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        NU[(1 + c) * N * N + qc] = (r[0][c] * d[0] + r[1][c] * d[1] + r[2][c] * d[2]) * inv;
                }
                __syncthreads();
                const R *I = D.tab + tab_off_I(N, no);   // [no][N]
                for (int i = l; i < N * no; i += WG) {
                    const int t1 = i % no, j2 = i / no;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        R acc = 0;
#pragma unroll
                        for (int j1 = 0; j1 < N; ++j1) acc += I[t1 * N + j1] * NU[c * N * N + j2 * N + j1];
                        NW[c * N * no + j2 * no + t1] = acc;
                    }
                }
                __syncthreads();
                const int so = rl32(nb_so, f), npo = no * no;
                const int64_t fo = rl64(nb_fo, f), to = rl64(nb_to, f);
                for (int i = l; i < npo; i += WG) {
                    const int t1 = i % no, t2 = i / no;
                    R w[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        R acc = 0;
#pragma unroll
                        for (int j2 = 0; j2 < N; ++j2) acc += I[t2 * N + j2] * NW[c * N * no + j2 * no + t1];
                        w[c] = acc;
                    }
                    const R *an = D.fgeo + fo + (so == 1 ? 1 : 4) * npo + i;
                    R *__restrict__ tb = D.tbuf + to + (so == 1 ? 0 : 2 * npo) + i;
                    tb[0] = w[0];
                    tb[npo] = -(an[0] * w[1] + an[npo] * w[2] + an[2 * npo] * w[3]);
                }
            }
            __syncthreads();
        }
    }
}

template <class R, int P, int BASIS = 0, bool P2P = false>
__global__ __launch_bounds__(Geo<P>::W) void k3t(Args A, Data<R> D) {
    if (A.skip && *A.skip) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    k3t_elem<R, P, BASIS, P2P>(A, D, blockIdx.x, smem_raw);
}

// Trace stage of every element of order <= 6 (traces <= 8 x 8) in one launch:
// block b takes element b of A.desc / A.fdesc, its order in ElemDesc::pad.
template <class R, int BASIS = 0, bool P2P = false, bool FOLD = false>
__global__ __launch_bounds__(W) void k3t_all(Args A, Data<R> D) {
    if (A.skip && *A.skip) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int i = blockIdx.x;
    switch (A.desc[i].pad & ELEM_ORDER_MASK) {
    case 1: k3t_elem<R, 1, BASIS, P2P, FOLD>(A, D, i, smem_raw); break;
    case 2: k3t_elem<R, 2, BASIS, P2P, FOLD>(A, D, i, smem_raw); break;
    case 3: k3t_elem<R, 3, BASIS, P2P, FOLD>(A, D, i, smem_raw); break;
    case 4: k3t_elem<R, 4, BASIS, P2P, FOLD>(A, D, i, smem_raw); break;
    case 5: k3t_elem<R, 5, BASIS, P2P, FOLD>(A, D, i, smem_raw); break;
    default: k3t_elem<R, 6, BASIS, P2P, FOLD>(A, D, i, smem_raw); break;
    }
}
__host__ __device__ constexpr int lds_trace_all() {
    int m = 0;
    const int v[6] = {TSz<1>::TOTAL, TSz<2>::TOTAL, TSz<3>::TOTAL, TSz<4>::TOTAL, TSz<5>::TOTAL, TSz<6>::TOTAL};
    for (int i = 0; i < 6; ++i) m = v[i] > m ? v[i] : m;
    return m;
}

// LDS (R units) of a launch: the trace kernel (mode 0) or the apply kernels
template <int P>
__host__ __device__ constexpr int lds_mode(int mode) {
    return mode == 0 ? TSz<P>::TOTAL : lds_total<P>(mode);
}

// Waves per SIMD the compiler sizes the registers of a kernel for.  The FP64
// map-geometry applies of orders 3 and 4 fit 3 waves (168 VGPRs; order 4 with
// a 60-byte spill) and gain 7 and 3 us on the 32^3 mesh; orders 5 and 6 spill
// 132 and 204 bytes there and lose, so they stay at 2.  The FP64 stored-factor
// apply of order 6 fits 3 waves (16-byte spill; its stash shares the face
// scratch, so its LDS allows 3 as well) and gains 5 us.
template <class R, int P, int MODE, int GEO = GEO_POINT>
struct Occ {
    static constexpr int V = (GEO == GEO_MAP && sizeof(R) == 8 && (P == 3 || P == 4)) ? 3
                             : (sizeof(R) == 8 && P == 6 && MODE == 1 && GEO == GEO_POINT) ? 3 : 2;
};

// One launch per order group (and per affine / deformed part of it): block b
// handles element b of A.desc.
template <class R, int P, int MODE, int GEO = GEO_POINT>
__global__ __launch_bounds__(Geo<P>::W) __attribute__((amdgpu_waves_per_eu(Occ<R, P, MODE, GEO>::V))) void k3g(Args A,
                                                                                                         Data<R> D) {
    if (A.skip && *A.skip) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    k3g_elem<R, P, MODE, GEO>(A, D, blockIdx.x, smem_raw);
}

// LDS of the persistent kernel: the largest order's.
template <int MODE>
__host__ __device__ constexpr int lds_persistent() {
    int m = 0;
    const int v[6] = {lds_mode<1>(MODE), lds_mode<2>(MODE), lds_mode<3>(MODE),
                      lds_mode<4>(MODE), lds_mode<5>(MODE), lds_mode<6>(MODE)};
    for (int i = 0; i < 6; ++i) m = v[i] > m ? v[i] : m;
    return m;
}

template <class R, int P, int MODE>
__device__ __forceinline__ void gf_elem(const Args &A, const Data<R> &D, int blk, unsigned char *smem_raw) {
    if constexpr (MODE == 0) k3t_elem<R, P>(A, D, blk, smem_raw);
    else k3g_elem<R, P, MODE>(A, D, blk, smem_raw);
}

// One persistent launch for elements of every order <= 6: A.desc / A.fdesc
// list them by decreasing order (the order in ElemDesc::pad); block b takes
// elements b, b + gridDim.x, ... until the list ends, so every block exits.
template <class R, int MODE>
__global__ __launch_bounds__(W) __attribute__((amdgpu_waves_per_eu(2))) void k3g_persistent(Args A, Data<R> D) {
    if (A.skip && *A.skip) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    for (int i = blockIdx.x; i < A.count; i += gridDim.x) {
        const int P = A.desc[i].pad & ELEM_ORDER_MASK;
        switch (P) {
        case 1: gf_elem<R, 1, MODE>(A, D, i, smem_raw); break;
        case 2: gf_elem<R, 2, MODE>(A, D, i, smem_raw); break;
        case 3: gf_elem<R, 3, MODE>(A, D, i, smem_raw); break;
        case 4: gf_elem<R, 4, MODE>(A, D, i, smem_raw); break;
        case 5: gf_elem<R, 5, MODE>(A, D, i, smem_raw); break;
        default: gf_elem<R, 6, MODE>(A, D, i, smem_raw); break;
        }
        __syncthreads();   // the next element reuses the LDS
    }
}

}  // namespace g3
}  // namespace sipdg
