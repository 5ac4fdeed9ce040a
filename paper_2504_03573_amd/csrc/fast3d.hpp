// Wavefront-per-element kernels for hexahedra with p <= 6 (n = p+2 <= 8, so
// an element's n x n point columns fit in one 64-lane wavefront).
//
// Volume terms (Xia & Moxey, Sec. 3.1 basic operators): lane (q0, q1) keeps
// the xi_2 column of its points in registers; BwdTrans, the collocation
// derivative and their transposes run as line contractions whose 1-D table
// entries are wave-uniform (scalar loads), with LDS only for the exchange
// between the two lane layouts.
//
// Face terms (Sec. 3.2 TracePhysEval, Sec. 3.3 shared trace space and
// TraceIProduct): u and grad_xi u are evaluated directly at the trace
// points from the coefficients (a reduction along the face normal with the
// endpoint values P_i(+-1), P'_i(+-1), then two contractions with the
// Legendre tables at the trace's GLL points), and the flux is projected back
// to the coefficients by the transposed contractions.  Face work never
// touches the volume layout.
//
// Two launch structures:
//   two-stage: k3_trace writes (u, g) of every interior face side to the
//              trace buffer, k3_apply<.., false> reads the neighbour's values;
//   fused:     k3_apply<.., true> evaluates the neighbour's trace from the
//              neighbour's coefficients (read through the cache), so one
//              launch per order group computes y = A x.
#pragma once

#include "context.hpp"
#include "launch.hpp"

namespace sipdg {
namespace f3 {

constexpr int W = 64;        // lanes per element
constexpr int NFM = 8;       // largest trace handled here (both sides p <= 6)
constexpr int S9 = PMAX + 1; // row stride of the BF/DBF tables

template <int P>
struct C {
    static constexpr int N = P + 2, NP = P + 1;
    static constexpr int NPTS = N * N * N, NM = NP * NP * NP;
};

struct Args3 {
    const int *elems;
    int count;
    int region;             // work region (R units) at the end of the block's LDS
    const int64_t *xoff;
    const int64_t *voff;
    const FaceRef *eface;
    const FaceTopo *faces;
    const int *order;
    const int64_t *foff;
    const int64_t *toff;
    const int *skip;
};

template <class R>
struct Data3 {
    const R *__restrict__ vgeo;
    const R *__restrict__ fgeo;
    const R *__restrict__ lam;
    const R *__restrict__ tau;
    const R *__restrict__ tab;
    const R *__restrict__ x;
    R *__restrict__ y;
    R *__restrict__ tbuf;
};

__device__ __forceinline__ int lane_id() { return threadIdx.x; }

// index of mode (ia, ib) on face direction k with normal index ik
template <int NP>
__device__ __forceinline__ int mode_index(int k, int ia, int ib, int ik) {
    if (k == 0) return ik + NP * (ia + NP * ib);
    if (k == 1) return ia + NP * (ik + NP * ib);
    return ia + NP * (ib + NP * ik);
}

// P_i(s) and P'_i(s) at s = +-1
template <class R>
__device__ __forceinline__ R end_val(int i, int s) { return (s || !(i & 1)) ? R(1) : R(-1); }
template <class R>
__device__ __forceinline__ R end_der(int i, int s) {
    const R v = R(0.5) * R(i) * R(i + 1);
    return (s || (i & 1)) ? v : -v;
}

// ---------------------------------------------------------------- faces
//
// The two faces normal to reference direction k (sides s = 0, 1) are handled
// together; every trace array is laid out on a zero-padded 8 x 8 grid
// (index t1 + 8 t2), so lane l of the wavefront owns grid entry
// (l & 7, l >> 3) in every phase.  For one element with NPX modes per
// direction a direction pass runs:
//   R   reduce the coefficients along k with P_i(s), P'_i(s)      -> U[s][2]
//   A   contract the first face direction with P, P' at the trace -> W[s][3]
//   B   contract the second face direction -> u, d_a u, d_b u, d_k u at every
//       trace point, then the flux there (or the stored trace values)
//   B'  transposed contraction of the flux along the second direction -> T[s][3]
//   A'  transposed contraction along the first direction, spread along k with
//       P_i(s), P'_i(s) into the coefficient accumulator Yf.
// The trace tables P_i(z_t), P'_i(z_t) of each side are copied to LDS with
// rows t >= nf and columns i >= NPX set to zero, so every contraction runs a
// fixed number of terms.
// Region layout (R units, 64 per array): TB[2][2] | U[2][2] | W[2][3] | V[2][4];
// T[2][3] aliases U and W once they are dead.

constexpr int G8 = 64;
constexpr int REG_TB = 0, REG_U = 4 * G8, REG_W = 8 * G8, REG_V = 14 * G8, REG_END = 22 * G8;
__host__ __device__ constexpr int dir_region() { return REG_END; }

__device__ __forceinline__ int face_dir(int k, int j) { return j == 0 ? (k == 0 ? 1 : 0) : (k == 2 ? 1 : 2); }

// mode index with a runtime number of modes per direction
__device__ __forceinline__ int mode_index_rt(int np, int k, int ia, int ib, int ik) {
    if (k == 0) return ik + np * (ia + np * ib);
    if (k == 1) return ia + np * (ik + np * ib);
    return ia + np * (ib + np * ik);
}

struct Side {
    int F, slot, nf, o;      // face id, slot (0 owner, 1 other, 2 boundary), trace size, orientation
};

// Per point, prefetched at kernel start: own C along (k, a, b), a = w J_s,
// neighbour (u, g) (two-stage) or the neighbour's C along its (k, a, b) (fused).
template <class R>
struct Pre {
    R ck, ca, cb, aw, n0, n1, n2;
};

__device__ __forceinline__ void side_info(const FaceRef *eface, int64_t e, int k, Side sd[2]) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const FaceRef fr = eface[e * 6 + 2 * k + s];
        sd[s].F = fr.F;
        sd[s].slot = face_slot(fr.info);
        sd[s].nf = face_nf(fr.info);
        sd[s].o = face_orient(fr.info);
    }
}

// MODE: 0 trace (own C only), 1 two-stage apply (C, a, neighbour u, g from the
// trace buffer), 2 fused apply (C, a, the neighbour's C).  Lane l holds grid
// point (l & 7, l >> 3) of both sides.
template <class R, int MODE>
__device__ __forceinline__ void prefetch_dir(const Args3 &A, const Data3<R> &D, int k, const Side sd[2],
                                             Pre<R> pf[2]) {
    const int t1 = lane_id() & 7, t2 = lane_id() >> 3;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        Pre<R> &q = pf[s];
        q.ck = q.ca = q.cb = q.aw = q.n0 = q.n1 = q.n2 = R(0);
        const Side &S = sd[s];
        const int nf = S.nf, npf = nf * nf;
        if (t1 >= nf || t2 >= nf) continue;
        if (MODE == 0 && S.slot == 2) continue;
        const int qc = canon_index(S.o, nf, t1, t2);
        const R *fg = D.fgeo + A.foff[S.F];
        const int gs = S.slot == 2 ? 0 : S.slot;
        const R *Cm = fg + npf * (1 + 3 * gs) + qc;
        q.ck = Cm[k * npf];
        q.ca = Cm[face_dir(k, 0) * npf];
        q.cb = Cm[face_dir(k, 1) * npf];
        if (MODE == 0) continue;
        q.aw = fg[qc];
        if (S.slot == 2) continue;
        if (MODE == 1) {
            const R *tb = D.tbuf + A.toff[S.F] + (1 - S.slot) * 2 * npf;
            q.n0 = tb[qc];
            q.n1 = tb[npf + qc];
        } else {
            // neighbour's own point at this lane: its C along its own directions
            const FaceTopo ft = A.faces[S.F];
            const int fn = S.slot == 0 ? ft.fR : ft.fL;
            const int on = S.slot == 0 ? ft.orient : 0;
            const int qn = canon_index(on, nf, t1, t2);
            const R *Cn = fg + npf * (1 + 3 * (1 - S.slot)) + qn;
            const int kn = fn >> 1;
            q.n0 = Cn[kn * npf];
            q.n1 = Cn[face_dir(kn, 0) * npf];
            q.n2 = Cn[face_dir(kn, 1) * npf];
        }
    }
}

// copy the trace tables of both sides into TB (zero padded)
template <class R>
__device__ __forceinline__ void load_tables(const Side sd[2], const R *__restrict__ tab, int npx, R *TB) {
    for (int i = lane_id(); i < 4 * G8; i += W) {
        const int s = i >> 7, c = (i >> 6) & 1, t = (i >> 3) & 7, m = i & 7;
        // s depends on the lane: select, so that sd stays in registers
        const int nf = s ? sd[1].nf : sd[0].nf;
        R v = R(0);
        if (t < nf && m < npx) v = tab[(c ? tab_off_DBF(nf) : tab_off_BF(nf)) + t * S9 + m];
        TB[i] = v;
    }
}

// R phase (compile-time modes): U[s][0] = sum_ik P_ik(s) X, U[s][1] = sum_ik P'_ik(s) X
template <class R, int NP>
__device__ __forceinline__ void phase_R(int k, const R *X, R *U) {
    const int ia = lane_id() & 7, ib = lane_id() >> 3;
    if (ia >= NP || ib >= NP) return;
    R a[2][2] = {{0, 0}, {0, 0}};
#pragma unroll
    for (int ik = 0; ik < NP; ++ik) {
        const R v = X[mode_index<NP>(k, ia, ib, ik)];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            a[s][0] += end_val<R>(ik, s) * v;
            a[s][1] += end_der<R>(ik, s) * v;
        }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        U[(2 * s) * G8 + lane_id()] = a[s][0];
        U[(2 * s + 1) * G8 + lane_id()] = a[s][1];
    }
}

// A phase: W[s][0] = BF U0, W[s][1] = DBF U0, W[s][2] = BF U1 (contract ia)
template <class R, int NPX>
__device__ __forceinline__ void phase_A(const R *TB, const R *U, R *Wt, const bool act[2]) {
    const int t1 = lane_id() & 7, ib = lane_id() >> 3;
    if (ib >= NPX) return;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        if (!act[s]) continue;
        const R *bf = TB + (2 * s) * G8 + 8 * t1, *dbf = bf + G8;
        const R *u0 = U + (2 * s) * G8 + 8 * ib, *u1 = u0 + G8;
        R w0 = 0, w0d = 0, w1 = 0;
#pragma unroll
        for (int ia = 0; ia < NPX; ++ia) {
            const R b = bf[ia], x0 = u0[ia];
            w0 += b * x0;
            w0d += dbf[ia] * x0;
            w1 += b * u1[ia];
        }
        Wt[(3 * s) * G8 + lane_id()] = w0;
        Wt[(3 * s + 1) * G8 + lane_id()] = w0d;
        Wt[(3 * s + 2) * G8 + lane_id()] = w1;
    }
}

// B phase at this lane's grid point of side s
template <class R, int NPX>
__device__ __forceinline__ void phase_B(const R *TB, const R *Wt, int s, R &u, R &da, R &db, R &dk) {
    const int t1 = lane_id() & 7, t2 = lane_id() >> 3;
    const R *bf = TB + (2 * s) * G8 + 8 * t2, *dbf = bf + G8;
    const R *w0 = Wt + (3 * s) * G8 + t1, *w0d = w0 + G8, *w1 = w0d + G8;
    u = da = db = dk = R(0);
#pragma unroll
    for (int ib = 0; ib < NPX; ++ib) {
        const R b = bf[ib], x = w0[8 * ib];
        u += b * x;
        da += b * w0d[8 * ib];
        db += dbf[ib] * x;
        dk += b * w1[8 * ib];
    }
}

// B' and A' phases: project V back to the coefficients of the element.
template <class R, int NP>
__device__ __forceinline__ void phase_lift(int k, const R *TB, const R *V, R *T, R *Yf) {
    const int lane = lane_id();
    {
        const int t1 = lane & 7, ib = lane >> 3;
        if (ib < NP) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const R *bf = TB + (2 * s) * G8 + ib, *dbf = bf + G8;
                const R *v = V + (4 * s) * G8 + t1;
                R a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
                for (int t2 = 0; t2 < 8; ++t2) {
                    const R b = bf[8 * t2], d = dbf[8 * t2];
                    a1 += b * v[8 * t2] + d * v[2 * G8 + 8 * t2];
                    a2 += b * v[G8 + 8 * t2];
                    a3 += b * v[3 * G8 + 8 * t2];
                }
                T[(3 * s) * G8 + lane] = a1;
                T[(3 * s + 1) * G8 + lane] = a2;
                T[(3 * s + 2) * G8 + lane] = a3;
            }
        }
    }
    __syncthreads();
    const int ia = lane & 7, ib = lane >> 3;
    if (ia < NP && ib < NP) {
        R q[2][2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const R *bf = TB + (2 * s) * G8 + ia, *dbf = bf + G8;
            const R *t = T + (3 * s) * G8 + 8 * ib;
            R q0 = 0, q1 = 0;
#pragma unroll
            for (int t1 = 0; t1 < 8; ++t1) {
                const R b = bf[8 * t1], d = dbf[8 * t1];
                q0 += b * t[t1] + d * t[G8 + t1];
                q1 += b * t[2 * G8 + t1];
            }
            q[s][0] = q0;
            q[s][1] = q1;
        }
#pragma unroll
        for (int ik = 0; ik < NP; ++ik)
            Yf[mode_index<NP>(k, ia, ib, ik)] += end_val<R>(ik, 0) * q[0][0] + end_der<R>(ik, 0) * q[0][1] +
                                                 end_val<R>(ik, 1) * q[1][0] + end_der<R>(ik, 1) * q[1][1];
    }
    __syncthreads();
}

// Neighbour evaluation for the fused apply (runtime number of modes per side):
// (u, g) of each neighbour at canonical points, padded grid NB[s][2][64].
template <class R>
__device__ __forceinline__ void nbr_eval(const Args3 &A, const Data3<R> &D, int k, const Side sd[2],
                                         const Pre<R> pf[2], R *XN, R *Rg, R *NB) {
    constexpr int NX = 7;
    int npn[2] = {0, 0}, fn[2] = {0, 0}, on[2] = {0, 0};
    bool act[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        act[s] = sd[s].slot != 2;
        if (act[s]) {
            const FaceTopo ft = A.faces[sd[s].F];
            const int en = sd[s].slot == 0 ? ft.eR : ft.eL;
            fn[s] = sd[s].slot == 0 ? ft.fR : ft.fL;
            on[s] = sd[s].slot == 0 ? ft.orient : 0;
            npn[s] = A.order[en] + 1;
            const int nm = npn[s] * npn[s] * npn[s];
            const int64_t off = A.xoff[en];
            for (int i = lane_id(); i < nm; i += W) XN[s * 344 + i] = D.x[off + i];
        }
    }
    if (!act[0] && !act[1]) return;
    R *TB = Rg + REG_TB, *U = Rg + REG_U, *Wt = Rg + REG_W;
    // tables padded to the neighbours' mode counts
    for (int i = lane_id(); i < 4 * G8; i += W) {
        const int s = i >> 7, c = (i >> 6) & 1, t = (i >> 3) & 7, m = i & 7;
        const int nf = s ? sd[1].nf : sd[0].nf;
        const bool as = s ? act[1] : act[0];
        const int nps = s ? npn[1] : npn[0];
        R v = R(0);
        if (as && t < nf && m < nps) v = D.tab[(c ? tab_off_DBF(nf) : tab_off_BF(nf)) + t * S9 + m];
        TB[i] = v;
    }
    __syncthreads();
    {
        const int ia = lane_id() & 7, ib = lane_id() >> 3;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            R a0 = 0, a1 = 0;
            if (act[s] && ia < npn[s] && ib < npn[s]) {
                const int kn = fn[s] >> 1, sn = fn[s] & 1, np = npn[s];
                const R *Xs = XN + s * 344;
#pragma unroll
                for (int ik = 0; ik < NX; ++ik) {
                    if (ik < np) {
                        const R v = Xs[mode_index_rt(np, kn, ia, ib, ik)];
                        a0 += end_val<R>(ik, sn) * v;
                        a1 += end_der<R>(ik, sn) * v;
                    }
                }
            }
            U[(2 * s) * G8 + lane_id()] = a0;   // zero outside the neighbour's modes
            U[(2 * s + 1) * G8 + lane_id()] = a1;
        }
    }
    __syncthreads();
    phase_A<R, NX>(TB, U, Wt, act);
    __syncthreads();
    const int t1 = lane_id() & 7, t2 = lane_id() >> 3;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        if (!act[s]) continue;
        const int nf = sd[s].nf;
        if (t1 >= nf || t2 >= nf) continue;
        R u, da, db, dk;
        phase_B<R, NX>(TB, Wt, s, u, da, db, dk);
        const int qc = canon_index(on[s], nf, t1, t2);
        const int qp = (qc % nf) + 8 * (qc / nf);
        NB[(2 * s) * G8 + qp] = u;
        NB[(2 * s + 1) * G8 + qp] = pf[s].n0 * dk + pf[s].n1 * da + pf[s].n2 * db;
    }
    __syncthreads();
}

// ---------------------------------------------------------------- volume

// y = B^T (lam w|J| u + sum_k D_k^T (G w grad u)) + Yf for one element; lane
// layout and table access as described at the top.  X holds the element's
// coefficients; A, Bv are two n^3 LDS arrays; tab holds B then D in LDS.
template <class R, int P>
__device__ __forceinline__ void volume(const R *X, R *A, R *Bv, const R *Yf, const R *__restrict__ vg,
                                       R lam, const R *__restrict__ tab, R *__restrict__ yout) {
    constexpr int N = C<P>::N, NP = C<P>::NP, NPTS = C<P>::NPTS;
    const R *Bt = tab;            // [q][i], n x NP  (LDS copy)
    const R *Dt = tab + N * NP;   // [q][j], n x n
    const int lane = lane_id();
    // BwdTrans along direction 0: lines (i1, i2)
    if (lane < NP * NP) {
        const R *in = X + NP * lane;
        R v[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) v[i] = in[i];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            R s = 0;
#pragma unroll
            for (int i = 0; i < NP; ++i) s += Bt[q * NP + i] * v[i];
            A[q + N * lane] = s;   // [i2][i1][q0]
        }
    }
    __syncthreads();
    // along direction 1: lines (q0, i2)
    if (lane < N * NP) {
        const int q0 = lane % N, i2 = lane / N;
        R v[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) v[i] = A[q0 + N * (i + NP * i2)];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            R s = 0;
#pragma unroll
            for (int i = 0; i < NP; ++i) s += Bt[q * NP + i] * v[i];
            Bv[q0 + N * (q + N * i2)] = s;  // [i2][q1][q0]
        }
    }
    __syncthreads();
    // along direction 2 into the register column of lane (q0, q1)
    const bool col = lane < N * N;
    const int q0 = lane % N, q1 = lane / N;
    R u[N], d0[N], d1[N], d2[N];
    if (col) {
        R v[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) v[i] = Bv[lane + N * N * i];
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
#pragma unroll
        for (int q = 0; q < N; ++q) A[lane + N * N * q] = u[q];  // [q2][q1][q0]
    }
    __syncthreads();
    // d0: lines (q1, q2) along direction 0
    if (col) {
        const R *in = A + N * lane;
        R v[N];
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] = in[j];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            R s = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) s += Dt[q * N + j] * v[j];
            Bv[q + N * lane] = s;
        }
    }
    __syncthreads();
    if (col) {
#pragma unroll
        for (int q = 0; q < N; ++q) d0[q] = Bv[lane + N * N * q];
    }
    __syncthreads();
    // d1: lines (q0, q2) along direction 1
    if (col) {
        const int a = lane % N, c = lane / N;  // a = q0, c = q2
        R v[N];
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] = A[a + N * (j + N * c)];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            R s = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) s += Dt[q * N + j] * v[j];
            Bv[a + N * (q + N * c)] = s;
        }
    }
    __syncthreads();
    if (col) {
#pragma unroll
        for (int q = 0; q < N; ++q) d1[q] = Bv[lane + N * N * q];
    }
    // pointwise: m = lam w|J| u, q = (G w) grad u  (in place: u <- m, d <- q)
    if (col) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const int p = lane + N * N * q;
            const R g00 = vg[p], g01 = vg[NPTS + p], g02 = vg[2 * NPTS + p];
            const R g11 = vg[3 * NPTS + p], g12 = vg[4 * NPTS + p], g22 = vg[5 * NPTS + p];
            const R wj = vg[6 * NPTS + p];
            const R a0 = d0[q], a1 = d1[q], a2 = d2[q];
            u[q] = lam * wj * u[q];
            d0[q] = g00 * a0 + g01 * a1 + g02 * a2;
            d1[q] = g01 * a0 + g11 * a1 + g12 * a2;
            d2[q] = g02 * a0 + g12 * a1 + g22 * a2;
        }
    }
    __syncthreads();
    // D_0^T q_0 and D_1^T q_1 through LDS, D_2^T q_2 in registers
    if (col) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            A[lane + N * N * q] = d0[q];
            Bv[lane + N * N * q] = d1[q];
        }
    }
    __syncthreads();
    if (col) {
        {   // direction 0, lines (q1, q2), in place
            R *io = A + N * lane;
            R v[N];
#pragma unroll
            for (int j = 0; j < N; ++j) v[j] = io[j];
#pragma unroll
            for (int j = 0; j < N; ++j) {
                R s = 0;
#pragma unroll
                for (int q = 0; q < N; ++q) s += Dt[q * N + j] * v[q];
                io[j] = s;
            }
        }
        {   // direction 1, lines (q0, q2), in place
            const int a = lane % N, c = lane / N;
            R v[N];
#pragma unroll
            for (int j = 0; j < N; ++j) v[j] = Bv[a + N * (j + N * c)];
#pragma unroll
            for (int j = 0; j < N; ++j) {
                R s = 0;
#pragma unroll
                for (int q = 0; q < N; ++q) s += Dt[q * N + j] * v[q];
                Bv[a + N * (j + N * c)] = s;
            }
        }
    }
    __syncthreads();
    R wv[NP];
    if (col) {
        R v[N];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            R s = u[j] + A[lane + N * N * j] + Bv[lane + N * N * j];
#pragma unroll
            for (int q = 0; q < N; ++q) s += Dt[q * N + j] * d2[q];
            v[j] = s;
        }
        // B^T along direction 2
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            R s = 0;
#pragma unroll
            for (int q = 0; q < N; ++q) s += Bt[q * NP + i] * v[q];
            wv[i] = s;
        }
    }
    __syncthreads();
    if (col) {
#pragma unroll
        for (int i = 0; i < NP; ++i) A[lane + N * N * i] = wv[i];   // [i2][q1][q0]
    }
    __syncthreads();
    // B^T along direction 1: lines (q0, i2)
    if (lane < N * NP) {
        const int a = lane % N, i2 = lane / N;
        R v[N];
#pragma unroll
        for (int q = 0; q < N; ++q) v[q] = A[a + N * (q + N * i2)];
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            R s = 0;
#pragma unroll
            for (int q = 0; q < N; ++q) s += Bt[q * NP + i] * v[q];
            Bv[a + N * (i + NP * i2)] = s;  // [i2][i1][q0]
        }
    }
    __syncthreads();
    // B^T along direction 0: lines (i1, i2), plus the face contributions
    if (lane < NP * NP) {
        const R *in = Bv + N * lane;
        R v[N];
#pragma unroll
        for (int q = 0; q < N; ++q) v[q] = in[q];
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            R s = Yf[i + NP * lane];
#pragma unroll
            for (int q = 0; q < N; ++q) s += Bt[q * NP + i] * v[q];
            yout[i + NP * lane] = s;
        }
    }
}

// ---------------------------------------------------------------- kernels

// Block LDS layout (R units):
//   X[NMX] | Yf[NMX] | VT[volume tables] | (fused: XN[2][344] | NB[2][2][64]) | Rg[region]
template <int P>
struct Lds {
    static constexpr int NMX = (C<P>::NM + 3) & ~3;
    static constexpr int VTAB = ((P + 2) * (P + 1) + (P + 2) * (P + 2) + 3) & ~3;
    static constexpr int region = dir_region() > 2 * C<P>::NPTS ? dir_region() : 2 * C<P>::NPTS;
    static constexpr int trace_total = NMX + dir_region();
    static constexpr int apply_total = 2 * NMX + VTAB + region;
    static constexpr int fused_total = 2 * NMX + VTAB + 2 * 344 + 4 * G8 + region;
};

// (u, g) of every interior face side of the element into the trace buffer.
template <class R, int P>
__global__ __launch_bounds__(W) void k3_trace(Args3 A, Data3<R> D) {
    using Cf = C<P>;
    constexpr int NP = Cf::NP;
    if (A.skip && *A.skip) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R *sm = reinterpret_cast<R *>(smem_raw);
    R *X = sm, *Rg = sm + Lds<P>::NMX;
    R *TB = Rg + REG_TB, *U = Rg + REG_U, *Wt = Rg + REG_W;
    const int64_t e = A.elems[blockIdx.x];
    const int lane = lane_id();
    Side sd[3][2];
    Pre<R> pf[3][2];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        side_info(A.eface, e, k, sd[k]);
        prefetch_dir<R, 0>(A, D, k, sd[k], pf[k]);
    }
    const int64_t xo = A.xoff[e];
    for (int i = lane; i < Cf::NM; i += W) X[i] = D.x[xo + i];
    __syncthreads();
    const int t1 = lane & 7, t2 = lane >> 3;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const bool act[2] = {sd[k][0].slot != 2, sd[k][1].slot != 2};
        if (!act[0] && !act[1]) continue;
        load_tables<R>(sd[k], D.tab, NP, TB);
        phase_R<R, NP>(k, X, U);
        __syncthreads();
        phase_A<R, NP>(TB, U, Wt, act);
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const Side &S = sd[k][s];
            const int nf = S.nf, npf = nf * nf;
            if (!act[s] || t1 >= nf || t2 >= nf) continue;
            R u, da, db, dk;
            phase_B<R, NP>(TB, Wt, s, u, da, db, dk);
            const int qc = canon_index(S.o, nf, t1, t2);
            R *tb = D.tbuf + A.toff[S.F] + S.slot * 2 * npf;
            tb[qc] = u;
            tb[npf + qc] = pf[k][s].ck * dk + pf[k][s].ca * da + pf[k][s].cb * db;
        }
        __syncthreads();
    }
}

// y = A x for the elements of one order group.  FUSED: neighbour traces are
// evaluated here from the neighbour's coefficients; otherwise read from the
// trace buffer written by k3_trace.
template <class R, int P, bool FUSED>
__global__ __launch_bounds__(W) void k3_apply(Args3 A, Data3<R> D) {
    using Cf = C<P>;
    constexpr int N = Cf::N, NP = Cf::NP, NMX = Lds<P>::NMX;
    if (A.skip && *A.skip) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R *sm = reinterpret_cast<R *>(smem_raw);
    R *X = sm, *Yf = sm + NMX, *VT = Yf + NMX;
    R *XN = VT + Lds<P>::VTAB, *NB = XN + 2 * 344;
    R *Rg = FUSED ? NB + 4 * G8 : VT + Lds<P>::VTAB;
    R *TB = Rg + REG_TB, *U = Rg + REG_U, *Wt = Rg + REG_W, *V = Rg + REG_V, *T = Rg + REG_U;
    const int64_t e = A.elems[blockIdx.x];
    const int lane = lane_id();
    Side sd[3][2];
    Pre<R> pf[3][2];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        side_info(A.eface, e, k, sd[k]);
        prefetch_dir<R, FUSED ? 2 : 1>(A, D, k, sd[k], pf[k]);
    }
    const int64_t xo = A.xoff[e];
    for (int i = lane; i < Cf::NM; i += W) X[i] = D.x[xo + i];
    for (int i = lane; i < NMX; i += W) Yf[i] = R(0);
    for (int i = lane; i < N * NP; i += W) VT[i] = D.tab[tab_off_B(P) + i];
    for (int i = lane; i < N * N; i += W) VT[N * NP + i] = D.tab[tab_off_D(N) + i];
    __syncthreads();
    const int t1 = lane & 7, t2 = lane >> 3;
    const bool both[2] = {true, true};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (FUSED) nbr_eval<R>(A, D, k, sd[k], pf[k], XN, Rg, NB);
        load_tables<R>(sd[k], D.tab, NP, TB);
        phase_R<R, NP>(k, X, U);
        __syncthreads();
        phase_A<R, NP>(TB, U, Wt, both);
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const Side &S = sd[k][s];
            const int nf = S.nf;
            R Fv = 0, Ga = 0, Gb = 0, Gk = 0;
            if (t1 < nf && t2 < nf) {
                R u, da, db, dk;
                phase_B<R, NP>(TB, Wt, s, u, da, db, dk);
                const Pre<R> &q = pf[k][s];
                const R g = q.ck * dk + q.ca * da + q.cb * db;
                R un, gn;
                if (S.slot == 2) {
                    un = -u;
                    gn = -g;
                } else if (FUSED) {
                    const int qc = canon_index(S.o, nf, t1, t2);
                    const int qp = (qc % nf) + 8 * (qc / nf);
                    un = NB[(2 * s) * G8 + qp];
                    gn = NB[(2 * s + 1) * G8 + qp];
                } else {
                    un = q.n0;
                    gn = q.n1;
                }
                const R jump = u - un;
                Fv = -R(0.5) * (g - gn) + D.tau[S.F] * q.aw * jump;
                const R Fg = R(-0.5) * jump;
                Ga = Fg * q.ca;
                Gb = Fg * q.cb;
                Gk = Fg * q.ck;
            }
            R *Vs = V + (4 * s) * G8 + lane;
            Vs[0] = Fv;
            Vs[G8] = Ga;
            Vs[2 * G8] = Gb;
            Vs[3 * G8] = Gk;
        }
        __syncthreads();
        phase_lift<R, NP>(k, TB, V, T, Yf);
    }
    volume<R, P>(X, Rg, Rg + Cf::NPTS, Yf, D.vgeo + A.voff[e], D.lam[e], VT, D.y + A.xoff[e]);
}

}  // namespace f3
}  // namespace sipdg
