// Device code of the matrix-free SIPG Helmholtz operator (gfx950).
//
// One application y = A x is two launches per order group (Xia & Moxey,
// Sec. 5.1: the LhsEval split into HelmholtzDGwithAverJump and
// HelmholtzIPDGTraceFlux, here without an exchange between them):
//
//   K1 (trace):  per element  BwdTrans -> PhysDeriv (collocation) -> for each
//                interior face gather u, grad_xi u at the face points,
//                interpolate to the shared trace (GLL with max(p_L,p_R)+2
//                points), form g = w J_s n . grad u with the side's own
//                metric, and store (u, g) in the trace buffer in the owner's
//                point order (Sec. 3.2 GathrInterp, Sec. 5.1 operator B:
//                gather, interpolate, permute; two values per trace point).
//   K2 (apply):  per element  BwdTrans -> PhysDeriv -> faces: own (u, g) as in
//                K1, neighbour (u, g) from the trace buffer (a mirrored value
//                on the boundary), flux of eq. IP at every trace point, and the
//                transposed interpolation back to the face points (the
//                inner product on the shared trace, TraceIProduct) -> volume
//                pointwise terms with the per-point factors G w and w|J| ->
//                IProduct with the transposed collocation derivative
//                -> y written once.
//
// No atomics: every element writes only its own rows, so results are
// deterministic.  All intermediate data of an element stays in LDS.
#pragma once

#include "context.hpp"

namespace sipdg {

constexpr int BLOCK = 256;

template <int DIM, int P>
struct Cfg {
    static constexpr int N = P + 2;
    static constexpr int NP = P + 1;
    static constexpr int NPTS = DIM == 3 ? N * N * N : N * N;
    static constexpr int NM = DIM == 3 ? NP * NP * NP : NP * NP;
    static constexpr int NFP = DIM == 3 ? N * N : N;      // element face points
    static constexpr int NQ = DIM + 1;                    // u and grad_xi u
    static constexpr int NGEO = DIM * (DIM + 1) / 2 + 1;  // G w (sym) + w|J|
    // elements per block: 2-D, one (measured on the 64 x 64 mixed-order mesh:
    // several per block left fewer blocks than compute units); 3-D, two up to
    // order 3
    static constexpr int EPB = DIM == 2 ? 1 : (NPTS <= 160 ? 2 : 1);
    static constexpr int TABSZ = N * NP + N * N;          // B and D in LDS
    static constexpr int TABPAD = (TABSZ + 3) & ~3;
};

// Per-element work-area size (R units) for a group whose largest trace has
// nfm points per direction.
template <int DIM, int P>
__host__ __device__ inline int work_size(int nfm) {
    using C = Cfg<DIM, P>;
    int nf = nfm < C::N ? C::N : nfm;
    int xs = DIM == 3 ? C::NQ * C::N * nf : 0;
    int ys = DIM == 3 ? C::NQ * nf * nf : C::NQ * nf;
    int t = 2 * (xs + ys);
    return t > 2 * C::NPTS ? t : 2 * C::NPTS;
}

template <int DIM, int P>
__host__ __device__ inline int elem_stride(int tsz, bool lift) {
    using C = Cfg<DIM, P>;
    int s = (1 + DIM) * C::NPTS + tsz + (lift ? 2 * DIM * C::NQ * C::NFP : 0);
    return (s + 3) & ~3;
}

template <int DIM, int P>
__host__ __device__ inline size_t lds_bytes(int tsz, bool lift, size_t rsize) {
    using C = Cfg<DIM, P>;
    return rsize * (size_t)(C::TABPAD + C::EPB * elem_stride<DIM, P>(tsz, lift));
}

// ---------------------------------------------------------------- contractions

// Apply a 1-D matrix along direction DIR of a tensor array held in LDS.
// Input extents: NIN along DIR, E0/E1/E2 along the other directions
// (direction 0 fastest).  The output has NOUT along DIR.  FWD: M is
// NOUT x NIN (out_o = sum_i M[o][i] in_i); TRANS: M is NIN x NOUT
// (out_o = sum_i M[i][o] in_i).  One work item = one line and a chunk of
// its outputs; the whole line is read once into registers.
template <int DIR, int NIN, int NOUT, int E0, int E1, int E2>
struct Lines {
    static constexpr int ext(int d) { return d == DIR ? NIN : (d == 0 ? E0 : (d == 1 ? E1 : E2)); }
    static constexpr int oext(int d) { return d == DIR ? NOUT : (d == 0 ? E0 : (d == 1 ? E1 : E2)); }
    static constexpr int istr(int d) { return d == 0 ? 1 : (d == 1 ? ext(0) : ext(0) * ext(1)); }
    static constexpr int ostr(int d) { return d == 0 ? 1 : (d == 1 ? oext(0) : oext(0) * oext(1)); }
    static constexpr int D1 = DIR == 0 ? 1 : 0;
    static constexpr int D2 = DIR == 2 ? 1 : 2;
    static constexpr int NL = ext(D1) * ext(D2);
};

enum { OUT_SET = 0, OUT_ADD = 1, OUT_SET_PLUS = 2 };

template <class R, int EPB, int DIR, int NIN, int NOUT, int E0, int E1, int E2, bool TRANS, int OUTM>
__device__ __forceinline__ void contract(const R *__restrict__ M, R *sm, int es, int in_off,
                                         int out_off, int plus_off, int nel) {
    using L = Lines<DIR, NIN, NOUT, E0, E1, E2>;
    constexpr int NCH0 = BLOCK / (EPB * L::NL);
    constexpr int NCH = NCH0 < 1 ? 1 : (NCH0 > NOUT ? NOUT : NCH0);
    constexpr int OC = (NOUT + NCH - 1) / NCH;
    const int total = nel * L::NL * NCH;
    for (int it = threadIdx.x; it < total; it += BLOCK) {
        const int el = it / (L::NL * NCH);
        const int r = it - el * (L::NL * NCH);
        const int line = r / NCH;
        const int ch = r - line * NCH;
        const int a = line % L::ext(L::D1);
        const int b = line / L::ext(L::D1);
        const R *in = sm + el * es + in_off + a * L::istr(L::D1) + b * L::istr(L::D2);
        const int obase = el * es + a * L::ostr(L::D1) + b * L::ostr(L::D2);
        R v[NIN];
#pragma unroll
        for (int i = 0; i < NIN; ++i) v[i] = in[i * L::istr(DIR)];
#pragma unroll
        for (int oo = 0; oo < OC; ++oo) {
            const int o = ch * OC + oo;
            if (OC * NCH == NOUT || o < NOUT) {
                R s = 0;
#pragma unroll
                for (int i = 0; i < NIN; ++i) s += (TRANS ? M[i * NOUT + o] : M[o * NIN + i]) * v[i];
                const int oi = obase + o * L::ostr(DIR);
                if (OUTM == OUT_ADD) sm[out_off + oi] += s;
                else if (OUTM == OUT_SET_PLUS) sm[out_off + oi] = s + sm[plus_off + oi];
                else sm[out_off + oi] = s;
            }
        }
    }
}

// ---------------------------------------------------------------- element fields

// Layout of one element's LDS region (R units).
template <int DIM, int P>
struct Lay {
    using C = Cfg<DIM, P>;
    static constexpr int U = 0;
    static constexpr int G = C::NPTS;                  // DIM arrays
    static constexpr int T = (1 + DIM) * C::NPTS;       // work area, tsz long
};

// u and grad_xi u at all GLL points of each element of the block:
// BwdTrans (B along each direction) then PhysDeriv (collocation D).
template <class R, int DIM, int P, bool DERIV = true>
__device__ __forceinline__ void element_fields(const R *x, const int64_t *xoff, const R *Bt,
                                              const R *Dt, R *sm, int es, const int *s_e, int nel) {
    using C = Cfg<DIM, P>;
    using Ly = Lay<DIM, P>;
    constexpr int N = C::N, NP = C::NP, EPB = C::EPB;
    const int TA = Ly::T, TB = Ly::T + C::NPTS;
    for (int it = threadIdx.x; it < nel * C::NM; it += BLOCK) {
        const int el = it / C::NM, i = it - el * C::NM;
        sm[el * es + TA + i] = x[xoff[s_e[el]] + i];
    }
    __syncthreads();
    if constexpr (DIM == 2) {
        contract<R, EPB, 0, NP, N, NP, NP, 1, false, OUT_SET>(Bt, sm, es, TA, TB, 0, nel);
        __syncthreads();
        contract<R, EPB, 1, NP, N, N, NP, 1, false, OUT_SET>(Bt, sm, es, TB, Ly::U, 0, nel);
        __syncthreads();
        if constexpr (!DERIV) return;
        contract<R, EPB, 0, N, N, N, N, 1, false, OUT_SET>(Dt, sm, es, Ly::U, Ly::G, 0, nel);
        contract<R, EPB, 1, N, N, N, N, 1, false, OUT_SET>(Dt, sm, es, Ly::U, Ly::G + C::NPTS, 0, nel);
        __syncthreads();
    } else {
        contract<R, EPB, 0, NP, N, NP, NP, NP, false, OUT_SET>(Bt, sm, es, TA, TB, 0, nel);
        __syncthreads();
        contract<R, EPB, 1, NP, N, N, NP, NP, false, OUT_SET>(Bt, sm, es, TB, TA, 0, nel);
        __syncthreads();
        contract<R, EPB, 2, NP, N, N, N, NP, false, OUT_SET>(Bt, sm, es, TA, Ly::U, 0, nel);
        __syncthreads();
        if constexpr (!DERIV) return;
        contract<R, EPB, 0, N, N, N, N, N, false, OUT_SET>(Dt, sm, es, Ly::U, Ly::G, 0, nel);
        contract<R, EPB, 1, N, N, N, N, N, false, OUT_SET>(Dt, sm, es, Ly::U, Ly::G + C::NPTS, 0, nel);
        contract<R, EPB, 2, N, N, N, N, N, false, OUT_SET>(Dt, sm, es, Ly::U, Ly::G + 2 * C::NPTS, 0, nel);
        __syncthreads();
    }
}

// Element point index of face point (a, b) on local face (k, s).
template <int DIM, int N>
__device__ __forceinline__ int face_point(int k, int s, int a, int b) {
    const int qk = s ? N - 1 : 0;
    if constexpr (DIM == 2) {
        return k == 0 ? (qk + N * a) : (a + N * qk);
    } else {
        if (k == 0) return qk + N * a + N * N * b;
        if (k == 1) return a + N * qk + N * N * b;
        return a + N * b + N * N * qk;
    }
}

enum { FACE_TRACE = 0, FACE_LIFT = 1 };

// Faces normal to reference direction k, both sides of every element of the
// block.  FACE_TRACE stores (u, g) of interior faces in the trace buffer.
// FACE_LIFT forms the flux and writes the face-point contributions to the
// element's u-test (value) and grad-test inputs into the staging area S
// (S[f][c][face point], f = 2k+s).
template <class R, int DIM, int P, int MODE>
__device__ __forceinline__ void faces_dir(const OpArgs<R> &A, int k, R *sm, int es, const int *s_e,
                                          const FaceRef *s_face, int nel, int nfm, int S_off) {
    using C = Cfg<DIM, P>;
    using Ly = Lay<DIM, P>;
    constexpr int N = C::N, NQ = C::NQ;
    const int xs = DIM == 3 ? NQ * N * nfm : 0;
    const int ys = DIM == 3 ? NQ * nfm * nfm : NQ * nfm;
    const int ysq = DIM == 3 ? nfm * nfm : nfm;  // stride of one quantity in Y
    auto X_of = [&](int el, int s) { return sm + el * es + Ly::T + s * xs; };
    auto Y_of = [&](int el, int s) { return sm + el * es + Ly::T + 2 * xs + s * ys; };
    auto fval = [&](int el, int c, int idx) -> R {
        return sm[el * es + (c == 0 ? Ly::U : Ly::G + (c - 1) * C::NPTS) + idx];
    };

    if constexpr (DIM == 3) {
        // F1: interpolate along the first face direction (nf > n only)
        const int per = NQ * N * nfm;
        for (int it = threadIdx.x; it < nel * 2 * per; it += BLOCK) {
            const int el = it / (2 * per);
            int r = it - el * 2 * per;
            const int s = r / per;
            r -= s * per;
            const int c = r / (N * nfm);
            r -= c * N * nfm;
            const int b = r / nfm, t1 = r - b * nfm;
            const FaceRef fr = s_face[el * 2 * DIM + 2 * k + s];
            const int nf = face_nf(fr.info);
            if (MODE == FACE_TRACE && face_slot(fr.info) == 2) continue;
            if (nf == N || t1 >= nf) continue;
            const R *I = A.tab + tab_off_I(N, nf);
            R acc = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) acc += I[t1 * N + j] * fval(el, c, face_point<DIM, N>(k, s, j, b));
            X_of(el, s)[c * N * nfm + b * nfm + t1] = acc;
        }
        __syncthreads();
    }
    {
        // F2: second direction (or a plain gather when the trace matches)
        const int per = NQ * ysq;
        for (int it = threadIdx.x; it < nel * 2 * per; it += BLOCK) {
            const int el = it / (2 * per);
            int r = it - el * 2 * per;
            const int s = r / per;
            r -= s * per;
            const int c = r / ysq;
            r -= c * ysq;
            const FaceRef fr = s_face[el * 2 * DIM + 2 * k + s];
            const int nf = face_nf(fr.info);
            if (MODE == FACE_TRACE && face_slot(fr.info) == 2) continue;
            R *Y = Y_of(el, s) + c * ysq;
            if constexpr (DIM == 3) {
                const int t2 = r / nfm, t1 = r - t2 * nfm;
                if (t1 >= nf || t2 >= nf) continue;
                if (nf == N) {
                    Y[t2 * nfm + t1] = fval(el, c, face_point<DIM, N>(k, s, t1, t2));
                } else {
                    const R *I = A.tab + tab_off_I(N, nf);
                    const R *X = X_of(el, s) + c * N * nfm;
                    R acc = 0;
#pragma unroll
                    for (int j = 0; j < N; ++j) acc += I[t2 * N + j] * X[j * nfm + t1];
                    Y[t2 * nfm + t1] = acc;
                }
            } else {
                const int t = r;
                if (t >= nf) continue;
                if (nf == N) {
                    Y[t] = fval(el, c, face_point<DIM, N>(k, s, t, 0));
                } else {
                    const R *I = A.tab + tab_off_I(N, nf);
                    R acc = 0;
#pragma unroll
                    for (int j = 0; j < N; ++j) acc += I[t * N + j] * fval(el, c, face_point<DIM, N>(k, s, j, 0));
                    Y[t] = acc;
                }
            }
        }
        __syncthreads();
    }
    {
        // F3: values at the trace points; store (TRACE) or flux (LIFT)
        for (int it = threadIdx.x; it < nel * 2 * ysq; it += BLOCK) {
            const int el = it / (2 * ysq);
            int r = it - el * 2 * ysq;
            const int s = r / ysq;
            r -= s * ysq;
            const FaceRef fr = s_face[el * 2 * DIM + 2 * k + s];
            const int nf = face_nf(fr.info);
            const int slot = face_slot(fr.info);
            if (MODE == FACE_TRACE && slot == 2) continue;
            int t, qc, npf;
            if constexpr (DIM == 3) {
                const int t2 = r / nfm, t1 = r - t2 * nfm;
                if (t1 >= nf || t2 >= nf) continue;
                t = t2 * nfm + t1;
                qc = canon_index(face_orient(fr.info), nf, t1, t2);
                npf = nf * nf;
            } else {
                if (r >= nf) continue;
                t = r;
                qc = (face_orient(fr.info) & 1) ? nf - 1 - r : r;
                npf = nf;
            }
            R *Y = Y_of(el, s);
            const R *fg = A.fgeo + A.foff[fr.F];
            const int gs = slot == 2 ? 0 : slot;
            R Cm[DIM];
            R u = Y[t], g = 0;
#pragma unroll
            for (int m = 0; m < DIM; ++m) {
                Cm[m] = fg[npf * (1 + DIM * gs) + m * npf + qc];
                g += Cm[m] * Y[(1 + m) * ysq + t];
            }
            if (MODE == FACE_TRACE) {
                R *tb = A.tbuf + A.toff[fr.F] + slot * 2 * npf;
                tb[qc] = u;
                tb[npf + qc] = g;
            } else {
                R un, gn;
                if (slot == 2) {
                    un = -u;
                    gn = -g;
                } else {
                    const R *tb = A.tbuf + A.toff[fr.F] + (1 - slot) * 2 * npf;
                    un = tb[qc];
                    gn = tb[npf + qc];
                }
                const R a = fg[qc];
                const R tau = A.tau[fr.F];
                const R jump = u - un;
                const R avg = R(0.5) * (g - gn);
                const R Fv = -avg + tau * a * jump;
                const R Fg = R(-0.5) * jump;
                Y[t] = Fv;
#pragma unroll
                for (int m = 0; m < DIM; ++m) Y[(1 + m) * ysq + t] = Fg * Cm[m];
            }
        }
        __syncthreads();
    }
    if constexpr (MODE == FACE_LIFT) {
        if constexpr (DIM == 3) {
            // F4: transposed interpolation along the second face direction
            const int per = NQ * N * nfm;
            for (int it = threadIdx.x; it < nel * 2 * per; it += BLOCK) {
                const int el = it / (2 * per);
                int r = it - el * 2 * per;
                const int s = r / per;
                r -= s * per;
                const int c = r / (N * nfm);
                r -= c * N * nfm;
                const int j = r / nfm, t1 = r - j * nfm;
                const FaceRef fr = s_face[el * 2 * DIM + 2 * k + s];
                const int nf = face_nf(fr.info);
                if (nf == N || t1 >= nf) continue;
                const R *I = A.tab + tab_off_I(N, nf);
                const R *Y = Y_of(el, s) + c * ysq;
                R acc = 0;
                for (int t2 = 0; t2 < nf; ++t2) acc += I[t2 * N + j] * Y[t2 * nfm + t1];
                X_of(el, s)[c * N * nfm + j * nfm + t1] = acc;
            }
            __syncthreads();
        }
        // F5: transposed interpolation along the first direction into S
        const int per = NQ * C::NFP;
        for (int it = threadIdx.x; it < nel * 2 * per; it += BLOCK) {
            const int el = it / (2 * per);
            int r = it - el * 2 * per;
            const int s = r / per;
            r -= s * per;
            const int c = r / C::NFP;
            const int fp = r - c * C::NFP;
            const FaceRef fr = s_face[el * 2 * DIM + 2 * k + s];
            const int nf = face_nf(fr.info);
            R *S = sm + el * es + S_off + ((2 * k + s) * NQ + c) * C::NFP;
            if constexpr (DIM == 3) {
                const int a = fp % N, b = fp / N;
                if (nf == N) {
                    S[fp] = Y_of(el, s)[c * ysq + b * nfm + a];
                } else {
                    const R *I = A.tab + tab_off_I(N, nf);
                    const R *X = X_of(el, s) + c * N * nfm + b * nfm;
                    R acc = 0;
                    for (int t1 = 0; t1 < nf; ++t1) acc += I[t1 * N + a] * X[t1];
                    S[fp] = acc;
                }
            } else {
                const R *Y = Y_of(el, s) + c * ysq;
                if (nf == N) {
                    S[fp] = Y[fp];
                } else {
                    const R *I = A.tab + tab_off_I(N, nf);
                    R acc = 0;
                    for (int t = 0; t < nf; ++t) acc += I[t * N + fp] * Y[t];
                    S[fp] = acc;
                }
            }
        }
        __syncthreads();
    }
}

// IProduct of point data held in U (value-test input m) and G (grad-test
// inputs q_k): y = B^T (m + sum_k D_k^T q_k), written once to y.
template <class R, int DIM, int P>
__device__ __forceinline__ void element_iproduct(R *y, const int64_t *xoff, const R *Bt, const R *Dt,
                                                 R *sm, int es, const int *s_e, int nel) {
    using C = Cfg<DIM, P>;
    using Ly = Lay<DIM, P>;
    constexpr int N = C::N, NP = C::NP, EPB = C::EPB, NPTS = C::NPTS;
    const int TA = Ly::T, TB = Ly::T + NPTS;
    if constexpr (DIM == 2) {
        contract<R, EPB, 0, N, N, N, N, 1, true, OUT_SET_PLUS>(Dt, sm, es, Ly::G, TA, Ly::U, nel);
        __syncthreads();
        contract<R, EPB, 1, N, N, N, N, 1, true, OUT_ADD>(Dt, sm, es, Ly::G + NPTS, TA, 0, nel);
        __syncthreads();
        contract<R, EPB, 1, N, NP, N, N, 1, true, OUT_SET>(Bt, sm, es, TA, TB, 0, nel);
        __syncthreads();
        contract<R, EPB, 0, N, NP, N, NP, 1, true, OUT_SET>(Bt, sm, es, TB, TA, 0, nel);
        __syncthreads();
    } else {
        contract<R, EPB, 0, N, N, N, N, N, true, OUT_SET_PLUS>(Dt, sm, es, Ly::G, TA, Ly::U, nel);
        __syncthreads();
        contract<R, EPB, 1, N, N, N, N, N, true, OUT_ADD>(Dt, sm, es, Ly::G + NPTS, TA, 0, nel);
        __syncthreads();
        contract<R, EPB, 2, N, N, N, N, N, true, OUT_ADD>(Dt, sm, es, Ly::G + 2 * NPTS, TA, 0, nel);
        __syncthreads();
        contract<R, EPB, 2, N, NP, N, N, N, true, OUT_SET>(Bt, sm, es, TA, TB, 0, nel);
        __syncthreads();
        contract<R, EPB, 1, N, NP, N, N, NP, true, OUT_SET>(Bt, sm, es, TB, Ly::U, 0, nel);
        __syncthreads();
        contract<R, EPB, 0, N, NP, N, NP, NP, true, OUT_SET>(Bt, sm, es, Ly::U, TA, 0, nel);
        __syncthreads();
    }
    for (int it = threadIdx.x; it < nel * C::NM; it += BLOCK) {
        const int el = it / C::NM, i = it - el * C::NM;
        y[xoff[s_e[el]] + i] = sm[el * es + TA + i];
    }
}

// Common block prologue: element ids, face descriptors and the B, D tables.
template <class R, int DIM, int P>
__device__ __forceinline__ int block_setup(const OpArgs<R> &A, R *tabs, int *s_e, FaceRef *s_face) {
    using C = Cfg<DIM, P>;
    constexpr int N = C::N, NP = C::NP, EPB = C::EPB;
    const int e0 = blockIdx.x * EPB;
    const int nel = min(EPB, A.count - e0);
    if (threadIdx.x < nel) s_e[threadIdx.x] = A.elems[e0 + threadIdx.x];
    for (int i = threadIdx.x; i < N * NP; i += BLOCK) tabs[i] = A.tab[tab_off_B(P) + i];
    for (int i = threadIdx.x; i < N * N; i += BLOCK) tabs[N * NP + i] = A.tab[tab_off_D(N) + i];
    __syncthreads();
    for (int i = threadIdx.x; i < nel * 2 * DIM; i += BLOCK) {
        const int el = i / (2 * DIM), f = i - el * 2 * DIM;
        s_face[i] = A.eface[(int64_t)s_e[el] * 2 * DIM + f];
    }
    __syncthreads();
    return nel;
}

// K1: trace values of every interior face side into the trace buffer.
template <class R, int DIM, int P>
__global__ __launch_bounds__(BLOCK) void k_trace(OpArgs<R> A, int nfm) {
    using C = Cfg<DIM, P>;
    if (A.skip && *A.skip) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R *tabs = reinterpret_cast<R *>(smem_raw);
    R *sm = tabs + C::TABPAD;
    __shared__ int s_e[C::EPB];
    __shared__ FaceRef s_face[C::EPB * 2 * DIM];
    const int es = elem_stride<DIM, P>(A.tsz, false);
    const int nel = block_setup<R, DIM, P>(A, tabs, s_e, s_face);
    element_fields<R, DIM, P>(A.x, A.xoff, tabs, tabs + C::N * C::NP, sm, es, s_e, nel);
    for (int k = 0; k < DIM; ++k) faces_dir<R, DIM, P, FACE_TRACE>(A, k, sm, es, s_e, s_face, nel, nfm, 0);
}

// Volume pointwise terms plus the staged face contributions, in place:
// U <- m = lambda w|J| u (+ face value terms), G <- q = G w grad_xi u (+ face
// gradient terms).  The staging area S (at S_off) holds per local face f the
// value-test and grad-test inputs at the element's own face points.
template <class R, int DIM, int P>
__device__ __forceinline__ void pointwise_faces(const OpArgs<R> &A, R *sm, int es, const int *s_e, int nel,
                                                int S_off) {
    using C = Cfg<DIM, P>;
    using Ly = Lay<DIM, P>;
    constexpr int N = C::N, NPTS = C::NPTS, NQ = C::NQ;
    for (int it = threadIdx.x; it < nel * NPTS; it += BLOCK) {
        const int el = it / NPTS, q = it - el * NPTS;
        const int e = s_e[el];
        const R *gb = A.vgeo + A.voff[e];
        R *U = sm + el * es + Ly::U;
        R *G = sm + el * es + Ly::G;
        const R *S = sm + el * es + S_off;
        R u = U[q];
        R m, q0, q1, q2 = 0;
        if constexpr (DIM == 2) {
            const R g00 = gb[q], g01 = gb[NPTS + q], g11 = gb[2 * NPTS + q], wj = gb[3 * NPTS + q];
            const R d0 = G[q], d1 = G[NPTS + q];
            m = A.lam[e] * wj * u;
            q0 = g00 * d0 + g01 * d1;
            q1 = g01 * d0 + g11 * d1;
            const int i0 = q % N, i1 = q / N;
            // faces k=0 (points (i0 fixed, a=i1)), k=1 (a=i0)
            if (i0 == 0 || i0 == N - 1) {
                const int f = i0 == 0 ? 0 : 1;
                const R *Sf = S + f * NQ * C::NFP;
                m += Sf[i1];
                q0 += Sf[C::NFP + i1];
                q1 += Sf[2 * C::NFP + i1];
            }
            if (i1 == 0 || i1 == N - 1) {
                const int f = i1 == 0 ? 2 : 3;
                const R *Sf = S + f * NQ * C::NFP;
                m += Sf[i0];
                q0 += Sf[C::NFP + i0];
                q1 += Sf[2 * C::NFP + i0];
            }
            U[q] = m;
            G[q] = q0;
            G[NPTS + q] = q1;
        } else {
            const R g00 = gb[q], g01 = gb[NPTS + q], g02 = gb[2 * NPTS + q];
            const R g11 = gb[3 * NPTS + q], g12 = gb[4 * NPTS + q], g22 = gb[5 * NPTS + q];
            const R wj = gb[6 * NPTS + q];
            const R d0 = G[q], d1 = G[NPTS + q], d2 = G[2 * NPTS + q];
            m = A.lam[e] * wj * u;
            q0 = g00 * d0 + g01 * d1 + g02 * d2;
            q1 = g01 * d0 + g11 * d1 + g12 * d2;
            q2 = g02 * d0 + g12 * d1 + g22 * d2;
            const int i0 = q % N, i1 = (q / N) % N, i2 = q / (N * N);
            const int idx[3] = {i0, i1, i2};
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) {
                const int ik = idx[kk];
                if (ik == 0 || ik == N - 1) {
                    const int f = 2 * kk + (ik == 0 ? 0 : 1);
                    const int a = kk == 0 ? i1 : i0;
                    const int b = kk == 2 ? i1 : i2;
                    const R *Sf = S + f * NQ * C::NFP + a + N * b;
                    m += Sf[0];
                    q0 += Sf[C::NFP];
                    q1 += Sf[2 * C::NFP];
                    q2 += Sf[3 * C::NFP];
                }
            }
            U[q] = m;
            G[q] = q0;
            G[NPTS + q] = q1;
            G[2 * NPTS + q] = q2;
        }
    }
    __syncthreads();

}

// K2: y = A x for the elements of the group.
template <class R, int DIM, int P>
__global__ __launch_bounds__(BLOCK) void k_apply(OpArgs<R> A, int nfm) {
    using C = Cfg<DIM, P>;
    using Ly = Lay<DIM, P>;
    constexpr int N = C::N, NP = C::NP, EPB = C::EPB, NPTS = C::NPTS, NQ = C::NQ;
    if (A.skip && *A.skip) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R *tabs = reinterpret_cast<R *>(smem_raw);
    R *sm = tabs + C::TABPAD;
    __shared__ int s_e[EPB];
    __shared__ FaceRef s_face[EPB * 2 * DIM];
    const int es = elem_stride<DIM, P>(A.tsz, true);
    const int S_off = Ly::T + A.tsz;
    const R *Bt = tabs, *Dt = tabs + N * NP;
    const int nel = block_setup<R, DIM, P>(A, tabs, s_e, s_face);
    element_fields<R, DIM, P>(A.x, A.xoff, Bt, Dt, sm, es, s_e, nel);
    for (int k = 0; k < DIM; ++k) faces_dir<R, DIM, P, FACE_LIFT>(A, k, sm, es, s_e, s_face, nel, nfm, S_off);

    // volume pointwise terms + face contributions, in place: U <- m, G <- q
    pointwise_faces<R, DIM, P>(A, sm, es, s_e, nel, S_off);

    element_iproduct<R, DIM, P>(A.y, A.xoff, Bt, Dt, sm, es, s_e, nel);
}

}  // namespace sipdg
