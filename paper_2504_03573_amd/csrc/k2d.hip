// 2-D wavefront kernels of the operator (quadrilaterals of order <= 6 whose
// faces carry at most 8 trace points): one 64-lane wavefront per element,
// every element of the handle in one launch (switching on its order;
// elements listed by decreasing order).
//
// Lanes take two roles in turn:
//   * volume (lane q0 + 8 q1 = quadrature point (q0, q1)): BwdTrans and the
//     collocation derivatives (Sec. 3.1), the pointwise terms with the
//     per-point factors, and at the end the IProduct with the transposed
//     collocation derivative, y written once;
//   * faces (lane 8 f + t = trace point t of local face f): the element's u
//     and grad_xi u at the shared trace points evaluated from its
//     coefficients (TracePhysEval, Sec. 3.2: reduction along the face normal
//     with the modes' end values, evaluation along the face), g = C . grad_xi u
//     with the side's own factors, the flux of eq. IP at the trace point,
//     and the transposed interpolation I^T back to the element's face points
//     (Sec. 3.3), where the lifted value- and gradient-test terms are added
//     to the pointwise terms, so one IProduct lifts faces and volume.
// Modes:
//   TRACE: each interior face side's (u, g) into the trace buffer (owner
//          point order), nothing else;
//   APPLY: the neighbour's (u, g) from the trace buffer (TRACE must have run
//          on the same x);
//   FUSED: the neighbour's (u, g) evaluated here from its coefficients (no
//          trace buffer, one launch per application).
// The tables are the handle's (Legendre or modified C0 modes): end values of
// the modes are the first and last rows of the mode table at the element's
// GLL points, which contain +-1.
#include "launch.hpp"

namespace sipdg {
namespace g2 {

constexpr int S9 = PMAX + 1;   // row stride of the BF / DBF tables
constexpr int NFM = 8;         // largest trace per face

enum { M_TRACE = 0, M_APPLY = 1, M_FUSED = 2 };

// LDS of one element (R units)
enum {
    L_XS = 0,        // own coefficients            [64]
    L_T = 64,        // half-transformed grid       [64]
    L_U = 128,       // u, later the IProduct input [64]
    L_Q0 = 192,      // q_0 = (G w grad u)_0        [64]
    L_Q1 = 256,      // q_1                         [64]
    L_FL = 320,      // flux terms at trace points  [4][3][8]
    L_LF = 416,      // the same at the face points [4][3][8]
    L_B = 512,       // B [n][N_P]                  [64]
    L_D = 576,       // D [n][n]                    [64]
    L_NX = 640,      // neighbours' coefficients    [4][64] (FUSED)
    L_TOTAL = 896
};

// u, d_k u and d_a u at trace point t of an element's face normal to k at
// side s: x has np modes per direction (first direction fastest), n the
// element's GLL points, nf the trace points.
// np <= NPM: the table entries are loaded into registers first (one round
// of loads), then the sums run fully unrolled over NPM with np guarding.
template <class R, int NPM>
__device__ __forceinline__ void face_eval(const R *x, int np, int n, int k, int s, const R *tab, int nf, int t,
                                          R &u, R &dk, R &da) {
    const int end = s ? n - 1 : 0;
    const R *Ep = tab + tab_off_BF(n) + end * S9, *Edp = tab + tab_off_DBF(n) + end * S9;
    const R *Fp = tab + tab_off_BF(nf) + t * S9, *Fdp = tab + tab_off_DBF(nf) + t * S9;
    R E[NPM], Ed[NPM], F[NPM], Fd[NPM];
#pragma unroll
    for (int i = 0; i < NPM; ++i) {
        const bool ok = i < np;
        E[i] = ok ? Ep[i] : R(0);
        Ed[i] = ok ? Edp[i] : R(0);
        F[i] = ok ? Fp[i] : R(0);
        Fd[i] = ok ? Fdp[i] : R(0);
    }
    u = dk = da = R(0);
#pragma unroll
    for (int ia = 0; ia < NPM; ++ia) {
        if (ia >= np) break;
        R r0 = 0, r1 = 0;
#pragma unroll
        for (int ik = 0; ik < NPM; ++ik) {
            if (ik >= np) break;
            const R xv = x[k == 0 ? ik + np * ia : ia + np * ik];
            r0 += xv * E[ik];
            r1 += xv * Ed[ik];
        }
        u += r0 * F[ia];
        dk += r1 * F[ia];
        da += r0 * Fd[ia];
    }
}

template <class R, int P, int MODE>
__device__ __forceinline__ void elem2(const Args2 &A, const Data2<R> &D, int i, R *sm) {
    constexpr int N = P + 2, NP = P + 1, NM = NP * NP, NPTS = N * N;
    static_assert(N <= NFM, "one lane per point of the 8 x 8 grid");
    const int l = threadIdx.x;
    const ElemDesc ed = A.desc[i];
    R *XS = sm + L_XS, *T = sm + L_T, *U = sm + L_U, *Q0 = sm + L_Q0, *Q1 = sm + L_Q1;
    R *FL = sm + L_FL, *LF = sm + L_LF, *BL = sm + L_B, *DL = sm + L_D, *NX = sm + L_NX;

    // face role: lane 8 f + t
    const int f = l >> 3, t = l & 7;
    const bool fl = f < 4;
    const int k = f >> 1, s = f & 1, a = 1 - k;
    FaceDesc fr{0, 0, 0, 0};
    R tau = 0;
    int nf = 0, slot = 2;
    if (fl) {
        fr = A.fdesc[(int64_t)i * 4 + f];   // with the neighbour record below: one round of loads
        nf = face_nf(fr.info);
        slot = face_slot(fr.info);
        if (MODE != M_TRACE) tau = D.tau[fr.F];
    }
    // the neighbour of this lane's face (FUSED): coefficients, order, local
    // face and orientation relative to the owner's point order
    int npn = 0, kn = 0, sn = 0, on = 0;
    int64_t xn = 0;
    if (MODE == M_FUSED && fl) {
        const NbDesc2 nd = A.nbdesc[(int64_t)i * 4 + f];
        npn = nd.code & 15;
        kn = (nd.code >> 5) & 1;
        sn = (nd.code >> 4) & 1;
        on = nd.code >> 6;
        xn = nd.xn;
    }

    // coefficients and tables into LDS
    if (l < NM) XS[l] = D.x[ed.xoff + l];
    if (MODE != M_TRACE) {
        if (l < N * NP) BL[l] = D.tab[tab_off_B(P) + l];
        if (l < N * N) DL[l] = D.tab[tab_off_D(N) + l];
    }
    if (MODE == M_FUSED && fl && slot != 2) {
        for (int j = t; j < npn * npn; j += 8) NX[f * 64 + j] = D.x[xn + j];
    }
    // the lane's volume factors meanwhile
    const int q0 = l & 7, q1 = l >> 3;
    const bool vl = q0 < N && q1 < N;
    R G00 = 0, G01 = 0, G11 = 0, WJ = 0;
    if (MODE != M_TRACE && vl) {
        const R *gb = D.vgeo + ed.voff + q0 + N * q1;
        G00 = gb[0];
        G01 = gb[NPTS];
        G11 = gb[2 * NPTS];
        WJ = gb[3 * NPTS];
    }
    __syncthreads();

    // faces: own (u, g), neighbour's (u, g), flux terms at the trace points
    if (fl && t < nf && (MODE != M_TRACE || slot != 2)) {
        const int o = face_orient(fr.info);
        const int qc = (o & 1) ? nf - 1 - t : t;
        const R *fg = D.fgeo + fr.fo;
        const int gs = slot == 2 ? 0 : slot;
        const R *Co = fg + nf * (1 + 2 * gs) + qc;
        const R Ck = Co[k * nf], Ca = Co[a * nf];
        R ou, odk, oda;
        face_eval<R, NP>(XS, NP, N, k, s, D.tab, nf, t, ou, odk, oda);
        const R og = Ck * odk + Ca * oda;
        const int so = slot == 1 ? 1 : 0;
        if (MODE == M_TRACE) {
            R *tb = D.tbuf + fr.to + so * 2 * nf;
            tb[qc] = ou;
            tb[nf + qc] = og;
        } else {
            R nu, ng;
            if (slot == 2) {   // mirrored exterior value
                nu = -ou;
                ng = -og;
            } else if (MODE == M_APPLY) {
                const R *tb = D.tbuf + fr.to + (1 - so) * 2 * nf;
                nu = tb[qc];
                ng = tb[nf + qc];
            } else {
                const int tn = (on & 1) ? nf - 1 - qc : qc;
                R ndk, nda;
                face_eval<R, 7>(NX + f * 64, npn, npn + 1, kn, sn, D.tab, nf, tn, nu, ndk, nda);
                const R *Cn = fg + nf * (1 + 2 * (1 - gs)) + qc;
                ng = Cn[kn * nf] * ndk + Cn[(1 - kn) * nf] * nda;
            }
            const R aw = fg[qc];
            const R jump = ou - nu;
            const R avg = R(0.5) * (og - ng);
            const R Fg = R(-0.5) * jump;
            R *fb = FL + f * 24 + t;
            fb[0] = -avg + tau * aw * jump;   // value-test term
            fb[8] = Fg * Ck;                  // gradient-test terms, own directions k, a
            fb[16] = Fg * Ca;
        }
    }
    if (MODE == M_TRACE) return;

    // BwdTrans along xi_0: lane (q0, i1)
    if (q0 < N && q1 < NP) {
        R sacc = 0;
#pragma unroll
        for (int i0 = 0; i0 < NP; ++i0) sacc += BL[q0 * NP + i0] * XS[i0 + NP * q1];
        T[q0 + 8 * q1] = sacc;
    }
    __syncthreads();
    R u = 0;
    if (vl) {
#pragma unroll
        for (int i1 = 0; i1 < NP; ++i1) u += BL[q1 * NP + i1] * T[q0 + 8 * i1];
        U[l] = u;
    }
    // lift: the flux terms back to the face points (I^T for finer traces)
    if (fl && t < N) {
        const R *fb = FL + f * 24;
        R *lb = LF + f * 24 + t;
        if (nf == N) {
            lb[0] = fb[t];
            lb[8] = fb[8 + t];
            lb[16] = fb[16 + t];
        } else {
            const R *I = D.tab + tab_off_I(N, nf);
            R wv[NFM];
#pragma unroll
            for (int tt = 0; tt < NFM; ++tt) wv[tt] = tt < nf ? I[tt * N + t] : R(0);
            R c0 = 0, c1 = 0, c2 = 0;
#pragma unroll
            for (int tt = 0; tt < NFM; ++tt) {
                if (tt >= nf) break;
                c0 += wv[tt] * fb[tt];
                c1 += wv[tt] * fb[8 + tt];
                c2 += wv[tt] * fb[16 + tt];
            }
            lb[0] = c0;
            lb[8] = c1;
            lb[16] = c2;
        }
    }
    __syncthreads();
    R m = 0, g0 = 0, g1 = 0;
    if (vl) {
        R d0 = 0, d1 = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            d0 += DL[q0 * N + j] * U[j + 8 * q1];
            d1 += DL[q1 * N + j] * U[q0 + 8 * j];
        }
        // pointwise terms: m = lambda w|J| u, q = (G w) grad_xi u
        m = D.lam[ed.e] * WJ * u;
        g0 = G00 * d0 + G01 * d1;
        g1 = G01 * d0 + G11 * d1;
        // the lifted face terms at the element's face points
        if (q0 == 0 || q0 == N - 1) {
            const R *lb = LF + (q0 == 0 ? 0 : 24) + q1;
            m += lb[0];
            g0 += lb[8];
            g1 += lb[16];
        }
        if (q1 == 0 || q1 == N - 1) {
            const R *lb = LF + (q1 == 0 ? 48 : 72) + q0;
            m += lb[0];
            g1 += lb[8];
            g0 += lb[16];
        }
    }
    __syncthreads();   // every lane has read U
    if (vl) {
        Q0[l] = g0;
        Q1[l] = g1;
    }
    __syncthreads();
    // IProduct: z = m + D^T q_0 + D^T q_1 at (q0, q1), then B^T in both directions
    if (vl) {
        R z = m;
#pragma unroll
        for (int j = 0; j < N; ++j) z += DL[j * N + q0] * Q0[j + 8 * q1] + DL[j * N + q1] * Q1[q0 + 8 * j];
        U[l] = z;
    }
    __syncthreads();
    if (q0 < NP && q1 < N) {
        R sacc = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) sacc += BL[j * NP + q0] * U[j + 8 * q1];
        T[q0 + 8 * q1] = sacc;
    }
    __syncthreads();
    if (q0 < NP && q1 < NP) {
        R sacc = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) sacc += BL[j * NP + q1] * T[q0 + 8 * j];
        D.y[ed.xoff + q0 + NP * q1] = sacc;
    }
}

template <class R, int MODE>
__global__ __launch_bounds__(64) void k2_all(Args2 A, Data2<R> D) {
    if (A.skip && *A.skip) return;
    __shared__ R sm[L_TOTAL];
    const int i = blockIdx.x;
    switch (A.desc[i].pad & ELEM_ORDER_MASK) {
    case 1: elem2<R, 1, MODE>(A, D, i, sm); break;
    case 2: elem2<R, 2, MODE>(A, D, i, sm); break;
    case 3: elem2<R, 3, MODE>(A, D, i, sm); break;
    case 4: elem2<R, 4, MODE>(A, D, i, sm); break;
    case 5: elem2<R, 5, MODE>(A, D, i, sm); break;
    default: elem2<R, 6, MODE>(A, D, i, sm); break;
    }
}

}  // namespace g2

template <class R>
hipError_t launch_wave2d(int mode, const Args2 &A, const Data2<R> &D, hipStream_t st) {
    if (A.count <= 0) return hipSuccess;
    if (mode == g2::M_TRACE) hipLaunchKernelGGL((g2::k2_all<R, g2::M_TRACE>), dim3(A.count), dim3(64), 0, st, A, D);
    else if (mode == g2::M_APPLY) hipLaunchKernelGGL((g2::k2_all<R, g2::M_APPLY>), dim3(A.count), dim3(64), 0, st, A, D);
    else if (mode == g2::M_FUSED) hipLaunchKernelGGL((g2::k2_all<R, g2::M_FUSED>), dim3(A.count), dim3(64), 0, st, A, D);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template hipError_t launch_wave2d<double>(int, const Args2 &, const Data2<double> &, hipStream_t);
template hipError_t launch_wave2d<float>(int, const Args2 &, const Data2<float> &, hipStream_t);

}  // namespace sipdg
