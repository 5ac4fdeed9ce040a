// Multi-element tiles of the gather-fold apply (two-stage structure, own and
// neighbour traces from the trace buffer), orders 1..5.
//
// One element of order p has (p+2)^2 point columns; one per wavefront lane
// leaves most lanes idle at low order (25 of 64 at p = 3).  A tile packs E
// elements into a workgroup of NW wavefronts: thread t holds column
// c = t mod n^2 of element t / n^2, so the volume work (BwdTrans, collocation
// derivatives, pointwise terms, IProduct: Sec. 3.1) runs for all E elements
// at once, each on its own pair of LDS point arrays.  The face work (flux on
// the shared trace and its lift, Sec. 3.3) needs a lane per trace point
// (traces up to 8 x 8): each wavefront takes one element's faces at a time,
// round after round, leaving the lifted flux of its two faces of the current
// direction in that element's LDS slot, from where the element's column
// threads add it to their pointwise terms.  The result is the one-element
// kernel's to rounding (same arithmetic per element, same order of sums).
#pragma once

#include "gfold3d.hpp"

namespace sipdg {
namespace g3 {

template <int P, int E, int NW>
struct MSz {
    static constexpr int N = P + 2, NP = P + 1, NC = N * N, T = 64 * NW, W = 64;
    static_assert(P <= 5, "multi-element tiles: orders whose traces fit the 8 x 8 lane grid, own traces buffered");
    static_assert(E >= 1 && E * NC <= T, "every column of the tile needs a thread");
    static_assert(6 * E <= 64, "face records of the tile in one wavefront");
    static constexpr int PTS = 2 * Sz<P>::ARR;   // SA, SB of one element
    // a field on the element's own face points (t1, t2 < n, lane t1 + 8 t2)
    static constexpr int FS = 8 * N;
    static constexpr int WSCR = 8 * W + 8 * FS;   // one wavefront's lift scratch
    static constexpr int FBE = 8 * FS;            // one element's lifted flux: [2 sides][4 fields][FS]
    static constexpr int FACE = E * FBE + NW * WSCR;
    static constexpr int BODY = E * PTS > FACE ? E * PTS : FACE;
    static constexpr int TOTAL = BODY + ((ITab<P>::SIZE + 3) & ~3);
};

// Face records of the tile's elements: lane j < 6 cnt of every wavefront
// loads face j % 6 of element j / 6 (one round of loads for all of them).
template <class R>
__device__ __forceinline__ MetaV<R> load_meta_tile(const Args &A, const Data<R> &D, int e0, int cnt) {
    MetaV<R> m;
    const int j = threadIdx.x & 63;
    if (j < 6 * cnt) {
        const FaceDesc fr = A.fdesc[(int64_t)e0 * 6 + j];
        m.F = fr.F;
        m.info = fr.info;
        m.fo = fr.fo;
        m.to = fr.to;
        m.tau = D.tau[fr.F];
    }
    return m;
}

template <class R, int P, int E, int NW, int GEO>
__device__ __forceinline__ void k3gm_elem(const Args &A, const Data<R> &D, int blk, unsigned char *smem_raw) {
    using S = Sz<P>;
    using M = MSz<P, E, NW>;
    constexpr int N = S::N, NP = S::NP, NC = M::NC, SG = 8, FS = M::FS;
    constexpr int ROUNDS = (E + NW - 1) / NW;
    static_assert(6 * (ROUNDS * NW - 1) + 5 < 64, "face records read from lanes of one wavefront");
    R *base = reinterpret_cast<R *>(smem_raw);
    const int t = threadIdx.x;
    const int h = t / NC, cc = t - h * NC, a = cc % N, b = cc / N;
    const int wv = t >> 6;
    const int e0 = blk * E;
    const int cnt = A.count - e0 < E ? A.count - e0 : E;
    const bool act = h < cnt;   // a column thread of an element present in the tile
    R *SA = base + (h < E ? h : 0) * M::PTS;
    R *SB = SA + S::ARR;
    ElemDesc ed;
    ed.xoff = ed.voff = 0;
    ed.e = ed.pad = 0;
    if (act) ed = A.desc[e0 + h];
    const ctab<R> Bt = as_const(D.tab) + tab_off_B(P);   // [N][NP]
    const ctab<R> Dt = as_const(D.tab) + tab_off_D(N);   // [N][N]
    const MetaV<R> meta = load_meta_tile<R>(A, D, e0, cnt);
    // interpolation tables of this order into LDS (read after several barriers)
    R *itl = base + M::BODY;
#pragma unroll
    for (int m = N + 1; m <= 8; ++m) {
        const R *__restrict__ src = D.tab + tab_off_I(N, m);
        for (int i = t; i < m * N; i += M::T) itl[itab_off<P>(m) + i] = src[i];
    }

    // BwdTrans along xi_0: thread (i1, i2) of each element
    if (act && a < NP && b < NP) {
        const R *__restrict__ xe = D.x + ed.xoff + NP * (a + NP * b);
        R v[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) v[i] = xe[i];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            R s = 0;
#pragma unroll
            for (int i = 0; i < NP; ++i) s += Bt[q * NP + i] * v[i];
            SA[pa<P>(q, a, b)] = s;
        }
    }
    __syncthreads();
    // along xi_1: thread (q0, i2)
    if (act && b < NP) {
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
    if (act) {
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
    if (act) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            SA[pa<P>(a, b, q)] = u[q];
            SB[pa<P>(a, b, q)] = d2[q];
        }
    }
    __syncthreads();
    // d_0 u along lines (q1, q2) = (a, b), d_1 u along lines (q0, q2) = (a, b)
    R l0[N], l1[N];
    if (act) {
        R v[N], w[N];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            v[j] = SA[pa<P>(j, a, b)];
            w[j] = SA[pa<P>(a, j, b)];
        }
#pragma unroll
        for (int q = 0; q < N; ++q) {
            R s = 0, r = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                s += Dt[q * N + j] * v[j];
                r += Dt[q * N + j] * w[j];
            }
            l0[q] = s;
            l1[q] = r;
        }
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            SA[pa<P>(q, a, b)] = l0[q];
            SB[pa<P>(a, q, b)] = l1[q];
        }
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            d0[q] = SA[pa<P>(a, b, q)];
            d1[q] = SB[pa<P>(a, b, q)];
        }
        // pointwise: m = lambda w|J| u, q = (G w) grad_xi u (in place)
        pointwise<R, P, GEO>(D, ed, a, b, u, d0, d1, d2);
    }
    __syncthreads();   // the point arrays become the face scratch

    // Faces, one direction at a time: each wavefront forms and lifts the flux
    // of its elements' two faces normal to xi_k (round after round), leaving
    // it in the element's slot FB[h]; then every column thread adds its
    // element's lifted flux to its pointwise terms.
    R *FB = base;                                   // [E][2 sides][4 fields][FS]
    R *WS = base + E * M::FBE + wv * M::WSCR;      // this wavefront's lift scratch
    const int ln = t & 63;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        for (int r = 0; r < ROUNDS; ++r) {
            const int hh = r * NW + wv;   // uniform in the wavefront
            if (NW == 1 && hh >= cnt) break;
            const FaceU<R> fA = face_uniform<R>(meta, 6 * hh + 2 * k);
            const FaceU<R> fB = face_uniform<R>(meta, 6 * hh + 2 * k + 1);
            const FaceD<R> dA = load_face<R, P, 1>(D, fA, k);
            const FaceD<R> dB = load_face<R, P, 1>(D, fB, k);
            R LA[4], LB[4];
            flux_tb<R, P>(fA, dA, LA);
            flux_tb<R, P>(fB, dB, LB);
            lift2<R, P, (NW > 1), M::FS>(itl, fA.nf, fB.nf, WS, LA, LB);
            if (hh < cnt && ln < M::FS) {
                R *fb = FB + hh * M::FBE;
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    fb[f * FS + ln] = LA[f];
                    fb[4 * FS + f * FS + ln] = LB[f];
                }
            }
        }
        __syncthreads();
        if (act) {
            const R *fe = FB + h * M::FBE;
            if (k == 0 && (a == 0 || a == N - 1)) {
                // faces normal to xi_0: face point (q1, q2) = (b, q)
                const R *fb = fe + (a == 0 ? 0 : 4 * FS) + b;
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    u[q] += fb[SG * q];
                    d0[q] += fb[FS + SG * q];
                    d1[q] += fb[2 * FS + SG * q];
                    d2[q] += fb[3 * FS + SG * q];
                }
            } else if (k == 1 && (b == 0 || b == N - 1)) {
                // faces normal to xi_1: face point (q0, q2) = (a, q)
                const R *fb = fe + (b == 0 ? 0 : 4 * FS) + a;
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    u[q] += fb[SG * q];
                    d1[q] += fb[FS + SG * q];
                    d0[q] += fb[2 * FS + SG * q];
                    d2[q] += fb[3 * FS + SG * q];
                }
            } else if (k == 2) {
                // faces normal to xi_2: face point (q0, q1) = (a, b), the column ends
                const R *fl = fe + a + SG * b, *fh = fl + 4 * FS;
                u[0] += fl[0];
                d2[0] += fl[FS];
                d0[0] += fl[2 * FS];
                d1[0] += fl[3 * FS];
                u[N - 1] += fh[0];
                d2[N - 1] += fh[FS];
                d0[N - 1] += fh[2 * FS];
                d1[N - 1] += fh[3 * FS];
            }
        }
        __syncthreads();
    }

    // IProduct: y = B^T (m + D_0^T q_0 + D_1^T q_1 + D_2^T q_2)
    R z[N];
    if (act) {
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
    if (act) {
        R v[N], w[N];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            v[j] = SA[pa<P>(j, a, b)];
            w[j] = SB[pa<P>(a, j, b)];
        }
#pragma unroll
        for (int j = 0; j < N; ++j) {
            R s = 0, r = 0;
#pragma unroll
            for (int q = 0; q < N; ++q) {
                s += Dt[q * N + j] * v[q];
                r += Dt[q * N + j] * w[q];
            }
            l0[j] = s;
            l1[j] = r;
        }
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            SA[pa<P>(q, a, b)] = l0[q];
            SB[pa<P>(a, q, b)] = l1[q];
        }
    }
    __syncthreads();
    R w2[NP];
    if (act) {
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
    if (act) {
#pragma unroll
        for (int i = 0; i < NP; ++i) SA[pa<P>(a, b, i)] = w2[i];
    }
    __syncthreads();
    // B^T along xi_1: thread (q0, i2)
    if (act && b < NP) {
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
    // B^T along xi_0: thread (i1, i2), y written once
    if (act && a < NP && b < NP) {
        R v[N];
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] = SB[pa<P>(j, a, b)];
        R *__restrict__ ye = D.y + ed.xoff + NP * (a + NP * b);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            R s = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) s += Bt[j * NP + i] * v[j];
            ye[i] = s;
        }
    }
}

// Register budget (waves per SIMD the compiler sizes the kernel for) of a
// tile instance: BUD.
template <class R, int P, int E, int NW, int GEO, int BUD>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(BUD))) void k3gm(Args A, Data<R> D) {
    if (A.skip && *A.skip) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    k3gm_elem<R, P, E, NW, GEO>(A, D, blockIdx.x, smem_raw);
}

}  // namespace g3
}  // namespace sipdg
