// Device code besides the operator: per-element kernels that reuse the
// operator's sum-factorisation (load vector, parameter gradients) and are
// instantiated per order next to it.
#pragma once

#include "operator.hpp"

namespace sipdg {

// Load vector b = (phi_i, s) + sum over boundary faces of
// [ -(g, grad phi_i . n) + 2 tau (g, phi_i) ]  (the Dirichlet data terms of the
// mirrored exterior value moved to the right-hand side).
template <int DIM, int P>
__global__ __launch_bounds__(BLOCK) void k_load(OpArgs<double> A, const int64_t *qoff,
                                                const int64_t *boff, const double *src,
                                                const double *gdir) {
    using C = Cfg<DIM, P>;
    using Ly = Lay<DIM, P>;
    constexpr int N = C::N, NP = C::NP, EPB = C::EPB, NPTS = C::NPTS, NFP = C::NFP;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *tabs = reinterpret_cast<double *>(smem_raw);
    double *sm = tabs + C::TABPAD;
    __shared__ int s_e[EPB];
    __shared__ FaceRef s_face[EPB * 2 * DIM];
    const int es = elem_stride<DIM, P>(A.tsz, false);
    const int nel = block_setup<double, DIM, P>(A, tabs, s_e, s_face);
    for (int it = threadIdx.x; it < nel * NPTS; it += BLOCK) {
        const int el = it / NPTS, q = it - el * NPTS;
        const int e = s_e[el];
        const double *gb = A.vgeo + A.voff[e];
        double m = gb[(C::NGEO - 1) * NPTS + q] * src[qoff[e] + q];
        double qq[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) qq[c] = 0.0;
        int idx[3] = {q % N, (q / N) % N, DIM == 3 ? q / (N * N) : 0};
        int nb = 0;  // ordinal of the boundary face within the element
        for (int f = 0; f < 2 * DIM; ++f) {
            const FaceRef fr = s_face[el * 2 * DIM + f];
            if (face_slot(fr.info) != 2) continue;
            const int k = f / 2, s = f & 1;
            const int ik = idx[k];
            if (ik == (s ? N - 1 : 0)) {
                int a, b;
                if constexpr (DIM == 2) {
                    a = k == 0 ? idx[1] : idx[0];
                    b = 0;
                } else {
                    a = k == 0 ? idx[1] : idx[0];
                    b = k == 2 ? idx[1] : idx[2];
                }
                const int fp = a + N * b;
                const double *fg = A.fgeo + A.foff[fr.F];
                const double g = gdir[boff[e] + (int64_t)nb * NFP + fp];
                const double tau = A.tau[fr.F];
                m += 2.0 * tau * fg[fp] * g;
#pragma unroll
                for (int c = 0; c < DIM; ++c) qq[c] -= g * fg[NFP + c * NFP + fp];
            }
            ++nb;
        }
        sm[el * es + Ly::U + q] = m;
#pragma unroll
        for (int c = 0; c < DIM; ++c) sm[el * es + Ly::G + c * NPTS + q] = qq[c];
    }
    __syncthreads();
    element_iproduct<double, DIM, P>(A.y, A.xoff, tabs, tabs + N * NP, sm, es, s_e, nel);
}

// Element part of the parameter gradients of a^T A b:
// dlam[e] = sum_q w|J| (B a)(B b)                       (volume mass term)
// bsig[e] = sum over boundary face points 2 tau0 a_q (B a)(B b)
template <int DIM, int P>
__global__ __launch_bounds__(BLOCK) void k_pgrad_elem(OpArgs<double> A, const double *av,
                                                      const double *bv, const double *tau0,
                                                      double *dlam, double *bsig) {
    using C = Cfg<DIM, P>;
    using Ly = Lay<DIM, P>;
    constexpr int N = C::N, NP = C::NP, EPB = C::EPB, NPTS = C::NPTS, NFP = C::NFP;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *tabs = reinterpret_cast<double *>(smem_raw);
    double *sm = tabs + C::TABPAD;
    __shared__ int s_e[EPB];
    __shared__ FaceRef s_face[EPB * 2 * DIM];
    const int es = elem_stride<DIM, P>(A.tsz, false);
    const int nel = block_setup<double, DIM, P>(A, tabs, s_e, s_face);
    element_fields<double, DIM, P, false>(av, A.xoff, tabs, tabs + N * NP, sm, es, s_e, nel);
    for (int it = threadIdx.x; it < nel * NPTS; it += BLOCK) {
        const int el = it / NPTS, q = it - el * NPTS;
        sm[el * es + Ly::G + q] = sm[el * es + Ly::U + q];
    }
    __syncthreads();
    element_fields<double, DIM, P, false>(bv, A.xoff, tabs, tabs + N * NP, sm, es, s_e, nel);
    // products in the work area: T[q] volume, T[NPTS+q] boundary
    for (int it = threadIdx.x; it < nel * NPTS; it += BLOCK) {
        const int el = it / NPTS, q = it - el * NPTS;
        const int e = s_e[el];
        const double *gb = A.vgeo + A.voff[e];
        const double uv = sm[el * es + Ly::U + q] * sm[el * es + Ly::G + q];
        sm[el * es + Ly::T + q] = gb[(C::NGEO - 1) * NPTS + q] * uv;
        int idx[3] = {q % N, (q / N) % N, DIM == 3 ? q / (N * N) : 0};
        double bs = 0.0;
        for (int f = 0; f < 2 * DIM; ++f) {
            const FaceRef fr = s_face[el * 2 * DIM + f];
            if (face_slot(fr.info) != 2) continue;
            const int k = f / 2, s = f & 1;
            if (idx[k] != (s ? N - 1 : 0)) continue;
            int a, b;
            if constexpr (DIM == 2) {
                a = k == 0 ? idx[1] : idx[0];
                b = 0;
            } else {
                a = k == 0 ? idx[1] : idx[0];
                b = k == 2 ? idx[1] : idx[2];
            }
            const double *fg = A.fgeo + A.foff[fr.F];
            bs += 2.0 * tau0[fr.F] * fg[a + N * b] * uv;
        }
        sm[el * es + Ly::T + NPTS + q] = bs;
    }
    __syncthreads();
    if (threadIdx.x < nel) {
        const int el = threadIdx.x;
        double s1 = 0.0, s2 = 0.0;
        for (int q = 0; q < NPTS; ++q) {
            s1 += sm[el * es + Ly::T + q];
            s2 += sm[el * es + Ly::T + NPTS + q];
        }
        dlam[s_e[el]] = s1;
        bsig[s_e[el]] = s2;
    }
}

}  // namespace sipdg
