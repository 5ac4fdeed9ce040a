// Setup and auxiliary kernels: per-point geometric factors, physical point
// coordinates, the Jacobi diagonal, the face part of the penalty gradient,
// deterministic segmented sums and precision casts.
#include "launch.hpp"
#include "operator.hpp"

namespace sipdg {

// Multilinear map at reference point xi: x and J[a][b] = dx_a / dxi_b.
template <int DIM>
__device__ inline void map_at(const double *X, const double *xi, double *x, double J[3][3]) {
    for (int a = 0; a < 3; ++a) {
        x[a] = 0.0;
        for (int b = 0; b < 3; ++b) J[a][b] = 0.0;
    }
    for (int v = 0; v < (1 << DIM); ++v) {
        double Nk[3], dN[3];
        for (int k = 0; k < DIM; ++k) {
            const int bit = (v >> k) & 1;
            Nk[k] = bit ? 0.5 * (1.0 + xi[k]) : 0.5 * (1.0 - xi[k]);
            dN[k] = bit ? 0.5 : -0.5;
        }
        double prod = 1.0;
        for (int k = 0; k < DIM; ++k) prod *= Nk[k];
        for (int b = 0; b < DIM; ++b) {
            double g = dN[b];
            for (int k = 0; k < DIM; ++k)
                if (k != b) g *= Nk[k];
            for (int a = 0; a < DIM; ++a) J[a][b] += X[v * DIM + a] * g;
        }
        for (int a = 0; a < DIM; ++a) x[a] += X[v * DIM + a] * prod;
    }
}

// adj(J) (so that J^{-1} = adj / det) and det.
template <int DIM>
__device__ inline double adjugate(const double J[3][3], double A[3][3]) {
    if constexpr (DIM == 2) {
        A[0][0] = J[1][1];
        A[0][1] = -J[0][1];
        A[1][0] = -J[1][0];
        A[1][1] = J[0][0];
        return J[0][0] * J[1][1] - J[0][1] * J[1][0];
    } else {
        A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
        A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
        A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
        A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        return J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
    }
}

// G = |J| J^{-1} J^{-T} = adj adj^T / det, entry (a, b).
template <int DIM>
__device__ inline double gtilde(const double A[3][3], double det, int a, int b) {
    double s = 0.0;
    for (int c = 0; c < DIM; ++c) s += A[a][c] * A[b][c];
    return s / det;
}

// Volume factors per element: G w (upper triangle, row-major: 00 01 (02) 11 (12 22))
// and w |J|, each an n^DIM array, element after element.
template <int DIM>
__global__ void k_geo_volume(const double *corners, const int *order, const int64_t *voff,
                             const double *tab, double *vgeo, int *flag) {
    const int64_t e = blockIdx.x;
    const int n = order[e] + 2;
    const int npts = DIM == 3 ? n * n * n : n * n;
    const double *X = corners + e * (1 << DIM) * DIM;
    const double *xs = tab + tab_off_X(n), *ws = tab + tab_off_W(n);
    constexpr int NG = DIM * (DIM + 1) / 2 + 1;
    double *out = vgeo + voff[e];
    for (int q = threadIdx.x; q < npts; q += blockDim.x) {
        const int q0 = q % n, q1 = (q / n) % n, q2 = q / (n * n);
        double xi[3] = {xs[q0], xs[q1], DIM == 3 ? xs[q2] : 0.0};
        const double w = ws[q0] * ws[q1] * (DIM == 3 ? ws[q2] : 1.0);
        double x[3], J[3][3], A[3][3];
        map_at<DIM>(X, xi, x, J);
        const double det = adjugate<DIM>(J, A);
        if (!(det > 0.0)) atomicOr(flag, 1);
        int c = 0;
        for (int a = 0; a < DIM; ++a)
            for (int b = a; b < DIM; ++b) out[(c++) * npts + q] = w * gtilde<DIM>(A, det, a, b);
        out[(NG - 1) * npts + q] = w * det;
    }
}

template <int DIM>
__device__ inline void embed(int f, const double *z, double *xi) {
    const int k = f / 2;
    int j = 0;
    for (int a = 0; a < DIM; ++a) xi[a] = (a == k) ? ((f & 1) ? 1.0 : -1.0) : z[j++];
}

// Face factors at the trace points, canonical (owner) order:
// a = w J_s from the owner's map; C_side[m] = s w G_side[k][m] with each
// side's own map at its own point.  Interior: [a][C_L x DIM][C_R x DIM],
// boundary: [a][C x DIM].
template <int DIM>
__global__ void k_geo_faces(const double *corners, const FaceTopo *ft, const int64_t *foff,
                            const double *tab, double *fgeo, int *flag) {
    const int64_t F = blockIdx.x;
    const FaceTopo t = ft[F];
    const int nf = t.nf;
    const int npf = DIM == 3 ? nf * nf : nf;
    const double *xs = tab + tab_off_X(nf), *ws = tab + tab_off_W(nf);
    double *out = fgeo + foff[F];
    for (int qc = threadIdx.x; qc < npf; qc += blockDim.x) {
        const int t1 = qc % nf, t2 = DIM == 3 ? qc / nf : 0;
        const double w = ws[t1] * (DIM == 3 ? ws[t2] : 1.0);
        for (int side = 0; side < (t.eR >= 0 ? 2 : 1); ++side) {
            const int e = side == 0 ? t.eL : t.eR;
            const int f = side == 0 ? t.fL : t.fR;
            int r1 = t1, r2 = t2;
            if (side == 1) {
                const int o = t.orient;
                int a1 = (o & 4) ? t2 : t1, a2 = (o & 4) ? t1 : t2;
                r1 = (o & 1) ? nf - 1 - a1 : a1;
                r2 = (o & 2) ? nf - 1 - a2 : a2;
                if (DIM == 2) r2 = 0;
            }
            const double z[2] = {xs[r1], DIM == 3 ? xs[r2] : 0.0};
            double xi[3], x[3], J[3][3], A[3][3];
            embed<DIM>(f, z, xi);
            map_at<DIM>(corners + (int64_t)e * (1 << DIM) * DIM, xi, x, J);
            const double det = adjugate<DIM>(J, A);
            if (!(det > 0.0)) atomicOr(flag, 2);
            const int k = f / 2;
            const double s = (f & 1) ? 1.0 : -1.0;
            if (side == 0) {
                double js = 0.0;
                for (int c = 0; c < DIM; ++c) js += A[k][c] * A[k][c];
                out[qc] = w * sqrt(js);
            }
            for (int m = 0; m < DIM; ++m) out[npf * (1 + DIM * side) + m * npf + qc] = s * w * gtilde<DIM>(A, det, k, m);
        }
    }
}

template <int DIM>
__global__ void k_points(const double *corners, const int *order, const FaceRef *eface,
                         const int64_t *qoff, const int64_t *boff, const double *tab, double *xq,
                         double *xb) {
    const int64_t e = blockIdx.x;
    const int n = order[e] + 2;
    const int npts = DIM == 3 ? n * n * n : n * n;
    const int nfp = DIM == 3 ? n * n : n;
    const double *X = corners + e * (1 << DIM) * DIM;
    const double *xs = tab + tab_off_X(n);
    for (int q = threadIdx.x; q < npts; q += blockDim.x) {
        const int q0 = q % n, q1 = (q / n) % n, q2 = q / (n * n);
        double xi[3] = {xs[q0], xs[q1], DIM == 3 ? xs[q2] : 0.0}, x[3], J[3][3];
        map_at<DIM>(X, xi, x, J);
        for (int a = 0; a < DIM; ++a) xq[(qoff[e] + q) * DIM + a] = x[a];
    }
    int nb = 0;
    for (int f = 0; f < 2 * DIM; ++f) {
        if (face_slot(eface[e * 2 * DIM + f].info) != 2) continue;
        for (int t = threadIdx.x; t < nfp; t += blockDim.x) {
            const int t1 = t % n, t2 = t / n;
            const double z[2] = {xs[t1], DIM == 3 ? xs[t2] : 0.0};
            double xi[3], x[3], J[3][3];
            embed<DIM>(f, z, xi);
            map_at<DIM>(X, xi, x, J);
            for (int a = 0; a < DIM; ++a) xb[(boff[e] + (int64_t)nb * nfp + t) * DIM + a] = x[a];
        }
        ++nb;
    }
}

// Jacobi diagonal a(phi_i, phi_i), sum-factorised, one block per element.
// Every term of the bilinear form at i = j factorises over the reference
// directions, so each is a tensor contraction with squared 1-D tables:
//  * volume: sum_q G_ab(q) g_a g_b, with g_a = D(q_a, i_a) prod_{c != a} B(q_c, i_c),
//    is the contraction of the per-point factor G_ab with, per direction d,
//    D^2 (d = a = b), B D (d one of a != b) or B^2 (otherwise); the lambda
//    term contracts w|J| with B^2 in every direction;
//  * face (k, s) at trace points t = (t1, t2) in the element's face
//    coordinates (directions a < b, both != k): phi = v_k(i_k) Bf(t1, i_a) Bf(t2, i_b)
//    with v_k, dv_k the mode values and derivatives at the end xi_k = s, and
//    phi (n.grad phi) w J_s = v_k dv_k C_k Bf^2 Bf^2 + v_k^2 (C_a (Bf Df) Bf^2 + C_b Bf^2 (Bf Df)),
//    so the face adds v_k^2 S_vv(i_a, i_b) + v_k dv_k S_vd(i_a, i_b) with two
//    2-D contractions over the trace (value-test and gradient-test terms of
//    eq. IP with the neighbour's coefficients zero; boundary faces by the
//    mirrored value, twice the consistency and penalty terms).
// The operation count is O(n^{d+1}) per term instead of O(n^d N_P^d).
// One launch per order group (elems: the group's element ids), LDS sized for
// the group's order.
template <int DIM, int P>
__global__ __launch_bounds__(256) void k_diag(const int *elems, const int64_t *xoff, const int64_t *voff,
                                              const FaceRef *eface, const int64_t *foff, const double *vgeo,
                                              const double *fgeo, const double *lam, const double *tau,
                                              const double *tab, double *diag) {
    constexpr int S = PMAX + 1, NM3 = DIM == 3 ? (P + 2) * (P + 2) * (P + 2) : (P + 2) * (P + 2);
    constexpr int NG = DIM * (DIM + 1) / 2 + 1;
    __shared__ double T[3][NMAX * S];   // B^2, D^2, B D at the volume points [q][i]
    __shared__ double G[NM3];           // one geometric factor at the volume points
    __shared__ double W1[NM3], W2[NM3]; // partial contractions
    __shared__ double acc[NM3];         // the diagonal of this element's modes
    __shared__ double FT[2][NMAX * S];  // Bf^2, Bf Df at the trace points [t][i]
    __shared__ double FW[4][NMAX * NMAX];   // a, C_k, C_a, C_b at (t1, t2)
    __shared__ double Y[3][NMAX * S];   // first face contraction [t2][i_a]
    __shared__ double SV[2][S * S];     // S_vv, S_vd [i_b][i_a]
    const int64_t e = elems[blockIdx.x];
    const int tid = threadIdx.x, nt = blockDim.x;
    constexpr int n = P + 2, np = P + 1;
    const int nm = DIM == 3 ? np * np * np : np * np;
    const int npts = DIM == 3 ? n * n * n : n * n;
    const double *Bn = tab + tab_off_BF(n), *Dn = tab + tab_off_DBF(n);
    const double *gb = vgeo + voff[e];
    for (int i = tid; i < n * np; i += nt) {
        const int q = i / np, j = i - q * np;
        const double b = Bn[q * S + j], d = Dn[q * S + j];
        T[0][q * S + j] = b * b;
        T[1][q * S + j] = d * d;
        T[2][q * S + j] = b * d;
    }
    for (int i = tid; i < nm; i += nt) acc[i] = 0.0;
    __syncthreads();
    // volume: components 00 01 02 11 12 22 (2-D: 00 01 11), then w|J| (lambda)
    int c = 0;
    for (int ta = 0; ta <= DIM; ++ta) {
        for (int tb = ta; tb < DIM || (ta == DIM && tb == DIM); ++tb) {
            const bool mass = ta == DIM;
            const double coef = mass ? lam[e] : (ta == tb ? 1.0 : 2.0);
            // table per direction: 0 = B^2, 1 = D^2, 2 = B D
            int td[3];
            for (int d = 0; d < 3; ++d)
                td[d] = mass ? 0 : (ta == d && tb == d ? 1 : ((ta == d || tb == d) ? 2 : 0));
            const double *gc = gb + (int64_t)(mass ? NG - 1 : c) * npts;
            for (int q = tid; q < npts; q += nt) G[q] = coef * gc[q];
            __syncthreads();
            const double *T0 = T[td[0]], *T1 = T[td[1]], *T2 = T[td[2]];
            if (DIM == 3) {
                // q0 -> i0: W1[i0 + np (q1 + n q2)]
                for (int i = tid; i < np * n * n; i += nt) {
                    const int i0 = i % np, r = i / np;
                    double s = 0.0;
                    for (int q = 0; q < n; ++q) s += T0[q * S + i0] * G[q + n * r];
                    W1[i] = s;
                }
                __syncthreads();
                // q1 -> i1: W2[i0 + np (i1 + np q2)]
                for (int i = tid; i < np * np * n; i += nt) {
                    const int i0 = i % np, i1 = (i / np) % np, q2 = i / (np * np);
                    double s = 0.0;
                    for (int q = 0; q < n; ++q) s += T1[q * S + i1] * W1[i0 + np * (q + n * q2)];
                    W2[i] = s;
                }
                __syncthreads();
                // q2 -> i2
                for (int i = tid; i < nm; i += nt) {
                    const int i01 = i % (np * np), i2 = i / (np * np);
                    double s = 0.0;
                    for (int q = 0; q < n; ++q) s += T2[q * S + i2] * W2[i01 + np * np * q];
                    acc[i] += s;
                }
            } else {
                for (int i = tid; i < np * n; i += nt) {
                    const int i0 = i % np, q1 = i / np;
                    double s = 0.0;
                    for (int q = 0; q < n; ++q) s += T0[q * S + i0] * G[q + n * q1];
                    W1[i] = s;
                }
                __syncthreads();
                for (int i = tid; i < nm; i += nt) {
                    const int i0 = i % np, i1 = i / np;
                    double s = 0.0;
                    for (int q = 0; q < n; ++q) s += T1[q * S + i1] * W1[i0 + np * q];
                    acc[i] += s;
                }
            }
            __syncthreads();
            if (mass) break;
            ++c;
        }
    }
    // faces
    for (int f = 0; f < 2 * DIM; ++f) {
        const FaceRef fr = eface[e * 2 * DIM + f];
        const int nf = face_nf(fr.info), slot = face_slot(fr.info), o = face_orient(fr.info);
        const int k = f / 2, end = (f & 1) ? n - 1 : 0;
        const int npf = DIM == 3 ? nf * nf : nf;
        const double *Bf = tab + tab_off_BF(nf), *Df = tab + tab_off_DBF(nf);
        const double *fg = fgeo + foff[fr.F];
        const int gs = slot == 2 ? 0 : slot;
        const double cw = slot == 2 ? 2.0 : 1.0;   // boundary: mirrored value
        const double tp = cw * tau[fr.F];
        const int da = k == 0 ? 1 : 0, db = k == 2 ? 1 : 2;
        for (int i = tid; i < nf * np; i += nt) {
            const int t = i / np, j = i - t * np;
            const double b = Bf[t * S + j], d = Df[t * S + j];
            FT[0][t * S + j] = b * b;
            FT[1][t * S + j] = b * d;
        }
        for (int t = tid; t < npf; t += nt) {
            const int t1 = t % nf, t2 = DIM == 3 ? t / nf : 0;
            const int qc = DIM == 3 ? canon_index(o, nf, t1, t2) : ((o & 1) ? nf - 1 - t1 : t1);
            const double *Cs = fg + npf * (1 + DIM * gs) + qc;
            FW[0][t] = tp * fg[qc];
            FW[1][t] = -cw * Cs[k * npf];
            FW[2][t] = -cw * Cs[da * npf];
            FW[3][t] = DIM == 3 ? -cw * Cs[db * npf] : 0.0;
        }
        __syncthreads();
        if (DIM == 3) {
            // along t1: Y0 = B2 a' + BD Ca', Y1 = B2 Cb', Y2 = B2 Ck'  [t2][i_a]
            for (int i = tid; i < nf * np; i += nt) {
                const int t2 = i / np, ia = i - t2 * np;
                double y0 = 0.0, y1 = 0.0, y2 = 0.0;
                for (int t1 = 0; t1 < nf; ++t1) {
                    const int t = t1 + nf * t2;
                    const double b2 = FT[0][t1 * S + ia], bd = FT[1][t1 * S + ia];
                    y0 += b2 * FW[0][t] + bd * FW[2][t];
                    y1 += b2 * FW[3][t];
                    y2 += b2 * FW[1][t];
                }
                Y[0][t2 * S + ia] = y0;
                Y[1][t2 * S + ia] = y1;
                Y[2][t2 * S + ia] = y2;
            }
            __syncthreads();
            for (int i = tid; i < np * np; i += nt) {
                const int ib = i / np, ia = i - ib * np;
                double vv = 0.0, vd = 0.0;
                for (int t2 = 0; t2 < nf; ++t2) {
                    const double b2 = FT[0][t2 * S + ib], bd = FT[1][t2 * S + ib];
                    vv += b2 * Y[0][t2 * S + ia] + bd * Y[1][t2 * S + ia];
                    vd += b2 * Y[2][t2 * S + ia];
                }
                SV[0][ib * S + ia] = vv;
                SV[1][ib * S + ia] = vd;
            }
        } else {
            for (int ia = tid; ia < np; ia += nt) {
                double vv = 0.0, vd = 0.0;
                for (int t1 = 0; t1 < nf; ++t1) {
                    const double b2 = FT[0][t1 * S + ia], bd = FT[1][t1 * S + ia];
                    vv += b2 * FW[0][t1] + bd * FW[2][t1];
                    vd += b2 * FW[1][t1];
                }
                SV[0][ia] = vv;
                SV[1][ia] = vd;
            }
        }
        __syncthreads();
        for (int i = tid; i < nm; i += nt) {
            const int ii[3] = {i % np, (i / np) % np, DIM == 3 ? i / (np * np) : 0};
            const double v = Bn[end * S + ii[k]], dv = Dn[end * S + ii[k]];
            const int s2 = DIM == 3 ? ii[db] * S + ii[da] : ii[da];
            acc[i] += v * v * SV[0][s2] + v * dv * SV[1][s2];
        }
        __syncthreads();
    }
    for (int i = tid; i < nm; i += nt) diag[xoff[e] + i] = acc[i];
}

// Interior-face part of d(a^T A b)/d sigma: per face
// sum_q tau0 a_q (uA_L - uA_R)(uB_L - uB_R) from the two trace buffers.
__global__ void k_pgrad_faces(int dim, const int *is_interior, const int64_t *toff,
                              const int64_t *foff, const int *nfv, const double *fgeo,
                              const double *tau0, const double *ta, const double *tb, double *out) {
    const int64_t F = blockIdx.x;
    __shared__ double red[BLOCK];
    double s = 0.0;
    if (is_interior[F]) {
        const int nf = nfv[F];
        const int npf = dim == 3 ? nf * nf : nf;
        const double *A = ta + toff[F], *B = tb + toff[F];
        const double *fg = fgeo + foff[F];
        for (int q = threadIdx.x; q < npf; q += BLOCK)
            s += fg[q] * (A[q] - A[2 * npf + q]) * (B[q] - B[2 * npf + q]);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[F] = tau0[F] * red[0];
}

__global__ void k_segsum(const int64_t *off, const double *v, double *out, int accumulate) {
    const int p = blockIdx.x;
    __shared__ double red[BLOCK];
    double s = 0.0;
    for (int64_t i = off[p] + threadIdx.x; i < off[p + 1]; i += BLOCK) s += v[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[p] = (accumulate ? out[p] : 0.0) + red[0];
}

__global__ void k_cast_f32(const double *in, float *out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}
__global__ void k_cast_f64(const float *in, double *out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (double)in[i];
}
__global__ void k_recip(const double *in, double *o64, float *o32, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double r = 1.0 / in[i];
        o64[i] = r;
        o32[i] = (float)r;
    }
}

static inline int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)(g < 8192 ? (g < 1 ? 1 : g) : 8192);
}

hipError_t launch_geo_volume(int dim, int64_t ne, const double *corners, const int *order,
                             const int64_t *voff, const double *tab, double *vgeo, int *flag,
                             hipStream_t st) {
    if (ne == 0) return hipSuccess;
    if (dim == 2) hipLaunchKernelGGL(k_geo_volume<2>, dim3(ne), dim3(128), 0, st, corners, order, voff, tab, vgeo, flag);
    else hipLaunchKernelGGL(k_geo_volume<3>, dim3(ne), dim3(256), 0, st, corners, order, voff, tab, vgeo, flag);
    return hipGetLastError();
}

hipError_t launch_geo_faces(int dim, int64_t nfaces, const double *corners, const FaceTopo *ft,
                            const int64_t *foff, const double *tab, double *fgeo, int *flag,
                            hipStream_t st) {
    if (nfaces == 0) return hipSuccess;
    if (dim == 2) hipLaunchKernelGGL(k_geo_faces<2>, dim3(nfaces), dim3(64), 0, st, corners, ft, foff, tab, fgeo, flag);
    else hipLaunchKernelGGL(k_geo_faces<3>, dim3(nfaces), dim3(128), 0, st, corners, ft, foff, tab, fgeo, flag);
    return hipGetLastError();
}

hipError_t launch_points(int dim, int64_t ne, const double *corners, const int *order,
                         const FaceRef *eface, const int64_t *qoff, const int64_t *boff,
                         const double *tab, double *xq, double *xb, hipStream_t st) {
    if (ne == 0) return hipSuccess;
    if (dim == 2) hipLaunchKernelGGL(k_points<2>, dim3(ne), dim3(128), 0, st, corners, order, eface, qoff, boff, tab, xq, xb);
    else hipLaunchKernelGGL(k_points<3>, dim3(ne), dim3(256), 0, st, corners, order, eface, qoff, boff, tab, xq, xb);
    return hipGetLastError();
}

hipError_t launch_diag(int dim, int P, int64_t count, const int *elems, const int64_t *xoff,
                       const int64_t *voff, const FaceRef *eface, const int64_t *foff,
                       const double *vgeo, const double *fgeo, const double *lam,
                       const double *tau, const double *tab, double *diag, hipStream_t st) {
    if (count == 0) return hipSuccess;
#define SIPDG_DIAG_CASE(PP)                                                                                      \
    case PP:                                                                                                    \
        if (dim == 2)                                                                                           \
            hipLaunchKernelGGL((k_diag<2, PP>), dim3(count), dim3(128), 0, st, elems, xoff, voff, eface, foff, \
                               vgeo, fgeo, lam, tau, tab, diag);                                                \
        else                                                                                                    \
            hipLaunchKernelGGL((k_diag<3, PP>), dim3(count), dim3(256), 0, st, elems, xoff, voff, eface, foff, \
                               vgeo, fgeo, lam, tau, tab, diag);                                                \
        break;
    switch (P) {
        SIPDG_DIAG_CASE(1) SIPDG_DIAG_CASE(2) SIPDG_DIAG_CASE(3) SIPDG_DIAG_CASE(4)
        SIPDG_DIAG_CASE(5) SIPDG_DIAG_CASE(6) SIPDG_DIAG_CASE(7) SIPDG_DIAG_CASE(8)
    default: return hipErrorInvalidValue;
    }
#undef SIPDG_DIAG_CASE
    return hipGetLastError();
}

hipError_t launch_pgrad_faces(int dim, int64_t nfaces, const int *is_interior,
                              const int64_t *toff, const int64_t *foff, const int *nf,
                              const double *fgeo, const double *tau0, const double *ta,
                              const double *tb, double *out, hipStream_t st) {
    if (nfaces == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pgrad_faces, dim3(nfaces), dim3(BLOCK), 0, st, dim, is_interior, toff, foff, nf, fgeo, tau0, ta, tb, out);
    return hipGetLastError();
}

hipError_t launch_segsum(int nseg, const int64_t *off, const double *v, double *out, int accumulate,
                         hipStream_t st) {
    if (nseg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_segsum, dim3(nseg), dim3(BLOCK), 0, st, off, v, out, accumulate);
    return hipGetLastError();
}

hipError_t launch_cast_f32(const double *in, float *out, int64_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cast_f32, dim3(grid_for(n)), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}
hipError_t launch_cast_f64(const float *in, double *out, int64_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cast_f64, dim3(grid_for(n)), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}
hipError_t launch_recip(const double *in, double *out64, float *out32, int64_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_recip, dim3(grid_for(n)), dim3(256), 0, st, in, out64, out32, n);
    return hipGetLastError();
}

}  // namespace sipdg
