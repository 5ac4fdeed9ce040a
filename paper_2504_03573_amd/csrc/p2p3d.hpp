// Point-to-point interpolation flux on hexahedra (Xia & Moxey, Sec. 3.3,
// ScatrInterp): the alternative to the shared trace space.  Every interior
// face is integrated twice, once per side, each side on its own GLL face
// quadrature (its own n = p+2 points per direction, weights and surface
// Jacobian), with the other side's value and physical gradient Lagrange-
// interpolated to its points.  The operator is not symmetric in general (the
// conditions of Sec. 3.3; Table 2).
//
//   K1 (trace): per element, at its own face points of every interior face:
//               u and grad_x u = J^-T grad_xi u into the point-to-point
//               buffer, in the owner's (canonical) orientation on the side's
//               own n x n grid (four values per point and side).
//   K2 (apply): per element: volume terms; per face direction, both faces:
//               the neighbour's four values interpolated from its n_o x n_o
//               grid to ours, one direction at a time in LDS (I(n_o -> n)
//               tables), and mapped to our face point order; then at our own
//               face points the flux of eq. IP with our outward normal,
//               weights and surface Jacobian (boundary faces: the mirrored
//               values), staged at the face points (no lift needed: the
//               quadrature points are the element's own); IProduct.
//
// Geometry at face points comes from the element's trilinear map (its 21
// coefficients): the columns of J, the rows of adj(J) as cross products of
// the columns, the area-weighted outward normal s * adj row k.
#pragma once

#include "launch.hpp"
#include "operator.hpp"

namespace sipdg {

// Columns of J = dx/dxi (J[c][k] = dx_c/dxi_k) at xi from the coefficients
// c1..c7 (each x, y, z) of x = c0 + c1 xi0 + c2 xi1 + c3 xi2 + c4 xi0 xi1 +
// c5 xi0 xi2 + c6 xi1 xi2 + c7 xi0 xi1 xi2; rows of adj(J) and det J.
template <class R>
__device__ __forceinline__ R map_adjugate(const R *cm, R x0, R x1, R x2, R r[3][3]) {
    R j0[3], j1[3], j2[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        j0[c] = cm[c] + cm[9 + c] * x1 + cm[12 + c] * x2 + cm[18 + c] * x1 * x2;
        j1[c] = cm[3 + c] + cm[9 + c] * x0 + cm[15 + c] * x2 + cm[18 + c] * x0 * x2;
        j2[c] = cm[6 + c] + cm[12 + c] * x0 + cm[15 + c] * x1 + cm[18 + c] * x0 * x1;
    }
    r[0][0] = j1[1] * j2[2] - j1[2] * j2[1];
    r[0][1] = j1[2] * j2[0] - j1[0] * j2[2];
    r[0][2] = j1[0] * j2[1] - j1[1] * j2[0];
    r[1][0] = j2[1] * j0[2] - j2[2] * j0[1];
    r[1][1] = j2[2] * j0[0] - j2[0] * j0[2];
    r[1][2] = j2[0] * j0[1] - j2[1] * j0[0];
    r[2][0] = j0[1] * j1[2] - j0[2] * j1[1];
    r[2][1] = j0[2] * j1[0] - j0[0] * j1[2];
    r[2][2] = j0[0] * j1[1] - j0[1] * j1[0];
    return j0[0] * r[0][0] + j0[1] * r[0][1] + j0[2] * r[0][2];
}

// Value, physical gradient and geometry at one face point.
template <class R>
struct P2PPoint {
    R u, gx[3];     // value and physical gradient
    R r[3][3], det; // rows of adj(J), det J
};

// Face point (a, b) (own face coordinates) of local face f = 2k + s of
// element e, whose fields u and grad_xi u are in LDS at sm.
template <class R, int P>
__device__ __forceinline__ P2PPoint<R> p2p_point(const OpArgs<R> &A, const R *sm, int e, int k, int s, int a,
                                                 int b) {
    using C = Cfg<3, P>;
    using Ly = Lay<3, P>;
    constexpr int N = C::N;
    P2PPoint<R> pt;
    const int q = face_point<3, N>(k, s, a, b);
    const int i0 = q % N, i1 = (q / N) % N, i2 = q / (N * N);
    const R *X = A.tab + tab_off_X(N);
    pt.det = map_adjugate<R>(A.emap + (int64_t)24 * e, X[i0], X[i1], X[i2], pt.r);
    pt.u = sm[Ly::U + q];
    const R d0 = sm[Ly::G + q], d1 = sm[Ly::G + C::NPTS + q], d2 = sm[Ly::G + 2 * C::NPTS + q];
    const R inv = R(1) / pt.det;
#pragma unroll
    for (int c = 0; c < 3; ++c) pt.gx[c] = (pt.r[0][c] * d0 + pt.r[1][c] * d1 + pt.r[2][c] * d2) * inv;
    return pt;
}

// K1: u and grad_x u at the own face points of every interior face side.
// Buffer: face F at 2 toff[F], side slot at + slot 4 nf^2, component c at
// + c nf^2, canonical index on the side's own n x n grid.
template <class R, int P>
__global__ __launch_bounds__(BLOCK) void k_p2p_trace(OpArgs<R> A) {
    using C = Cfg<3, P>;
    constexpr int N = C::N, NFP = C::NFP;
    if (A.skip && *A.skip) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R *tabs = reinterpret_cast<R *>(smem_raw);
    R *sm = tabs + C::TABPAD;
    __shared__ int s_e[C::EPB];
    __shared__ FaceRef s_face[C::EPB * 6];
    const int es = elem_stride<3, P>(A.tsz, false);
    const int nel = block_setup<R, 3, P>(A, tabs, s_e, s_face);
    element_fields<R, 3, P>(A.x, A.xoff, tabs, tabs + N * C::NP, sm, es, s_e, nel);
    for (int it = threadIdx.x; it < nel * 6 * NFP; it += BLOCK) {
        const int el = it / (6 * NFP);
        const int r = it - el * 6 * NFP;
        const int f = r / NFP, fp = r - f * NFP;
        const FaceRef fr = s_face[el * 6 + f];
        const int slot = face_slot(fr.info);
        if (slot == 2) continue;
        const int a = fp % N, b = fp / N;
        const P2PPoint<R> pt = p2p_point<R, P>(A, sm + el * es, s_e[el], f / 2, f & 1, a, b);
        const int nf = face_nf(fr.info), npf = nf * nf;
        const int qc = canon_index(face_orient(fr.info), N, a, b);
        R *tb = A.tbuf + 2 * A.toff[fr.F] + (int64_t)slot * 4 * npf;
        tb[qc] = pt.u;
        tb[npf + qc] = pt.gx[0];
        tb[2 * npf + qc] = pt.gx[1];
        tb[3 * npf + qc] = pt.gx[2];
    }
}

// Own face coordinates (a, b) of canonical index qc on an n x n grid (the
// inverse of canon_index for orientation code o).
__device__ __forceinline__ int own_of_canon(int o, int n, int qc) {
    const int c1 = qc % n, c2 = qc / n;
    const int a1 = (o & 4) ? c2 : c1, a2 = (o & 4) ? c1 : c2;
    const int r1 = (o & 1) ? n - 1 - a1 : a1;
    const int r2 = (o & 2) ? n - 1 - a2 : a2;
    return r1 + n * r2;
}

// K2: y = A_p2p x for the elements of the group (nfm: the group's largest
// trace, which bounds every neighbour's n_o).
template <class R, int P>
__global__ __launch_bounds__(BLOCK) void k_p2p_apply(OpArgs<R> A, int nfm) {
    using C = Cfg<3, P>;
    using Ly = Lay<3, P>;
    constexpr int N = C::N, NP = C::NP, NFP = C::NFP, NQ = C::NQ;
    if (A.skip && *A.skip) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R *tabs = reinterpret_cast<R *>(smem_raw);
    R *sm = tabs + C::TABPAD;
    __shared__ int s_e[C::EPB];
    __shared__ FaceRef s_face[C::EPB * 6];
    const int es = elem_stride<3, P>(A.tsz, true);
    const int S_off = Ly::T + A.tsz;
    const R *Bt = tabs, *Dt = tabs + N * NP;
    const int nel = block_setup<R, 3, P>(A, tabs, s_e, s_face);
    element_fields<R, 3, P>(A.x, A.xoff, Bt, Dt, sm, es, s_e, nel);
    const R *W = A.tab + tab_off_W(N);
    const int fs = 4 * nfm * N;   // work-area floats per face side of one direction
    for (int k = 0; k < 3; ++k) {
        // P1: the neighbour's grid interpolated along the first canonical
        // direction to our N points (work area: [s][c][j2][t1])
        for (int it = threadIdx.x; it < nel * 2 * fs; it += BLOCK) {
            const int el = it / (2 * fs);
            int r = it - el * 2 * fs;
            const int s = r / fs;
            r -= s * fs;
            const int c = r / (nfm * N);
            r -= c * nfm * N;
            const int j2 = r / N, t1 = r - j2 * N;
            const FaceRef fr = s_face[el * 6 + 2 * k + s];
            const int slot = face_slot(fr.info);
            if (slot == 2) continue;
            const FaceTopo ft = A.faces[fr.F];
            const int no = A.order[slot == 0 ? ft.eR : ft.eL] + 2;
            if (j2 >= no) continue;
            const int nf = face_nf(fr.info), npf = nf * nf;
            const R *src = A.tbuf + 2 * A.toff[fr.F] + (int64_t)(1 - slot) * 4 * npf + c * npf + j2 * no;
            const R *I = A.tab + tab_off_I(no, N) + t1 * no;
            R acc = 0;
            for (int j1 = 0; j1 < no; ++j1) acc += I[j1] * src[j1];
            sm[el * es + Ly::T + s * fs + (c * nfm + j2) * N + t1] = acc;
        }
        __syncthreads();
        // P2: along the second direction, stored at our own face point order
        for (int it = threadIdx.x; it < nel * 2 * 4 * NFP; it += BLOCK) {
            const int el = it / (8 * NFP);
            int r = it - el * 8 * NFP;
            const int s = r / (4 * NFP);
            r -= s * 4 * NFP;
            const int c = r / NFP, qc = r - c * NFP;
            const FaceRef fr = s_face[el * 6 + 2 * k + s];
            const int slot = face_slot(fr.info);
            if (slot == 2) continue;
            const FaceTopo ft = A.faces[fr.F];
            const int no = A.order[slot == 0 ? ft.eR : ft.eL] + 2;
            const int t1 = qc % N, t2 = qc / N;
            const R *I = A.tab + tab_off_I(no, N) + t2 * no;
            const R *tmp = sm + el * es + Ly::T + s * fs + c * nfm * N + t1;
            R acc = 0;
            for (int j2 = 0; j2 < no; ++j2) acc += I[j2] * tmp[j2 * N];
            const int fp = own_of_canon(face_orient(fr.info), N, qc);
            sm[el * es + S_off + ((2 * k + s) * NQ + c) * NFP + fp] = acc;
        }
        __syncthreads();
        // P3: flux of eq. IP at our own face points, staged in place
        for (int it = threadIdx.x; it < nel * 2 * NFP; it += BLOCK) {
            const int el = it / (2 * NFP);
            int r = it - el * 2 * NFP;
            const int s = r / NFP, fp = r - s * NFP;
            const int f = 2 * k + s;
            const FaceRef fr = s_face[el * 6 + f];
            const int slot = face_slot(fr.info);
            const int a = fp % N, b = fp / N;
            const P2PPoint<R> pt = p2p_point<R, P>(A, sm + el * es, s_e[el], k, s, a, b);
            // area-weighted outward normal times the quadrature weight: w s adj row k
            const R w = W[a] * W[b];
            R an[3];
            R js2 = 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const R v = s ? pt.r[k][c] : -pt.r[k][c];
                js2 += v * v;
                an[c] = w * v;
            }
            const R aw = w * sqrt(js2);   // w J_s
            const R g = an[0] * pt.gx[0] + an[1] * pt.gx[1] + an[2] * pt.gx[2];
            R *S = sm + el * es + S_off + f * NQ * NFP + fp;
            R un, go;
            if (slot == 2) {
                // mirrored exterior: u+ = -u-, grad u+ = grad u-
                un = -pt.u;
                go = g;
            } else {
                un = S[0];
                go = an[0] * S[NFP] + an[1] * S[2 * NFP] + an[2] * S[3 * NFP];
            }
            const R jump = pt.u - un;
            const R Fv = R(-0.5) * (g + go) + A.tau[fr.F] * aw * jump;
            const R Fg = R(-0.5) * jump;
            const R inv = R(1) / pt.det;
            S[0] = Fv;
#pragma unroll
            for (int m = 0; m < 3; ++m)
                S[(1 + m) * NFP] = Fg * (an[0] * pt.r[m][0] + an[1] * pt.r[m][1] + an[2] * pt.r[m][2]) * inv;
        }
    }
    __syncthreads();
    pointwise_faces<R, 3, P>(A, sm, es, s_e, nel, S_off);
    element_iproduct<R, 3, P>(A.y, A.xoff, Bt, Dt, sm, es, s_e, nel);
}

// ---------------------------------------------------------------------------
// Point-to-point flux through the gather-fold apply (k3g, unchanged): each
// face side gets its own point set (nf = its own n) with
//   factors  (canonical order on its own n x n grid, w the own GLL weights):
//            a = w J_s, C_m = w J_s n . J^-T e_m, and an = w J_s n (vector),
//            laid out [a | C | an] on the owner side and [a | an | C] on the
//            other side (the apply reads C at 1 or 4 npf by slot);
//   buffer   own (u, g = an . grad u) and the neighbour's (u, -an . I grad u_o),
//            both on this side's grid, at the slots the apply reads.
// The gather-fold trace kernel (k3t_elem with its point-to-point flag) writes
// both: its own pair, and its trace interpolated to the neighbour's points
// for the neighbour (Sec. 3.3, ScatrInterp), using the neighbour's an.

// Factors of every face side (one block per side, FP64); boundary faces have
// one side (slot 0 layout).  side[F * 4 + 2 s] = factor offset of side s,
// side[F * 4 + 2 s + 1] = its buffer offset.
__global__ __launch_bounds__(BLOCK) void k_p2p_factors(const FaceTopo *faces, const int *order, const int64_t *side,
                                                       const double *emap, const double *tab, double *fg) {
    const int F = blockIdx.x, s = blockIdx.y;
    const FaceTopo ft = faces[F];
    if (s == 1 && ft.eR < 0) return;
    const int e = s ? ft.eR : ft.eL, f = s ? ft.fR : ft.fL, o = s ? ft.orient : 0;
    const int n = order[e] + 2, npf = n * n;
    const int k = f / 2, sg = f & 1;
    double *out = fg + side[(int64_t)F * 4 + 2 * s];
    const double *X = tab + tab_off_X(n), *W = tab + tab_off_W(n);
    const int co = s == 1 ? 4 : 1, ao = s == 1 ? 1 : 4;
    for (int c = threadIdx.x; c < npf; c += BLOCK) {
        const int fp = own_of_canon(o, n, c), a = fp % n, b = fp / n;
        double xi[3];
        xi[k] = sg ? 1.0 : -1.0;
        xi[k == 0 ? 1 : 0] = X[a];
        xi[k == 2 ? 1 : 2] = X[b];
        double r[3][3];
        const double det = map_adjugate<double>(emap + (int64_t)24 * e, xi[0], xi[1], xi[2], r);
        const double w = W[a] * W[b];
        double an[3], js2 = 0.0;
        for (int cc = 0; cc < 3; ++cc) {
            const double v = sg ? r[k][cc] : -r[k][cc];
            js2 += v * v;
            an[cc] = w * v;
        }
        out[c] = w * sqrt(js2);
        for (int m = 0; m < 3; ++m) {
            out[(co + m) * npf + c] = (an[0] * r[m][0] + an[1] * r[m][1] + an[2] * r[m][2]) / det;
            out[(ao + m) * npf + c] = an[m];
        }
    }
}

}  // namespace sipdg
