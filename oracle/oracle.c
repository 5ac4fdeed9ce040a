/*
 * Oracle: a plain, slow, FP64 CPU evaluation of the symmetric interior
 * penalty (SIPG) Helmholtz operator on quad/hex spectral elements with
 * polynomial non-conforming faces evaluated on a shared trace space.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may call,
 * link or include this file; only the tests, the smoke check and the CPU
 * baseline of the benchmark use it.
 *
 * What it computes (Xia & Moxey, arXiv 2504.03573):
 *   - element expansion u = sum_j phi_j(xi) u_j, tensor-product bases
 *     (Sec. 2.1, expansion eq. and tensor basis eq.): the orthogonal
 *     (Legendre) basis of Table 1, or its modified C0 modal basis;
 *   - tensor Gauss-Lobatto-Legendre quadrature with the Jacobian determinant
 *     (Sec. 2.1, inner-product eq.), p+2 points per direction (Sec. 5.2), or
 *     for the volume terms Gauss-Legendre points (Sec. 3.2, the point sets
 *     that do not contain the element boundary);
 *   - the element-wise SIPG form (Sec. 2.2, eq. IP) with the average and
 *     jump operators of Sec. 2.2; summing it over elements gives the primal
 *     form (eq. primal);
 *   - interface integrals evaluated on a shared trace space whose GLL
 *     quadrature follows the higher-order side (Sec. 3.3, shared trace
 *     space), with the solution of each side evaluated pointwise at the
 *     trace points (Sec. 3.3, the physical-space mortar equivalence);
 *   - Dirichlet boundaries through exterior values u+ = -u- + 2 g,
 *     grad u+ = grad u- (Sec. 2.2, boundary values set by the boundary
 *     condition, mirror principle of the cited work).
 *
 * No sum-factorisation, no interpolation and no collocation: every basis
 * function and every geometric quantity is evaluated directly at every
 * quadrature point, gradients and normals are physical, and each element
 * accumulates its own rows (faces are visited from both sides).
 *
 * Reading of unstated details: tau_F = sigma * 2 (p_F+1)^2 / h with
 * p_F = max(p_L, p_R) (boundary: p_e); trace coordinates are those of the
 * owner (the lower element id); the trace weight a_q = w_q J_s comes from the
 * owner's map and each side's normal and gradient from its own map.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXN 16   /* max quadrature points per direction */

typedef struct {
    int dim;
    long ne;
    const double *coords;   /* [nv][dim] */
    const long *ev;         /* [ne][2^dim] lexicographic corners */
    const int *order;       /* [ne] */
    const double *lambda;   /* [ne] */
    const long *dof_off;    /* [ne+1] natural layout */
    double h, sigma;
    const long *nb;         /* [ne][2dim] neighbour element, -1 on boundary */
    const int *nb_face;     /* [ne][2dim] neighbour's local face */
    const int *owner;       /* [ne][2dim] 1 if this element owns the face */
    const int *amap;        /* [ne][2dim][4] owner face coords -> other side's */
    const double *gll_x;    /* [OR_MAXN+1][OR_MAXN] nodes, row n holds n nodes */
    const double *gll_w;    /* same shape, weights */
    int basis;              /* 0: Legendre (orthogonal), 1: modified C0 modal */
    const double *vol_x;    /* volume quadrature of the operator, same shape: */
    const double *vol_w;    /* the GLL tables, or Gauss-Legendre nodes/weights */
} omesh;

/* Legendre polynomials P_0..P_p and their derivatives at x (Bonnet's
 * recurrence; P'_{i+1} = (i+1) P_i + x P'_i). */
static void legendre(int p, double x, double *P, double *dP)
{
    P[0] = 1.0; dP[0] = 0.0;
    if (p >= 1) { P[1] = x; dP[1] = 1.0; }
    for (int i = 1; i < p; ++i) {
        P[i + 1] = ((2.0 * i + 1.0) * x * P[i] - i * P[i - 1]) / (i + 1.0);
        dP[i + 1] = (i + 1.0) * P[i] + x * dP[i];
    }
}

/* Jacobi polynomials P^(1,1)_0..P^(1,1)_n at x and their derivatives: the
 * three-term recurrence of the Jacobi family with alpha = beta = 1,
 * 2k(k+2)(2k) P_k = (2k+1)(2k+2)(2k) x P_{k-1} - 2k^2(2k+2) P_{k-2}. */
static void jacobi11(int n, double x, double *J, double *dJ)
{
    J[0] = 1.0; dJ[0] = 0.0;
    if (n >= 1) { J[1] = 2.0 * x; dJ[1] = 2.0; }
    for (int k = 2; k <= n; ++k) {
        double a = 2.0 * k * (k + 2.0) * (2.0 * k);
        double b = (2.0 * k + 1.0) * (2.0 * k + 2.0) * (2.0 * k);
        double c = 2.0 * k * k * (2.0 * k + 2.0);
        J[k] = (b * x * J[k - 1] - c * J[k - 2]) / a;
        dJ[k] = (b * (J[k - 1] + x * dJ[k - 1]) - c * dJ[k - 2]) / a;
    }
}

/* 1-D modes 0..p at x and their derivatives.  basis 0: Legendre P_i
 * (Table 1, orthogonal).  basis 1: the modified C0 modal basis of Table 1
 * (Karniadakis & Sherwin), vertex modes first: psi_0 = (1-x)/2,
 * psi_1 = (1+x)/2, psi_i = (1-x)/2 (1+x)/2 P^(1,1)_{i-2}(x) for i >= 2. */
static void modes_1d(int basis, int p, double x, double *P, double *dP)
{
    if (basis == 0) { legendre(p, x, P, dP); return; }
    double J[OR_MAXN], dJ[OR_MAXN];
    P[0] = 0.5 * (1.0 - x); dP[0] = -0.5;
    if (p >= 1) { P[1] = 0.5 * (1.0 + x); dP[1] = 0.5; }
    if (p >= 2) jacobi11(p - 2, x, J, dJ);
    for (int i = 2; i <= p; ++i) {
        double b = 0.25 * (1.0 - x) * (1.0 + x);
        P[i] = b * J[i - 2];
        dP[i] = -0.5 * x * J[i - 2] + b * dJ[i - 2];
    }
}

/* Multilinear element map: physical point x(xi) and J[a][b] = dx_a/dxi_b. */
static void element_map(const omesh *m, long e, const double *xi, double *x, double J[3][3])
{
    int d = m->dim, nvert = 1 << d;
    for (int a = 0; a < 3; ++a) { x[a] = 0.0; for (int b = 0; b < 3; ++b) J[a][b] = 0.0; }
    for (int v = 0; v < nvert; ++v) {
        const double *X = m->coords + m->ev[e * nvert + v] * d;
        double N[3], dN[3];
        for (int k = 0; k < d; ++k) {
            int bit = (v >> k) & 1;
            N[k] = bit ? 0.5 * (1.0 + xi[k]) : 0.5 * (1.0 - xi[k]);
            dN[k] = bit ? 0.5 : -0.5;
        }
        double prod = 1.0;
        for (int k = 0; k < d; ++k) prod *= N[k];
        for (int b = 0; b < d; ++b) {
            double g = dN[b];
            for (int k = 0; k < d; ++k) if (k != b) g *= N[k];
            for (int a = 0; a < d; ++a) J[a][b] += X[a] * g;
        }
        for (int a = 0; a < d; ++a) x[a] += X[a] * prod;
    }
}

/* det(J) and J^{-1} by the adjugate. */
static double invert(int d, double J[3][3], double Ji[3][3])
{
    double det;
    if (d == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        Ji[0][0] = J[1][1] / det;  Ji[0][1] = -J[0][1] / det;
        Ji[1][0] = -J[1][0] / det; Ji[1][1] = J[0][0] / det;
    } else {
        double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        Ji[0][0] = c00 / det;
        Ji[1][0] = c01 / det;
        Ji[2][0] = c02 / det;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    }
    return det;
}

/* All basis functions phi_i(xi) = prod_k psi_{i_k}(xi_k) of order p (1-D
 * modes of the given basis) and their physical gradients
 * grad phi_i = J^{-T} grad_xi phi_i.  Modes lexicographic, first direction
 * fastest. */
static int basis_at(int basis, int d, int p, const double *xi, double Ji[3][3], double *phi, double *gphi)
{
    double P[3][OR_MAXN], dP[3][OR_MAXN];
    for (int k = 0; k < d; ++k) modes_1d(basis, p, xi[k], P[k], dP[k]);
    int np = p + 1, nm = 0;
    int n3 = (d == 3) ? np : 1;
    for (int i3 = 0; i3 < n3; ++i3)
        for (int i2 = 0; i2 < np; ++i2)
            for (int i1 = 0; i1 < np; ++i1) {
                double g[3];
                if (d == 2) {
                    phi[nm] = P[0][i1] * P[1][i2];
                    g[0] = dP[0][i1] * P[1][i2];
                    g[1] = P[0][i1] * dP[1][i2];
                } else {
                    phi[nm] = P[0][i1] * P[1][i2] * P[2][i3];
                    g[0] = dP[0][i1] * P[1][i2] * P[2][i3];
                    g[1] = P[0][i1] * dP[1][i2] * P[2][i3];
                    g[2] = P[0][i1] * P[1][i2] * dP[2][i3];
                }
                for (int a = 0; a < d; ++a) {
                    double s = 0.0;
                    for (int b = 0; b < d; ++b) s += Ji[b][a] * g[b];
                    gphi[nm * 3 + a] = s;
                }
                ++nm;
            }
    return nm;
}

static int ipow(int b, int e) { int r = 1; while (e--) r *= b; return r; }

/* Reference point on local face f = 2k + (s>0) from face coordinates z
 * (the remaining reference directions in increasing order). */
static void embed(int d, int f, const double *z, double *xi)
{
    int k = f / 2, j = 0;
    for (int a = 0; a < d; ++a) xi[a] = (a == k) ? ((f & 1) ? 1.0 : -1.0) : z[j++];
}

/* Everything one side of a face needs at a trace point. */
typedef struct {
    double xi[3], J[3][3], Ji[3][3], det;
    double n[3];      /* outward unit normal of this side */
    double Js;        /* surface Jacobian of this side */
} side_geo;

static void side_geometry(const omesh *m, long e, int f, const double *z, side_geo *g)
{
    int d = m->dim, k = f / 2;
    double s = (f & 1) ? 1.0 : -1.0, x[3];
    embed(d, f, z, g->xi);
    element_map(m, e, g->xi, x, g->J);
    g->det = invert(d, g->J, g->Ji);
    /* area-weighted outward normal: s * det(J) * J^{-T} e_k = s * det * row k of J^{-1} */
    double nn = 0.0, v[3];
    for (int a = 0; a < d; ++a) { v[a] = s * g->det * g->Ji[k][a]; nn += v[a] * v[a]; }
    g->Js = sqrt(nn);
    for (int a = 0; a < d; ++a) g->n[a] = v[a] / g->Js;
}

static void apply_amap(int d, const int *A, const double *z, double *zo)
{
    if (d == 2) zo[0] = A[0] * z[0];
    else { zo[0] = A[0] * z[0] + A[1] * z[1]; zo[1] = A[2] * z[0] + A[3] * z[1]; }
}

/* Value and physical gradient of the expansion with coefficients c. */
static void field_at(int d, int nm, const double *phi, const double *gphi, const double *c,
                     double *u, double *gu)
{
    double uu = 0.0, g[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < nm; ++j) {
        uu += phi[j] * c[j];
        for (int a = 0; a < d; ++a) g[a] += gphi[j * 3 + a] * c[j];
    }
    *u = uu;
    for (int a = 0; a < d; ++a) gu[a] = g[a];
}

/* Trace point grid of a face with nF points per direction: point t has face
 * coordinates z and weight w (products of 1-D GLL nodes / weights). */
static void trace_point(const omesh *m, int d, int nF, int t, double *z, double *w)
{
    const double *gx = m->gll_x + nF * OR_MAXN, *gw = m->gll_w + nF * OR_MAXN;
    if (d == 2) { z[0] = gx[t]; *w = gw[t]; }
    else { int t1 = t % nF, t2 = t / nF; z[0] = gx[t1]; z[1] = gx[t2]; *w = gw[t1] * gw[t2]; }
}

enum { MODE_APPLY = 0, MODE_DIAG = 1, MODE_APPLY_P2P = 2 };

/* Lagrange basis polynomial i of the n GLL nodes gx at z. */
static double lagrange(int n, const double *gx, int i, double z)
{
    double v = 1.0;
    for (int k = 0; k < n; ++k)
        if (k != i) v *= (z - gx[k]) / (gx[i] - gx[k]);
    return v;
}

/* Point-to-point interpolation (Sec. 3.3, ScatrInterp): the other side's value
 * and physical gradient at its own face quadrature points (its GLL grid, in
 * its face coordinates), Lagrange-interpolated to the point zn given in those
 * coordinates.  F holds [nn^(d-1)][1 + d] samples. */
static void interp_other(int d, int nn, const double *gx, const double *F, const double *zn,
                         double *u, double *gu)
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int np = d == 2 ? nn : nn * nn;
    for (int t = 0; t < np; ++t) {
        int t1 = t % nn, t2 = t / nn;
        double l = lagrange(nn, gx, t1, zn[0]);
        if (d == 3) l *= lagrange(nn, gx, t2, zn[1]);
        for (int c = 0; c <= d; ++c) acc[c] += l * F[t * 4 + c];
    }
    *u = acc[0];
    for (int c = 0; c < d; ++c) gu[c] = acc[1 + c];
}

/* Rows of element e of A x (mode APPLY) or of diag(A) (mode DIAG). */
static void element_rows(const omesh *m, long e, const double *x, double *y, int mode,
                         double *phi, double *gphi, double *phn, double *gphn)
{
    int d = m->dim, p = m->order[e], n = p + 2;
    int nm = ipow(p + 1, d), nq = ipow(n, d);
    /* volume quadrature: n = p + 2 points per direction, GLL or Gauss (the
     * latter leaves out the element boundary; the faces keep the trace's
     * own GLL points either way) */
    const double *gx = m->vol_x + n * OR_MAXN, *gw = m->vol_w + n * OR_MAXN;
    const double *xe = x ? x + m->dof_off[e] : NULL;
    double *ye = y + m->dof_off[e];
    double lam = m->lambda[e];
    for (int i = 0; i < nm; ++i) ye[i] = 0.0;

    /* volume: (grad v, grad u) + lambda (v, u), eq. IP first line */
    for (int q = 0; q < nq; ++q) {
        int q1 = q % n, q2 = (q / n) % n, q3 = q / (n * n);
        double xi[3] = {gx[q1], gx[q2], d == 3 ? gx[q3] : 0.0};
        double w = gw[q1] * gw[q2] * (d == 3 ? gw[q3] : 1.0);
        double X[3], J[3][3], Ji[3][3];
        element_map(m, e, xi, X, J);
        double det = invert(d, J, Ji);
        basis_at(m->basis, d, p, xi, Ji, phi, gphi);
        if (mode != MODE_DIAG) {
            double u, gu[3];
            field_at(d, nm, phi, gphi, xe, &u, gu);
            for (int i = 0; i < nm; ++i) {
                double s = lam * phi[i] * u;
                for (int a = 0; a < d; ++a) s += gphi[i * 3 + a] * gu[a];
                ye[i] += w * det * s;
            }
        } else {
            for (int i = 0; i < nm; ++i) {
                double s = lam * phi[i] * phi[i];
                for (int a = 0; a < d; ++a) s += gphi[i * 3 + a] * gphi[i * 3 + a];
                ye[i] += w * det * s;
            }
        }
    }

    /* faces: -(grad v, 1/2 [[u]]) - (v, {grad u}.n) + (v, tau [[u]].n), eq. IP */
    for (int f = 0; f < 2 * d; ++f) {
        long nbr = m->nb[e * 2 * d + f];
        int own = m->owner[e * 2 * d + f];
        const int *A = m->amap + (e * 2 * d + f) * 4;
        int fn = m->nb_face[e * 2 * d + f];
        int pn = nbr >= 0 ? m->order[nbr] : p;
        int pF = p > pn ? p : pn, nF = pF + 2;
        double tau = m->sigma * 2.0 * (pF + 1.0) * (pF + 1.0) / m->h;
        int nmn = nbr >= 0 ? ipow(pn + 1, d) : 0;
        const double *xn = (nbr >= 0 && x) ? x + m->dof_off[nbr] : NULL;
        if (mode == MODE_APPLY_P2P && nbr >= 0) {
            /* point to point: this side's own face quadrature (n = p + 2 GLL
             * points per direction, its own weights and surface Jacobian);
             * the neighbour's u and grad u sampled at its own face points and
             * interpolated to ours; same penalty tau_F.  Face coordinates:
             * the owner's are canonical, the other side's are A times them. */
            int nn = pn + 2, npn = d == 2 ? nn : nn * nn, nown = d == 2 ? n : n * n;
            const double *gxn = m->gll_x + nn * OR_MAXN;
            double F[OR_MAXN * OR_MAXN * 4];
            for (int t = 0; t < npn; ++t) {
                double z[2], wz;
                trace_point(m, d, nn, t, z, &wz);
                side_geo gq;
                side_geometry(m, nbr, fn, z, &gq);
                basis_at(m->basis, d, pn, gq.xi, gq.Ji, phn, gphn);
                double un, gun[3] = {0.0, 0.0, 0.0};
                field_at(d, nmn, phn, gphn, xn, &un, gun);
                F[t * 4] = un;
                for (int c = 0; c < d; ++c) F[t * 4 + 1 + c] = gun[c];
            }
            for (int t = 0; t < nown; ++t) {
                double z[2], wz, c2[2], zn[2];
                trace_point(m, d, n, t, z, &wz);
                if (own) apply_amap(d, A, z, zn);
                else {   /* canonical = A^T (own coordinates); the neighbour owns */
                    if (d == 2) c2[0] = A[0] * z[0];
                    else { c2[0] = A[0] * z[0] + A[2] * z[1]; c2[1] = A[1] * z[0] + A[3] * z[1]; }
                    zn[0] = c2[0];
                    zn[1] = d == 3 ? c2[1] : 0.0;
                }
                side_geo ge;
                side_geometry(m, e, f, z, &ge);
                double a = wz * ge.Js;
                basis_at(m->basis, d, p, ge.xi, ge.Ji, phi, gphi);
                double ue, gue[3], un, gun[3] = {0.0, 0.0, 0.0};
                field_at(d, nm, phi, gphi, xe, &ue, gue);
                interp_other(d, nn, gxn, F, zn, &un, gun);
                double jump = ue - un, avg = 0.0;
                for (int c = 0; c < d; ++c) avg += 0.5 * (gue[c] + gun[c]) * ge.n[c];
                for (int i = 0; i < nm; ++i) {
                    double dn = 0.0;
                    for (int c = 0; c < d; ++c) dn += gphi[i * 3 + c] * ge.n[c];
                    ye[i] += a * (-0.5 * jump * dn - phi[i] * avg + tau * jump * phi[i]);
                }
            }
            continue;
        }
        int nt = (d == 2) ? nF : nF * nF;
        for (int t = 0; t < nt; ++t) {
            double z[2], wz, zo[2], zn[2];
            trace_point(m, d, nF, t, z, &wz);
            side_geo ge, gn;
            if (nbr < 0 || own) { zo[0] = z[0]; zo[1] = z[1]; }
            else apply_amap(d, A, z, zo);
            side_geometry(m, e, f, zo, &ge);
            double a;
            if (nbr >= 0) {
                if (own) apply_amap(d, A, z, zn); else { zn[0] = z[0]; zn[1] = z[1]; }
                side_geometry(m, nbr, fn, zn, &gn);
                a = wz * (own ? ge.Js : gn.Js);
            } else {
                a = wz * ge.Js;
            }
            basis_at(m->basis, d, p, ge.xi, ge.Ji, phi, gphi);
            if (mode != MODE_DIAG) {
                double ue, gue[3], un, gun[3];
                field_at(d, nm, phi, gphi, xe, &ue, gue);
                if (nbr >= 0) {
                    basis_at(m->basis, d, pn, gn.xi, gn.Ji, phn, gphn);
                    field_at(d, nmn, phn, gphn, xn, &un, gun);
                } else {               /* homogeneous mirror: u+ = -u-, grad u+ = grad u- */
                    un = -ue;
                    for (int c = 0; c < d; ++c) gun[c] = gue[c];
                }
                double jump = ue - un, avg = 0.0;
                for (int c = 0; c < d; ++c) avg += 0.5 * (gue[c] + gun[c]) * ge.n[c];
                for (int i = 0; i < nm; ++i) {
                    double dn = 0.0;
                    for (int c = 0; c < d; ++c) dn += gphi[i * 3 + c] * ge.n[c];
                    ye[i] += a * (-0.5 * jump * dn - phi[i] * avg + tau * jump * phi[i]);
                }
            } else {
                /* diagonal: u = phi_i on this element, zero elsewhere */
                for (int i = 0; i < nm; ++i) {
                    double dn = 0.0;
                    for (int c = 0; c < d; ++c) dn += gphi[i * 3 + c] * ge.n[c];
                    double ue = phi[i], un = (nbr >= 0) ? 0.0 : -ue;
                    double gnn = (nbr >= 0) ? 0.0 : dn;
                    double jump = ue - un, avg = 0.5 * (dn + gnn);
                    ye[i] += a * (-0.5 * jump * dn - phi[i] * avg + tau * jump * phi[i]);
                }
            }
        }
    }
}

static int max_modes(const omesh *m)
{
    int pm = 0;
    for (long e = 0; e < m->ne; ++e) if (m->order[e] > pm) pm = m->order[e];
    return ipow(pm + 1, m->dim);
}

/* Rows of A x for every element (or the listed ones) in the given mode. */
static int apply_mode(const omesh *m, const double *x, double *y, const long *elems, long nsel,
                      int mode)
{
    int mm = max_modes(m);
    long cnt = elems ? nsel : m->ne;
    int bad = 0;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * (size_t)mm * 8);
        if (!buf) {
#pragma omp atomic write
            bad = 1;
        } else {
#pragma omp for schedule(dynamic, 4)
            for (long i = 0; i < cnt; ++i) {
                long e = elems ? elems[i] : i;
                element_rows(m, e, x, y, mode, buf, buf + mm, buf + 4 * mm, buf + 5 * mm);
            }
            free(buf);
        }
    }
    return bad ? -1 : 0;
}

/* y = A x.  If elems != NULL only the rows of the listed elements are
 * written (the rest of y is untouched). */
int oracle_apply(const omesh *m, const double *x, double *y, const long *elems, long nsel)
{
    return apply_mode(m, x, y, elems, nsel, MODE_APPLY);
}

/* y = A_p2p x: the same form with every interior face integrated twice,
 * once per side on that side's own face quadrature with the other side's
 * trace interpolated point to point (Sec. 3.3, point-to-point
 * interpolation).  Boundary faces as in oracle_apply.  Not symmetric in
 * general (Sec. 3.3 conditions; Table 2). */
int oracle_apply_p2p(const omesh *m, const double *x, double *y, const long *elems, long nsel)
{
    return apply_mode(m, x, y, elems, nsel, MODE_APPLY_P2P);
}

/* diag(A): a(phi_i, phi_i) with every other coefficient zero (Jacobi). */
int oracle_diagonal(const omesh *m, double *dg)
{
    int mm = max_modes(m);
    int bad = 0;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * (size_t)mm * 8);
        if (!buf) {
#pragma omp atomic write
            bad = 1;
        } else {
#pragma omp for schedule(dynamic, 4)
            for (long e = 0; e < m->ne; ++e)
                element_rows(m, e, NULL, dg, MODE_DIAG, buf, buf + mm, buf + 4 * mm, buf + 5 * mm);
            free(buf);
        }
    }
    return bad ? -1 : 0;
}

/* Physical coordinates of the volume quadrature points (element by element,
 * points lexicographic) and of the boundary trace points (element by element,
 * boundary faces in local-face order, points lexicographic in face
 * coordinates).  Returns the two counts through nq_out / nb_out when the
 * arrays are NULL. */
int oracle_points(const omesh *m, double *xq, double *xb, long *nq_out, long *nb_out)
{
    int d = m->dim;
    long cq = 0, cb = 0;
    for (long e = 0; e < m->ne; ++e) {
        int n = m->order[e] + 2;
        const double *gx = m->gll_x + n * OR_MAXN;
        int nq = ipow(n, d);
        for (int q = 0; q < nq; ++q) {
            int q1 = q % n, q2 = (q / n) % n, q3 = q / (n * n);
            double xi[3] = {gx[q1], gx[q2], d == 3 ? gx[q3] : 0.0}, X[3], J[3][3];
            if (xq) { element_map(m, e, xi, X, J); for (int a = 0; a < d; ++a) xq[cq * d + a] = X[a]; }
            ++cq;
        }
        for (int f = 0; f < 2 * d; ++f) {
            if (m->nb[e * 2 * d + f] >= 0) continue;
            int nt = (d == 2) ? n : n * n;
            for (int t = 0; t < nt; ++t) {
                double z[2], w, xi[3], X[3], J[3][3];
                trace_point(m, d, n, t, z, &w);
                embed(d, f, z, xi);
                if (xb) { element_map(m, e, xi, X, J); for (int a = 0; a < d; ++a) xb[cb * d + a] = X[a]; }
                ++cb;
            }
        }
    }
    if (nq_out) *nq_out = cq;
    if (nb_out) *nb_out = cb;
    return 0;
}

/* Right-hand side: b_i = (phi_i, s)_Omega plus the Dirichlet data terms of
 * the mirrored exterior value u+ = -u- + 2 g moved to the right:
 * sum over boundary points of a [ -g grad phi_i . n + 2 tau g phi_i ]. */
int oracle_rhs(const omesh *m, const double *s_q, const double *g_b, double *b)
{
    int d = m->dim, mm = max_modes(m);
    long *qoff = (long *)malloc(sizeof(long) * (m->ne + 1));
    long *boff = (long *)malloc(sizeof(long) * (m->ne + 1));
    if (!qoff || !boff) { free(qoff); free(boff); return -1; }
    qoff[0] = boff[0] = 0;
    for (long e = 0; e < m->ne; ++e) {
        int n = m->order[e] + 2, nbf = 0;
        for (int f = 0; f < 2 * d; ++f) nbf += m->nb[e * 2 * d + f] < 0;
        qoff[e + 1] = qoff[e] + ipow(n, d);
        boff[e + 1] = boff[e] + (long)nbf * ipow(n, d - 1);
    }
    int bad = 0;
#pragma omp parallel
    {
        double *phi = (double *)malloc(sizeof(double) * (size_t)mm * 4);
        if (!phi) {
#pragma omp atomic write
            bad = 1;
        } else {
            double *gphi = phi + mm;
#pragma omp for schedule(dynamic, 4)
            for (long e = 0; e < m->ne; ++e) {
                int p = m->order[e], n = p + 2, nm = ipow(p + 1, d), nq = ipow(n, d);
                const double *gx = m->gll_x + n * OR_MAXN, *gw = m->gll_w + n * OR_MAXN;
                double *be = b + m->dof_off[e];
                for (int i = 0; i < nm; ++i) be[i] = 0.0;
                for (int q = 0; q < nq; ++q) {
                    int q1 = q % n, q2 = (q / n) % n, q3 = q / (n * n);
                    double xi[3] = {gx[q1], gx[q2], d == 3 ? gx[q3] : 0.0};
                    double w = gw[q1] * gw[q2] * (d == 3 ? gw[q3] : 1.0);
                    double X[3], J[3][3], Ji[3][3];
                    element_map(m, e, xi, X, J);
                    double det = invert(d, J, Ji);
                    basis_at(m->basis, d, p, xi, Ji, phi, gphi);
                    double sv = s_q[qoff[e] + q];
                    for (int i = 0; i < nm; ++i) be[i] += w * det * phi[i] * sv;
                }
                double tau = m->sigma * 2.0 * (p + 1.0) * (p + 1.0) / m->h;
                long cb = boff[e];
                for (int f = 0; f < 2 * d; ++f) {
                    if (m->nb[e * 2 * d + f] >= 0) continue;
                    int nt = (d == 2) ? n : n * n;
                    for (int t = 0; t < nt; ++t, ++cb) {
                        double z[2], wz;
                        side_geo ge;
                        trace_point(m, d, n, t, z, &wz);
                        side_geometry(m, e, f, z, &ge);
                        basis_at(m->basis, d, p, ge.xi, ge.Ji, phi, gphi);
                        double a = wz * ge.Js, g = g_b[cb];
                        for (int i = 0; i < nm; ++i) {
                            double dn = 0.0;
                            for (int c = 0; c < d; ++c) dn += gphi[i * 3 + c] * ge.n[c];
                            be[i] += a * (-g * dn + 2.0 * tau * g * phi[i]);
                        }
                    }
                }
            }
            free(phi);
        }
    }
    free(qoff);
    free(boff);
    return bad ? -1 : 0;
}

/* Gradients of the bilinear form value aT A b with respect to lambda_e and
 * the penalty scale sigma:
 *   d/dlambda_e = (a, b)_{Omega_e}, on the operator's volume quadrature
 *                 (GLL or Gauss points: the one the lambda term of apply uses)
 *   d/dsigma    = sum_F (tau_F/sigma) ([[a]], [[b]])_F  (boundary: 2 a b). */
int oracle_param_grad(const omesh *m, const double *av, const double *bv,
                      double *dlam, double *dsig_per_elem)
{
    int d = m->dim, mm = max_modes(m);
    int bad = 0;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * (size_t)mm * 8);
        if (!buf) {
#pragma omp atomic write
            bad = 1;
        } else {
            double *phi = buf, *gphi = buf + mm, *phn = buf + 4 * mm, *gphn = buf + 5 * mm;
#pragma omp for schedule(dynamic, 4)
            for (long e = 0; e < m->ne; ++e) {
                int p = m->order[e], n = p + 2, nm = ipow(p + 1, d), nq = ipow(n, d);
                /* the lambda term lives on the operator's own volume points */
                const double *gx = m->vol_x + n * OR_MAXN, *gw = m->vol_w + n * OR_MAXN;
                const double *ae = av + m->dof_off[e], *be = bv + m->dof_off[e];
                double sl = 0.0;
                for (int q = 0; q < nq; ++q) {
                    int q1 = q % n, q2 = (q / n) % n, q3 = q / (n * n);
                    double xi[3] = {gx[q1], gx[q2], d == 3 ? gx[q3] : 0.0};
                    double w = gw[q1] * gw[q2] * (d == 3 ? gw[q3] : 1.0);
                    double X[3], J[3][3], Ji[3][3], ua, ub, g[3];
                    element_map(m, e, xi, X, J);
                    double det = invert(d, J, Ji);
                    basis_at(m->basis, d, p, xi, Ji, phi, gphi);
                    field_at(d, nm, phi, gphi, ae, &ua, g);
                    field_at(d, nm, phi, gphi, be, &ub, g);
                    sl += w * det * ua * ub;
                }
                dlam[e] = sl;
                double ss = 0.0;
                for (int f = 0; f < 2 * d; ++f) {
                    long nbr = m->nb[e * 2 * d + f];
                    int own = m->owner[e * 2 * d + f];
                    if (nbr >= 0 && !own) continue;      /* each interior face once */
                    const int *A = m->amap + (e * 2 * d + f) * 4;
                    int fn = m->nb_face[e * 2 * d + f];
                    int pn = nbr >= 0 ? m->order[nbr] : p;
                    int pF = p > pn ? p : pn, nF = pF + 2;
                    double tau0 = 2.0 * (pF + 1.0) * (pF + 1.0) / m->h;
                    int nt = (d == 2) ? nF : nF * nF, nmn = nbr >= 0 ? ipow(pn + 1, d) : 0;
                    for (int t = 0; t < nt; ++t) {
                        double z[2], wz, zn[2], g[3];
                        side_geo ge, gn;
                        trace_point(m, d, nF, t, z, &wz);
                        side_geometry(m, e, f, z, &ge);
                        double a = wz * ge.Js;
                        basis_at(m->basis, d, p, ge.xi, ge.Ji, phi, gphi);
                        double ua, ub, una = 0.0, unb = 0.0;
                        field_at(d, nm, phi, gphi, ae, &ua, g);
                        field_at(d, nm, phi, gphi, be, &ub, g);
                        if (nbr >= 0) {
                            apply_amap(d, A, z, zn);
                            side_geometry(m, nbr, fn, zn, &gn);
                            basis_at(m->basis, d, pn, gn.xi, gn.Ji, phn, gphn);
                            field_at(d, nmn, phn, gphn, av + m->dof_off[nbr], &una, g);
                            field_at(d, nmn, phn, gphn, bv + m->dof_off[nbr], &unb, g);
                            ss += tau0 * a * (ua - una) * (ub - unb);
                        } else {
                            ss += 2.0 * tau0 * a * ua * ub;
                        }
                    }
                }
                dsig_per_elem[e] = ss;
            }
            free(buf);
        }
    }
    return bad ? -1 : 0;
}

/* Values of the expansion x, physical points and w|J| at a tensor set of
 * reference points per element: for order p the caller provides
 * nr = p + extra nodes in ref_x[p] / weights ref_w[p] (row stride OR_MAXN+4).
 * Output is element by element, points lexicographic. */
int oracle_sample(const omesh *m, const double *x, int extra, const double *ref_x,
                  const double *ref_w, double *xyz, double *wdet, double *uval)
{
    int d = m->dim, mm = max_modes(m);
    long *off = (long *)malloc(sizeof(long) * (m->ne + 1));
    if (!off) return -1;
    off[0] = 0;
    for (long e = 0; e < m->ne; ++e) off[e + 1] = off[e] + ipow(m->order[e] + extra, d);
    int bad = 0;
#pragma omp parallel
    {
        double *phi = (double *)malloc(sizeof(double) * (size_t)mm * 4);
        if (!phi) {
#pragma omp atomic write
            bad = 1;
        } else {
            double *gphi = phi + mm;
#pragma omp for schedule(dynamic, 4)
            for (long e = 0; e < m->ne; ++e) {
                int p = m->order[e], nr = p + extra, nm = ipow(p + 1, d), nq = ipow(nr, d);
                const double *rx = ref_x + p * (OR_MAXN + 4), *rw = ref_w + p * (OR_MAXN + 4);
                for (int q = 0; q < nq; ++q) {
                    int q1 = q % nr, q2 = (q / nr) % nr, q3 = q / (nr * nr);
                    double xi[3] = {rx[q1], rx[q2], d == 3 ? rx[q3] : 0.0};
                    double w = rw[q1] * rw[q2] * (d == 3 ? rw[q3] : 1.0);
                    double X[3], J[3][3], Ji[3][3], u, g[3];
                    element_map(m, e, xi, X, J);
                    double det = invert(d, J, Ji);
                    basis_at(m->basis, d, p, xi, Ji, phi, gphi);
                    field_at(d, nm, phi, gphi, x + m->dof_off[e], &u, g);
                    long o = off[e] + q;
                    for (int a = 0; a < d; ++a) xyz[o * d + a] = X[a];
                    wdet[o] = w * det;
                    uval[o] = u;
                }
            }
            free(phi);
        }
    }
    free(off);
    return bad ? -1 : 0;
}

/* Per-point geometry the invariants check: det J at volume points
 * (element by element) for the orientation / validity check. */
int oracle_min_detj(const omesh *m, double *mindet)
{
    int d = m->dim;
    for (long e = 0; e < m->ne; ++e) {
        int n = m->order[e] + 2, nq = ipow(n, d);
        const double *gx = m->gll_x + n * OR_MAXN;
        double mn = 1e300;
        for (int q = 0; q < nq; ++q) {
            int q1 = q % n, q2 = (q / n) % n, q3 = q / (n * n);
            double xi[3] = {gx[q1], gx[q2], d == 3 ? gx[q3] : 0.0}, X[3], J[3][3], Ji[3][3];
            element_map(m, e, xi, X, J);
            double det = invert(d, J, Ji);
            if (det < mn) mn = det;
        }
        mindet[e] = mn;
    }
    return 0;
}

/* Face geometry used by the invariant tests: for every element and every
 * local face, sum over the face's own GLL points (n_e per direction) of
 * w * det(J) * J^{-T} e_k * s (the area-weighted outward normal), and the
 * face area.  out_n is [ne][2d][d], out_area [ne][2d]. */
int oracle_face_moments(const omesh *m, double *out_n, double *out_area)
{
    int d = m->dim;
    for (long e = 0; e < m->ne; ++e) {
        int n = m->order[e] + 2, nt = (d == 2) ? n : n * n;
        for (int f = 0; f < 2 * d; ++f) {
            double sn[3] = {0, 0, 0}, ar = 0.0;
            for (int t = 0; t < nt; ++t) {
                double z[2], w;
                side_geo g;
                trace_point(m, d, n, t, z, &w);
                side_geometry(m, e, f, z, &g);
                for (int a = 0; a < d; ++a) sn[a] += w * g.Js * g.n[a];
                ar += w * g.Js;
            }
            for (int a = 0; a < d; ++a) out_n[(e * 2 * d + f) * d + a] = sn[a];
            out_area[e * 2 * d + f] = ar;
        }
    }
    return 0;
}

/* Threads the OpenMP loops of this library use. */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of threads of the OpenMP loops (n >= 1); returns the new count. */
int oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
