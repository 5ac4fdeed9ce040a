// Host preprocessing of one or several meshes: validation, face matching,
// owner / orientation of every interior face, trace sizes, offsets.
//
// Faces are matched by their sorted corner vertex ids; the element with the
// lower id owns the face and the trace points are laid out in the owner's
// face coordinates (Xia & Moxey, Sec. 3.3: one shared trace per face;
// Sec. 5.1: orientation of the adjacent side, at most 8 in 3-D).
#include <algorithm>
#include <array>
#include <cmath>
#include <string>

#include "sipdg.h"
#include "topology.hpp"

namespace sipdg {

namespace {

struct FaceKey {
    std::array<int64_t, 4> ids;  // sorted corner ids (unused slots = -1)
    int64_t e;
    int f;
};

// Corner ids of local face f = 2k + s in face-coordinate order
// (c = c1 + 2 c2, face coordinates = remaining directions, increasing).
void face_corners(int dim, const int64_t *ev, int f, int64_t *out) {
    const int k = f / 2, s = f & 1;
    int others[2], j = 0;
    for (int a = 0; a < dim; ++a)
        if (a != k) others[j++] = a;
    for (int c = 0; c < (1 << (dim - 1)); ++c) {
        int v = s << k;
        for (int jj = 0; jj < dim - 1; ++jj) v |= ((c >> jj) & 1) << others[jj];
        out[c] = ev[v];
    }
}

// Canonical (owner) corner (c1, c2) -> the other side's corner under code o.
void corner_map(int dim, int o, int c1, int c2, int &d1, int &d2) {
    if (dim == 2) {
        d1 = (o & 1) ? 1 - c1 : c1;
        d2 = 0;
        return;
    }
    int a1 = (o & 4) ? c2 : c1, a2 = (o & 4) ? c1 : c2;
    d1 = (o & 1) ? 1 - a1 : a1;
    d2 = (o & 2) ? 1 - a2 : a2;
}

double corner_det(int dim, const double *X, int corner) {
    // J at reference corner: columns dx/dxi_b
    double J[3][3] = {{0}};
    double xi[3];
    for (int k = 0; k < dim; ++k) xi[k] = ((corner >> k) & 1) ? 1.0 : -1.0;
    for (int v = 0; v < (1 << dim); ++v) {
        double Nk[3], dN[3];
        for (int k = 0; k < dim; ++k) {
            int bit = (v >> k) & 1;
            Nk[k] = bit ? 0.5 * (1 + xi[k]) : 0.5 * (1 - xi[k]);
            dN[k] = bit ? 0.5 : -0.5;
        }
        for (int b = 0; b < dim; ++b) {
            double g = dN[b];
            for (int k = 0; k < dim; ++k)
                if (k != b) g *= Nk[k];
            for (int a = 0; a < dim; ++a) J[a][b] += X[v * dim + a] * g;
        }
    }
    if (dim == 2) return J[0][0] * J[1][1] - J[0][1] * J[1][0];
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

}  // namespace

int build_topology(int nprob, const sipdg_mesh_desc *descs, Topology &T, std::string &err) {
    if (nprob <= 0 || !descs) {
        err = "no problems";
        return SIPDG_EINVAL;
    }
    const int dim = descs[0].dim;
    if (dim != 2 && dim != 3) {
        err = "dim must be 2 or 3";
        return SIPDG_EINVAL;
    }
    const int nvert = 1 << dim, nlf = 2 * dim;
    T = Topology();
    T.dim = dim;
    T.nprob = nprob;
    T.prob_elem_off.assign(nprob + 1, 0);
    T.prob_dof_off.assign(nprob + 1, 0);
    int64_t vbase = 0;
    std::vector<int64_t> vert_base(nprob);
    for (int p = 0; p < nprob; ++p) {
        const sipdg_mesh_desc &d = descs[p];
        if (d.dim != dim) {
            err = "all problems must have the same dim";
            return SIPDG_EINVAL;
        }
        if (d.n_elems < 0 || d.n_vertices < 0 || (d.n_elems > 0 && (!d.coords || !d.elem_vertices || !d.order || !d.lambda))) {
            err = "null array in mesh description";
            return SIPDG_EINVAL;
        }
        if (!(d.h > 0.0) || !(d.penalty_scale > 0.0) || !std::isfinite(d.h) || !std::isfinite(d.penalty_scale)) {
            err = "h and penalty_scale must be positive";
            return SIPDG_EINVAL;
        }
        if (d.quad_extra != 0 && d.quad_extra != 2) {
            err = "quad_extra must be 2 (p + 2 GLL points per direction) or 0 for that default";
            return SIPDG_EINVAL;
        }
        if (d.basis != SIPDG_BASIS_LEGENDRE && d.basis != SIPDG_BASIS_MODAL) {
            err = "unknown basis";
            return SIPDG_EINVAL;
        }
        if (d.basis != descs[0].basis) {
            err = "every problem of a batch must use the same basis";
            return SIPDG_EINVAL;
        }
        T.prob_elem_off[p + 1] = T.prob_elem_off[p] + d.n_elems;
        vert_base[p] = vbase;
        vbase += d.n_vertices;
    }
    const int64_t ne = T.prob_elem_off[nprob];
    T.ne = ne;
    T.order.resize(ne);
    T.lambda.resize(ne);
    T.elem_prob.resize(ne);
    T.corners.resize((size_t)ne * nvert * dim);
    T.h.resize(nprob);
    T.sigma.resize(nprob);
    std::vector<int64_t> gev((size_t)ne * nvert);
    for (int p = 0; p < nprob; ++p) {
        const sipdg_mesh_desc &d = descs[p];
        T.h[p] = d.h;
        T.sigma[p] = d.penalty_scale;
        for (int64_t i = 0; i < d.n_elems; ++i) {
            const int64_t e = T.prob_elem_off[p] + i;
            const int o = d.order[i];
            if (o < 1 || o > PMAX) {
                err = "element " + std::to_string(i) + ": order " + std::to_string(o) + " outside [1, 8]";
                return SIPDG_EINVAL;
            }
            if (!std::isfinite(d.lambda[i])) {
                err = "non-finite lambda";
                return SIPDG_EINVAL;
            }
            T.order[e] = o;
            T.lambda[e] = d.lambda[i];
            T.elem_prob[e] = p;
            for (int v = 0; v < nvert; ++v) {
                const int64_t id = d.elem_vertices[i * nvert + v];
                if (id < 0 || id >= d.n_vertices) {
                    err = "element " + std::to_string(i) + ": vertex id out of range";
                    return SIPDG_EINVAL;
                }
                gev[(size_t)e * nvert + v] = vert_base[p] + id;
                for (int a = 0; a < dim; ++a) T.corners[((size_t)e * nvert + v) * dim + a] = d.coords[id * dim + a];
            }
            for (int c = 0; c < nvert; ++c) {
                if (!(corner_det(dim, &T.corners[(size_t)e * nvert * dim], c) > 0.0)) {
                    err = "element " + std::to_string(i) + " of problem " + std::to_string(p) +
                          ": non-positive Jacobian at a corner";
                    return SIPDG_EMESH;
                }
            }
        }
    }

    // face matching
    std::vector<FaceKey> keys((size_t)ne * nlf);
    for (int64_t e = 0; e < ne; ++e) {
        for (int f = 0; f < nlf; ++f) {
            FaceKey &K = keys[(size_t)e * nlf + f];
            K.ids = {-1, -1, -1, -1};
            int64_t c[4];
            face_corners(dim, &gev[(size_t)e * nvert], f, c);
            const int nc = 1 << (dim - 1);
            for (int j = 0; j < nc; ++j) K.ids[j] = c[j];
            std::sort(K.ids.begin(), K.ids.begin() + nc);
            for (int j = 1; j < nc; ++j)
                if (K.ids[j] == K.ids[j - 1]) {
                    err = "degenerate face (repeated vertex)";
                    return SIPDG_EMESH;
                }
            K.e = e;
            K.f = f;
        }
    }
    std::sort(keys.begin(), keys.end(), [](const FaceKey &a, const FaceKey &b) {
        if (a.ids != b.ids) return a.ids < b.ids;
        if (a.e != b.e) return a.e < b.e;
        return a.f < b.f;
    });
    struct RawFace {
        int64_t eL, eR;
        int fL, fR, orient;
    };
    std::vector<RawFace> raw;
    raw.reserve(keys.size() / 2 + 16);
    for (size_t i = 0; i < keys.size();) {
        size_t j = i + 1;
        while (j < keys.size() && keys[j].ids == keys[i].ids) ++j;
        if (j - i == 1) {
            raw.push_back({keys[i].e, -1, keys[i].f, -1, 0});
        } else if (j - i == 2) {
            const FaceKey &L = keys[i], &Rk = keys[i + 1];
            if (L.e == Rk.e) {
                err = "element meets itself across a face";
                return SIPDG_EMESH;
            }
            int64_t cL[4], cR[4];
            face_corners(dim, &gev[(size_t)L.e * nvert], L.f, cL);
            face_corners(dim, &gev[(size_t)Rk.e * nvert], Rk.f, cR);
            int found = -1;
            for (int o = 0; o < (dim == 3 ? 8 : 2) && found < 0; ++o) {
                bool ok = true;
                for (int c = 0; c < (1 << (dim - 1)) && ok; ++c) {
                    int d1, d2;
                    corner_map(dim, o, c & 1, c >> 1, d1, d2);
                    ok = cL[c] == cR[d1 + 2 * d2];
                }
                if (ok) found = o;
            }
            if (found < 0) {
                err = "faces do not match by a symmetry of the square";
                return SIPDG_EMESH;
            }
            raw.push_back({L.e, Rk.e, L.f, Rk.f, found});
        } else {
            err = "face shared by more than two elements";
            return SIPDG_EMESH;
        }
        i = j;
    }
    std::sort(raw.begin(), raw.end(), [](const RawFace &a, const RawFace &b) {
        if (a.eL != b.eL) return a.eL < b.eL;
        return a.fL < b.fL;
    });
    const int64_t nf = (int64_t)raw.size();
    T.nfaces = nf;
    T.faces.resize(nf);
    T.eface.assign((size_t)ne * nlf, FaceRef{-1, 0});
    T.tau0.resize(nf);
    T.face_prob.resize(nf);
    T.foff.resize(nf + 1);
    T.toff.assign(nf, -1);
    T.prob_face_off.assign(nprob + 1, 0);
    int64_t fo = 0, to = 0;
    for (int64_t F = 0; F < nf; ++F) {
        const RawFace &r = raw[F];
        const int pL = T.order[r.eL];
        const int pR = r.eR >= 0 ? T.order[r.eR] : pL;
        const int pF = std::max(pL, pR), nF = pF + 2;
        const int npf = dim == 3 ? nF * nF : nF;
        const int prob = T.elem_prob[r.eL];
        T.faces[F] = {(int)r.eL, r.fL, (int)r.eR, r.fR, r.orient, nF};
        T.face_prob[F] = prob;
        T.prob_face_off[prob + 1] = F + 1;
        T.tau0[F] = 2.0 * (pF + 1.0) * (pF + 1.0) / T.h[prob];
        T.foff[F] = fo;
        if (r.eR >= 0) {
            fo += (int64_t)npf * (1 + 2 * dim);
            T.toff[F] = to;
            to += 4 * (int64_t)npf;
            T.eface[(size_t)r.eL * nlf + r.fL] = {(int)F, 0 | (0 << 2) | (nF << 5)};
            T.eface[(size_t)r.eR * nlf + r.fR] = {(int)F, 1 | (r.orient << 2) | (nF << 5)};
            T.n_interior++;
            T.n_int_trace_points += npf;
            if (pL != pR) T.n_nonconf++;
            T.orient_count[r.orient]++;
        } else {
            fo += (int64_t)npf * (1 + dim);
            T.toff[F] = to;   // one side: the element's own (u, g)
            to += 2 * (int64_t)npf;
            T.eface[(size_t)r.eL * nlf + r.fL] = {(int)F, 2 | (nF << 5)};
            T.n_boundary++;
            T.n_bnd_trace_points += npf;
        }
        T.n_trace_points += npf;
    }
    for (int p = 0; p < nprob; ++p)
        if (T.prob_face_off[p + 1] < T.prob_face_off[p]) T.prob_face_off[p + 1] = T.prob_face_off[p];
    T.foff[nf] = fo;
    T.fgeo_len = fo;
    T.tbuf_len = to;

    // element offsets
    T.xoff.resize(ne + 1);
    T.voff.resize(ne + 1);
    T.qoff.resize(ne + 1);
    T.boff.resize(ne + 1);
    T.xoff[0] = T.voff[0] = T.qoff[0] = T.boff[0] = 0;
    const int ng = dim * (dim + 1) / 2 + 1;
    for (int64_t e = 0; e < ne; ++e) {
        const int n = T.order[e] + 2, np = T.order[e] + 1;
        const int64_t npts = dim == 3 ? (int64_t)n * n * n : (int64_t)n * n;
        const int64_t nm = dim == 3 ? (int64_t)np * np * np : (int64_t)np * np;
        int nbf = 0;
        for (int f = 0; f < nlf; ++f) nbf += face_slot(T.eface[(size_t)e * nlf + f].info) == 2;
        T.xoff[e + 1] = T.xoff[e] + nm;
        T.voff[e + 1] = T.voff[e] + npts * ng;
        T.qoff[e + 1] = T.qoff[e] + npts;
        T.boff[e + 1] = T.boff[e] + (int64_t)nbf * (dim == 3 ? n * n : n);
    }
    for (int p = 0; p < nprob; ++p) T.prob_dof_off[p + 1] = T.xoff[T.prob_elem_off[p + 1]];
    T.ndof = T.xoff[ne];
    T.vgeo_len = T.voff[ne];
    return SIPDG_OK;
}

}  // namespace sipdg
