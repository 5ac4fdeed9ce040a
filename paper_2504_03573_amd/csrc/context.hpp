// Library-internal state of one handle and the kernel argument blocks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "tables.hpp"

namespace sipdg {

// Packed description of one local face of an element, as seen by kernels:
//   x = global face id F
//   y = slot | orient << 2 | NF << 5
// slot 0: this element owns F (lower id), 1: the other side, 2: boundary.
// orient: map between the owner's face coordinates (canonical trace order)
// and this side's (bit0 flip first, bit1 flip second, bit2 swap).
// NF: GLL points per direction on the shared trace.
struct FaceRef {
    int F;
    int info;
};

__host__ __device__ inline int face_slot(int info) { return info & 3; }
__host__ __device__ inline int face_orient(int info) { return (info >> 2) & 7; }
__host__ __device__ inline int face_nf(int info) { return (info >> 5) & 31; }

// Own face coordinates (r1, r2) on a trace with nf points per direction ->
// canonical (owner) index.
__host__ __device__ inline int canon_index(int orient, int nf, int r1, int r2) {
    int a1 = (orient & 1) ? nf - 1 - r1 : r1;
    int a2 = (orient & 2) ? nf - 1 - r2 : r2;
    return (orient & 4) ? (a2 + nf * a1) : (a1 + nf * a2);
}

template <class R>
struct OpArgs {
    const int *elems;       // element ids of this order group
    int count;
    int tsz;                // per-element work-area size (R units)
    const int64_t *xoff;    // [ne+1] coefficient offsets
    const int64_t *voff;    // [ne] volume-factor offsets
    const FaceRef *eface;   // [ne][2 dim]
    const int64_t *foff;    // [nf] face-factor offsets
    const int64_t *toff;    // [nf] trace-buffer offsets (interior: 2 sides, boundary: 1)
    const R *vgeo;          // volume factors
    const R *fgeo;          // face factors
    const R *lam;           // [ne]
    const R *tau;           // [nf] penalty tau_F
    const R *tab;           // 1-D tables
    const R *x;
    R *y;
    R *tbuf;                // trace buffer
    const int *skip;        // optional: return at once when *skip != 0
    // point-to-point flux (3-D) only
    const int *order = nullptr;             // [ne]
    const struct FaceTopo *faces = nullptr; // [nf]
    const R *emap = nullptr;                // [ne][24] trilinear map coefficients
};

// Per-element descriptors of an order group (3-D), indexed by the position in
// the group, so that a kernel reaches its element's offsets and the records
// of its six faces in one round of loads.
struct ElemDesc {
    int64_t xoff, voff;     // coefficient and volume-factor offsets
    int e, pad;             // element id; pad: order (persistent lists) | AFFINE
};
constexpr int ELEM_AFFINE = 0x100;   // the element's map is affine: constant G~ and |J|
constexpr int ELEM_ORDER_MASK = 0xff;
struct FaceDesc {
    int64_t fo, to;         // face-factor and trace-buffer offsets
    int F, info;            // face id and FaceRef::info
};

struct Group {
    int P;
    int count;
    int nfmax;              // largest trace that touches the group
    int *d_elems;
    ElemDesc *d_desc = nullptr;      // [count]      (3-D); split: the naff affine elements first
    int naff = 0;                    // affine elements of the group (3-D)
    bool split = false;              // apply: affine part and deformed part launched apart
    FaceDesc *d_fdesc = nullptr;     // [count][6]   (3-D)
    FaceDesc *d_fdesc_p2p = nullptr; // [count][6]   point-to-point flux: own point sets
    double alg_bytes[2] = {0, 0};    // algorithmic bytes of the group's elements (FP64, FP32)
};

// Optional record of HIP events around each kernel launch of an application.
struct LaunchRec {
    hipEvent_t *ev = nullptr;   // [2 * cap]
    int cap = 0, n = 0;
    int stage[64], group[64];
};

struct CgWork;  // defined in the solver
struct FaceTopo;
struct NbDesc2;

}  // namespace sipdg

struct sipdg_ctx {
    int dim = 0;
    int nprob = 0;
    int device = 0;
    int64_t ne = 0, ndof = 0, nfaces = 0;
    int64_t nvq = 0, nbq = 0;          // volume / boundary points
    int64_t vgeo_len = 0, fgeo_len = 0, tbuf_len = 0;

    // host copies (topology)
    std::vector<int> order;
    std::vector<int64_t> xoff, prob_dof_off, prob_elem_off, prob_face_off;
    std::vector<double> tau0, sigma;
    std::vector<int> face_prob;

    // device
    int64_t *d_xoff = nullptr, *d_voff = nullptr, *d_foff = nullptr, *d_toff = nullptr;
    int64_t *d_qoff = nullptr, *d_boff = nullptr;
    int64_t *d_prob_elem_off = nullptr, *d_prob_face_off = nullptr, *d_prob_dof_off = nullptr;
    sipdg::FaceRef *d_eface = nullptr;
    sipdg::FaceTopo *d_faces = nullptr;
    int *d_order = nullptr, *d_is_interior = nullptr, *d_face_nf = nullptr, *d_flag = nullptr;
    double *d_corners = nullptr;
    double *d_tab64 = nullptr;
    float *d_tab32 = nullptr;
    // the table set of Gauss volume points (X, W, B, D at the Gauss points)
    double *d_tabgl64 = nullptr;
    float *d_tabgl32 = nullptr;
    int points = 0;         // SIPDG_POINTS_GLL or SIPDG_POINTS_GAUSS (volume quadrature)
    double *d_vgeo64 = nullptr, *d_fgeo64 = nullptr, *d_lam64 = nullptr, *d_tau64 = nullptr;
    float *d_vgeo32 = nullptr, *d_fgeo32 = nullptr, *d_lam32 = nullptr, *d_tau32 = nullptr;
    // per element [8]: G~ (00 01 02 11 12 22) and |J| of an affine (parallelepiped)
    // element, zero otherwise; ElemDesc::pad bit AFFINE marks the affine elements
    double *d_egeo64 = nullptr;
    float *d_egeo32 = nullptr;
    // per element [24]: trilinear map coefficients c1..c7 (x, y, z) and a pad
    // (3-D), for the apply's on-the-fly geometry of deformed elements
    double *d_emap64 = nullptr;
    float *d_emap32 = nullptr;
    bool geo_map = false;   // deformed elements: geometry from the map, not the stored factors
    int flux = 0;           // SIPDG_FLUX_SHARED or SIPDG_FLUX_P2P
    int basis = 0;          // SIPDG_BASIS_LEGENDRE or SIPDG_BASIS_MODAL
    bool fast_ok0 = false, gfold_ok0 = false;   // structures the mesh allows (Legendre basis)
    void *d_tbuf_p2p = nullptr;   // point-to-point trace buffer (FP64 units: 2 x tbuf_len)
    int64_t *d_p2p_side = nullptr;           // [nf][2][factor offset, buffer offset] (gather-fold p2p)
    sipdg::FaceDesc *d_pfdesc_p2p = nullptr; // point-to-point face descriptors of the persistent list
    double *d_fgeo_p2p64 = nullptr;          // per face side: a, C, an on its own grid
    float *d_fgeo_p2p32 = nullptr;
    double *d_tau0 = nullptr;
    double *d_tbuf = nullptr;              // FP64-sized; the FP32 path reuses it
    double *d_tbuf2 = nullptr;             // second trace buffer (gradients)
    double *d_face_tmp = nullptr, *d_elem_tmp = nullptr;
    double *d_diag64 = nullptr, *d_dinv64 = nullptr;
    float *d_dinv32 = nullptr;
    std::vector<sipdg::Group> groups;
    sipdg::CgWork *cg = nullptr;
    int variant = 0;        // SIPDG_VARIANT_*
    // side streams (default priority) and events: the order groups of one
    // stage run concurrently, joined back into the caller's stream
    std::vector<hipStream_t> gstreams;
    std::vector<hipEvent_t> gevents;   // [0] fork, [1 + g] group g done
    // partly affine order groups: the affine part's apply launch runs on this
    // side stream beside the deformed part's, so that their tails overlap
    hipStream_t aff_stream = nullptr;
    hipEvent_t aff_ev[2] = {nullptr, nullptr};   // fork, join
    bool concurrent = false;
    // persistent gather-fold launch: every element of the order <= 6 groups
    // (with traces <= 8 x 8), by decreasing order; ElemDesc::pad = order
    sipdg::ElemDesc *d_pdesc = nullptr;
    sipdg::FaceDesc *d_pfdesc = nullptr;
    int pcount = 0;
    // 2-D wavefront list: every element of order <= 6 with traces <= 8
    // points, by decreasing order (ElemDesc::pad = order), four faces each
    sipdg::ElemDesc *d_w2desc = nullptr;
    sipdg::FaceDesc *d_w2fdesc = nullptr;
    sipdg::NbDesc2 *d_w2nb = nullptr;
    int w2count = 0;
    int *d_eprob = nullptr;   // [n_elems] problem of each element
    int num_cu = 256;
    int blocks_per_cu = 8;            // persistent grid = num_cu * blocks_per_cu
    uint64_t signature = 0;           // mesh signature (autotuner cache key)
    bool tune_from_cache = false;     // the current tuning came from a cache file
    // gather-fold apply tile shape per order: elements per workgroup, and the
    // register budget (waves per SIMD) of the kernel instance
    int tile[9] = {1, 1, 1, 1, 1, 1, 1, 1, 1};
    int budget[9] = {2, 2, 2, 2, 2, 2, 2, 2, 2};
    bool fast_ok = false;   // 3-D with every order <= 6
    bool gfold_ok = false;  // 3-D: gather-fold (general kernels for groups <= 6 next to orders 7-8)
};
