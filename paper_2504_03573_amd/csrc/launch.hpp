// Host-side launchers (implemented next to their kernels).
#pragma once

#include <vector>

#include "context.hpp"

namespace sipdg {

enum OpKind { OP_TRACE = 0, OP_APPLY = 1 };

// Tile shapes of the gather-fold apply launch of one order group that the
// library is built with: elements per workgroup and the register budget
// (waves per SIMD the kernel instance is compiled for).  The first entry is
// the default; the autotuner chooses among them.
struct TileShape {
    int tile, budget;
};
std::vector<TileShape> tile_shapes(int P);

// Operator kernels for one order group.  tsz must be work_size(nfm).
template <class R>
hipError_t launch_op(int dim, int P, int kind, const OpArgs<R> &A, int nfm, hipStream_t st);
// Point-to-point flux kernels (3-D) for one order group: stage 1 trace, 2 apply;
// tsz must be work_size(nfm).
template <class R>
hipError_t launch_p2p(int P, int stage, const OpArgs<R> &A, int nfm, hipStream_t st);
// Point-to-point flux through the gather-fold kernels: per-side factors
// (FP64, every face side; side: [nf][2][factor offset, buffer offset]).
hipError_t launch_p2p_factors(int64_t nfaces, const FaceTopo *faces, const int *order, const int64_t *side,
                              const double *emap, const double *tab, double *fg, hipStream_t st);

int work_size_for(int dim, int P, int nfm);
size_t lds_for(int dim, int P, int tsz, bool lift, size_t rsize);
int elems_per_block(int dim, int P);

hipError_t launch_load(int dim, int P, const OpArgs<double> &A, const int64_t *qoff,
                       const int64_t *boff, const double *src, const double *gdir,
                       hipStream_t st);
hipError_t launch_pgrad_elem(int dim, int P, const OpArgs<double> &A, const double *a,
                             const double *b, const double *tau0, double *dlam, double *bsig,
                             hipStream_t st);

// Setup and auxiliary kernels (aux.hip).
struct FaceTopo {
    int eL, fL, eR, fR, orient, nf;
};

// 2-D wavefront kernels (k2d.hip): every quadrilateral of order <= 6 whose
// faces carry at most 8 trace points, one wavefront each, one launch.
// The neighbour across one face of a 2-D wavefront element (fused mode):
// its coefficient offset, and code = N_P | local face << 4 | orientation
// relative to the owner's point order << 6 (0 on boundary faces).
struct NbDesc2 {
    int64_t xn;
    int code, pad;
};
struct Args2 {
    const ElemDesc *desc;    // [count], by decreasing order; pad: order
    const FaceDesc *fdesc;   // [count][4]
    const NbDesc2 *nbdesc;   // [count][4]
    int count;
    const int *skip;         // stop flag of a captured solver loop, or null
};
template <class R>
struct Data2 {
    const R *__restrict__ vgeo;
    const R *__restrict__ fgeo;
    const R *__restrict__ lam;
    const R *__restrict__ tau;
    const R *__restrict__ tab;
    const R *__restrict__ x;
    R *__restrict__ y;
    R *__restrict__ tbuf;
};
// mode 0: trace values into the buffer; 1: apply (neighbours from the
// buffer); 2: fused apply (neighbours' traces from their coefficients)
template <class R>
hipError_t launch_wave2d(int mode, const Args2 &A, const Data2<R> &D, hipStream_t st);
hipError_t launch_geo_volume(int dim, int64_t ne, const double *corners, const int *order,
                             const int64_t *voff, const double *tab, double *vgeo, int *flag,
                             hipStream_t st);
hipError_t launch_geo_faces(int dim, int64_t nfaces, const double *corners, const FaceTopo *ft,
                            const int64_t *foff, const double *tab, double *fgeo, int *flag,
                            hipStream_t st);
hipError_t launch_points(int dim, int64_t ne, const double *corners, const int *order,
                         const FaceRef *eface, const int64_t *qoff, const int64_t *boff,
                         const double *tab, double *xq, double *xb, hipStream_t st);
// Jacobi diagonal of one order group (elems: its element ids)
hipError_t launch_diag(int dim, int P, int64_t count, const int *elems, const int64_t *xoff,
                       const int64_t *voff, const FaceRef *eface, const int64_t *foff,
                       const double *vgeo, const double *fgeo, const double *lam,
                       const double *tau, const double *tab, double *diag, hipStream_t st);
hipError_t launch_pgrad_faces(int dim, int64_t nfaces, const int *is_interior,
                              const int64_t *toff, const int64_t *foff, const int *nf,
                              const double *fgeo, const double *tau0, const double *ta,
                              const double *tb, double *out, hipStream_t st);
// out[p] = sum_{i in [off[p], off[p+1])} v[i]  (fixed-order, deterministic)
hipError_t launch_segsum(int nseg, const int64_t *off, const double *v, double *out, int accumulate,
                         hipStream_t st);
hipError_t launch_cast_f32(const double *in, float *out, int64_t n, hipStream_t st);
hipError_t launch_cast_f64(const float *in, double *out, int64_t n, hipStream_t st);
hipError_t launch_recip(const double *in, double *out64, float *out32, int64_t n, hipStream_t st);

}  // namespace sipdg
