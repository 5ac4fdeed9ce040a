// Dimension / order dispatch of the per-order kernels.
#include "op_instances.hpp"
#include "tile_shapes.hpp"

namespace sipdg {

template <class R>
hipError_t launch_op_2d(int P, int kind, const OpArgs<R> &A, int nfm, hipStream_t st);
template <class R>
hipError_t launch_op_3d(int P, int kind, const OpArgs<R> &A, int nfm, hipStream_t st);
hipError_t launch_load_2d(int P, const OpArgs<double> &A, const int64_t *qoff, const int64_t *boff,
                          const double *src, const double *gdir, hipStream_t st);
hipError_t launch_load_3d(int P, const OpArgs<double> &A, const int64_t *qoff, const int64_t *boff,
                          const double *src, const double *gdir, hipStream_t st);
hipError_t launch_pgrad_2d(int P, const OpArgs<double> &A, const double *a, const double *b,
                           const double *tau0, double *dlam, double *bsig, hipStream_t st);
hipError_t launch_pgrad_3d(int P, const OpArgs<double> &A, const double *a, const double *b,
                           const double *tau0, double *dlam, double *bsig, hipStream_t st);

template <class R>
hipError_t launch_op(int dim, int P, int kind, const OpArgs<R> &A, int nfm, hipStream_t st) {
    return dim == 2 ? launch_op_2d<R>(P, kind, A, nfm, st) : launch_op_3d<R>(P, kind, A, nfm, st);
}
template hipError_t launch_op<double>(int, int, int, const OpArgs<double> &, int, hipStream_t);
template hipError_t launch_op<float>(int, int, int, const OpArgs<float> &, int, hipStream_t);

hipError_t launch_load(int dim, int P, const OpArgs<double> &A, const int64_t *qoff,
                       const int64_t *boff, const double *src, const double *gdir, hipStream_t st) {
    return dim == 2 ? launch_load_2d(P, A, qoff, boff, src, gdir, st)
                    : launch_load_3d(P, A, qoff, boff, src, gdir, st);
}

hipError_t launch_pgrad_elem(int dim, int P, const OpArgs<double> &A, const double *a,
                             const double *b, const double *tau0, double *dlam, double *bsig,
                             hipStream_t st) {
    return dim == 2 ? launch_pgrad_2d(P, A, a, b, tau0, dlam, bsig, st)
                    : launch_pgrad_3d(P, A, a, b, tau0, dlam, bsig, st);
}

#define SIZE_CASE(D, p) \
    case p: return work_size<D, p>(nfm);
int work_size_for(int dim, int P, int nfm) {
    if (dim == 2) {
        switch (P) { SIZE_CASE(2, 1) SIZE_CASE(2, 2) SIZE_CASE(2, 3) SIZE_CASE(2, 4) SIZE_CASE(2, 5) SIZE_CASE(2, 6) SIZE_CASE(2, 7) SIZE_CASE(2, 8) }
    } else {
        switch (P) { SIZE_CASE(3, 1) SIZE_CASE(3, 2) SIZE_CASE(3, 3) SIZE_CASE(3, 4) SIZE_CASE(3, 5) SIZE_CASE(3, 6) SIZE_CASE(3, 7) SIZE_CASE(3, 8) }
    }
    return 0;
}
#undef SIZE_CASE
#define LDS_CASE(D, p) \
    case p: return lds_bytes<D, p>(tsz, lift, rsize);
size_t lds_for(int dim, int P, int tsz, bool lift, size_t rsize) {
    if (dim == 2) {
        switch (P) { LDS_CASE(2, 1) LDS_CASE(2, 2) LDS_CASE(2, 3) LDS_CASE(2, 4) LDS_CASE(2, 5) LDS_CASE(2, 6) LDS_CASE(2, 7) LDS_CASE(2, 8) }
    } else {
        switch (P) { LDS_CASE(3, 1) LDS_CASE(3, 2) LDS_CASE(3, 3) LDS_CASE(3, 4) LDS_CASE(3, 5) LDS_CASE(3, 6) LDS_CASE(3, 7) LDS_CASE(3, 8) }
    }
    return 0;
}
#undef LDS_CASE
#define EPB_CASE(D, p) \
    case p: return Cfg<D, p>::EPB;
int elems_per_block(int dim, int P) {
    if (dim == 2) {
        switch (P) { EPB_CASE(2, 1) EPB_CASE(2, 2) EPB_CASE(2, 3) EPB_CASE(2, 4) EPB_CASE(2, 5) EPB_CASE(2, 6) EPB_CASE(2, 7) EPB_CASE(2, 8) }
    } else {
        switch (P) { EPB_CASE(3, 1) EPB_CASE(3, 2) EPB_CASE(3, 3) EPB_CASE(3, 4) EPB_CASE(3, 5) EPB_CASE(3, 6) EPB_CASE(3, 7) EPB_CASE(3, 8) }
    }
    return 1;
}
#undef EPB_CASE

std::vector<TileShape> tile_shapes(int P) {
    std::vector<TileShape> v = {{1, 2}};   // one wavefront per element: the default kernel
#define SIPDG_TILE_ENTRY(PP, EE, BB) \
    if (P == PP) v.push_back({EE, BB});
    SIPDG_TILE_SHAPES(SIPDG_TILE_ENTRY)
#undef SIPDG_TILE_ENTRY
    return v;
}

}  // namespace sipdg
