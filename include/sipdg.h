/*
 * sipdg.h - C ABI of the MI355X SIPG Helmholtz library.
 *
 * The library applies, matrix-free, the symmetric interior penalty DG
 * discretisation of  -lap u + lambda u = s  on unstructured quadrilateral
 * (2-D) or hexahedral (3-D) spectral elements with per-element polynomial
 * order (Xia & Moxey, arXiv 2504.03573: Sec. 2.2 eq. IP and eq. primal).
 * Interfaces between elements of different order are evaluated on a shared
 * trace space whose Gauss-Lobatto quadrature follows the higher-order side
 * (Sec. 3.3, "shared trace space"); each side's solution is evaluated at the
 * trace points and the flux is projected back to the element by the
 * transposed evaluation, so the operator is symmetric (Appendix A).
 *
 * Discretisation fixed by this library (part of the ABI):
 *   - element e has order p_e in [1, 8], N_P = p_e+1 modes per direction,
 *     orthogonal (Legendre) basis phi_i = prod_k P_{i_k}(xi_k) with
 *     P_i(1) = 1 (Table 1, "Orthogonal"), modes lexicographic with the first
 *     reference direction fastest;
 *   - tensor Gauss-Lobatto-Legendre quadrature with p_e+2 points per
 *     direction in the element (Sec. 5.2 benchmark setting), and
 *     max(p_L,p_R)+2 per direction on an interior face;
 *   - element map: multilinear from the 2^dim corners, corners stored
 *     lexicographically (corner with reference coordinates (c_1..c_d) in
 *     {-1,1}^d at index sum_k ((c_k+1)/2) 2^k);
 *   - penalty tau_F = sigma * 2 (p_F+1)^2 / h, p_F = max(p_L, p_R) (on a
 *     boundary face p_e); Dirichlet boundaries by the mirrored exterior
 *     value u+ = -u- + 2 g, grad u+ = grad u- (Sec. 2.2, boundary values set
 *     by the boundary condition), hence penalty 2 tau_F on boundary faces.
 *
 * Vector layout: natural element order; element e's (p_e+1)^dim
 * coefficients start at elem_offsets[e].  In a batch, problem after problem.
 *
 * Conventions for every function:
 *   - return 0 (SIPDG_OK) or a negative error code; sipdg_last_error()
 *     returns a thread-local message for the last failure;
 *   - "device" pointers are HIP device memory (e.g. torch tensor
 *     data_ptr()), contiguous, owned by the caller; "host" pointers are
 *     ordinary memory, read during the call only;
 *   - stream is a hipStream_t passed as void* (NULL = default stream);
 *     functions documented "async" only enqueue work on that stream;
 *   - a handle may be used by one stream at a time;
 *   - a mesh with no elements is valid: on its handle every vector call
 *     (apply, transpose, stages, diagonal, points, load vector, lambda,
 *     parameter gradient, CG) does nothing and accepts null vectors; CG
 *     reports convergence after 0 iterations and the penalty gradient of
 *     each problem is 0.  A batch may hold such problems among others.
 */
#ifndef SIPDG_H
#define SIPDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIPDG_OK          0
#define SIPDG_EINVAL     -1   /* bad argument: null pointer, order out of range, size */
#define SIPDG_EMESH      -2   /* non-positive Jacobian, face shared by >2 elements,
                                 faces that do not match by a symmetry of the square */
#define SIPDG_ENOMEM     -3   /* device or host allocation failed */
#define SIPDG_EHIP       -4   /* a HIP runtime call failed (no device, launch error) */
#define SIPDG_ENOCONV    -5   /* CG reached maxit without meeting the tolerance */
#define SIPDG_EBREAKDOWN -6   /* CG found p^T A p <= 0 (operator not SPD) */

#define SIPDG_F64 0
#define SIPDG_F32 1

#define SIPDG_MAX_ORDER 8

typedef struct sipdg_ctx *sipdg_handle;

/* One mesh (one problem).  All arrays are host memory, read during create.
 * A zero-initialised description plus the arrays and sizes is valid: basis 0
 * is the Legendre basis and quad_extra 0 selects the default (2). */
typedef struct {
    int dim;                       /* 2 or 3 */
    int64_t n_vertices;
    const double *coords;          /* [n_vertices][dim] */
    int64_t n_elems;
    const int64_t *elem_vertices;  /* [n_elems][2^dim], lexicographic corners */
    const int32_t *order;          /* [n_elems], 1..SIPDG_MAX_ORDER */
    const double *lambda;          /* [n_elems] Helmholtz coefficient per element */
    double h;                      /* nominal mesh size in tau_F (> 0) */
    double penalty_scale;          /* sigma in tau_F (> 0) */
    int basis;                     /* SIPDG_BASIS_LEGENDRE (0) or SIPDG_BASIS_MODAL (1) (Table 1);
                                      every problem of a batch the same (EINVAL otherwise) */
    int quad_extra;                /* GLL points per direction n = p + quad_extra in the
                                      element and n_F = p_F + quad_extra on a face
                                      (Sec. 5.2 benchmark setting: 2).  0 or 2; any other value
                                      returns EINVAL (the kernels are built for p + 2) */
} sipdg_mesh_desc;

/* Mesh statistics computed on the host without a device. */
typedef struct {
    int64_t n_elems, n_dofs;
    int64_t n_interior_faces, n_boundary_faces;
    int64_t n_nonconforming_faces;   /* interior faces with p_L != p_R */
    int64_t orientation_count[8];    /* interior faces per orientation code */
    int64_t n_volume_points, n_trace_points;
    int64_t n_interior_trace_points, n_boundary_trace_points;
    int64_t elems_per_order[SIPDG_MAX_ORDER + 1];
} sipdg_mesh_stats;

/* Sets up the discrete SIPG operator of Sec. 2.2 (eq. IP, the primal form)
 * on the mesh: faces matched by sorted corner ids (owner = lower element
 * id, orientation of the non-owner side, Sec. 5.1), the shared trace of each
 * interior face with max(p_L, p_R) + 2 GLL points per direction (Sec. 3.3),
 * per-point geometric factors |J| J^-1 J^-T w and |J| w (Sec. 2.1; FP64 and an
 * FP32 copy rounded once), per-trace-point a = w J_s and each side's
 * s w (|J| J^-1 J^-T)[k], tau_F, and the Jacobi diagonal, on the current
 * device.  Every device buffer the handle's calls use (trace buffers, CG
 * work vectors, gradient scratch) is allocated here.  desc and its arrays
 * are host memory read during the call; *out receives a handle owned by
 * the caller until sipdg_destroy.  Synchronous.  Errors: EINVAL (null
 * pointer, order outside [1, 8], dim, h, sigma, basis or quad_extra), EMESH
 * (non-positive Jacobian, face shared by more than two elements, faces that
 * do not match), ENOMEM, EHIP (no device). */
int sipdg_create(const sipdg_mesh_desc *desc, sipdg_handle *out);

/* Several independent problems in one handle: one vector holds them one
 * after the other, one launch per kernel covers all of them (elements are
 * grouped by order across problems), and CG keeps separate scalars and a
 * separate stopping test per problem. */
int sipdg_create_batch(int n_problems, const sipdg_mesh_desc *descs, sipdg_handle *out);

void sipdg_destroy(sipdg_handle h);

/* Host-only inspection of a mesh (no device needed).  Same validation and
 * error codes as sipdg_create. */
int sipdg_mesh_inspect(const sipdg_mesh_desc *desc, sipdg_mesh_stats *stats);

int sipdg_num_dofs(sipdg_handle h, int64_t *n);
int sipdg_num_elems(sipdg_handle h, int64_t *n);
int sipdg_num_problems(sipdg_handle h, int *n);
/* host [n_elems+1] coefficient offsets of each element */
int sipdg_elem_offsets(sipdg_handle h, int64_t *off);
/* host [n_problems+1] coefficient / element offsets of each problem */
int sipdg_problem_offsets(sipdg_handle h, int64_t *dof_off, int64_t *elem_off);

/* y = A x, the matrix-free application of the operator of Sec. 2.2 (eq. IP
 * summed over elements and faces, i.e. the primal form), with the interface
 * terms on the shared trace (Sec. 3.3) and the launch structure of Sec. 5.1
 * (LhsEval: trace stage, then volume and flux stage).  x, y: device,
 * [n_dofs] in the natural layout, owned by the caller; they must not
 * overlap.  precision SIPDG_F64: double; SIPDG_F32: float, computed with the
 * FP32 copy of the geometric factors.  Scratch (the trace buffer) is owned by
 * the handle.  Async on stream.  Errors: EINVAL (null handle or vector), EHIP
 * (launch failure). */
int sipdg_apply(sipdg_handle h, const void *x, void *y, int precision, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): y = A x
 * exactly as sipdg_apply (same kernels, same results bit for bit), but the
 * trace buffer between the two stages is a fixed device array of
 * SIPDG_NOALLOC_SCRATCH_BYTES inside the library (one per GPU, held until
 * the process ends, its address looked up at sipdg_create) instead of the
 * handle's buffer.  The call itself allocates nothing and enqueues only
 * kernel launches on stream (async).  Every call on one GPU shares that
 * array and leaves its contents behind (no call needs it cleared): calls on
 * one GPU that overlap in time, from any handle or stream, race and give
 * wrong results; serialise them.  Errors: EINVAL (null handle or vector,
 * x == y, precision, point-to-point flux set, or a trace buffer of
 * 4 (n_interior_trace_points) + 2 (n_boundary_trace_points) values at this
 * precision larger than the scratch), EHIP (launch failure, no scratch
 * address for the handle's device). */
#define SIPDG_NOALLOC_SCRATCH_BYTES (160ll << 20)
int sipdg_apply_noalloc(sipdg_handle h, const void *x, void *y, int precision, void *stream);

/* One of the two stages of sipdg_apply, async (Sec. 5.1 splits LhsEval the
 * same way, with the trace exchange between the two parts):
 *   stage 1: trace values (u and w J_s n.grad u, owner point order) of every
 *            interior face side into the handle's trace buffer (reads x);
 *   stage 2: volume terms, shared-trace fluxes (neighbour values from the
 *            trace buffer, so stage 1 must have run on the same x) and the
 *            inner products, y written once.
 * sipdg_apply == stage 1 then stage 2.  For timing and for overlapping the
 * two parts with other work. */
int sipdg_apply_stage(sipdg_handle h, const void *x, void *y, int precision, int stage,
                      void *stream);

/* Measurement: run `reps` applications y = A x back to back with a HIP event
 * recorded around every kernel launch on the stream, then return per launch
 * of one application (at most max_launches, in launch order; *n_launches
 * receives the count):
 *   ms        mean duration over the reps,
 *   stage     1 (trace kernels) or 2 (apply kernels),
 *   order     the polynomial order of the launch's element group (0 for
 *             the persistent launch of all orders <= 6),
 *   elements  the elements it processes,
 *   alg_bytes the algorithmic bytes of those elements at this precision
 *             (stage 2 only, 0 for stage 1): each element's coefficients in
 *             and out, its volume factors and lambda, all of its boundary
 *             faces' factors and half of its interior faces' factors (7 values
 *             per trace point: a and both sides' C), plus 32 bytes of
 *             connectivity per face shared the same way; summed over all
 *             elements this is the algorithmic traffic of one application.
 * x, y device; info host.  Synchronous. */
typedef struct {
    double ms;
    int stage;
    int order;
    int64_t elements;
    double alg_bytes;
} sipdg_launch_info;
int sipdg_apply_timed(sipdg_handle h, const void *x, void *y, int precision, int reps,
                      sipdg_launch_info *info, int max_launches, int *n_launches, void *stream);

/* Kernel structure of sipdg_apply (same results to rounding):
 *   GATHER:    trace values gathered from the element's quadrature points and
 *              interpolated to the trace (Sec. 3.2 GathrInterp), lifted by the
 *              transposed interpolation; two launches per order group; any
 *              dimension and order.
 *   TWO_STAGE: trace values evaluated directly from the coefficients
 *              (TracePhysEval) and lifted by TraceIProduct, one wavefront per
 *              element; trace kernel then apply kernel.  3-D, orders <= 6.
 *   FUSED:     as TWO_STAGE, but each element evaluates its neighbours'
 *              traces from their coefficients, so one launch per order group
 *              and no trace buffer.  3-D, orders <= 6.
 *   GATHER_FOLD: two stages.  The trace stage evaluates every face side's
 *              (u, g) at the shared trace points from the element's
 *              coefficients (TracePhysEval, Sec. 3.2), one launch for every
 *              element of order <= 6 and one per order-7/8 group.  The apply
 *              runs one wavefront per element (two for orders 7-8) with the
 *              volume in registers; the flux from both sides' (u, g) is
 *              lifted by the transposed interpolation and added to the
 *              volume's pointwise terms so that one IProduct lifts faces and
 *              volume (Sec. 3.3).  3-D; an order group <= 6 touching a
 *              neighbour above 6 uses the GATHER kernels (same trace buffer).
 *              In 2-D: one wavefront per quadrilateral of order <= 6 whose
 *              faces carry at most 8 trace points, all of them in one trace
 *              launch and one apply launch; each face side's (u, g) at the
 *              trace points from the element's coefficients (TracePhysEval),
 *              the flux lifted by the transposed interpolation and folded
 *              into the pointwise terms; the other elements on the GATHER
 *              kernels.  Default in 3-D, and in 2-D when an element fits.
 *   GATHER_FOLD_PERSISTENT: as GATHER_FOLD, but each stage is one
 *              persistent launch for the elements of every order <= 6 of all
 *              problems (listed by decreasing order; a fixed number of blocks
 *              per compute unit, chosen by sipdg_autotune, loops over them).
 *              3-D.
 *   GATHER_FOLD_FUSED: as GATHER_FOLD, but the neighbour's traces are
 *              evaluated from its coefficients (TracePhysEval): one launch
 *              per order group, no trace buffer.  3-D, orders <= 6; 2-D
 *              when every element takes the 2-D wavefront kernel (one launch
 *              for the whole mesh). */
#define SIPDG_VARIANT_GATHER            0
#define SIPDG_VARIANT_TWO_STAGE         1
#define SIPDG_VARIANT_FUSED             2
#define SIPDG_VARIANT_GATHER_FOLD       3
#define SIPDG_VARIANT_GATHER_FOLD_FUSED 4
#define SIPDG_VARIANT_GATHER_FOLD_PERSISTENT 5
#define SIPDG_NUM_VARIANTS              6
int sipdg_set_variant(sipdg_handle h, int variant);   /* EINVAL if not allowed */
int sipdg_get_variant(sipdg_handle h, int *variant);

/* Where the default gather-fold apply takes a deformed element's geometric
 * factors G~ w = |J| J^-1 J^-T w and |J| w (Sec. 2.1):
 *   STORED: the per-point values computed at create (7 per quadrature point;
 *           the default, and what every other kernel structure reads).
 *   MAP:    derived at every quadrature point from the element's trilinear
 *           map (21 coefficients per element, stored at create): more
 *           arithmetic, far fewer bytes, the trade-off of Sec. 5.1.
 * Same operator to rounding (FP64 within a few ulp of STORED).  Affine
 * elements always use their 7 per-element constants.  3-D only (EINVAL for
 * MAP on a 2-D handle).  Captured CG iterations are captured again after a
 * change. */
/* Interface flux of interior faces:
 *   SHARED: the shared trace space (Sec. 3.3): both sides evaluated at one
 *           GLL set of max(p_L, p_R) + 2 points per direction; A symmetric.
 *           The default, and the only flux of every other entry point.
 *   P2P:    point-to-point interpolation (Sec. 3.3, ScatrInterp): each side
 *           integrates on its own p + 2 GLL face points with the other
 *           side's value and physical gradient Lagrange-interpolated to them.
 *           Not symmetric in general (Sec. 3.3 conditions, Table 2).  3-D.
 *           While set, sipdg_apply, sipdg_apply_stage, sipdg_apply_timed
 *           (default kernel structure ignored: one trace and one apply
 *           launch per order group) and sipdg_gmres_solve use it; CG,
 *           transpose, diagonal, parameter gradients and autotuning return
 *           EINVAL.
 *           The first switch allocates a buffer of 8 values per trace point
 *           of each interior face side (EHIP if that fails). */

/* Modal basis of the coefficients (Table 1, quadrilateral / hexahedron):
 *   LEGENDRE: the orthogonal basis, tensor products of Legendre P_i (default).
 *   MODAL:    the modified C0 modal basis (Karniadakis & Sherwin), per
 *             direction psi_0 = (1-x)/2, psi_1 = (1+x)/2 (vertex modes
 *             first), psi_i = (1-x)/2 (1+x)/2 P^(1,1)_{i-2}(x), i >= 2.
 * Same space, so the operator changes by a congruence with the per-element
 * change of basis.  Switching rebuilds the 1-D tables and the Jacobi
 * diagonal (synchronous).  GATHER and GATHER_FOLD (the default) take either
 * basis; TWO_STAGE, FUSED, GATHER_FOLD_FUSED and GATHER_FOLD_PERSISTENT use
 * Legendre endpoint values in closed form and return EINVAL under MODAL.
 * Every entry point and both fluxes work. */
#define SIPDG_BASIS_LEGENDRE 0
#define SIPDG_BASIS_MODAL 1
int sipdg_set_basis(sipdg_handle h, int basis);
int sipdg_get_basis(sipdg_handle h, int *basis);

/* Volume quadrature points (Sec. 3.2: point sets that contain the element
 * boundary, where the trace is gathered from the volume points, and point
 * sets that do not, where it is evaluated from the coefficients):
 *   GLL:   n = p + 2 Gauss-Lobatto-Legendre points per direction (default).
 *   GAUSS: n = p + 2 Gauss-Legendre points per direction.  Exact for
 *          polynomial integrands of degree 2p + 3 per direction (GLL:
 *          2p + 1), so on trilinear elements the lambda term is integrated
 *          exactly; on affine elements both give the same operator.
 * The interface integrals keep the shared trace's GLL points (max p + 2 per
 * direction) either way: under GAUSS each side's u and C.grad u there come
 * from its coefficients (the trace stage), and the flux terms go back to the
 * modes by the transposed evaluation.  GAUSS takes the geometry of deformed
 * elements from their trilinear maps (no stored factors at the Gauss
 * points) and affine elements' constants, whatever sipdg_set_geometry says.
 * Requirements (EINVAL otherwise): a 3-D mesh, the shared-trace flux, and
 * every order group on the gather-fold kernels (no element of order <= 6
 * with a neighbour of order 7 or 8).  Switching to GAUSS selects the
 * GATHER_FOLD structure; while set, sipdg_set_variant accepts only that one
 * and sipdg_set_flux refuses the point-to-point flux.  sipdg_apply,
 * sipdg_apply_stage, sipdg_apply_timed, sipdg_apply_transpose (the operator
 * stays symmetric), sipdg_cg_solve and sipdg_gmres_solve use it (the solvers'
 * Jacobi preconditioner stays the GLL operator's diagonal); sipdg_diagonal,
 * sipdg_param_grad, sipdg_autotune, sipdg_quad_points and sipdg_load_vector
 * return EINVAL.  Either basis.  No allocation (both table sets are built at
 * create and by sipdg_set_basis). */
#define SIPDG_POINTS_GLL 0
#define SIPDG_POINTS_GAUSS 1
int sipdg_set_points(sipdg_handle h, int points);
int sipdg_get_points(sipdg_handle h, int *points);

#define SIPDG_FLUX_SHARED 0
#define SIPDG_FLUX_P2P 1
int sipdg_set_flux(sipdg_handle h, int flux);
int sipdg_get_flux(sipdg_handle h, int *flux);

#define SIPDG_GEOMETRY_STORED 0
#define SIPDG_GEOMETRY_MAP 1
int sipdg_set_geometry(sipdg_handle h, int source);
int sipdg_get_geometry(sipdg_handle h, int *source);
/* Autotuner (the per-order, compile-time specialised kernels of Sec. 5.1,
 * chosen by measurement).  Times one FP64 application (reps each, HIP events
 * on the stream, on the handle's CG work vectors: nothing is allocated) for
 * every allowed kernel structure, the persistent structure's grid (blocks
 * per compute unit), and for the gather-fold structure the tile shape of
 * each order group (elements per workgroup and the register budget, see
 * sipdg_tuning), and keeps the fastest.  A tile shape is timed in
 * alternation with the order group's best shape so far (twice each, the
 * faster run of each kept) and replaces it only if it is more than 2 %
 * faster.
 * cache_path (host string, may be NULL): a JSON file of earlier results, one
 * record per key "<mesh signature>-<library source hash>-<GPU arch>-<CUs>".
 * A record with this handle's key is applied without timing; otherwise the
 * result is added to the file (written to a temporary file, then renamed).
 * ms_out (host, [SIPDG_NUM_VARIANTS], may be NULL) receives the times (from
 * the record on a cache hit; 0 for structures not allowed).  Synchronous.
 * Errors: EINVAL (point-to-point flux or Gauss points set), EHIP; a cache
 * file that cannot be read or written is ignored (the tuning still runs). */
int sipdg_autotune(sipdg_handle h, const char *cache_path, int reps, double *ms_out, void *stream);

/* The handle's current tuning: kernel structure, persistent grid, whether it
 * came from a cache file, the mesh signature (FNV-1a of dim, problems,
 * orders, element corner ids and coordinates) and per order p the tile
 * shape of the gather-fold apply launch: tile[p] = elements per workgroup
 * (1 = one wavefront per element), budget[p] = waves per SIMD the register
 * allocation targets. */
typedef struct {
    int variant;
    int blocks_per_cu;
    int from_cache;
    uint64_t signature;
    int tile[SIPDG_MAX_ORDER + 1];
    int budget[SIPDG_MAX_ORDER + 1];
} sipdg_tuning;
int sipdg_get_tuning(sipdg_handle h, sipdg_tuning *t);

/* Set the tile shape of order p's gather-fold apply launch by hand (what the
 * autotuner chooses): tile = elements per workgroup, budget = waves per SIMD
 * of the kernel's register allocation; (1, 2) is the one-wavefront-per-
 * element kernel.  Tiles apply to the shared-trace apply of orders <= 5 with
 * stored or map geometry (affine and Gauss-point launches keep one element
 * per wavefront); results equal the one-element kernel's bit for bit.
 * Errors: EINVAL (null handle, order outside [1, 8], a shape the library is
 * not built with). */
int sipdg_set_tile(sipdg_handle h, int order, int tile, int budget);

/* xbar = A^T g, async.  The shared-trace SIPG operator is symmetric, so this
 * evaluates the same dataflow as sipdg_apply (Appendix A conditions hold by
 * construction). */
int sipdg_apply_transpose(sipdg_handle h, const void *g, void *xbar, int precision,
                          void *stream);

/* d = diag(A) in FP64 (device [n_dofs]), async: a(phi_i, phi_i) of eq. IP
 * with the neighbours' coefficients zero, sum-factorised per element (every
 * volume and face term of the diagonal is a tensor contraction of squared
 * 1-D mode tables with the geometric factors).  The Jacobi preconditioner of
 * sipdg_cg_solve. */
int sipdg_diagonal(sipdg_handle h, double *d, void *stream);

/* Gradients of the scalar a^T A b with respect to the parameters (the
 * differentiable operator, a project addition to the paper's method): the
 * operator is affine in lambda and sigma, so
 * dlambda (device [n_elems]) = (a, b) on each element, the lambda term of
 * eq. IP integrated with the volume quadrature, and
 * dsigma (device [n_problems]) = sum_F tau_F/sigma ([[a]], [[b]])_F per problem
 * (boundary faces: 2 a b), the penalty term.  a, b: device FP64 [n_dofs].
 * Scratch (a second trace buffer) comes from create.  Async.  Errors:
 * EINVAL (null pointer, point-to-point flux or Gauss points set), EHIP. */
int sipdg_param_grad(sipdg_handle h, const double *a, const double *b, double *dlambda,
                     double *dsigma, void *stream);

/* Replace lambda (device FP64 [n_elems]) / sigma (host, per problem or all
 * when problem < 0).  Refreshes the Jacobi diagonal.  Synchronous. */
int sipdg_set_lambda(sipdg_handle h, const double *lambda_dev, void *stream);
int sipdg_set_penalty_scale(sipdg_handle h, int problem, double sigma);

/* Number of volume quadrature points and of boundary trace points. */
int sipdg_num_points(sipdg_handle h, int64_t *n_volume, int64_t *n_boundary);

/* Number of elements found affine at create (3-D: the 8 corners span a
 * parallelepiped to within 1e-14 of the longest edge plus 16 ulp of the
 * largest corner coordinate, so the Jacobian is constant to rounding).
 * These are the regular elements of Sec. 5.1: the default gather-fold apply
 * reads their 6 entries of |J| J^-1 J^-T and |J| once per element instead of
 * 7 values per quadrature point, in a launch of their own.
 * Detection is off when the environment variable SIPDG_NO_AFFINE is "1" at
 * create.  2-D handles: 0.  Errors: EINVAL (null handle or pointer). */
int sipdg_num_affine(sipdg_handle h, int64_t *n_affine);
/* Physical coordinates (device FP64, [n][dim]) of the volume quadrature
 * points (element by element, points lexicographic) and of the boundary
 * trace points (element by element, boundary faces in local face order
 * 2k+(s>0), points lexicographic in face coordinates).  Async. */
int sipdg_quad_points(sipdg_handle h, double *xq, double *xb, void *stream);
/* Right-hand side of the primal form (Sec. 2.2) with Dirichlet data by the
 * mirrored exterior value u+ = -u- + 2 g (the boundary treatment of
 * Sec. 2.2, penalty 2 tau_F):
 * b = (phi_i, s) + the boundary data terms -(g, grad phi_i . n) + 2 tau (g, phi_i),
 * from source values s at the volume points and Dirichlet values g at the
 * boundary points (device FP64, in sipdg_quad_points' order; g may be NULL
 * when there are no boundary points).  b: device FP64 [n_dofs].  Async.
 * Errors: EINVAL (null pointer, Gauss points set), EHIP. */
int sipdg_load_vector(sipdg_handle h, const double *s, const double *g, double *b,
                      void *stream);

#define SIPDG_CG_F64     0   /* FP64 Jacobi-PCG */
#define SIPDG_CG_F32_IR  1   /* FP32 inner PCG inside FP64 iterative refinement */
#define SIPDG_CG_F32_RU  2   /* FP32 PCG with FP64 reliable updates: as F32_IR, but at each
                                FP64 residual replacement the FP32 recursion continues with its
                                search direction (renormalised) instead of restarting */

typedef struct {
    double tol;        /* stop when ||b - A x||_2 <= tol ||b||_2 per problem (1e-10) */
    int maxit;         /* max total (inner) iterations, per solve */
    int mode;          /* SIPDG_CG_F64, SIPDG_CG_F32_IR or SIPDG_CG_F32_RU */
    double inner_tol;  /* F32_IR, F32_RU: smallest relative reduction one inner FP32 cycle is
                          asked for (1e-4); each inner solve asks for what the outer
                          residual still needs, max(inner_tol, tol ||b|| / (2 ||r||)) */
    int precond;       /* 1 = Jacobi, 0 = none */
    int graph_k;       /* iterations per captured HIP graph / per host check; 0 = no graph */
    int max_outer;     /* F32_IR / F32_RU: max refinement steps / residual replacements;
                          F64: max restarts from the true residual, plus one (50) */
    /* optional checkpoint: called every checkpoint_every iterations with the
     * device pointers of the FP64 iterate x and residual r and the iteration
     * count; x0_given = 1 starts from the x passed in (resume). */
    void (*checkpoint)(void *user, const double *x, const double *r, int iter);
    void *checkpoint_user;
    int checkpoint_every;
    int x0_given;
    double ru_delta;   /* F32_RU: replace the residual once the FP32 residual has dropped by
                          this factor (0.1); a problem whose true residual then exceeds 1.5x
                          its recursive estimate restarts instead of continuing */
} sipdg_cg_opts;

typedef struct {
    int iters;              /* total (inner) iterations */
    int outer_iters;        /* refinement steps (F32_IR); F64: 1 + restarts from the true residual */
    int converged;          /* all problems met tol */
    double rel_resid;       /* max over problems of true ||b-Ax||/||b|| (FP64) */
    double time_ms;         /* wall time of the solve */
} sipdg_cg_info;

void sipdg_cg_default_opts(sipdg_cg_opts *o);

/* Restarted GMRES(restart) for A x = b with the handle's current operator,
 * either interface flux: the point-to-point flux makes A nonsymmetric, and
 * the paper solves those systems with GMRES (Table 2).  FP64 throughout.
 * Right preconditioning with the Jacobi diagonal of the shared-trace
 * operator (precond = 1; an approximation of the point-to-point diagonal),
 * Arnoldi by classical Gram-Schmidt applied twice, Givens rotations.  x
 * starts from zero; stop when ||b - A x||_2 <= tol ||b||_2 (the true residual
 * at a restart; inside a cycle the Arnoldi estimate).  maxit bounds the
 * Arnoldi steps.  A batched handle is solved as one system (tol applies to
 * the whole vector).  Device memory: (restart + 3) vectors for the call.
 * Synchronous.  Errors: EINVAL, ENOCONV (info filled), EHIP. */
typedef struct {
    double tol;       /* 1e-10 */
    int restart;      /* Krylov vectors per cycle, 1..1000 (30) */
    int maxit;        /* max Arnoldi steps in total (100000) */
    int precond;      /* 1 = Jacobi (shared-trace diagonal), 0 = none */
} sipdg_gmres_opts;

typedef struct {
    int iters;          /* Arnoldi steps */
    int restarts;       /* completed cycles */
    int converged;
    double rel_resid;   /* true ||b - A x|| / ||b|| at the end */
    double time_ms;
} sipdg_gmres_info;

void sipdg_gmres_default_opts(sipdg_gmres_opts *o);
int sipdg_gmres_solve(sipdg_handle h, const double *b, double *x, const sipdg_gmres_opts *opts,
                      sipdg_gmres_info *info, void *stream);

/* Solve A x = b by Jacobi-preconditioned conjugate gradients: the SIPG
 * operator is symmetric and, for lambda > 0, positive definite, which is
 * what the symmetric interior penalty is chosen for (Sec. 2.2); FP64, or
 * FP32 inner solves inside FP64 iterative refinement (mode, a project
 * addition).  b, x: device FP64 [n_dofs], owned by the caller (x is the
 * initial guess when opts->x0_given).  CG iterations are captured in HIP
 * graphs of opts->graph_k iterations.  When the 3-D gather-fold structure
 * evaluates every element's traces in one launch, each iteration's updates
 * of x and of the search direction run inside the next application's trace
 * stage (one pass over r, p and x instead of two vector kernels; the same
 * values bit for bit; the environment variable SIPDG_NO_FOLD=1 keeps the
 * separate kernels).  Synchronous: returns when done.
 * Errors: ENOCONV (maxit reached, info filled), EBREAKDOWN (p^T A p <= 0),
 * EINVAL (null pointer, options, point-to-point flux set), EHIP. */
int sipdg_cg_solve(sipdg_handle h, const double *b, double *x, const sipdg_cg_opts *opts,
                   sipdg_cg_info *info, void *stream);

const char *sipdg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SIPDG_H */
