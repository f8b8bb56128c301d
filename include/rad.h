/*
 * rad.h — C-ABI of librad: hierarchical low-rank view-factor matrices and
 * radiosity solves on one AMD Instinct MI355X (gfx950).
 *
 * Method: Potter, Bertone, Schorghofer, Mazarico, "Fast hierarchical low-rank
 * view factor matrices for thermal irradiance on planetary surfaces"
 * (arXiv 2209.07632).  Equation and algorithm names below are the paper's.
 *
 * Conventions (all entry points)
 *  - Status codes only; no C++ exception crosses this boundary.  On any status
 *    other than RAD_OK, rad_last_error() returns a thread-local message.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *    memory of the device the matrix was built on.  The caller owns every
 *    pointer it passes; the library never frees caller memory.
 *  - Vectors and blocks of right-hand sides are column-major N x R with a
 *    leading dimension >= N, facets in the caller's original face order
 *    unless RAD_ORDER_TREE is passed.
 *  - hip_stream may be NULL (the null stream).  Work is enqueued on it;
 *    matvec returns without waiting, solve synchronises on it because its
 *    stopping test reads residuals back to the host.
 *  - A rad_hmat is immutable after build; concurrent matvecs on different
 *    streams need separate workspaces and are not supported: calls on one
 *    matrix must be serialised by the caller.
 */
#ifndef RAD_H
#define RAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rad_hmat rad_hmat;

typedef enum {
    RAD_OK = 0,
    RAD_EINVAL = 1,  /* bad argument: null pointer, size, ld < N, non-finite input, bad mesh */
    RAD_ENOMEM = 2,  /* device or host allocation failed                                       */
    RAD_EDEVICE = 3, /* a HIP call failed                                                      */
    RAD_ENOCONV = 4, /* iterative solve hit max_iter before rtol (results and info still filled) */
    RAD_EUNSUP = 5   /* valid request this build does not implement                            */
} rad_status;

typedef enum { RAD_F64 = 0, RAD_F32 = 1, RAD_F16 = 2, RAD_BF16 = 3 } rad_dtype;

/* Visibility V_ij of eq. FF-def (section 3.2). */
typedef enum {
    RAD_VIS_BACKFACE = 0, /* n_i.d_ij > 0 and n_j.d_ji > 0 only (no occlusion test) */
    RAD_VIS_RAYCAST = 1   /* back-face test, then the centroid segment must miss every other triangle */
} rad_visibility;

/* Storage of leaf blocks next to the diagonal (Algorithm 4, the leaf case). */
typedef enum {
    RAD_NEAR_AUTO = 0,  /* fewer bytes of dense or CSR, as the paper states */
    RAD_NEAR_DENSE = 1, /* always dense                                      */
    RAD_NEAR_CSR = 2    /* always CSR                                        */
} rad_nearfield;

/*
 * Layout of vectors and blocks of right-hand sides:
 *  RAD_ORDER_ORIGINAL: column-major N x R, rows in the caller's face order;
 *  RAD_ORDER_TREE: column-major N x R, rows in tree order (rad_hmat_perm);
 *  RAD_ORDER_TREE_RMAJOR: the library's internal layout, rows in tree order
 *      with the R values of a facet contiguous: element (t, r) at t * ld + r,
 *      where ld must equal R rounded up to a multiple of 4 and the pointer must
 *      be 16-byte aligned.  No layout conversion is done on this path.
 */
typedef enum { RAD_ORDER_ORIGINAL = 0, RAD_ORDER_TREE = 1, RAD_ORDER_TREE_RMAJOR = 2 } rad_order;

/*
 * Device-memory hook.  When rad_build_opts.allocator is non-NULL, every device
 * allocation of the matrix (operator, geometry, ray-casting grid, solve and
 * product workspace) and of its build's temporaries goes through alloc, and is
 * returned through free, instead of hipMalloc/hipFree; for example a caching
 * allocator of the caller's framework.  alloc returns device memory of at
 * least `bytes` bytes on `device`, 256-byte aligned, or NULL on failure (the
 * call then fails with RAD_ENOMEM); free receives the same pointer, byte count
 * and device.  The library copies the struct at build or load time; ctx and
 * both functions must stay valid until rad_hmat_free of that matrix (and of
 * groups built from it).  Both are called from the thread that calls into the
 * library, only during rad_hmat_build*, rad_hmat_load, rad_hmat_group,
 * rad_insolation (its sun list) and rad_hmat_free; products and solves never
 * allocate.
 */
typedef struct {
    void *ctx;
    void *(*alloc)(void *ctx, size_t bytes, int32_t device);
    void (*free)(void *ctx, void *ptr, size_t bytes, int32_t device);
} rad_allocator;

typedef struct {
    double tol;           /* compression tolerance eps of Algorithm 3 (> 0)           */
    int32_t leaf_size;    /* quadtree leaf capacity, Algorithm 2 (default 64, <= 4096) */
    int32_t max_depth;    /* quadtree depth limit (0: none)                           */
    int32_t nearfield;    /* rad_nearfield                                            */
    int32_t visibility;   /* rad_visibility                                           */
    int32_t storage;      /* RAD_F64 or RAD_F32: precision of stored blocks and of matvec/solve */
    int32_t oversample;   /* extra sketch columns in the randomized rank search (default 8) */
    int32_t power_iters;  /* subspace iterations of the rank search (default 1)       */
    int32_t max_rhs;      /* workspace is sized for up to this many right-hand sides (default 1) */
    int32_t device;       /* HIP device ordinal (default 0)                           */
    uint64_t seed;        /* seed of the sketch's random signs                        */
    int32_t verbose;      /* 1: print build progress and statistics to stderr         */
    int32_t max_rank;     /* 0: no limit; else Algorithm 3 gives up above this rank   */
    int32_t lowp;         /* 0: none; RAD_F16 or RAD_BF16: also keep a 16-bit copy of the
                             operator (needs storage RAD_F32) for refined solves       */
    const rad_allocator *allocator; /* NULL: hipMalloc/hipFree; else the hook above     */
} rad_build_opts;

/* Fills *opts with the defaults listed above (tol 1e-3). */
void rad_build_opts_default(rad_build_opts *opts);

/*
 * Builds the compressed view-factor matrix F-hat (Algorithms 2-4) from a
 * triangle mesh: host arrays verts (nv x 3, row-major, FP64) and faces
 * (nf x 3, row-major, 0-based int32).  Facet i is face i; its centroid,
 * unit normal (right-hand rule) and area follow section 3.  F_ij is eq. FF-def
 * (it includes the column area A_j), F_ii = 0.  The matrix lives on
 * opts->device until rad_hmat_free.
 * Errors: RAD_EINVAL for null pointers, nf < 1, indices outside [0, nv),
 * non-finite coordinates, zero-area faces or bad options; RAD_ENOMEM;
 * RAD_EDEVICE.  *out is NULL on error.
 */
rad_status rad_hmat_build(const double *verts, int64_t nv, const int32_t *faces, int64_t nf,
                          const rad_build_opts *opts, rad_hmat **out);

/*
 * rad_hmat_build with a choice of tree (Algorithm 2; section 4.1 names the
 * octree as its 3-D analogue for overhangs and small bodies):
 * tree_dims = 2 splits the centroids on (x, y), a quadtree, as rad_hmat_build;
 * tree_dims = 3 splits them on (x, y, z), an octree of at most eight children
 * per node (x the most significant side, then y, then z), for closed bodies.
 * Everything after the tree (block pairs from the root's children, rank
 * search, layout, products) is the same.  Errors as rad_hmat_build, and
 * RAD_EINVAL for another tree_dims.
 */
rad_status rad_hmat_build_tree(const double *verts, int64_t nv, const int32_t *faces, int64_t nf,
                               const rad_build_opts *opts, int32_t tree_dims, rad_hmat **out);

/*
 * rad_hmat_build from facet geometry instead of a mesh (section 3 states the
 * view factors of eq. FF-def through centroids, unit normals and areas alone):
 * host arrays x (N x 3 centroids), n (N x 3 unit normals, |n| within 1e-6 of 1,
 * used as given), area (N, > 0), all row-major FP64 in the caller's facet
 * order.  tri_verts (N x 9: the three vertices of facet i's triangle, row-major)
 * supplies the occluders of ray-cast visibility (section 3.2) and the shadows
 * of rad_insolation; it may be NULL only with visibility RAD_VIS_BACKFACE, and
 * then rad_insolation casts no shadows.  tree_dims as rad_hmat_build_tree.
 * Errors: RAD_EINVAL for null arrays, N < 1, non-finite values, non-unit
 * normals, areas <= 0, bad options or RAD_VIS_RAYCAST without triangles;
 * RAD_ENOMEM; RAD_EDEVICE.  *out is NULL on error.
 */
rad_status rad_hmat_build_facets(const double *x, const double *n, const double *area, int64_t N,
                                 const double *tri_verts, const rad_build_opts *opts, int32_t tree_dims,
                                 rad_hmat **out);

/*
 * Writes the blocks of F-hat to a binary file at path, for use outside the
 * library (for example to form F-hat densely on the host).  The blocks are
 * the leaves of the partition Algorithm 4 chose: every non-zero block of F-hat
 * once, rows and columns as ranges of the tree order (rad_hmat_perm maps tree
 * position t to original facet perm[t]); zero blocks are not listed.  All
 * integers little-endian, values FP64 (the stored values converted exactly):
 *   char magic[8] = "RADHBLKS"; uint32 version = 1; int32 storage dtype;
 *   int64 N; int64 nblocks; int32 perm[N];
 *   per block: int32 kind (1 dense, 2 CSR, 3 low rank), i0, m, j0, n, rank
 *              (0 unless low rank); int64 nnz (non-zero entries of the block
 *              of F; for CSR the stored entries); then
 *     dense:    double A[m * n], column-major (F-hat[i0 + r, j0 + c] = A[r + c m]);
 *     CSR:      int32 rowptr[m + 1] (rowptr[0] = 0), int32 col[nnz] (0 .. n-1),
 *               double val[nnz];
 *     low rank: double U[m * rank], double V[n * rank], both column-major, with
 *               F-hat block = U V^T (U = U Sigma of Algorithm 3).
 * Errors: RAD_EINVAL (null, a group), RAD_EDEVICE (file or HIP failure).
 */
rad_status rad_hmat_export(const rad_hmat *H, const char *path);

/*
 * Saves the complete compressed operator (device layout, geometry, ray-casting
 * grid, 16-bit copy, launch configurations) to a versioned binary file, so
 * that it is built once and used elsewhere (section 10 names reuse of the
 * assembled matrix).  rad_hmat_load reads it back onto `device` with
 * workspace for max_rhs right-hand sides (0: the saved max_rhs); every
 * product and solve of the loaded matrix equals that of the saved one bit for
 * bit.  The file holds raw little-endian structures of this library version:
 * a file from another version or with other structure sizes is refused.
 * allocator: as rad_build_opts.allocator (NULL: hipMalloc).
 * Errors: RAD_EINVAL (null, bad file), RAD_ENOMEM, RAD_EDEVICE (file or HIP
 * failure).  *out is NULL on error.
 */
rad_status rad_hmat_save(const rad_hmat *H, const char *path);

/*
 * A new matrix with the compressed operator of H (same partition, ranks and
 * layout) stored in dtype (RAD_F64 or RAD_F32): FP32 values widen exactly,
 * FP64 values round.  This gives, for example, the FP64 form of an operator
 * built in FP32 without a second assembly, so both precisions can be compared
 * on one F-hat.  The 16-bit copy is not carried over; max_rhs as
 * rad_hmat_load (0: H's); H's allocator hook serves the new matrix too.
 * Errors: RAD_EINVAL (null, a group, bad dtype), RAD_ENOMEM, RAD_EDEVICE.
 */
rad_status rad_hmat_convert(const rad_hmat *H, int32_t dtype, int32_t max_rhs, rad_hmat **out);
rad_status rad_hmat_load(const char *path, int32_t device, int32_t max_rhs, const rad_allocator *allocator,
                         rad_hmat **out);

/*
 * Y = F-hat X (Algorithm 5) for R right-hand sides.  X and Y are device
 * arrays of the matrix's compute dtype (rad_hmat_dtype) in the layout named
 * by order (rad_order; leading dimensions ldx, ldy as that layout requires).
 * X and Y must not overlap.  1 <= R <= max_rhs.
 * dtype equal to the matrix's lowp (RAD_F16 or RAD_BF16) applies the 16-bit
 * copy of the operator instead, with FP32 X and Y and FP32 accumulation
 * (R >= 16 only).
 * Errors: RAD_EINVAL (null, R out of range, ld < N, dtype mismatch), RAD_EDEVICE.
 */
rad_status rad_hmat_matvec(const rad_hmat *H, int64_t R, int32_t dtype, const void *X, int64_t ldx,
                           void *Y, int64_t ldy, int32_t order, void *hip_stream);

/*
 * Allocation-free variant of rad_hmat_matvec, for callers that cannot
 * allocate device memory at call time (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same product, same
 * kernels, same arguments and layouts as rad_hmat_matvec with 1 <= R <= 15
 * (the single-RHS kernels); R is not limited by the matrix's max_rhs.
 * Its scratch (the projections T = V^T X, t_ld x R values, and for the
 * original and R-major orders X and Y in tree order, N x R values each) lives
 * in a file-scope device array of rad_noalloc_scratch_bytes() bytes (8 MiB)
 * that every device running the library holds until the process ends; the
 * call allocates nothing (no hipMalloc, no host-side allocating library
 * call).  Every value read from the scratch is written earlier in the same
 * call, so nothing needs clearing.  All calls on one device share that
 * device's array: calls that overlap in time on one device (different
 * streams, host threads or matrices) race and must be serialised by the
 * caller.  The first call on a device looks the array's device address up
 * with that device current (H's device).
 * Errors: as rad_hmat_matvec; RAD_EINVAL for R outside [1, 15], for a group,
 * and when the scratch needed exceeds the array (the message states both).
 */
rad_status rad_hmat_matvec_noalloc(const rad_hmat *H, int64_t R, int32_t dtype, const void *X, int64_t ldx,
                                   void *Y, int64_t ldy, int32_t order, void *hip_stream);

/* Size in bytes of the static scratch array of rad_hmat_matvec_noalloc. */
size_t rad_noalloc_scratch_bytes(void);

typedef struct {
    double rtol;      /* stop column c when ||B^{k+1}-B^k||_2 <= rtol ||E_c||_2 (default 1e-3) */
    int32_t max_iter; /* default 100                                                     */
    int32_t order;    /* rad_order of E and B                                            */
    int32_t check_every; /* read residuals back every this many iterations (default 1) */
    int32_t use_graph;   /* 1: replay each iteration as a cached HIP graph (default 1) */
    int32_t refine;      /* 0: Jacobi on F-hat; 1: iterative refinement: FP64 residual with the
                            FP32 operator, inner Jacobi with the 16-bit copy (needs lowp, R >= 16) */
    int32_t inner_iters; /* inner Jacobi iterations per refinement step (default 3)  */
    int32_t warm;        /* 1: B holds a starting guess on entry (same layout as the output);
                            each column keeps it only if its first residual is no larger
                            than the cold start's (default 0)                          */
    int32_t method;      /* a rad_solve_method; default RAD_SOLVE_JACOBI                 */
    double lam_lo, lam_hi; /* Chebyshev: an interval containing the (real) spectrum of
                            F-hat; both 0 (default): [-s, s] with s = 1.01 max_i (F-hat 1)_i */
    int32_t restart;     /* GMRES: Arnoldi steps per cycle (default 30)                  */
} rad_solve_opts;

/*
 * Iterations of rad_solve.  The paper relaxes with Jacobi (section 5.1:
 * O(1) iterations for its systems).  Chebyshev and GMRES are not in the paper:
 * they serve systems whose spectral radius rho max|lambda(F)| approaches one
 * (closed or deep bodies in the infrared band, rho = 1), where Jacobi needs
 * many products.
 *  RAD_SOLVE_CHEBYSHEV: the three-term Chebyshev iteration for
 *    (I - rho F-hat) B = E from B^0 = E (Saad, Iterative Methods for Sparse
 *    Linear Systems, 2nd ed., section 12.1), one product per iteration.  F is
 *    self-adjoint in the area-weighted inner product (reciprocity, eq. FF-def),
 *    so its spectrum is real; [lam_lo, lam_hi] must contain it (F-hat's), and
 *    1 - rho lam_hi > 0.  Column c stops counting at the first iteration whose
 *    recurrence residual has ||r_c|| <= rtol ||E_c||; all columns step until
 *    every one has (one scalar recurrence), and B holds that iterate.  Needs a
 *    scalar rho (rho == NULL), no refinement, no warm start, no group.
 *  RAD_SOLVE_GMRES: restarted GMRES (same reference, section 6.5) from B = 0,
 *    every column its own Krylov space, all columns advancing together (one
 *    multi-column product per Arnoldi step); Arnoldi with classical
 *    Gram-Schmidt applied twice, Givens rotations on the host.  A column stops
 *    when its residual estimate meets rtol ||E_c||; each cycle ends with the
 *    true residual.  info->iters counts each column's Arnoldi steps (products).
 *    Allocates its Krylov basis ((restart + 1) N R values) for the call.  Needs
 *    no refinement, no warm start, no group; rho may be per facet.
 */
typedef enum { RAD_SOLVE_JACOBI = 0, RAD_SOLVE_CHEBYSHEV = 1, RAD_SOLVE_GMRES = 2 } rad_solve_method;

void rad_solve_opts_default(rad_solve_opts *opts);

typedef struct {
    int32_t *iters;      /* host, length R (R x instances for a group, instance-major; or NULL):
                            iterations at which column met rtol (-1: never)                      */
    double *rel_change;  /* host, same length (or NULL): last ||B^{k+1}-B^k|| / ||E||            */
    int32_t total_iters; /* iterations run (refinement steps when refine = 1)                      */
    int32_t inner_iters; /* inner iterations run in total (refine = 1)                              */
    int32_t warm_columns; /* columns that kept the starting guess (warm = 1)                        */
} rad_solve_info;

/*
 * Solves (I - diag(rho) F-hat) B = E, the radiosity system eq.
 * radiosity-system, for R right-hand sides by Jacobi relaxation
 * B^{k+1} = E + rho (F-hat B^k), B^0 = E (sections 3 and 5.1).  Column c has
 * converged at the first k with ||B^k - B^{k-1}||^2 <= rtol^2 ||E_c||^2 (rtol^2
 * when E_c = 0); the solve returns when every column has converged (per
 * instance and column for a group) and B holds that iterate.  With R >= 16
 * and check_every = 1 the test also runs on the device and one iteration is
 * queued ahead of it (skipped on the device once every column has converged);
 * the returned iterate and info are those of the host's test.
 * With opts->refine = 1 (mixed precision): B (FP64 accumulator) starts at 0;
 * each step forms r = E - B + rho (F-hat B) in FP64 from the FP32 operator,
 * stops columns with ||r|| <= rtol ||E||, runs inner_iters Jacobi iterations of
 * (I - rho F16) d = r with the 16-bit operator (FP32 accumulation) and adds d.
 * Warm start (opts->warm = 1; the solve accepts any B^0): per column, the
 * guess G in B is judged against the cold start by their first residuals.
 * Jacobi: ||E + rho F G - G|| against ||rho F E||, both from one iteration;
 * the smaller one's iterate continues (one extra product).  Refinement:
 * ||E - G + rho F32 G|| against ||rho F16 E||; a rejected column restarts
 * from B = 0.  A column whose guess already meets rtol is kept, and when
 * every column's does, the cold-start product is skipped.  info->iters then
 * counts from the chosen start (0 when the guess already meets rtol under
 * refinement).  An R-major B is read in place (the guess may be B itself).
 * rho: device array of N reflectances (original order for RAD_ORDER_ORIGINAL,
 * tree order otherwise), or NULL to use rho_scalar for every facet.  E and B
 * are device arrays of the compute dtype in the layout opts->order names; they
 * may not overlap.  With RAD_ORDER_TREE_RMAJOR, lde and ldb must both equal
 * R rounded up to a multiple of 4.
 * Errors: RAD_EINVAL, RAD_ENOCONV (B holds the last iterate, info filled),
 * RAD_EDEVICE.
 */
rad_status rad_solve(const rad_hmat *H, const void *rho, double rho_scalar, int64_t R, int32_t dtype,
                     const void *E, int64_t lde, void *B, int64_t ldb, const rad_solve_opts *opts,
                     rad_solve_info *info, void *hip_stream);

/*
 * Direct insolation for R point-sun directions (eq. insolation, section 2;
 * used for the right-hand sides of section 5.1):
 *   Q[i, k] = flux * max(0, n_i . s_k) * V_sun(i, k),
 * where V_sun(i, k) = 1 when the ray x_i + t s_k, t > 1e-9, hits no mesh
 * triangle other than facet i.  suns: host array, R x 3 row-major unit vectors
 * (direction towards the sun).  flux = S / d^2 in W/m^2 (d in AU).
 * Q: device, layout named by order (rad_order), compute dtype of H.
 * Runs asynchronously on hip_stream except for the upload of suns.
 * Errors: RAD_EINVAL (null, R < 1, non-finite or zero-length direction,
 * ld < N, dtype mismatch), RAD_ENOMEM, RAD_EDEVICE.
 */
rad_status rad_insolation(const rad_hmat *H, int64_t R, const double *suns, double flux, int32_t dtype,
                          void *Q, int64_t ldq, int32_t order, void *hip_stream);

/*
 * Equilibrium surface temperature for R sun positions (section 5.1 with
 * eqs. 3d-equilbr, Qvis and QIR; subsurface flux H = 0), all on the device:
 *   short wave: (I - albedo F-hat) B_s = albedo Q_dir,   Q_refl = F-hat B_s,
 *               Q_vis = Q_dir + Q_refl;
 *   long wave:  (I - F-hat) B_IR = (1 - albedo) Q_vis,   Q_IR = F-hat B_IR;
 *   T = ( max(0, (1 - albedo) Q_vis + emissivity Q_IR) / (emissivity sigma) )^(1/4),
 * sigma = 5.670374419e-8.  Qdir, T, Qvis, Qir: device arrays of the compute
 * dtype in the layout opts->order names, all with leading dimension ld (N for
 * the column-major layouts, R rounded up to 4 for RAD_ORDER_TREE_RMAJOR); Qvis
 * and Qir may be NULL.  albedo in [0, 1), emissivity in (0, 1].  The two
 * solves use opts (rtol, max_iter, graphs; refine and warm are ignored: both
 * bands run plain Jacobi from B^0 = E); info_sw / info_ir may be NULL.
 * Errors: as rad_solve, plus RAD_EINVAL for albedo/emissivity out of range.
 */
rad_status rad_equilibrium(const rad_hmat *H, int64_t R, int32_t dtype, const void *Qdir, int64_t ld, double albedo,
                           double emissivity, void *T, void *Qvis, void *Qir, const rad_solve_opts *opts,
                           rad_solve_info *info_sw, rad_solve_info *info_ir, void *hip_stream);

typedef struct {
    int64_t n;                 /* facets                                              */
    int64_t n_leaves;          /* quadtree leaves                                     */
    int32_t depth;             /* quadtree depth                                      */
    int32_t dtype;             /* compute/storage dtype                               */
    int64_t n_dense, n_csr, n_lowrank, n_zero; /* final blocks by kind                */
    int64_t bytes_dense, bytes_csr, bytes_lowrank; /* stored value+index bytes by kind */
    int64_t bytes_total;       /* all device bytes of the operator incl. task lists   */
    int64_t nnz_near;          /* stored near-field entries (dense + CSR)             */
    int64_t sum_rank;          /* sum of ranks of low-rank blocks                     */
    int64_t lowrank_elems;     /* sum over low-rank blocks of (m+n) k                 */
    int32_t max_rank;
    double build_seconds;
    double flops_per_rhs;      /* 2 (sum (m+n)k + nnz_near): matvec flops per column   */
    int64_t lowrank_row_elems; /* sum over low-rank blocks of m k (U' factors)        */
    int64_t lowrank_col_elems; /* sum over low-rank blocks of n k (V factors)         */
    int64_t max_panel_cols;    /* widest 64-row tile panel: dense columns plus ranks of the
                                  blocks covering the tile (the longest reduction of the
                                  expansion)                                          */
    int64_t bytes_csr_panels;  /* device copy of the CSR slices as compressed 64-row
                                  panels (values over the union of each tile's nonzero
                                  columns, and their X rows), read by the FP32/FP64
                                  products; included in bytes_total                   */
} rad_hmat_stats;

rad_status rad_hmat_info(const rad_hmat *H, rad_hmat_stats *stats);

/*
 * Diagnostic timing of the multi-RHS kernels of one Jacobi iteration on the
 * caller's stream, measured with HIP events over nrep back-to-back launches of
 * each kernel on the library's own workspace (contents irrelevant):
 *   ms[0] = projections T = V^T X (split-K GEMM),
 *   ms[1] = sum of the split-K partial tiles,
 *   ms[2] = expansion and near field with the fused Jacobi update.
 * Averages per launch in milliseconds.  Requires 16 <= R <= max_rhs.  dtype
 * is the matrix's dtype, or its lowp to time the 16-bit kernels.
 */
rad_status rad_hmat_time_phases(const rad_hmat *H, int64_t R, int32_t dtype, int32_t nrep, void *hip_stream,
                                double *ms);

/*
 * Groups of independent matrices (many craters, each with its own suns) as
 * one block-diagonal operator, so that every product and Jacobi iteration of
 * all instances runs in one launch per kernel over all of their blocks.
 * parts: count built matrices on one device with equal dtype and lowp (not
 * groups).  The group copies their device data (parts may be freed after).
 * Layout: instance k's facets, in its tree order, are rows
 * [offsets[k], offsets[k] + sizes[k]) of an RAD_ORDER_TREE_RMAJOR block of
 * rad_hmat_n(group) rows; offsets are multiples of 64 and the rows between
 * instances are padding that must be zero in E (solves keep them zero).
 * Column c of instance k is right-hand side c of that instance; solves track
 * convergence per (instance, column).  A group supports rad_hmat_matvec and
 * rad_solve with RAD_ORDER_TREE_RMAJOR and 16 <= R <= max_rhs (no warm
 * start); rad_insolation and rad_equilibrium return RAD_EUNSUP (run them on
 * the parts and write into the group layout at the offsets).
 * Errors: RAD_EINVAL, RAD_ENOMEM, RAD_EDEVICE.  *out is NULL on error.
 */
rad_status rad_hmat_group(const rad_hmat *const *parts, int32_t count, int32_t max_rhs, rad_hmat **out);

/*
 * Autotuner of the multi-RHS kernels for R right-hand sides (R >= 16).  The
 * candidates are 64-, 128- or (FP32, R > 128) 256-column workgroup tiles of the
 * expansion, each as a flat grid (one
 * workgroup per 64-row tile and column tile) or as a persistent grid of 1, 2
 * or 4 workgroups per compute unit pulling tiles, in decreasing order of
 * their reduction length, from a work counter.  Each candidate runs nrep
 * Jacobi iterations on the matrix's own blocks (timed with HIP events on
 * hip_stream); the fastest is used by every later product and solve with
 * this R.  cache_path (may be NULL) names a JSON file of earlier results
 * keyed by the matrix signature (dtype, tile count, hash of the tile-cost
 * histogram, compute units) and R: a hit is used without timing (ms = 0);
 * a miss is timed and added.  config (host int32[3], may be NULL) receives
 * (tn, persistent, blocks_per_cu); ms (may be NULL) the chosen time per
 * iteration.  All candidates give identical products.  Synchronises.
 * Errors: RAD_EINVAL (R out of range, bad cache file path), RAD_EDEVICE.
 */
rad_status rad_hmat_autotune(rad_hmat *H, int64_t R, int32_t nrep, const char *cache_path, int32_t *config,
                             double *ms, void *hip_stream);

/* Forces the configuration (tn 64|128|256 (FP32), persistent 0|1, blocks_per_cu 1..64)
 * for R right-hand sides, or reads the one in use (default: tn 64 for
 * R <= 64 else 128, flat grid). */
rad_status rad_hmat_set_config(rad_hmat *H, int64_t R, const int32_t *config);
rad_status rad_hmat_get_config(const rad_hmat *H, int64_t R, int32_t *config);

/* Instances in H (1 for a matrix built by rad_hmat_build; -1 for NULL). */
int32_t rad_hmat_instances(const rad_hmat *H);

/* Row offset and facet count of every instance (host arrays of
 * rad_hmat_instances(H) entries; either may be NULL). */
rad_status rad_hmat_group_layout(const rad_hmat *H, int64_t *offsets, int64_t *sizes);

/* Number of facets N and compute dtype of H (-1 when H is NULL).  For a group,
 * N counts the rows of its layout, padding included. */
int64_t rad_hmat_n(const rad_hmat *H);
int32_t rad_hmat_dtype(const rad_hmat *H);

/* The 16-bit copy's dtype (0: none) and the right-hand sides the workspace
 * holds (max_rhs) of H; -1 when H is NULL. */
int32_t rad_hmat_lowp(const rad_hmat *H);
int32_t rad_hmat_max_rhs(const rad_hmat *H);

/* perm (host, length N): perm[t] = original index of the facet in tree position t. */
rad_status rad_hmat_perm(const rad_hmat *H, int32_t *perm);

/* Releases H and its device memory.  NULL is allowed. */
void rad_hmat_free(rad_hmat *H);

/* Message of the last failed call on this thread ("" if none). */
const char *rad_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RAD_H */
