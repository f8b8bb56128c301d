// Internal declarations of librad (not part of the public C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "rad.h"

namespace rad {

struct Error : std::runtime_error {
    rad_status code;
    Error(rad_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define RAD_HIP(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            throw ::rad::Error(RAD_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define RAD_REQUIRE(cond, msg)                                 \
    do {                                                       \
        if (!(cond))                                           \
            throw ::rad::Error(RAD_EINVAL, std::string(msg));  \
    } while (0)

// Caller-supplied device allocator (rad_allocator) in force on this thread,
// and the device it allocates on: set by AllocScope for the duration of a
// build, load, group or insolation call; nullptr means hipMalloc/hipFree.
struct AllocCtx {
    const rad_allocator *al = nullptr;
    int32_t device = 0;
};
inline AllocCtx &alloc_ctx() {
    static thread_local AllocCtx c;
    return c;
}
struct AllocScope {
    AllocCtx saved;
    AllocScope(const rad_allocator *al, int32_t device) : saved(alloc_ctx()) {
        alloc_ctx().al = (al && al->alloc && al->free) ? al : nullptr;
        alloc_ctx().device = device;
    }
    ~AllocScope() { alloc_ctx() = saved; }
    AllocScope(const AllocScope &) = delete;
    AllocScope &operator=(const AllocScope &) = delete;
};

// Owning device allocation (through the allocator in force when it was made).
template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    const rad_allocator *al = nullptr;
    int32_t dev = 0;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n), al(o.al), dev(o.dev) { o.p = nullptr; o.n = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p; n = o.n; al = o.al; dev = o.dev;
            o.p = nullptr; o.n = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count == 0) return;
        al = alloc_ctx().al;
        dev = alloc_ctx().device;
        if (al) {
            p = (T *)al->alloc(al->ctx, count * sizeof(T), dev);
            if (!p) throw Error(RAD_ENOMEM, "allocator hook returned NULL for " + std::to_string(count * sizeof(T)) + " bytes");
        } else {
            hipError_t e = hipMalloc((void **)&p, count * sizeof(T));
            if (e != hipSuccess) {
                p = nullptr;
                throw Error(RAD_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
            }
        }
        n = count;
    }
    void release() {
        if (p) {
            if (al)
                al->free(al->ctx, p, n * sizeof(T), dev);
            else
                (void)hipFree(p);
        }
        p = nullptr;
        n = 0;
    }
    void upload(const std::vector<T> &h) {
        alloc(h.size());
        if (!h.empty()) RAD_HIP(hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    }
    std::vector<T> download(size_t count) const {
        std::vector<T> h(count);
        if (count) RAD_HIP(hipMemcpy(h.data(), p, count * sizeof(T), hipMemcpyDeviceToHost));
        return h;
    }
    size_t bytes() const { return n * sizeof(T); }
};

// ----------------------------------------------------------------------------
// Quadtree (Algorithm 2) and block pairs (Algorithm 4)
// ----------------------------------------------------------------------------
struct TreeNode {
    int32_t start;        // first facet (tree order)
    int32_t size;         // number of facets
    int32_t depth;
    int32_t first_child;  // index of first child node, children contiguous; -1 for a leaf
    int32_t nchild;
    int32_t leaf_index;   // position among leaves (DFS order), -1 for internal nodes
    int32_t leaf_first;   // first leaf under this node
    int32_t leaf_count;   // leaves under this node
};

enum BlockKind : int8_t { BK_ZERO = 0, BK_DENSE = 1, BK_CSR = 2, BK_LOWRANK = 3, BK_HIER = 4 };

struct BlockPair {
    int32_t I, J;          // tree node indices
    int32_t level;         // 0 = pairs of the root's children
    int32_t first_child;   // -1 for a leaf pair
    int32_t nchild;
    int64_t nnz;           // non-zero entries of F_IJ
    int64_t best_bytes;    // bytes of the chosen representation
    int8_t kind;           // chosen BlockKind
    int32_t rank;          // accepted SVD rank (0: none)
    int64_t svd_bytes;     // bytes of the accepted SVD (-1: none)
    int64_t cand_off;      // offset of the candidate factors in its level pool (doubles)
    int32_t cand_level;
};

// Sketch task for the randomized rank search: one block of F.
struct SketchBlock {
    int32_t i0, m;         // rows [i0, i0+m) in tree order
    int32_t j0, n;         // cols [j0, j0+n)
    int32_t ell;           // sketch width
    int32_t pad_;
    int64_t y_off;         // m x ell (col-major, ld = m) in the Y workspace
    int64_t z_off;         // n x ell (col-major, ld = n) in the Z workspace
    uint64_t seed;
};

enum TaskType : int32_t { TASK_DENSE = 0, TASK_CSR = 1, TASK_LOWRANK = 2 };

// One 64-row tile of the tree order: its packed panel of dense and U' rows
// (64 x kpad, column-major, ld 64, kpad a multiple of 32) with the operand
// row of each panel column in brow[brow_off + k] (X row if >= 0, T row
// -1 - v if < 0), and its CSR tasks [csr_begin, csr_end).
struct TileInfo {
    int64_t panel_off;
    int64_t brow_off;
    int32_t kpad;          // panel columns, a multiple of 32 (the 16-bit chunk width)
    int32_t csr_begin, csr_end;
    int32_t k16;           // panel columns that hold values, rounded up to 16 (the FP32/FP64 chunk)
};

// Batched copy-with-cast of a column-major FP64 block into the value pool.
struct CopyDesc {
    const double *src;
    int64_t dst_off;
    int32_t rows, cols;
    int32_t lds, ldd;
};

// CSR task of one 64-row tile: rows [r_lo, r_hi) of the tile are block rows
// row_off + r; row pointers at aux_off are relative to the value base a_off;
// column indices (local to the block) at a_off - csr_val_start.
struct TileTask {
    int32_t type;
    int32_t ncol;
    int32_t ld;
    int32_t col0;
    int64_t a_off;
    int64_t aux_off;
    int32_t row_off;
    int32_t r_lo, r_hi;
    int32_t full;          // 1: every row in [r_lo, r_hi) holds all ncol columns (values row-major, ld ncol)
};

// A tile's CSR slices as one compressed panel for the multi-RHS kernels:
// 64 x k16 values (column-major, ld 64) over the union of the columns where
// any of the tile's rows has an entry (zeros elsewhere, k16 a multiple of 16),
// and the X row each column multiplies.
struct CsrPanel {
    int64_t panel_off;     // into the compressed-panel values
    int64_t brow_off;      // into their X-row indices
    int32_t k16;           // 0: no CSR slice in this tile
    int32_t pad_;
};

// Segment of a single-RHS tile product: column groups [g0, g1) of the panel
// of tile `tile` (groups of 16 / sizeof(T) columns; g1 = -1: all), the
// tile's CSR tasks when csr is set, partial row sums to slot `slot`.
struct GemvSeg {
    int32_t tile, g0, g1, csr, slot;
};

// Segment of the wide 16-bit tile-pair expansion: kp panel columns of the two
// tiles of a pair, whose 16-bit panels start at element offsets pa and pb
// of the value pool and whose operand-row list starts at br; its partial
// tile goes to slot `slot` (a pair's segments hold consecutive slots, in order).
// The wide BF16 projection runs the same kernel on panels of the 16-bit V
// copy (two 64-row slabs of V_J^T per item, operand rows the facets of the
// column node): its rows 0..63 go to partial tile `slot`, rows 64..127 to
// `slot2` (-1: the item has one slab).
struct WideSeg {
    int64_t pa, pb, br;
    int32_t kp, slot;
    int32_t slot2, pad_;   // pad_ = 1: pa, pb, br index the compressed CSR pair panels
};

// Phase-1 group: all low-rank blocks sharing column node J.
struct ProjGroup {
    int32_t j0, n;         // X rows
    int32_t ktot;          // stacked rank
    int32_t ld;            // leading dimension of stacked V (>= n, multiple of 4)
    int64_t v_off;         // value offset of V_J (n x ktot, col-major)
    int32_t t_off;         // row offset of T_J in T
    int32_t pad_;
};

// Launch configuration of the multi-RHS kernels for one R (rad_hmat_autotune).
struct MmConfig {
    int32_t tn = 128;          // right-hand-side columns per workgroup: 64 or 128
    int32_t persistent = 0;    // 1: fixed grid pulling work items from a counter
    int32_t blocks_per_cu = 2; // grid of the persistent form, per compute unit
};

// Phase-1 split-K work item of the multi-RHS path: rows [krow0, krow0+64) of
// stacked V_J^T times facets [jb, je) of the column node, into partial tile `part`.
struct P1Work {
    int32_t group, krow0, jb, je;
    int32_t part, pad_;
};

// Sum of the partial tiles of one 64-row slab of T.
struct P1Red {
    int32_t t_row0, nrows, part_begin, part_count;
};

// One final block of the partition Algorithm 4 chose (zero blocks are not
// kept), rows [i0, i0 + m) x columns [j0, j0 + n) of the tree order, and
// where its values live: dense values and U' rows in the tile panels (see
// BlockPiece); V columns [vcol, vcol + rank) of the stacked V of projection
// group `group`; CSR row pointers at ptr_off of the CSR pointer pool and
// values at csr_val_start + val_base (column indices at val_base).
struct BlockRec {
    int32_t kind;          // BlockKind: BK_DENSE, BK_CSR or BK_LOWRANK
    int32_t i0, m, j0, n, rank;
    int64_t nnz;
    int32_t group, vcol;
    int64_t ptr_off, val_base;
};

// Rows [r_lo, r_hi) of 64-row tile `tile` of block `block` sit in that tile's
// panel at columns [col, col + width) (width n for dense, rank for low rank).
struct BlockPiece {
    int32_t block, tile, col, r_lo, r_hi;
};

}  // namespace rad

// Opaque matrix handle (device-resident operator + host metadata).
struct rad_hmat {
    rad_allocator allocator{};         // device-memory hook (all null: hipMalloc)
    int device = 0;
    int64_t N = 0;
    int32_t dtype = RAD_F64;   // storage and compute dtype
    int32_t max_rhs = 1;
    int32_t leaf_size = 64;
    std::vector<int32_t> perm;        // tree position -> original facet
    std::vector<rad::TreeNode> nodes;
    rad_hmat_stats stats{};

    // device operator
    rad::DevBuf<int32_t> d_perm;       // tree -> original
    rad::DevBuf<unsigned char> d_vals; // value pool (dtype)
    rad::DevBuf<int32_t> d_csr_idx;    // CSR column indices (local to the block)
    rad::DevBuf<int32_t> d_csr_ptr;    // CSR row pointers per leaf slice
    rad::DevBuf<rad::ProjGroup> d_groups;
    int32_t n_leaves = 0, n_groups = 0, t_rows = 0, t_ld = 0;
    int64_t csr_val_start = 0;
    std::vector<rad::ProjGroup> h_groups;
    rad::DevBuf<rad::TileTask> d_tile_tasks;
    rad::DevBuf<rad::TileInfo> d_tiles;
    rad::DevBuf<int32_t> d_brow;
    int32_t n_tiles = 0;
    rad::DevBuf<rad::P1Work> d_p1work;
    rad::DevBuf<rad::P1Red> d_p1red;
    int32_t n_p1work = 0, n_p1red = 0, n_parts = 0;

    // geometry and ray-casting grid (tree order, FP64)
    rad::DevBuf<double> d_x, d_n, d_a, d_tri, d_cell_zmax;
    rad::DevBuf<int32_t> d_cell_start, d_cell_tris;
    double grid_x0 = 0, grid_y0 = 0, grid_h = 1, grid_ztop = 0;
    int32_t grid_gx = 1, grid_gy = 1;

    // cached HIP graphs of one solve iteration (see api.cpp)
    struct GraphEntry {
        int path;
        int64_t R;
        const void *Bold, *E, *rho;
        void *Bnew;
        double rho_s;
        double *hn;
        const int32_t *stop;
        bool first;
        double rtol2;
        hipGraph_t g;
        hipGraphExec_t ex;
    };
    std::vector<GraphEntry> graphs;
    hipStream_t cap_stream = nullptr;
    // pinned: kNormSlots slots of per-column changes (one per iteration in
    // flight), then ||E||^2
    static constexpr int kNormSlots = 4;
    double *h_norms = nullptr;
    double *d_hnorms = nullptr;  // the same memory as the device addresses it
    hipEvent_t ev[kNormSlots] = {};   // ends of the iterations in flight
    ~rad_hmat();

    // workspace (sized for max_rhs)
    rad::DevBuf<unsigned char> w_x, w_y, w_t, w_b, w_e, w_rho, w_red, w_part, w_q1, w_q2;
    rad::DevBuf<double> w_b64;            // FP64 accumulator of refined solves
    rad::DevBuf<uint16_t> w_x16, w_t16;   // BF16 operand rows (X and T) of the wide 16-bit kernel

    // 16-bit copy of the operator (panels and stacked V, power-of-two scales)
    int32_t lowp = 0;
    rad::DevBuf<uint16_t> d_vals16;
    rad::DevBuf<float> d_pscale, d_tscale;
    rad::DevBuf<double> w_norms;
    rad::DevBuf<int32_t> w_flags;         // per-column choices of warm-started solves
    rad::DevBuf<double> w_thr;            // per-column stopping thresholds of a solve
    rad::DevBuf<double> w_ered;           // per-tile partial sums of E^2 (first iteration)
    rad::DevBuf<int32_t> w_conv;          // per-column "met rtol", then the stop flag

    // group of independent matrices (block diagonal): instance k owns rows
    // [inst_off[k], inst_off[k] + inst_n[k]) and tiles [inst_tile[k], inst_tile[k+1])
    int32_t n_inst = 1;

    // multi-RHS launch configurations (autotuned per R), tile order by
    // decreasing cost and the work counter of the persistent kernels
    std::vector<std::pair<int64_t, rad::MmConfig>> tuned;
    rad::DevBuf<int32_t> d_tile_order, d_queue;
    rad::DevBuf<int32_t> d_p1pairs;  // phase-1 work items taken two at a time (second -1 if single)
    int32_t n_p1pairs = 0;
    // per pair: the T row its slabs start at when each slab is reduced by that
    // one work item (the kernel then writes T itself), else -1; and the slabs
    // of several work items, which the split-K sum of the FP32/FP64 path adds
    rad::DevBuf<int32_t> d_p1direct;
    rad::DevBuf<rad::P1Red> d_p1red_multi;
    int32_t n_p1red_multi = 0;
    // the CSR slices of every tile as compressed panels (multi-RHS FP32/FP64
    // expansion); n_cpan = 0: none, the kernels expand the CSR rows themselves
    rad::DevBuf<rad::CsrPanel> d_cpan;
    rad::DevBuf<unsigned char> d_cvals;
    rad::DevBuf<int32_t> d_cbrow;
    int32_t n_cpan = 0;
    int64_t cpan_elems = 0;
    // the same for the wide BF16 expansion, one panel per tile pair over the
    // union of both tiles' columns (16-bit chunk layout; segments with pad_ = 1
    // read these buffers); wide_csr = 1: every CSR slice lies in a tile pair
    rad::DevBuf<uint16_t> d_cvals16;
    rad::DevBuf<int32_t> d_cbrow16;
    int32_t wide_csr = 0;
    // wide 16-bit expansion: first tiles of consecutive tile pairs with identical
    // operand-row lists (one 128-row workgroup each), and the remaining tiles
    rad::DevBuf<int32_t> d_wpairs, d_wsingles;
    int32_t n_wpairs = 0, n_wsingles = 0;
    // single-RHS products: panel segments (longest first), each tile's slots
    // [gseg_of_tile[t], gseg_of_tile[t+1]), and the segments' partial row sums
    rad::DevBuf<int32_t> d_pwide;        // (group, column) items of k_proj_wide (groups of n >= kProjWideN)
    int32_t n_pwide = 0;
    rad::DevBuf<int32_t> d_pcols;        // (group, column) items of k_proj_cols (the other groups)
    int32_t n_pcols = 0;
    rad::DevBuf<rad::GemvSeg> d_gsegs;
    rad::DevBuf<int32_t> d_gseg_of_tile;
    int32_t n_gsegs = 0;
    rad::DevBuf<unsigned char> w_gpart;
    rad::DevBuf<rad::WideSeg> d_wsegs;    // the pairs' reduction segments (index = partial slot)
    int32_t n_wsegs = 0;
    rad::DevBuf<int32_t> d_wseg_order;    // their launch table (xcd_region_order)
    int32_t n_wseg_blocks = 0;
    // wide BF16 projection: V panels (64 rows x 32 facets per chunk), the
    // facet lists of the column nodes, the items (longest first) and the sums
    // of partial tiles per 64-row slab of T
    rad::DevBuf<uint16_t> d_vpan16;
    rad::DevBuf<int32_t> d_pbrow;
    rad::DevBuf<rad::WideSeg> d_psegs;
    rad::DevBuf<int32_t> d_pseg_order;
    rad::DevBuf<rad::P1Red> d_wpred;
    int32_t n_psegs = 0, n_pseg_blocks = 0, n_wpred = 0;
    rad::DevBuf<int32_t> d_wslot;         // pair p's segments' partial tiles: slots [wslot[p], wslot[p+1])
    rad::DevBuf<float> w_wpart;           // partial tiles of the segments (128 x 256 FP32 each)
    int32_t n_cu = 256;
    std::string sched_sig;           // dtype, tile count and tile-cost histogram hash (autotuner cache key)
    std::vector<int64_t> inst_off, inst_n;
    std::vector<int32_t> inst_tile;
    rad::DevBuf<int32_t> d_inst_tile;

    // final blocks and their places in the layout (rad_hmat_export)
    std::vector<rad::BlockRec> blocks;
    std::vector<rad::BlockPiece> pieces;

    // allocator hook of this matrix, or nullptr
    const rad_allocator *hook() const { return allocator.alloc && allocator.free ? &allocator : nullptr; }
};

namespace rad {

// thread-local error text
void set_error(const std::string &msg);

// Allocates the solve/matvec workspace of H for max_rhs right-hand sides.
void alloc_workspace(rad_hmat *H);

// Runs f, translating exceptions into a status code and the thread's last error.
template <class F>
rad_status guard(F &&f) {
    try {
        f();
        return RAD_OK;
    } catch (const Error &e) {
        set_error(e.what());
        return e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return RAD_ENOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return RAD_EDEVICE;
    }
}

// One-sided Jacobi SVD of the l x l column-major matrix A (host, FP64), in
// place: columns of A become U Sigma sorted by decreasing norm, V the right
// singular vectors, sv the singular values.
void jacobi_svd(int l, std::vector<double> &A, std::vector<double> &V, std::vector<double> &sv);

// builder entry (build.cpp)
// tree_dims: 2 = quadtree on (x, y), 3 = octree on (x, y, z)
void build_hmat(rad_hmat *H, const double *verts, int64_t nv, const int32_t *faces, int64_t nf,
                const rad_build_opts &o, int tree_dims = 2);
// block export, save and load (serialize.cpp)
void export_blocks(const rad_hmat *H, const char *path);
void save_hmat(const rad_hmat *H, const char *path);
void load_hmat(rad_hmat *H, const char *path, int32_t device, int32_t max_rhs);
// G = the operator of H with its values in dtype (same structure and layout)
void convert_hmat(rad_hmat *G, const rad_hmat *H, int32_t dtype, int32_t max_rhs);
// the same from centroids, unit normals, areas and optional triangles (N x 9)
void build_hmat_facets(rad_hmat *H, const double *x, const double *n, const double *area, int64_t N,
                       const double *tri_verts, const rad_build_opts &o, int tree_dims);

// device geometry used by the build kernels (tree order, FP64)
struct DevGeom {
    const double *x;   // N x 3
    const double *n;   // N x 3
    const double *a;   // N
    const uint32_t *vis;  // optional visibility bitmap (N x N bits, row-major), nullptr = back-face only
    int64_t vis_words_per_row;
};

// build kernels (build_kernels.hip)
void launch_leaf_nnz(const DevGeom &g, const int32_t *pairs /*4 per pair: i0,m,j0,n*/, int64_t npairs,
                     int64_t *nnz_out, hipStream_t s);
void launch_fill_rademacher(double *Z, const SketchBlock *blocks, int32_t nblocks, hipStream_t s);
void launch_sketch_apply(const DevGeom &g, const SketchBlock *blocks, int32_t nblocks, int transpose,
                         const double *in, double *out, int32_t max_rows, int32_t max_ell, hipStream_t s);
void launch_cgs2(double *Ybase, const SketchBlock *blocks, int32_t nblocks, int use_z, double *Rout,
                 const int64_t *roff, hipStream_t s);
void launch_cgs2_tall(double *base, const SketchBlock *blocks, int32_t nblocks, int use_z, double *Rout,
                      const int64_t *roff, int32_t max_rows, int32_t max_ell, double *part, double *normpart,
                      double *norm0part, hipStream_t s);
void launch_small_gemm(const double *Qbase, const SketchBlock *blocks, const int64_t *small_off,
                       const double *small, const int32_t *qk, const int64_t *out_off, double *out,
                       int32_t nblocks, int use_z, int32_t max_rows, hipStream_t s);
void launch_dense_fill(const DevGeom &g, const int32_t *tiles /*6 per: i0,m,j0,n,ld,pad*/,
                       const int64_t *offs, int64_t ntiles, void *vals, int32_t dtype, hipStream_t s);
void launch_csr_count(const DevGeom &g, const int32_t *tiles, int64_t ntiles, int32_t *row_counts,
                      const int64_t *row_offs, hipStream_t s);
void launch_csr_fill(const DevGeom &g, const int32_t *tiles, int64_t ntiles, const int32_t *rowptr,
                     const int64_t *row_offs, const int64_t *val_base, void *vals, int32_t *cols,
                     int32_t dtype, hipStream_t s);
void launch_copy_batched(const CopyDesc *d, int64_t n, void *vals, int32_t dtype, hipStream_t s);
// out[dst[i]] = vals[i] for i < n with dst[i] >= 0 (values of the matrix's dtype)
void launch_csr_panel_scatter(const void *vals, const int64_t *dst, int64_t n, void *out, int32_t dtype,
                              hipStream_t s);
// the same from FP32 values into BF16
void launch_csr_panel_scatter16(const float *vals, const int64_t *dst, int64_t n, uint16_t *out, hipStream_t s);
// ray casting (raycast.hip)
void build_grid(rad_hmat *H, const std::vector<double> &tri);
// visibility bits of rows [row0, row0 + rows) of the N x N pair matrix
void launch_vis_grid(const rad_hmat *H, uint32_t *bits, int64_t wpr, int64_t row0, int64_t rows, hipStream_t s);
void launch_insolation(const rad_hmat *H, const double *suns_dev, int64_t R, double flux, int32_t dtype, void *Q,
                       int64_t ldq, int32_t order, hipStream_t s);

// matvec / solve kernels (matvec_kernels.hip)
void mv_gather(const rad_hmat *H, const void *src, int64_t lds, void *dst, int64_t ldd, int64_t R, hipStream_t s);
void mv_scatter(const rad_hmat *H, const void *src, int64_t lds, void *dst, int64_t ldd, int64_t R, hipStream_t s);
void mv_apply(const rad_hmat *H, const void *X, int64_t ldx, void *Y, int64_t ldy, int64_t R, hipStream_t s);
// the same product with the projections T in caller-chosen device memory
// (t_ld x R values of the matrix's dtype)
void mv_apply_ws(const rad_hmat *H, const void *X, int64_t ldx, void *Y, int64_t ldy, int64_t R, void *Tb,
                 hipStream_t s);
// Device address of the file-scope scratch array of the allocation-free
// product on `device` (which must be current); looked up once per device.
constexpr size_t kStaticScratchBytes = size_t(8) << 20;
void *static_scratch(int device);
void col_norms2(const rad_hmat *H, const void *E, int64_t ld, int64_t R, double *out, hipStream_t s);
size_t reduction_doubles(int64_t R);

// elementwise operations on N x R blocks (column-major or R-major, leading dimension ld)
enum EwOp : int32_t {
    EW_SCALE = 0,   // z = a x
    EW_ADD = 1,     // z = x + y
    EW_TEMP = 2     // z = (max(0, a x + b y) / c)^(1/4)
};
void launch_elementwise(const rad_hmat *H, int32_t op, double a, double b, double c, const void *x, const void *y,
                        void *z, int64_t R, int64_t ld, bool rmajor, hipStream_t s);

// multi-RHS path (matmat_kernels.hip), R-major tree-ordered buffers
constexpr int64_t kMfmaMinRhs = 16;
// column nodes of at least this many facets project with one workgroup per V column
constexpr int32_t kProjWideN = 4096;
int64_t mm_ldr(int64_t R);
int mm_part_rows();
void mm_to_rmajor(const rad_hmat *H, const void *src, int64_t lds, bool permute, void *dst, int64_t ldr, int64_t R,
                  hipStream_t s);
void mm_from_rmajor(const rad_hmat *H, const void *src, int64_t ldr, bool permute, void *dst, int64_t ldd, int64_t R,
                    hipStream_t s);
void mm_apply(const rad_hmat *H, const void *X, void *Y, int64_t ldr, int64_t R, hipStream_t s);
void mm_col_norms2(const rad_hmat *H, const void *E, int64_t ldr, int64_t R, double *out, hipStream_t s);
// Device-side stopping test of a Jacobi solve, run on the sums of a column
// reduction (out) right after it:
// mode 1 (out = squared changes): conv[c] |= out[c] <= thr[c] (skipped while
//        *stop is set);
// mode 2 (out = ||E||^2, dn given): thr[c] = rtol2 out[c] (rtol2 when 0),
//        conv[c] = dn[c] <= thr[c];
// then stop = all(conv[0..nc)).  hdn (and hen, mode 2), when given: pinned
// host memory that receives the squared changes (and ||E||^2) directly.
struct ConvTest {
    int mode;
    int nc;
    const double *dn;
    double *thr;
    double rtol2;
    int32_t *conv, *stop;
    double *hdn = nullptr, *hen = nullptr;
};

void mm_jacobi_step(const rad_hmat *H, const void *E, const void *rho, double rho_scalar, const void *Bold, void *Bnew,
                    int64_t ldr, int64_t R, double *norms, hipStream_t s, const int32_t *stop = nullptr,
                    double *enorms = nullptr, const ConvTest *test = nullptr);
// The same iteration on the single-RHS kernels (column-major tree order,
// leading dimension ld for E, B_old and B_new): the Jacobi update, the squared
// changes (and ||E||^2 with enorms) are fused into the tile kernel.
void mv_jacobi_step(const rad_hmat *H, const void *E, const void *rho, double rho_scalar, const void *Bold, void *Bnew,
                    int64_t ld, int64_t R, double *norms, hipStream_t s, const int32_t *stop = nullptr,
                    double *enorms = nullptr, const ConvTest *test = nullptr);
size_t mm_reduction_doubles_for(const rad_hmat *H, int64_t R);
rad::MmConfig mm_config(const rad_hmat *H, int64_t R);
void mm_prepare_schedule(rad_hmat *H);
// times every candidate configuration of one Jacobi iteration for R columns
// and records the fastest in H->tuned; returns (config, ms) of every candidate
std::vector<std::pair<rad::MmConfig, double>> mm_autotune(rad_hmat *H, int64_t R, int nrep, hipStream_t s);
void mm_reduce_cols(const rad_hmat *H, const double *partial, int nparts, int64_t R, double *out, hipStream_t s,
                    const int32_t *stop = nullptr, const ConvTest *test = nullptr);
// thr[c] = rtol2 enorm2[c] (rtol2 when 0); clears conv[0..nc) and stop
void conv_init(const double *enorm2, double rtol2, int64_t nc, double *thr, int32_t *conv, int32_t *stop,
               hipStream_t s);

// blocks of R columns in the solve's working layout (R-major with ld when
// rmajor, else column-major with ld) for Chebyshev and GMRES (krylov.hip);
// column sums per 64-row tile in part (tile-major), then in a fixed order
void krylov_cheb_init(const rad_hmat *H, bool rmajor, int64_t ld, int64_t R, double rho, double theta, const void *Y,
                      void *r, void *d, double *part, hipStream_t s);
void krylov_cheb_step(const rad_hmat *H, bool rmajor, int64_t ld, int64_t R, double rho, double a, double b,
                      const void *Y, void *B, void *r, void *d, double *part, hipStream_t s);
void krylov_apply_a(const rad_hmat *H, bool rmajor, int64_t ld, int64_t R, double rho, const void *rhov, const void *e,
                    const void *v, const void *Y, void *w, hipStream_t s);
void krylov_dots(const rad_hmat *H, bool rmajor, int64_t ld, int64_t R, const void *V, int64_t vstride, int nv,
                 const void *w, double *part, double *out, hipStream_t s);
void krylov_combine(const rad_hmat *H, bool rmajor, int64_t ld, int64_t R, const void *V, int64_t vstride, int nv,
                    const double *h, double sign, void *w, hipStream_t s);
void krylov_scale(const rad_hmat *H, bool rmajor, int64_t ld, int64_t R, const void *w, const double *nrm2, void *v,
                  hipStream_t s);

// 16-bit operator (lowp_kernels.hip)
void ir_select(const rad_hmat *H, double *B64, float *B32, float *r, const float *E, const int32_t *flag, int64_t ldr,
               int64_t R, hipStream_t s);
void ir_load(const rad_hmat *H, double *B64, float *B32, const float *B0, int64_t ldr, int64_t R, hipStream_t s);
void select_columns(const rad_hmat *H, const void *a, const void *b, const int32_t *flag, void *out, int64_t ld,
                    int64_t R, bool rmajor, hipStream_t s);
void lowp_time_phases(const rad_hmat *H, int64_t R, int nrep, hipStream_t s, double *ms);
void lowp_convert(rad_hmat *H, hipStream_t s);
void lowp_prepare_proj(rad_hmat *H);
// Launch table for independent work items on the 8 XCDs (workgroup i of a
// 1-D grid runs on XCD i mod 8).  The items of one group read the same
// operand rows: they go to one XCD back to back, so that its L2 serves those
// rows once.  Groups are dealt, longest item first, to the XCD with the least
// work so far; entry 8 s + x is the s-th item of XCD x (-1: none, the
// workgroup exits).
std::vector<int32_t> xcd_launch_order(const std::vector<std::vector<int32_t>> &groups,
                                      const std::vector<int64_t> &cost);
// Launch table that keeps the order of the groups: they are cut into 8
// contiguous runs of near-equal cost, run x going to XCD x in order (layout of
// the table as for xcd_launch_order).
std::vector<int32_t> xcd_region_order(const std::vector<std::vector<int32_t>> &groups,
                                      const std::vector<int64_t> &cost);
void lowp_step(const rad_hmat *H, const void *E, const void *rho, double rho_s, const void *Bold, void *Bnew,
               int64_t ldr, int64_t R, double *norms, hipStream_t s);
void ir_residual(const rad_hmat *H, const float *E, const double *B64, const float *FB, const float *rho, double rho_s,
                 float *r, int64_t ldr, int64_t R, double *norms, hipStream_t s);
void ir_update(const rad_hmat *H, double *B64, const float *d, float *B32, int64_t ldr, int64_t R, hipStream_t s);
void mm_time_phases(const rad_hmat *H, int64_t R, int nrep, hipStream_t s, double *ms);

}  // namespace rad
