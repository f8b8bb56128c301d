// Files of a compressed operator: the block export (host blocks of the
// partition of Algorithm 4, FP64) and the save/load of the whole device
// layout, so that a matrix assembled once is used elsewhere.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <memory>

#include "rad_internal.h"

namespace rad {

namespace {

struct FileCloser {
    void operator()(std::FILE *f) const {
        if (f) std::fclose(f);
    }
};
using File = std::unique_ptr<std::FILE, FileCloser>;

File open_file(const char *path, const char *mode) {
    RAD_REQUIRE(path != nullptr && path[0] != '\0', "null or empty path");
    File f(std::fopen(path, mode));
    if (!f) throw Error(RAD_EDEVICE, std::string("cannot open ") + path);
    return f;
}

struct Writer {
    std::FILE *f;
    void raw(const void *p, size_t bytes) {
        if (bytes && std::fwrite(p, 1, bytes, f) != bytes) throw Error(RAD_EDEVICE, "write failed");
    }
    template <class T>
    void val(const T &v) {
        raw(&v, sizeof(T));
    }
    template <class T>
    void vec(const std::vector<T> &v) {
        val<uint64_t>(v.size());
        raw(v.data(), v.size() * sizeof(T));
    }
    template <class T>
    void dev(const DevBuf<T> &b) {
        val<uint64_t>(b.n);
        if (b.n) {
            std::vector<T> h = b.download(b.n);
            raw(h.data(), b.n * sizeof(T));
        }
    }
};

struct Reader {
    std::FILE *f;
    void raw(void *p, size_t bytes) {
        if (bytes && std::fread(p, 1, bytes, f) != bytes) throw Error(RAD_EINVAL, "file ends early");
    }
    template <class T>
    T val() {
        T v;
        raw(&v, sizeof(T));
        return v;
    }
    uint64_t count(size_t elem) {
        const uint64_t n = val<uint64_t>();
        RAD_REQUIRE(n < ((uint64_t)1 << 40) / elem, "implausible array length in file");
        return n;
    }
    template <class T>
    void vec(std::vector<T> &v) {
        v.resize(count(sizeof(T)));
        raw(v.data(), v.size() * sizeof(T));
    }
    template <class T>
    void dev(DevBuf<T> &b) {
        std::vector<T> h(count(sizeof(T)));
        raw(h.data(), h.size() * sizeof(T));
        b.upload(h);
    }
};

// value i of the pool, converted to FP64 (exactly)
inline double pool_value(const std::vector<unsigned char> &pool, int32_t dtype, int64_t i) {
    if (dtype == RAD_F64) {
        double v;
        std::memcpy(&v, pool.data() + i * 8, 8);
        return v;
    }
    float v;
    std::memcpy(&v, pool.data() + i * 4, 4);
    return v;
}

// values [off, off + count) of the pool, converted to FP64
std::vector<double> pool_values(const std::vector<unsigned char> &pool, int32_t dtype, int64_t off, int64_t count) {
    std::vector<double> out(count);
    for (int64_t i = 0; i < count; ++i) out[i] = pool_value(pool, dtype, off + i);
    return out;
}

constexpr char kExportMagic[8] = {'R', 'A', 'D', 'H', 'B', 'L', 'K', 'S'};
constexpr char kSaveMagic[8] = {'R', 'A', 'D', 'H', 'M', 'A', 'T', 'X'};
constexpr uint32_t kSaveVersion = 1;

// sizes of every raw structure in a saved file: a file whose sizes differ
// comes from another build of the library and is refused
std::vector<uint32_t> layout_sizes() {
    return {(uint32_t)sizeof(rad_hmat_stats), (uint32_t)sizeof(TreeNode), (uint32_t)sizeof(ProjGroup),
            (uint32_t)sizeof(TileTask),      (uint32_t)sizeof(TileInfo), (uint32_t)sizeof(P1Work),
            (uint32_t)sizeof(P1Red),         (uint32_t)sizeof(MmConfig), (uint32_t)sizeof(BlockRec),
            (uint32_t)sizeof(BlockPiece)};
}

}  // namespace

void export_blocks(const rad_hmat *H, const char *path) {
    RAD_REQUIRE(H->n_inst == 1, "export takes a single matrix, not a group");
    const int es = H->dtype == RAD_F64 ? 8 : 4;
    RAD_HIP(hipSetDevice(H->device));
    std::vector<unsigned char> pool = H->d_vals.download(H->d_vals.n);
    std::vector<int32_t> cptr = H->d_csr_ptr.download(H->d_csr_ptr.n);
    std::vector<int32_t> cidx = H->d_csr_idx.download(H->d_csr_idx.n);
    std::vector<TileInfo> tiles = H->d_tiles.download((size_t)H->n_tiles);
    const int64_t npool = (int64_t)pool.size() / es;
    // the pieces of every block (its rows spread over 64-row tile panels)
    std::vector<std::vector<const BlockPiece *>> by_block(H->blocks.size());
    for (const BlockPiece &pc : H->pieces) by_block[pc.block].push_back(&pc);

    File f = open_file(path, "wb");
    Writer w{f.get()};
    w.raw(kExportMagic, 8);
    w.val<uint32_t>(1);
    w.val<int32_t>(H->dtype);
    w.val<int64_t>(H->N);
    w.val<int64_t>((int64_t)H->blocks.size());
    w.raw(H->perm.data(), H->perm.size() * sizeof(int32_t));
    for (size_t b = 0; b < H->blocks.size(); ++b) {
        const BlockRec &r = H->blocks[b];
        w.val<int32_t>(r.kind);
        w.val<int32_t>(r.i0);
        w.val<int32_t>(r.m);
        w.val<int32_t>(r.j0);
        w.val<int32_t>(r.n);
        w.val<int32_t>(r.rank);
        if (r.kind == BK_CSR) {
            const int32_t *p = cptr.data() + r.ptr_off;
            const int64_t nnz = p[r.m] - p[0];
            w.val<int64_t>(nnz);
            for (int32_t i = 0; i <= r.m; ++i) w.val<int32_t>(p[i] - p[0]);
            const int64_t base = r.val_base + p[0];
            RAD_REQUIRE(base + nnz <= (int64_t)cidx.size(), "CSR indices out of range");
            w.raw(cidx.data() + base, nnz * sizeof(int32_t));
            std::vector<double> v = pool_values(pool, H->dtype, H->csr_val_start + base, nnz);
            w.raw(v.data(), nnz * sizeof(double));
            continue;
        }
        const int32_t width = r.kind == BK_DENSE ? r.n : r.rank;
        w.val<int64_t>(r.nnz);
        // dense values or U' (m x width, column-major) from the tile panels
        std::vector<double> A((size_t)r.m * width, 0.0);
        for (const BlockPiece *pc : by_block[b]) {
            const TileInfo &ti = tiles[pc->tile];
            for (int32_t k = 0; k < width; ++k)
                for (int32_t rr = pc->r_lo; rr < pc->r_hi; ++rr) {
                    const int64_t src = ti.panel_off + (int64_t)(pc->col + k) * 64 + rr;
                    RAD_REQUIRE(src < npool, "panel offset out of range");
                    const int64_t row = (int64_t)pc->tile * 64 + rr - r.i0;
                    A[row + (int64_t)k * r.m] = pool_value(pool, H->dtype, src);
                }
        }
        w.raw(A.data(), A.size() * sizeof(double));
        if (r.kind == BK_LOWRANK) {
            const ProjGroup &g = H->h_groups[r.group];
            std::vector<double> V((size_t)r.n * r.rank);
            for (int32_t k = 0; k < r.rank; ++k) {
                std::vector<double> col = pool_values(pool, H->dtype, g.v_off + (int64_t)(r.vcol + k) * g.ld, r.n);
                std::copy(col.begin(), col.end(), V.begin() + (int64_t)k * r.n);
            }
            w.raw(V.data(), V.size() * sizeof(double));
        }
    }
    if (std::fflush(f.get()) != 0) throw Error(RAD_EDEVICE, "write failed");
}

void save_hmat(const rad_hmat *H, const char *path) {
    RAD_HIP(hipSetDevice(H->device));
    File f = open_file(path, "wb");
    Writer w{f.get()};
    w.raw(kSaveMagic, 8);
    w.val<uint32_t>(kSaveVersion);
    w.vec(layout_sizes());
    w.val<int64_t>(H->N);
    w.val<int32_t>(H->dtype);
    w.val<int32_t>(H->max_rhs);
    w.val<int32_t>(H->leaf_size);
    w.vec(H->perm);
    w.vec(H->nodes);
    w.val(H->stats);
    w.dev(H->d_perm);
    w.dev(H->d_vals);
    w.dev(H->d_csr_idx);
    w.dev(H->d_csr_ptr);
    w.dev(H->d_groups);
    w.val<int32_t>(H->n_leaves);
    w.val<int32_t>(H->n_groups);
    w.val<int32_t>(H->t_rows);
    w.val<int32_t>(H->t_ld);
    w.val<int64_t>(H->csr_val_start);
    w.vec(H->h_groups);
    w.dev(H->d_tile_tasks);
    w.dev(H->d_tiles);
    w.dev(H->d_brow);
    w.val<int32_t>(H->n_tiles);
    w.dev(H->d_p1work);
    w.dev(H->d_p1red);
    w.val<int32_t>(H->n_p1work);
    w.val<int32_t>(H->n_p1red);
    w.val<int32_t>(H->n_parts);
    w.dev(H->d_x);
    w.dev(H->d_n);
    w.dev(H->d_a);
    w.dev(H->d_tri);
    w.dev(H->d_cell_zmax);
    w.dev(H->d_cell_start);
    w.dev(H->d_cell_tris);
    w.val(H->grid_x0);
    w.val(H->grid_y0);
    w.val(H->grid_h);
    w.val(H->grid_ztop);
    w.val<int32_t>(H->grid_gx);
    w.val<int32_t>(H->grid_gy);
    w.val<int32_t>(H->lowp);
    w.dev(H->d_vals16);
    w.dev(H->d_pscale);
    w.dev(H->d_tscale);
    w.val<int32_t>(H->n_inst);
    w.vec(H->inst_off);
    w.vec(H->inst_n);
    w.vec(H->inst_tile);
    w.dev(H->d_inst_tile);
    std::vector<int64_t> tuned_r;
    std::vector<MmConfig> tuned_c;
    for (const auto &e : H->tuned) {
        tuned_r.push_back(e.first);
        tuned_c.push_back(e.second);
    }
    w.vec(tuned_r);
    w.vec(tuned_c);
    w.vec(H->blocks);
    w.vec(H->pieces);
    w.raw(kSaveMagic, 8);   // end marker
    if (std::fflush(f.get()) != 0) throw Error(RAD_EDEVICE, "write failed");
}

void load_hmat(rad_hmat *H, const char *path, int32_t device, int32_t max_rhs) {
    File f = open_file(path, "rb");
    Reader r{f.get()};
    char magic[8];
    r.raw(magic, 8);
    RAD_REQUIRE(std::memcmp(magic, kSaveMagic, 8) == 0, std::string(path) + " is not a saved rad_hmat");
    RAD_REQUIRE(r.val<uint32_t>() == kSaveVersion, std::string(path) + " has another format version");
    std::vector<uint32_t> sizes;
    r.vec(sizes);
    RAD_REQUIRE(sizes == layout_sizes(), std::string(path) + " was written by a build with other structure sizes");
    H->device = device;
    RAD_HIP(hipSetDevice(device));
    H->N = r.val<int64_t>();
    H->dtype = r.val<int32_t>();
    const int32_t saved_rhs = r.val<int32_t>();
    H->max_rhs = max_rhs > 0 ? max_rhs : saved_rhs;
    H->leaf_size = r.val<int32_t>();
    RAD_REQUIRE(H->N >= 1 && (H->dtype == RAD_F64 || H->dtype == RAD_F32) && H->max_rhs >= 1, "bad header values");
    r.vec(H->perm);
    r.vec(H->nodes);
    H->stats = r.val<rad_hmat_stats>();
    r.dev(H->d_perm);
    r.dev(H->d_vals);
    r.dev(H->d_csr_idx);
    r.dev(H->d_csr_ptr);
    r.dev(H->d_groups);
    H->n_leaves = r.val<int32_t>();
    H->n_groups = r.val<int32_t>();
    H->t_rows = r.val<int32_t>();
    H->t_ld = r.val<int32_t>();
    H->csr_val_start = r.val<int64_t>();
    r.vec(H->h_groups);
    r.dev(H->d_tile_tasks);
    r.dev(H->d_tiles);
    r.dev(H->d_brow);
    H->n_tiles = r.val<int32_t>();
    r.dev(H->d_p1work);
    r.dev(H->d_p1red);
    H->n_p1work = r.val<int32_t>();
    H->n_p1red = r.val<int32_t>();
    H->n_parts = r.val<int32_t>();
    r.dev(H->d_x);
    r.dev(H->d_n);
    r.dev(H->d_a);
    r.dev(H->d_tri);
    r.dev(H->d_cell_zmax);
    r.dev(H->d_cell_start);
    r.dev(H->d_cell_tris);
    H->grid_x0 = r.val<double>();
    H->grid_y0 = r.val<double>();
    H->grid_h = r.val<double>();
    H->grid_ztop = r.val<double>();
    H->grid_gx = r.val<int32_t>();
    H->grid_gy = r.val<int32_t>();
    H->lowp = r.val<int32_t>();
    r.dev(H->d_vals16);
    r.dev(H->d_pscale);
    r.dev(H->d_tscale);
    H->n_inst = r.val<int32_t>();
    r.vec(H->inst_off);
    r.vec(H->inst_n);
    r.vec(H->inst_tile);
    r.dev(H->d_inst_tile);
    std::vector<int64_t> tuned_r;
    std::vector<MmConfig> tuned_c;
    r.vec(tuned_r);
    r.vec(tuned_c);
    RAD_REQUIRE(tuned_r.size() == tuned_c.size(), "bad launch configuration table");
    for (size_t i = 0; i < tuned_r.size(); ++i) H->tuned.push_back({tuned_r[i], tuned_c[i]});
    r.vec(H->blocks);
    r.vec(H->pieces);
    r.raw(magic, 8);
    RAD_REQUIRE(std::memcmp(magic, kSaveMagic, 8) == 0, std::string(path) + " is truncated or corrupt");
    RAD_REQUIRE((int64_t)H->perm.size() == H->N && H->d_tiles.n == (size_t)H->n_tiles &&
                    H->d_p1work.n == (size_t)H->n_p1work && H->h_groups.size() == (size_t)H->n_groups,
                "inconsistent table sizes in file");
}

namespace {

__global__ void k_cast_f32_f64(const float *src, double *dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (double)src[i];
}

__global__ void k_cast_f64_f32(const double *src, float *dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

template <class T>
void copy_dev(DevBuf<T> &dst, const DevBuf<T> &src) {
    dst.alloc(src.n);
    if (src.n) RAD_HIP(hipMemcpy(dst.p, src.p, src.n * sizeof(T), hipMemcpyDeviceToDevice));
}

}  // namespace

void convert_hmat(rad_hmat *G, const rad_hmat *H, int32_t dtype, int32_t max_rhs) {
    RAD_REQUIRE(H->n_inst == 1, "convert takes a single matrix, not a group");
    RAD_REQUIRE(dtype == RAD_F64 || dtype == RAD_F32, "dtype must be RAD_F64 or RAD_F32");
    RAD_HIP(hipSetDevice(H->device));
    G->device = H->device;
    G->N = H->N;
    G->dtype = dtype;
    G->max_rhs = max_rhs > 0 ? max_rhs : H->max_rhs;
    G->leaf_size = H->leaf_size;
    G->perm = H->perm;
    G->nodes = H->nodes;
    G->stats = H->stats;
    copy_dev(G->d_perm, H->d_perm);
    // the value pool, element by element in the new precision (same offsets)
    const int64_t nvals = (int64_t)(H->d_vals.n / (H->dtype == RAD_F64 ? 8 : 4));
    G->d_vals.alloc((size_t)nvals * (dtype == RAD_F64 ? 8 : 4));
    if (dtype == H->dtype) {
        RAD_HIP(hipMemcpy(G->d_vals.p, H->d_vals.p, H->d_vals.n, hipMemcpyDeviceToDevice));
    } else {
        const unsigned blocks = (unsigned)std::min<int64_t>((nvals + 255) / 256, 65536);
        if (dtype == RAD_F64)
            hipLaunchKernelGGL(k_cast_f32_f64, dim3(blocks), dim3(256), 0, nullptr, (const float *)H->d_vals.p,
                               (double *)G->d_vals.p, nvals);
        else
            hipLaunchKernelGGL(k_cast_f64_f32, dim3(blocks), dim3(256), 0, nullptr, (const double *)H->d_vals.p,
                               (float *)G->d_vals.p, nvals);
        RAD_HIP(hipGetLastError());
        RAD_HIP(hipDeviceSynchronize());
    }
    copy_dev(G->d_csr_idx, H->d_csr_idx);
    copy_dev(G->d_csr_ptr, H->d_csr_ptr);
    copy_dev(G->d_groups, H->d_groups);
    G->n_leaves = H->n_leaves;
    G->n_groups = H->n_groups;
    G->t_rows = H->t_rows;
    G->t_ld = H->t_ld;
    G->csr_val_start = H->csr_val_start;
    G->h_groups = H->h_groups;
    copy_dev(G->d_tile_tasks, H->d_tile_tasks);
    copy_dev(G->d_tiles, H->d_tiles);
    copy_dev(G->d_brow, H->d_brow);
    G->n_tiles = H->n_tiles;
    copy_dev(G->d_p1work, H->d_p1work);
    copy_dev(G->d_p1red, H->d_p1red);
    G->n_p1work = H->n_p1work;
    G->n_p1red = H->n_p1red;
    G->n_parts = H->n_parts;
    copy_dev(G->d_x, H->d_x);
    copy_dev(G->d_n, H->d_n);
    copy_dev(G->d_a, H->d_a);
    copy_dev(G->d_tri, H->d_tri);
    copy_dev(G->d_cell_zmax, H->d_cell_zmax);
    copy_dev(G->d_cell_start, H->d_cell_start);
    copy_dev(G->d_cell_tris, H->d_cell_tris);
    G->grid_x0 = H->grid_x0;
    G->grid_y0 = H->grid_y0;
    G->grid_h = H->grid_h;
    G->grid_ztop = H->grid_ztop;
    G->grid_gx = H->grid_gx;
    G->grid_gy = H->grid_gy;
    G->lowp = 0;   // the 16-bit copy is not carried over
    G->blocks = H->blocks;
    G->pieces = H->pieces;
    // stored bytes at the new value size (eq. nbytes-comparison, reading 8)
    const int64_t sz = dtype == RAD_F64 ? 8 : 4;
    rad_hmat_stats &st = G->stats;
    st.dtype = dtype;
    st.bytes_dense = st.bytes_csr = st.bytes_lowrank = 0;
    for (const BlockRec &b : G->blocks) {
        if (b.kind == BK_DENSE)
            st.bytes_dense += (int64_t)b.m * b.n * sz;
        else if (b.kind == BK_CSR)
            st.bytes_csr += 4 * ((int64_t)b.m + 1) + b.nnz * (4 + sz);
        else
            st.bytes_lowrank += ((int64_t)b.m + b.n) * b.rank * sz + b.rank * sz;
    }
    st.bytes_total = (int64_t)G->d_vals.bytes() + (int64_t)G->d_csr_idx.bytes() + (int64_t)G->d_csr_ptr.bytes() +
                     (int64_t)G->d_tiles.bytes() + (int64_t)G->d_brow.bytes() + (int64_t)G->d_groups.bytes() +
                     (int64_t)G->d_tile_tasks.bytes() + (int64_t)G->d_perm.bytes();
    st.bytes_csr_panels = 0;   // (the schedule adds the converted matrix's own)
}

}  // namespace rad
