// GPU kernels of the builder (FP64 throughout).
//
// Entries of F are never stored for the rank search: every product with a
// block recomputes F_ij = [n_i.(x_j-x_i)][n_j.(x_i-x_j)] A_j / (pi |x_i-x_j|^4) V_ij
// (eq. FF-def) from the tree-ordered geometry, with V_ij the back-face test
// of section 3.2 and, when a visibility bitmap is present, its ray-cast bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <hip/hip_fp16.h>

#include "rad_internal.h"

namespace rad {

namespace {

constexpr double kPi = 3.14159265358979323846;

// The back-face decisions are taken without contraction so that they match a
// plain FP64 evaluation of the same dot products.
__device__ __forceinline__ double dot3_exact(double a0, double a1, double a2, double b0, double b1, double b2) {
    double p0 = __dmul_rn(a0, b0);
    double p1 = __dmul_rn(a1, b1);
    double p2 = __dmul_rn(a2, b2);
    return __dadd_rn(__dadd_rn(p0, p1), p2);
}

__device__ __forceinline__ double vf_entry(const DevGeom &g, int64_t i, int64_t j) {
    if (i == j) return 0.0;
    const double *xi = g.x + 3 * i, *xj = g.x + 3 * j;
    const double *ni = g.n + 3 * i, *nj = g.n + 3 * j;
    double r0 = __dsub_rn(xj[0], xi[0]);
    double r1 = __dsub_rn(xj[1], xi[1]);
    double r2 = __dsub_rn(xj[2], xi[2]);
    double ci = dot3_exact(ni[0], ni[1], ni[2], r0, r1, r2);
    double cj = -dot3_exact(nj[0], nj[1], nj[2], r0, r1, r2);
    if (!(ci > 0.0) || !(cj > 0.0)) return 0.0;
    if (g.vis) {
        uint32_t w = g.vis[i * g.vis_words_per_row + (j >> 5)];
        if (!((w >> (j & 31)) & 1u)) return 0.0;
    }
    double rr = dot3_exact(r0, r1, r2, r0, r1, r2);
    return ci * cj * g.a[j] / (kPi * rr * rr);
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// non-zero count of each leaf block: one wave per block
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_leaf_nnz(DevGeom g, const int32_t *pairs, int64_t npairs,
                                                   int64_t *nnz) {
    int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (p >= npairs) return;
    int32_t i0 = pairs[4 * p], m = pairs[4 * p + 1], j0 = pairs[4 * p + 2], n = pairs[4 * p + 3];
    int64_t cnt = 0;
    int64_t tot = (int64_t)m * n;
    for (int64_t e = lane; e < tot; e += 64) {
        int64_t r = e / n, c = e - r * n;
        cnt += vf_entry(g, i0 + r, j0 + c) != 0.0;
    }
    cnt = wave_sum_i64(cnt);
    if (lane == 0) nnz[p] = cnt;
}

// random signs Omega (n x ell) of each sketch block, written into Z
__global__ void k_fill_rademacher(double *Z, const SketchBlock *blocks) {
    const SketchBlock b = blocks[blockIdx.y];
    int64_t tot = (int64_t)b.n * b.ell;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        uint64_t h = mix64(b.seed ^ mix64((uint64_t)e));
        Z[b.z_off + e] = (h & 1) ? 1.0 : -1.0;
    }
}

// ---------------------------------------------------------------------------
// out = F_b in (transpose = 0: m x ell from n x ell) or F_b^T in (n x ell from
// m x ell), entries recomputed per 64 x 32 tile.  Block: 256 threads =
// 64 output rows x 4 column groups of 16 sketch columns.
// ---------------------------------------------------------------------------
constexpr int SK_ROWS = 64, SK_K = 32, SK_COLS = 64;

__global__ void __launch_bounds__(256) k_sketch_apply(DevGeom g, const SketchBlock *blocks, int transpose,
                                                       const double *in, double *out) {
    const SketchBlock b = blocks[blockIdx.y];
    const int M = transpose ? b.n : b.m;
    const int K = transpose ? b.m : b.n;
    const int row0 = blockIdx.x * SK_ROWS;
    const int col0 = blockIdx.z * SK_COLS;
    if (row0 >= M || col0 >= b.ell) return;
    const double *src = in + (transpose ? b.y_off : b.z_off);
    double *dst = out + (transpose ? b.z_off : b.y_off);
    const int ncol = min(SK_COLS, b.ell - col0);

    __shared__ double sF[SK_K][SK_ROWS + 1];
    __shared__ double sP[SK_K][SK_COLS];
    const int t = threadIdx.x;
    const int r = t & 63;
    const int cg = t >> 6;
    double acc[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] = 0.0;

    for (int k0 = 0; k0 < K; k0 += SK_K) {
        // entries: 64 rows x 32 k = 2048, 8 per thread
        for (int e = t; e < SK_ROWS * SK_K; e += 256) {
            int rr = e & 63, kk = e >> 6;
            int orow = row0 + rr, kidx = k0 + kk;
            double v = 0.0;
            if (orow < M && kidx < K) {
                int64_t i, j;
                if (!transpose) {
                    i = b.i0 + orow;
                    j = b.j0 + kidx;
                } else {
                    i = b.i0 + kidx;
                    j = b.j0 + orow;
                }
                v = vf_entry(g, i, j);
            }
            sF[kk][rr] = v;
        }
        for (int e = t; e < SK_K * SK_COLS; e += 256) {
            int kk = e >> 6, c = e & 63;
            int kidx = k0 + kk;
            sP[kk][c] = (kidx < K && c < ncol) ? src[(int64_t)kidx + (int64_t)(col0 + c) * K] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < SK_K; ++kk) {
            double a = sF[kk][r];
#pragma unroll
            for (int c = 0; c < 16; ++c) acc[c] += a * sP[kk][cg * 16 + c];
        }
        __syncthreads();
    }
    int orow = row0 + r;
    if (orow < M) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            int cc = cg * 16 + c;
            if (cc < ncol) dst[(int64_t)orow + (int64_t)(col0 + cc) * M] = acc[c];
        }
    }
}

// ---------------------------------------------------------------------------
// Classical Gram-Schmidt, applied twice per column (CGS2), FP64, one
// workgroup per block.  The projections d = Q[:, :c]^T v are formed 32
// columns at a time with per-thread partial sums over the thread's rows;
// the update v -= Q d runs with one thread per row.  Columns whose norm
// collapses below 1e-13 of their starting norm are set to zero (dependent).
// Optionally records R.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_cgs2(double *base, const SketchBlock *blocks, int use_z, double *Rout,
                                               const int64_t *roff) {
    const SketchBlock b = blocks[blockIdx.x];
    const int rows = use_z ? b.n : b.m;
    const int ell = b.ell;
    double *Q = base + (use_z ? b.z_off : b.y_off);
    double *R = Rout ? Rout + roff[blockIdx.x] : nullptr;
    __shared__ double sd[4][64];
    __shared__ double sdot[64];
    __shared__ double sred[4];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;

    if (R) {
        for (int e = t; e < ell * ell; e += 256) R[e] = 0.0;
        __syncthreads();
    }
    for (int c = 0; c < ell; ++c) {
        double *v = Q + (int64_t)c * rows;
        double s = 0.0;
        for (int r = t; r < rows; r += 256) s += v[r] * v[r];
        s = wave_sum(s);
        if (lane == 0) sred[w] = s;
        __syncthreads();
        const double norm0 = sqrt(sred[0] + sred[1] + sred[2] + sred[3]);
        __syncthreads();
        for (int pass = 0; pass < 2 && c > 0; ++pass) {
            for (int j0 = 0; j0 < c; j0 += 32) {
                const int jn = min(32, c - j0);
                // d_j = Q[:, j0+j]^T v: every thread keeps 32 partial sums over
                // its rows (coalesced loads), then the block reduces them.
                double pj[32];
#pragma unroll
                for (int jj = 0; jj < 32; ++jj) pj[jj] = 0.0;
                for (int r = t; r < rows; r += 256) {
                    const double vr = v[r];
#pragma unroll
                    for (int jj = 0; jj < 32; ++jj)
                        if (jj < jn) pj[jj] += Q[(int64_t)(j0 + jj) * rows + r] * vr;
                }
#pragma unroll
                for (int jj = 0; jj < 32; ++jj) {
                    double q = wave_sum(pj[jj]);
                    if (lane == 0) sd[w][jj] = q;
                }
                __syncthreads();
                if (t < 32) sdot[t] = (t < jn) ? sd[0][t] + sd[1][t] + sd[2][t] + sd[3][t] : 0.0;
                __syncthreads();
                for (int r = t; r < rows; r += 256) {
                    double acc = v[r];
                    for (int jj = 0; jj < jn; ++jj) acc -= Q[(int64_t)(j0 + jj) * rows + r] * sdot[jj];
                    v[r] = acc;
                }
                if (R && t < jn) R[(j0 + t) + (int64_t)c * ell] += sdot[t];
                __syncthreads();
            }
        }
        s = 0.0;
        for (int r = t; r < rows; r += 256) s += v[r] * v[r];
        s = wave_sum(s);
        if (lane == 0) sred[w] = s;
        __syncthreads();
        const double nrm = sqrt(sred[0] + sred[1] + sred[2] + sred[3]);
        __syncthreads();
        const bool dep = !(nrm > 1e-13 * norm0) || !(nrm > 0.0);
        const double inv = dep ? 0.0 : 1.0 / nrm;
        for (int r = t; r < rows; r += 256) v[r] = dep ? 0.0 : v[r] * inv;
        if (R && t == 0) R[c + (int64_t)c * ell] = dep ? 0.0 : nrm;
        __syncthreads();
    }
}

__global__ void k_zero_r(const SketchBlock *blocks, double *Rout, const int64_t *roff) {
    const SketchBlock b = blocks[blockIdx.x];
    double *R = Rout + roff[blockIdx.x];
    for (int e = threadIdx.x; e < b.ell * b.ell; e += blockDim.x) R[e] = 0.0;
}

// ---------------------------------------------------------------------------
// CGS2 for tall blocks, spread over many workgroups: for each column c the
// rows are split in chunks of kCgsRows; every chunk writes partial dot
// products (or norms), and the next launch sums them in a fixed order.
// One column needs five launches: dots, update, dots, update, normalize.
// ---------------------------------------------------------------------------
constexpr int kCgsRows = 2048;

// part[(b * nch + ch) * stride + j] = sum over the chunk of Q[:, j] v (j < c);
// with first != 0 also writes the chunk's sum of v^2 at index stride - 1.
__global__ void __launch_bounds__(256) k_cgs2_dots(double *base, const SketchBlock *blocks, int use_z, int c,
                                                    int nch, int stride, double *part, int first) {
    const SketchBlock b = blocks[blockIdx.y];
    const int rows = use_z ? b.n : b.m;
    const int ch = blockIdx.x;
    if (c >= b.ell || ch * kCgsRows >= rows) return;
    const double *Q = base + (use_z ? b.z_off : b.y_off);
    const double *v = Q + (int64_t)c * rows;
    const int r0 = ch * kCgsRows, r1 = min(rows, r0 + kCgsRows);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    __shared__ double sd[4][33];
    double *out = part + ((int64_t)blockIdx.y * nch + ch) * stride;
    for (int j0 = 0; j0 < c; j0 += 32) {
        const int jn = min(32, c - j0);
        double pj[32];
#pragma unroll
        for (int jj = 0; jj < 32; ++jj) pj[jj] = 0.0;
        for (int r = r0 + t; r < r1; r += 256) {
            const double vr = v[r];
#pragma unroll
            for (int jj = 0; jj < 32; ++jj)
                if (jj < jn) pj[jj] += Q[(int64_t)(j0 + jj) * rows + r] * vr;
        }
#pragma unroll
        for (int jj = 0; jj < 32; ++jj) {
            double q = wave_sum(pj[jj]);
            if (lane == 0) sd[w][jj] = q;
        }
        __syncthreads();
        if (t < jn) out[j0 + t] = sd[0][t] + sd[1][t] + sd[2][t] + sd[3][t];
        __syncthreads();
    }
    if (first) {
        double s = 0.0;
        for (int r = r0 + t; r < r1; r += 256) s += v[r] * v[r];
        s = wave_sum(s);
        if (lane == 0) sd[w][32] = s;
        __syncthreads();
        if (t == 0) out[stride - 1] = sd[0][32] + sd[1][32] + sd[2][32] + sd[3][32];
    }
}

// v -= Q[:, :c] d with d = sum of the chunk partials; chunk 0 adds d to R.
// Writes the chunk's sum of the updated v^2 at normpart[b * nch + ch].
__global__ void __launch_bounds__(256) k_cgs2_update(double *base, const SketchBlock *blocks, int use_z, int c,
                                                      int nch, int stride, const double *part, double *Rout,
                                                      const int64_t *roff, double *normpart) {
    const SketchBlock b = blocks[blockIdx.y];
    const int rows = use_z ? b.n : b.m;
    const int ch = blockIdx.x;
    if (c >= b.ell || ch * kCgsRows >= rows) return;
    double *Q = base + (use_z ? b.z_off : b.y_off);
    double *v = Q + (int64_t)c * rows;
    const int r0 = ch * kCgsRows, r1 = min(rows, r0 + kCgsRows);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int nchb = (rows + kCgsRows - 1) / kCgsRows;
    __shared__ double sdot[512];
    __shared__ double sred[4];
    double s = 0.0;
    for (int j0 = 0; j0 < c; j0 += 512) {
        const int jn = min(512, c - j0);
        for (int jj = t; jj < jn; jj += 256) {
            double d = 0.0;
            for (int k = 0; k < nchb; ++k) d += part[((int64_t)blockIdx.y * nch + k) * stride + j0 + jj];
            sdot[jj] = d;
            if (Rout && ch == 0) Rout[roff[blockIdx.y] + (j0 + jj) + (int64_t)c * b.ell] += d;
        }
        __syncthreads();
        for (int r = r0 + t; r < r1; r += 256) {
            double acc = v[r];
            for (int jj = 0; jj < jn; ++jj) acc -= Q[(int64_t)(j0 + jj) * rows + r] * sdot[jj];
            v[r] = acc;
        }
        __syncthreads();
    }
    for (int r = r0 + t; r < r1; r += 256) s += v[r] * v[r];
    s = wave_sum(s);
    if (lane == 0) sred[w] = s;
    __syncthreads();
    if (t == 0) normpart[(int64_t)blockIdx.y * nch + ch] = sred[0] + sred[1] + sred[2] + sred[3];
}

// normalize column c (or zero it when it collapsed below 1e-13 of its start)
__global__ void __launch_bounds__(256) k_cgs2_norm(double *base, const SketchBlock *blocks, int use_z, int c, int nch,
                                                    int stride, const double *part, const double *normpart,
                                                    double *Rout, const int64_t *roff) {
    const SketchBlock b = blocks[blockIdx.y];
    const int rows = use_z ? b.n : b.m;
    const int ch = blockIdx.x;
    if (c >= b.ell || ch * kCgsRows >= rows) return;
    double *v = base + (use_z ? b.z_off : b.y_off) + (int64_t)c * rows;
    const int nchb = (rows + kCgsRows - 1) / kCgsRows;
    double n0 = 0.0, n1 = 0.0;
    for (int k = 0; k < nchb; ++k) {
        n0 += part[((int64_t)blockIdx.y * nch + k) * stride + stride - 1];
        n1 += normpart[(int64_t)blockIdx.y * nch + k];
    }
    const double norm0 = sqrt(n0), nrm = sqrt(n1);
    const bool dep = !(nrm > 1e-13 * norm0) || !(nrm > 0.0);
    const double inv = dep ? 0.0 : 1.0 / nrm;
    const int r0 = ch * kCgsRows, r1 = min(rows, r0 + kCgsRows);
    for (int r = r0 + threadIdx.x; r < r1; r += 256) v[r] = dep ? 0.0 : v[r] * inv;
    if (Rout && ch == 0 && threadIdx.x == 0) Rout[roff[blockIdx.y] + c + (int64_t)c * b.ell] = dep ? 0.0 : nrm;
}

// out (rows x q) = Q (rows x ell) * small (ell x q) for each accepted block
__global__ void k_small_gemm(const double *Qbase, const SketchBlock *blocks, const int64_t *soff,
                             const double *small, const int32_t *qk, const int64_t *ooff, double *out, int use_z) {
    const SketchBlock b = blocks[blockIdx.y];
    const int rows = use_z ? b.n : b.m;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const double *Q = Qbase + (use_z ? b.z_off : b.y_off);
    const double *S = small + soff[blockIdx.y];
    const int q = qk[blockIdx.y], ell = b.ell;
    double *o = out + ooff[blockIdx.y];
    for (int c = 0; c < q; ++c) {
        double acc = 0.0;
        for (int k = 0; k < ell; ++k) acc += Q[(int64_t)k * rows + r] * S[k + (int64_t)c * ell];
        o[r + (int64_t)c * rows] = acc;
    }
}

template <class T>
__device__ __forceinline__ T cast_to(double v);
template <>
__device__ __forceinline__ double cast_to<double>(double v) { return v; }
template <>
__device__ __forceinline__ float cast_to<float>(double v) { return (float)v; }

template <class T>
__global__ void k_dense_fill(DevGeom g, const int32_t *tiles, const int64_t *offs, T *vals) {
    const int32_t *tl = tiles + 6 * (int64_t)blockIdx.x;
    int32_t i0 = tl[0], m = tl[1], j0 = tl[2], n = tl[3], ld = tl[4];
    T *dst = vals + offs[blockIdx.x];
    int64_t tot = (int64_t)m * n;
    for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
        int64_t c = e / m, r = e - c * m;
        dst[r + c * ld] = cast_to<T>(vf_entry(g, i0 + r, j0 + c));
    }
}

__global__ void k_csr_count(DevGeom g, const int32_t *tiles, int32_t *cnt, const int64_t *row_offs) {
    const int32_t *tl = tiles + 6 * (int64_t)blockIdx.x;
    int32_t i0 = tl[0], m = tl[1], j0 = tl[2], n = tl[3];
    int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int r = w; r < m; r += blockDim.x / 64) {
        int64_t c = 0;
        for (int j = lane; j < n; j += 64) c += vf_entry(g, i0 + r, j0 + j) != 0.0;
        c = wave_sum_i64(c);
        if (lane == 0) cnt[row_offs[blockIdx.x] + r] = (int32_t)c;
    }
}

template <class T>
__global__ void k_csr_fill(DevGeom g, const int32_t *tiles, const int32_t *rowptr, const int64_t *row_offs,
                           const int64_t *val_base, T *vals, int32_t *cols_at_val) {
    const int32_t *tl = tiles + 6 * (int64_t)blockIdx.x;
    int32_t i0 = tl[0], m = tl[1], j0 = tl[2], n = tl[3];
    const int32_t *ptr = rowptr + row_offs[blockIdx.x];
    int64_t vb = val_base[blockIdx.x];
    for (int r = threadIdx.x; r < m; r += blockDim.x) {
        int64_t k = vb + ptr[r];
        for (int j = 0; j < n; ++j) {
            double v = vf_entry(g, i0 + r, j0 + j);
            if (v != 0.0) {
                vals[k] = cast_to<T>(v);
                cols_at_val[k] = j;
                ++k;
            }
        }
    }
}

// one workgroup per copy descriptor: FP64 source block -> value pool (cast)
template <class T>
__global__ void k_copy_batched(const CopyDesc *d, T *vals) {
    const CopyDesc c = d[blockIdx.x];
    T *dst = vals + c.dst_off;
    const int64_t tot = (int64_t)c.rows * c.cols;
    for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
        int64_t col = e / c.rows, r = e - col * c.rows;
        dst[r + col * c.ldd] = cast_to<T>(c.src[r + col * c.lds]);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_leaf_nnz(const DevGeom &g, const int32_t *pairs, int64_t npairs, int64_t *nnz, hipStream_t s) {
    if (npairs <= 0) return;
    int64_t blocks = (npairs + 3) / 4;
    hipLaunchKernelGGL(k_leaf_nnz, dim3((unsigned)blocks), dim3(256), 0, s, g, pairs, npairs, nnz);
    RAD_HIP(hipGetLastError());
}

void launch_fill_rademacher(double *Z, const SketchBlock *blocks, int32_t nblocks, hipStream_t s) {
    if (nblocks <= 0) return;
    hipLaunchKernelGGL(k_fill_rademacher, dim3(64, nblocks), dim3(256), 0, s, Z, blocks);
    RAD_HIP(hipGetLastError());
}

void launch_sketch_apply(const DevGeom &g, const SketchBlock *blocks, int32_t nblocks, int transpose,
                         const double *in, double *out, int32_t max_rows, int32_t max_ell, hipStream_t s) {
    if (nblocks <= 0) return;
    dim3 grid((max_rows + SK_ROWS - 1) / SK_ROWS, nblocks, (max_ell + SK_COLS - 1) / SK_COLS);
    hipLaunchKernelGGL(k_sketch_apply, grid, dim3(256), 0, s, g, blocks, transpose, in, out);
    RAD_HIP(hipGetLastError());
}

void launch_cgs2(double *base, const SketchBlock *blocks, int32_t nblocks, int use_z, double *Rout,
                 const int64_t *roff, hipStream_t s) {
    if (nblocks <= 0) return;
    hipLaunchKernelGGL(k_cgs2, dim3(nblocks), dim3(256), 0, s, base, blocks, use_z, Rout, roff);
    RAD_HIP(hipGetLastError());
}

void launch_cgs2_tall(double *base, const SketchBlock *blocks, int32_t nblocks, int use_z, double *Rout,
                      const int64_t *roff, int32_t max_rows, int32_t max_ell, double *part, double *normpart,
                      double *norm0part, hipStream_t s) {
    (void)norm0part;
    if (nblocks <= 0) return;
    const int nch = (max_rows + kCgsRows - 1) / kCgsRows;
    const int stride = max_ell + 1;
    dim3 grid(nch, nblocks);
    if (Rout) {
        // R = 0 before accumulation: one small kernel per block would also do; reuse the fill
        hipLaunchKernelGGL(k_zero_r, dim3(nblocks), dim3(256), 0, s, blocks, Rout, roff);
        RAD_HIP(hipGetLastError());
    }
    for (int c = 0; c < max_ell; ++c) {
        hipLaunchKernelGGL(k_cgs2_dots, grid, dim3(256), 0, s, base, blocks, use_z, c, nch, stride, part, 1);
        hipLaunchKernelGGL(k_cgs2_update, grid, dim3(256), 0, s, base, blocks, use_z, c, nch, stride,
                           (const double *)part, Rout, roff, normpart);
        hipLaunchKernelGGL(k_cgs2_dots, grid, dim3(256), 0, s, base, blocks, use_z, c, nch, stride, part, 0);
        hipLaunchKernelGGL(k_cgs2_update, grid, dim3(256), 0, s, base, blocks, use_z, c, nch, stride,
                           (const double *)part, Rout, roff, normpart);
        hipLaunchKernelGGL(k_cgs2_norm, grid, dim3(256), 0, s, base, blocks, use_z, c, nch, stride,
                           (const double *)part, (const double *)normpart, Rout, roff);
        RAD_HIP(hipGetLastError());
    }
}

void launch_small_gemm(const double *Qbase, const SketchBlock *blocks, const int64_t *soff, const double *small,
                       const int32_t *qk, const int64_t *ooff, double *out, int32_t nblocks, int use_z,
                       int32_t max_rows, hipStream_t s) {
    if (nblocks <= 0) return;
    dim3 grid((max_rows + 255) / 256, nblocks);
    hipLaunchKernelGGL(k_small_gemm, grid, dim3(256), 0, s, Qbase, blocks, soff, small, qk, ooff, out, use_z);
    RAD_HIP(hipGetLastError());
}

void launch_dense_fill(const DevGeom &g, const int32_t *tiles, const int64_t *offs, int64_t ntiles, void *vals,
                       int32_t dtype, hipStream_t s) {
    if (ntiles <= 0) return;
    if (dtype == RAD_F64)
        hipLaunchKernelGGL(k_dense_fill<double>, dim3((unsigned)ntiles), dim3(256), 0, s, g, tiles, offs,
                           (double *)vals);
    else
        hipLaunchKernelGGL(k_dense_fill<float>, dim3((unsigned)ntiles), dim3(256), 0, s, g, tiles, offs,
                           (float *)vals);
    RAD_HIP(hipGetLastError());
}

void launch_csr_count(const DevGeom &g, const int32_t *tiles, int64_t ntiles, int32_t *cnt, const int64_t *row_offs,
                      hipStream_t s) {
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(k_csr_count, dim3((unsigned)ntiles), dim3(256), 0, s, g, tiles, cnt, row_offs);
    RAD_HIP(hipGetLastError());
}

void launch_csr_fill(const DevGeom &g, const int32_t *tiles, int64_t ntiles, const int32_t *rowptr,
                     const int64_t *row_offs, const int64_t *val_base, void *vals, int32_t *cols, int32_t dtype,
                     hipStream_t s) {
    if (ntiles <= 0) return;
    if (dtype == RAD_F64)
        hipLaunchKernelGGL(k_csr_fill<double>, dim3((unsigned)ntiles), dim3(64), 0, s, g, tiles, rowptr, row_offs,
                           val_base, (double *)vals, cols);
    else
        hipLaunchKernelGGL(k_csr_fill<float>, dim3((unsigned)ntiles), dim3(64), 0, s, g, tiles, rowptr, row_offs,
                           val_base, (float *)vals, cols);
    RAD_HIP(hipGetLastError());
}

void launch_copy_batched(const CopyDesc *d, int64_t n, void *vals, int32_t dtype, hipStream_t s) {
    for (int64_t b0 = 0; b0 < n; b0 += (int64_t)1 << 30) {
        unsigned nb = (unsigned)std::min<int64_t>(n - b0, (int64_t)1 << 30);
        if (dtype == RAD_F64)
            hipLaunchKernelGGL(k_copy_batched<double>, dim3(nb), dim3(256), 0, s, d + b0, (double *)vals);
        else
            hipLaunchKernelGGL(k_copy_batched<float>, dim3(nb), dim3(256), 0, s, d + b0, (float *)vals);
        RAD_HIP(hipGetLastError());
    }
}

}  // namespace rad
