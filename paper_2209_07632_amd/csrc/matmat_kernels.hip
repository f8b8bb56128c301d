// Multi-RHS H-matvec on the matrix cores (Algorithm 5 with X an N x R block).
//
// Internal layout: tree-ordered, right-hand-side-minor ("R-major"): element
// (facet t, column r) at t * ldr + r.  Both phases are tiled GEMMs on
// v_mfma_{f32,f64}_16x16x4 with 64 x 128 output tiles per workgroup (four
// waves, each 64 rows x 32 columns), operands staged through LDS in chunks of
// 32 along the reduction dimension:
//   phase 1 (projections), split along the facets of the column node:
//       P_s = V_J[rows of split s]^T X_J[rows of split s]; T_J = sum_s P_s
//       (the sum over splits runs in a second, deterministic kernel);
//   phase 2 (expansion and near field), one workgroup per (leaf, column tile):
//       Y_L = sum_dense A X_J + sum_csr A X_J + sum_lowrank U'_L T_b,
//       CSR slices are expanded to dense chunks in LDS.
#include <hip/hip_runtime.h>

#include "rad_internal.h"
#include "mm_epilogue.h"

namespace rad {

namespace {

constexpr int TM = 64;    // output rows per workgroup
constexpr int TN = 128;   // output columns (right-hand sides) per workgroup
constexpr int KC = 16;    // reduction chunk
constexpr int PADA = 4, PADB = 4;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <class T>
struct Mfma;
// Operands of both instructions: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16].  Result register v of lane l holds column l % 16 and
// row 4 (l / 16) + v for FP32, row (l / 16) + 4 v for FP64 (checked on gfx950).
template <>
struct Mfma<float> {
    typedef f32x4 acc_t;
    static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};
template <>
struct Mfma<double> {
    typedef f64x4 acc_t;
    static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};

// acc[i][j]: row tile i (16 rows), column tile j (16 columns of this wave's 32)
template <class T>
struct Tile {
    typename Mfma<T>::acc_t acc[4][2];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;
    }
    // one chunk of KC from LDS: sA[k][row], sB[k][col]
    __device__ __forceinline__ void mma(const T (*sA)[TM + PADA], const T (*sB)[TN + PADB], int lane, int w) {
        const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int s = 0; s < KC / 4; ++s) {
            const int k = s * 4 + lk;
            T a[4], b[2];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = sA[k][i * 16 + lr];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = sB[k][w * 32 + j * 16 + lr];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = Mfma<T>::run(a[i], b[j], acc[i][j]);
        }
    }
};

// B chunk: rows [brow, brow + kcount) of an R-major matrix, columns [r0, r0+TN).
// ldr and r0 are multiples of 4, so groups of four columns are loaded as one
// 16-byte (FP32) or two 16-byte (FP64) vectors.
template <class T>
__device__ __forceinline__ void load_b_rmajor(T (*sB)[TN + PADB], const T *src, int64_t brow, int kcount,
                                              int64_t ldr, int r0, int R, int t) {
    for (int e = t; e < KC * TN / 4; e += 256) {
        int k = e / (TN / 4), c = (e - k * (TN / 4)) * 4;
        T v0 = 0, v1 = 0, v2 = 0, v3 = 0;
        if (k < kcount) {
            const T *p = src + (brow + k) * ldr + r0 + c;
            if (r0 + c + 3 < R) {
                if constexpr (sizeof(T) == 4) {
                    float4 q = *(const float4 *)p;
                    v0 = q.x; v1 = q.y; v2 = q.z; v3 = q.w;
                } else {
                    double2 q0 = *(const double2 *)p, q1 = *(const double2 *)(p + 2);
                    v0 = q0.x; v1 = q0.y; v2 = q1.x; v3 = q1.y;
                }
            } else {
                if (r0 + c < R) v0 = p[0];
                if (r0 + c + 1 < R) v1 = p[1];
                if (r0 + c + 2 < R) v2 = p[2];
            }
        }
        sB[k][c] = v0;
        sB[k][c + 1] = v1;
        sB[k][c + 2] = v2;
        sB[k][c + 3] = v3;
    }
}

// A chunk from a column-major slice (rows x cols, leading dimension ld)
template <class T>
__device__ __forceinline__ void load_a_colmajor(T (*sA)[TM + PADA], const T *src, int64_t ld, int rows, int kbase,
                                                int kcount, int t) {
    for (int e = t; e < KC * TM; e += 256) {
        int k = e / TM, r = e - k * TM;
        T v = 0;
        if (k < kcount && r < rows) v = src[(int64_t)r + (int64_t)(kbase + k) * ld];
        sA[k][r] = v;
    }
}

// One reduction chunk of a GEMM, staged through registers so that the global
// loads of chunk c+1 are in flight while chunk c runs on the matrix cores.
// A[r][k]: kind 0 = column-major block rows (row_off + r, r in [r_lo, r_hi)),
//          kind 1 = transposed V (A[r][k] = V[k + r * ld], r < r_hi).
template <class T>
struct Stage {
    T a[KC * TM / 256];
    T b[KC * TN / 256];
    __device__ __forceinline__ void fetch(int kind, const T *A, int64_t ld, int row_off, int r_lo, int r_hi, int kb,
                                          int kcount, const T *B, int64_t brow, int64_t ldr, int r0, int R, int t) {
#pragma unroll
        for (int q = 0; q < KC * TM / 256; ++q) {
            int e = t + q * 256;
            T v = 0;
            if (kind == 0) {
                int k = e / TM, r = e - k * TM;
                if (k < kcount && r >= r_lo && r < r_hi) v = A[(int64_t)(row_off + r) + (int64_t)(kb + k) * ld];
            } else {
                int r = e / KC, k = e - r * KC;
                if (k < kcount && r < r_hi) v = A[(int64_t)(kb + k) + (int64_t)r * ld];
            }
            a[q] = v;
        }
#pragma unroll
        for (int q = 0; q < KC * TN / 1024; ++q) {
            int e = t + q * 256;
            int k = e / (TN / 4), c = (e - k * (TN / 4)) * 4;
            T v0 = 0, v1 = 0, v2 = 0, v3 = 0;
            if (k < kcount) {
                const T *p = B + (brow + k) * ldr + r0 + c;
                if (r0 + c + 3 < R) {
                    if constexpr (sizeof(T) == 4) {
                        float4 qv = *(const float4 *)p;
                        v0 = qv.x; v1 = qv.y; v2 = qv.z; v3 = qv.w;
                    } else {
                        double2 q0 = *(const double2 *)p, q1 = *(const double2 *)(p + 2);
                        v0 = q0.x; v1 = q0.y; v2 = q1.x; v3 = q1.y;
                    }
                } else {
                    if (r0 + c < R) v0 = p[0];
                    if (r0 + c + 1 < R) v1 = p[1];
                    if (r0 + c + 2 < R) v2 = p[2];
                }
            }
            b[4 * q] = v0;
            b[4 * q + 1] = v1;
            b[4 * q + 2] = v2;
            b[4 * q + 3] = v3;
        }
    }
    __device__ __forceinline__ void commit(int kind, T (*sA)[TM + PADA], T (*sB)[TN + PADB], int t) {
#pragma unroll
        for (int q = 0; q < KC * TM / 256; ++q) {
            int e = t + q * 256;
            if (kind == 0) {
                int k = e / TM, r = e - k * TM;
                sA[k][r] = a[q];
            } else {
                int r = e / KC, k = e - r * KC;
                sA[k][r] = a[q];
            }
        }
#pragma unroll
        for (int q = 0; q < KC * TN / 1024; ++q) {
            int e = t + q * 256;
            int k = e / (TN / 4), c = (e - k * (TN / 4)) * 4;
            sB[k][c] = b[4 * q];
            sB[k][c + 1] = b[4 * q + 1];
            sB[k][c + 2] = b[4 * q + 2];
            sB[k][c + 3] = b[4 * q + 3];
        }
    }
};

// Chunk of a packed panel (64 x KC contiguous, ld 64) and of the operand rows
// it multiplies (gathered through brow: X row if >= 0, T row -1-v if < 0).
template <class T>
struct PanelStage {
    T a[KC * TM / 256];
    T b[KC * TN / 256];
    __device__ __forceinline__ void fetch(const T *pan, const int32_t *brc, const T *X, const T *Tb, int64_t ldr, int r0,
                                          int R, int t) {
#pragma unroll
        for (int q = 0; q < KC * TM / 1024; ++q) {
            const T *p = pan + 4 * (t + q * 256);
            if constexpr (sizeof(T) == 4) {
                float4 v = *(const float4 *)p;
                a[4 * q] = v.x; a[4 * q + 1] = v.y; a[4 * q + 2] = v.z; a[4 * q + 3] = v.w;
            } else {
                double2 v0 = *(const double2 *)p, v1 = *(const double2 *)(p + 2);
                a[4 * q] = v0.x; a[4 * q + 1] = v0.y; a[4 * q + 2] = v1.x; a[4 * q + 3] = v1.y;
            }
        }
#pragma unroll
        for (int q = 0; q < KC * TN / 1024; ++q) {
            int e = t + q * 256;
            int k = e / (TN / 4), c = (e - k * (TN / 4)) * 4;
            int32_t v = brc[k];
            const T *p = (v >= 0 ? X + (int64_t)v * ldr : Tb + (int64_t)(-1 - v) * ldr) + r0 + c;
            T v0 = 0, v1 = 0, v2 = 0, v3 = 0;
            if (r0 + c + 3 < R) {
                if constexpr (sizeof(T) == 4) {
                    float4 qv = *(const float4 *)p;
                    v0 = qv.x; v1 = qv.y; v2 = qv.z; v3 = qv.w;
                } else {
                    double2 q0 = *(const double2 *)p, q1 = *(const double2 *)(p + 2);
                    v0 = q0.x; v1 = q0.y; v2 = q1.x; v3 = q1.y;
                }
            } else {
                if (r0 + c < R) v0 = p[0];
                if (r0 + c + 1 < R) v1 = p[1];
                if (r0 + c + 2 < R) v2 = p[2];
            }
            b[4 * q] = v0;
            b[4 * q + 1] = v1;
            b[4 * q + 2] = v2;
            b[4 * q + 3] = v3;
        }
    }
    __device__ __forceinline__ void commit(T (*sA)[TM + PADA], T (*sB)[TN + PADB], int t) {
#pragma unroll
        for (int q = 0; q < KC * TM / 1024; ++q) {
            int e = 4 * (t + q * 256);
            int k = e / TM, r = e - k * TM;
            sA[k][r] = a[4 * q];
            sA[k][r + 1] = a[4 * q + 1];
            sA[k][r + 2] = a[4 * q + 2];
            sA[k][r + 3] = a[4 * q + 3];
        }
#pragma unroll
        for (int q = 0; q < KC * TN / 1024; ++q) {
            int e = t + q * 256;
            int k = e / (TN / 4), c = (e - k * (TN / 4)) * 4;
            sB[k][c] = b[4 * q];
            sB[k][c + 1] = b[4 * q + 1];
            sB[k][c + 2] = b[4 * q + 2];
            sB[k][c + 3] = b[4 * q + 3];
        }
    }
};

// ---------------------------------------------------------------------------
// phase 1: partial projections
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) k_proj_mm(const ProjGroup *groups, const P1Work *work, const T *vals,
                                                  const T *X, int64_t ldr, int R, T *part) {
    const P1Work wk = work[blockIdx.x];
    const ProjGroup g = groups[wk.group];
    const int r0 = blockIdx.y * TN;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    __shared__ T sA[2][KC][TM + PADA];
    __shared__ T sB[2][KC][TN + PADB];
    Tile<T> tile;
    tile.zero();
    const int rows = min(TM, g.ktot - wk.krow0);
    const T *V = vals + g.v_off + (int64_t)wk.krow0 * g.ld;
    Stage<T> st;
    int buf = 0;
    st.fetch(1, V, g.ld, 0, 0, rows, wk.jb, min(KC, wk.je - wk.jb), X, (int64_t)g.j0 + wk.jb, ldr, r0, R, t);
    for (int kb = wk.jb; kb < wk.je; kb += KC) {
        st.commit(1, sA[buf], sB[buf], t);
        __syncthreads();
        const int nk = kb + KC;
        if (nk < wk.je) st.fetch(1, V, g.ld, 0, 0, rows, nk, min(KC, wk.je - nk), X, (int64_t)g.j0 + nk, ldr, r0, R, t);
        tile.mma(sA[buf], sB[buf], lane, w);
        buf ^= 1;
    }
    T *out = part + (int64_t)wk.part * TM * ldr;
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int row = i * 16 + Mfma<T>::row(lk, v);
                int col = r0 + w * 32 + j * 16 + lr;
                if (col < R) out[(int64_t)row * ldr + col] = tile.acc[i][j][v];
            }
}

// T rows = sum of the partial tiles of every split (fixed order); one thread
// per (row of T, column)
template <class T>
__global__ void __launch_bounds__(256) k_proj_reduce(const P1Red *red, const T *part, int64_t ldr, int R, T *Tb) {
    const P1Red rd = red[blockIdx.x / TM];
    const int row = blockIdx.x % TM;
    const int c = blockIdx.y * 256 + threadIdx.x;
    if (c >= R || row >= rd.nrows) return;
    T s = 0;
    for (int p = 0; p < rd.part_count; ++p) s += part[((int64_t)(rd.part_begin + p) * TM + row) * ldr + c];
    Tb[(int64_t)(rd.t_row0 + row) * ldr + c] = s;
}

// ---------------------------------------------------------------------------
// phase 2: one workgroup per (64-row tile, 128-column tile).  With E given,
// the epilogue performs the Jacobi update B_new = E + rho * (F B_old) and
// writes the per-column partial sums of (B_new - B_old)^2 for this tile.
// ---------------------------------------------------------------------------
template <class T, bool kFused>
__global__ void __launch_bounds__(256) k_tile_mm(const TileInfo *tiles, const int32_t *brow, const TileTask *ctasks,
                                                  const T *vals, const int32_t *csr_ptr, const int32_t *csr_idx,
                                                  int64_t csr_val_start, const T *X, const T *Tb, int64_t ldr, int R,
                                                  int64_t N, T *Y, const T *E, const T *rho, T rho_s,
                                                  double *partial) {
    const int tile = blockIdx.x;
    const TileInfo ti = tiles[tile];
    const int64_t tile0 = (int64_t)tile * TM;
    const int r0 = blockIdx.y * TN;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    // pipeline buffers during the reduction, the 64 x 128 result tile after it
    constexpr int kPipe = 2 * KC * (TM + PADA) + 2 * KC * (TN + PADB);
    constexpr int kOut = TM * (TN + PADB);
    __shared__ T smem[kPipe > kOut ? kPipe : kOut];
    static_assert(8 * TN * sizeof(double) <= sizeof(T) * (kPipe > kOut ? kPipe : kOut), "partial sums fit");
    T (*sA)[KC][TM + PADA] = (T (*)[KC][TM + PADA])smem;
    T (*sB)[KC][TN + PADB] = (T (*)[KC][TN + PADB])(smem + 2 * KC * (TM + PADA));
    Tile<T> acc;
    acc.zero();
    // CSR tasks: rows expanded into dense chunks in LDS
    for (int c = ti.csr_begin; c < ti.csr_end; ++c) {
        const TileTask tk = ctasks[c];
        const T *v = vals + tk.a_off;
        const int32_t *ci = csr_idx + (tk.a_off - csr_val_start);
        int cur = 0, end = 0;
        if (t >= tk.r_lo && t < tk.r_hi) {
            cur = csr_ptr[tk.aux_off + tk.row_off + t];
            end = csr_ptr[tk.aux_off + tk.row_off + t + 1];
        }
        for (int kb = 0; kb < tk.ncol; kb += KC) {
            const int kcount = min(KC, tk.ncol - kb);
            for (int e = t; e < KC * TM; e += 256) sA[0][e / TM][e % TM] = 0;
            __syncthreads();
            while (cur < end && ci[cur] < kb + KC) {
                sA[0][ci[cur] - kb][t] = v[cur];
                ++cur;
            }
            load_b_rmajor(sB[0], X, (int64_t)tk.col0 + kb, kcount, ldr, r0, R, t);
            __syncthreads();
            acc.mma(sA[0], sB[0], lane, w);
            __syncthreads();
        }
    }
    // packed panel: software-pipelined chunks
    if (ti.kpad > 0) {
        const T *pan = vals + ti.panel_off;
        const int32_t *br = brow + ti.brow_off;
        PanelStage<T> st;
        st.fetch(pan, br, X, Tb, ldr, r0, R, t);
        int buf = 0;
        for (int kb = 0; kb < ti.kpad; kb += KC) {
            st.commit(sA[buf], sB[buf], t);
            __syncthreads();
            if (kb + KC < ti.kpad) st.fetch(pan + (int64_t)(kb + KC) * TM, br + kb + KC, X, Tb, ldr, r0, R, t);
            acc.mma(sA[buf], sB[buf], lane, w);
            buf ^= 1;
        }
    }
    // epilogue through LDS: the 64 x 128 result tile is written to LDS, then
    // every thread streams 16-byte groups of whole rows (coalesced E, B_old,
    // B_new accesses).  Per-column partial sums are reduced in a fixed order.
    __syncthreads();
    T (*sC)[TN + PADB] = (T (*)[TN + PADB])smem;
    {
        const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) sC[i * 16 + Mfma<T>::row(lk, v)][w * 32 + j * 16 + lr] = acc.acc[i][j][v];
    }
    __syncthreads();
    tile_epilogue<T, kFused, TM, TN, TN + PADB>(sC, smem, tile, tile0, r0, ldr, R, N, Y, E, X, rho, rho_s, partial);
}

// col-major (original or tree order) <-> R-major tree order, 64 x 64 tiles
// through LDS so that both the column-major and the R-major side are walked
// along their contiguous dimension.
template <class T>
__global__ void __launch_bounds__(256) k_to_rmajor(const int32_t *perm, const T *src, int64_t lds, T *dst,
                                                    int64_t ldr, int64_t N, int R) {
    __shared__ T sm[64][65];
    const int64_t t0 = (int64_t)blockIdx.x * 64;
    const int r0 = blockIdx.y * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        int tt = e & 63, rr = e >> 6;
        int64_t t = t0 + tt;
        T v = 0;
        if (t < N && r0 + rr < R) v = src[(perm ? (int64_t)perm[t] : t) + (int64_t)(r0 + rr) * lds];
        sm[rr][tt] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        int rr = e & 63, tt = e >> 6;
        int64_t t = t0 + tt;
        if (t < N && r0 + rr < R) dst[t * ldr + r0 + rr] = sm[rr][tt];
    }
}

template <class T>
__global__ void __launch_bounds__(256) k_from_rmajor(const int32_t *perm, const T *src, int64_t ldr, T *dst,
                                                      int64_t ldd, int64_t N, int R) {
    __shared__ T sm[64][65];
    const int64_t t0 = (int64_t)blockIdx.x * 64;
    const int r0 = blockIdx.y * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        int rr = e & 63, tt = e >> 6;
        int64_t t = t0 + tt;
        T v = 0;
        if (t < N && r0 + rr < R) v = src[t * ldr + r0 + rr];
        sm[rr][tt] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        int tt = e & 63, rr = e >> 6;
        int64_t t = t0 + tt;
        if (t < N && r0 + rr < R) dst[(perm ? (int64_t)perm[t] : t) + (int64_t)(r0 + rr) * ldd] = sm[rr][tt];
    }
}

// out[r] = sum_i partial[i * R + r]: 16 columns x 16 part groups per
// workgroup, fixed summation order (deterministic)
__global__ void __launch_bounds__(256) k_reduce_rm(const double *partial, int nparts, int R, double *out) {
    const int cl = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int r = blockIdx.x * 16 + cl;
    double s = 0.0;
    if (r < R)
        for (int i = g; i < nparts; i += 16) s += partial[(int64_t)i * R + r];
    __shared__ double red[16][17];
    red[g][cl] = s;
    __syncthreads();
    if (g == 0 && r < R) {
        double tot = 0.0;
        for (int k = 0; k < 16; ++k) tot += red[k][cl];
        out[r] = tot;
    }
}

// Groups: out[k * R + r] = sum over the tiles of instance k, fixed order
__global__ void __launch_bounds__(256) k_reduce_inst(const double *partial, const int32_t *inst_tile, int R,
                                                      double *out) {
    const int k = blockIdx.y;
    const int cl = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int r = blockIdx.x * 16 + cl;
    const int t0 = inst_tile[k], t1 = inst_tile[k + 1];
    double s = 0.0;
    if (r < R)
        for (int i = t0 + g; i < t1; i += 16) s += partial[(int64_t)i * R + r];
    __shared__ double red[16][17];
    red[g][cl] = s;
    __syncthreads();
    if (g == 0 && r < R) {
        double tot = 0.0;
        for (int q = 0; q < 16; ++q) tot += red[q][cl];
        out[(int64_t)k * R + r] = tot;
    }
}

// partial[tile * R + r] = sum over the tile's 64 facets of E^2 (R-major)
template <class T>
__global__ void __launch_bounds__(256) k_colnorm_tiles(const T *E, int64_t N, int64_t ldr, int R, double *partial) {
    const int r = blockIdx.y * 256 + threadIdx.x;
    if (r >= R) return;
    const int64_t t0 = (int64_t)blockIdx.x * 64, t1 = min(N, t0 + 64);
    double s = 0.0;
    for (int64_t t = t0; t < t1; ++t) {
        double v = (double)E[t * ldr + r];
        s += v * v;
    }
    partial[(int64_t)blockIdx.x * R + r] = s;
}

constexpr int kRmParts = 64;

template <class T>
void proj_mm_t(const rad_hmat *H, const T *X, int64_t ldr, int R, hipStream_t s) {
    unsigned rtiles = (unsigned)((R + TN - 1) / TN);
    if (H->n_p1work > 0) {
        hipLaunchKernelGGL(k_proj_mm<T>, dim3(H->n_p1work, rtiles), dim3(256), 0, s, H->d_groups.p, H->d_p1work.p,
                           (const T *)H->d_vals.p, X, ldr, R, (T *)H->w_part.p);
        RAD_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_proj_reduce<T>, dim3(H->n_p1red * TM, (R + 255) / 256), dim3(256), 0, s, H->d_p1red.p,
                           (const T *)H->w_part.p, ldr, R, (T *)H->w_t.p);
        RAD_HIP(hipGetLastError());
    }
}

template <class T>
void apply_mm_t(const rad_hmat *H, const T *X, T *Y, int64_t ldr, int R, const T *E, const T *rho, T rho_s,
                double *partial, hipStream_t s) {
    proj_mm_t<T>(H, X, ldr, R, s);
    unsigned rtiles = (unsigned)((R + TN - 1) / TN);
    if (E)
        hipLaunchKernelGGL((k_tile_mm<T, true>), dim3(H->n_tiles, rtiles), dim3(256), 0, s, H->d_tiles.p, H->d_brow.p,
                           H->d_tile_tasks.p, (const T *)H->d_vals.p, H->d_csr_ptr.p, H->d_csr_idx.p,
                           H->csr_val_start, X, (const T *)H->w_t.p, ldr, R, H->N, Y, E, rho, rho_s, partial);
    else
        hipLaunchKernelGGL((k_tile_mm<T, false>), dim3(H->n_tiles, rtiles), dim3(256), 0, s, H->d_tiles.p,
                           H->d_brow.p, H->d_tile_tasks.p, (const T *)H->d_vals.p, H->d_csr_ptr.p, H->d_csr_idx.p,
                           H->csr_val_start, X, (const T *)H->w_t.p, ldr, R, H->N, Y, E, rho, rho_s, partial);
    RAD_HIP(hipGetLastError());
}

}  // namespace

int64_t mm_ldr(int64_t R) { return (R + 3) & ~(int64_t)3; }
int mm_part_rows() { return TM; }

void mm_to_rmajor(const rad_hmat *H, const void *src, int64_t lds, bool permute, void *dst, int64_t ldr, int64_t R,
                  hipStream_t s) {
    dim3 grid((unsigned)((H->N + 63) / 64), (unsigned)((R + 63) / 64));
    const int32_t *perm = permute ? H->d_perm.p : nullptr;
    if (H->dtype == RAD_F64)
        hipLaunchKernelGGL(k_to_rmajor<double>, grid, dim3(256), 0, s, perm, (const double *)src, lds, (double *)dst,
                           ldr, H->N, (int)R);
    else
        hipLaunchKernelGGL(k_to_rmajor<float>, grid, dim3(256), 0, s, perm, (const float *)src, lds, (float *)dst, ldr,
                           H->N, (int)R);
    RAD_HIP(hipGetLastError());
}

void mm_from_rmajor(const rad_hmat *H, const void *src, int64_t ldr, bool permute, void *dst, int64_t ldd, int64_t R,
                    hipStream_t s) {
    dim3 grid((unsigned)((H->N + 63) / 64), (unsigned)((R + 63) / 64));
    const int32_t *perm = permute ? H->d_perm.p : nullptr;
    if (H->dtype == RAD_F64)
        hipLaunchKernelGGL(k_from_rmajor<double>, grid, dim3(256), 0, s, perm, (const double *)src, ldr, (double *)dst,
                           ldd, H->N, (int)R);
    else
        hipLaunchKernelGGL(k_from_rmajor<float>, grid, dim3(256), 0, s, perm, (const float *)src, ldr, (float *)dst,
                           ldd, H->N, (int)R);
    RAD_HIP(hipGetLastError());
}

void mm_apply(const rad_hmat *H, const void *X, void *Y, int64_t ldr, int64_t R, hipStream_t s) {
    if (H->dtype == RAD_F64)
        apply_mm_t<double>(H, (const double *)X, (double *)Y, ldr, (int)R, nullptr, nullptr, 0.0, nullptr, s);
    else
        apply_mm_t<float>(H, (const float *)X, (float *)Y, ldr, (int)R, nullptr, nullptr, 0.0f, nullptr, s);
}

// one Jacobi iteration: B_new = E + rho * (F-hat B_old), norms[r] = ||B_new - B_old||^2
void mm_jacobi_step(const rad_hmat *H, const void *E, const void *rho, double rho_scalar, const void *Bold, void *Bnew,
                    int64_t ldr, int64_t R, double *norms, hipStream_t s) {
    double *part = (double *)H->w_red.p;
    if (H->dtype == RAD_F64)
        apply_mm_t<double>(H, (const double *)Bold, (double *)Bnew, ldr, (int)R, (const double *)E,
                           (const double *)rho, rho_scalar, part, s);
    else
        apply_mm_t<float>(H, (const float *)Bold, (float *)Bnew, ldr, (int)R, (const float *)E, (const float *)rho,
                          (float)rho_scalar, part, s);
    mm_reduce_cols(H, part, H->n_tiles, R, norms, s);
    RAD_HIP(hipGetLastError());
}

template <class T>
void time_phases_t(const rad_hmat *H, int R, int nrep, hipStream_t s, double *ms) {
    const int64_t ldr = mm_ldr(R);
    const T *X = (const T *)H->w_x.p;
    T *Y = (T *)H->w_b.p;
    const T *E = (const T *)H->w_e.p;
    double *part = (double *)H->w_red.p;
    unsigned rtiles = (unsigned)((R + TN - 1) / TN);
    hipEvent_t e0, e1;
    RAD_HIP(hipEventCreate(&e0));
    RAD_HIP(hipEventCreate(&e1));
    float t = 0;
    ms[0] = ms[1] = ms[2] = 0.0;
    if (H->n_p1work > 0) {
        RAD_HIP(hipEventRecord(e0, s));
        for (int i = 0; i < nrep; ++i)
            hipLaunchKernelGGL(k_proj_mm<T>, dim3(H->n_p1work, rtiles), dim3(256), 0, s, H->d_groups.p,
                               H->d_p1work.p, (const T *)H->d_vals.p, X, ldr, R, (T *)H->w_part.p);
        RAD_HIP(hipEventRecord(e1, s));
        RAD_HIP(hipEventSynchronize(e1));
        RAD_HIP(hipEventElapsedTime(&t, e0, e1));
        ms[0] = t / nrep;
        RAD_HIP(hipEventRecord(e0, s));
        for (int i = 0; i < nrep; ++i)
            hipLaunchKernelGGL(k_proj_reduce<T>, dim3(H->n_p1red * TM, (R + 255) / 256), dim3(256), 0, s,
                               H->d_p1red.p, (const T *)H->w_part.p, ldr, R, (T *)H->w_t.p);
        RAD_HIP(hipEventRecord(e1, s));
        RAD_HIP(hipEventSynchronize(e1));
        RAD_HIP(hipEventElapsedTime(&t, e0, e1));
        ms[1] = t / nrep;
    }
    RAD_HIP(hipEventRecord(e0, s));
    for (int i = 0; i < nrep; ++i)
        hipLaunchKernelGGL((k_tile_mm<T, true>), dim3(H->n_tiles, rtiles), dim3(256), 0, s, H->d_tiles.p, H->d_brow.p,
                           H->d_tile_tasks.p, (const T *)H->d_vals.p, H->d_csr_ptr.p, H->d_csr_idx.p,
                           H->csr_val_start, X, (const T *)H->w_t.p, ldr, R, H->N, Y, E, (const T *)nullptr, (T)0.3,
                           part);
    RAD_HIP(hipEventRecord(e1, s));
    RAD_HIP(hipEventSynchronize(e1));
    RAD_HIP(hipEventElapsedTime(&t, e0, e1));
    ms[2] = t / nrep;
    RAD_HIP(hipGetLastError());
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

void mm_time_phases(const rad_hmat *H, int64_t R, int nrep, hipStream_t s, double *ms) {
    if (H->dtype == RAD_F64)
        time_phases_t<double>(H, (int)R, nrep, s, ms);
    else
        time_phases_t<float>(H, (int)R, nrep, s, ms);
}

void mm_reduce_cols(const rad_hmat *H, const double *partial, int nparts, int64_t R, double *out, hipStream_t s) {
    if (H->n_inst > 1)
        hipLaunchKernelGGL(k_reduce_inst, dim3((unsigned)((R + 15) / 16), (unsigned)H->n_inst), dim3(256), 0, s,
                           partial, (const int32_t *)H->d_inst_tile.p, (int)R, out);
    else
        hipLaunchKernelGGL(k_reduce_rm, dim3((unsigned)((R + 15) / 16)), dim3(256), 0, s, partial, nparts, (int)R,
                           out);
    RAD_HIP(hipGetLastError());
}

size_t mm_reduction_doubles_for(const rad_hmat *H, int64_t R) {
    return (size_t)std::max<int64_t>(H->n_tiles, kRmParts) * (size_t)R;
}

void mm_col_norms2(const rad_hmat *H, const void *E, int64_t ldr, int64_t R, double *out, hipStream_t s) {
    dim3 grid((unsigned)H->n_tiles, (unsigned)((R + 255) / 256));
    double *part = (double *)H->w_red.p;
    if (H->dtype == RAD_F64)
        hipLaunchKernelGGL(k_colnorm_tiles<double>, grid, dim3(256), 0, s, (const double *)E, H->N, ldr, (int)R, part);
    else
        hipLaunchKernelGGL(k_colnorm_tiles<float>, grid, dim3(256), 0, s, (const float *)E, H->N, ldr, (int)R, part);
    mm_reduce_cols(H, part, H->n_tiles, R, out, s);
    RAD_HIP(hipGetLastError());
}

}  // namespace rad
