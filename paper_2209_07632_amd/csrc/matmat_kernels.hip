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

namespace rad {

namespace {

constexpr int TM = 64;    // output rows per workgroup
constexpr int TN = 128;   // output columns (right-hand sides) per workgroup
constexpr int KC = 32;    // reduction chunk
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

// B chunk: rows [brow, brow + kcount) of an R-major matrix, columns [r0, r0+TN)
template <class T>
__device__ __forceinline__ void load_b_rmajor(T (*sB)[TN + PADB], const T *src, int64_t brow, int kcount,
                                              int64_t ldr, int r0, int R, int t) {
    for (int e = t; e < KC * TN; e += 256) {
        int k = e / TN, c = e - k * TN;
        T v = 0;
        if (k < kcount && r0 + c < R) v = src[(brow + k) * ldr + r0 + c];
        sB[k][c] = v;
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
    __shared__ T sA[KC][TM + PADA];
    __shared__ T sB[KC][TN + PADB];
    Tile<T> tile;
    tile.zero();
    const int rows = min(TM, g.ktot - wk.krow0);
    const T *V = vals + g.v_off + (int64_t)wk.krow0 * g.ld;
    for (int kb = wk.jb; kb < wk.je; kb += KC) {
        const int kcount = min(KC, wk.je - kb);
        // A[row][k] = V[(kb + k) + row * ld]: threads walk k fastest (contiguous in V)
        for (int e = t; e < KC * TM; e += 256) {
            int r = e / KC, k = e - r * KC;
            T v = 0;
            if (k < kcount && r < rows) v = V[(int64_t)(kb + k) + (int64_t)r * g.ld];
            sA[k][r] = v;
        }
        load_b_rmajor(sB, X, (int64_t)g.j0 + kb, kcount, ldr, r0, R, t);
        __syncthreads();
        tile.mma(sA, sB, lane, w);
        __syncthreads();
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

// T rows = sum of the partial tiles of every split (fixed order)
template <class T>
__global__ void __launch_bounds__(256) k_proj_reduce(const P1Red *red, const T *part, int64_t ldr, int R, T *Tb) {
    const P1Red rd = red[blockIdx.x];
    const int c = blockIdx.y * 256 + threadIdx.x;
    if (c >= R) return;
    for (int row = 0; row < rd.nrows; ++row) {
        T s = 0;
        for (int p = 0; p < rd.part_count; ++p) s += part[((int64_t)(rd.part_begin + p) * TM + row) * ldr + c];
        Tb[(int64_t)(rd.t_row0 + row) * ldr + c] = s;
    }
}

// ---------------------------------------------------------------------------
// phase 2: per leaf
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) k_leaf_mm(const LeafInfo *leaves, const LeafTask *tasks, const T *vals,
                                                  const int32_t *csr_ptr, const int32_t *csr_idx,
                                                  int64_t csr_val_start, const T *X, const T *Tb, int64_t ldr, int R,
                                                  T *Y) {
    const LeafInfo L = leaves[blockIdx.x];
    const int r0 = blockIdx.y * TN;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    __shared__ T sA[KC][TM + PADA];
    __shared__ T sB[KC][TN + PADB];
    for (int rb = 0; rb < L.size; rb += TM) {
        const int rows = min(TM, L.size - rb);
        Tile<T> tile;
        tile.zero();
        for (int ti = L.task_begin; ti < L.task_end; ++ti) {
            const LeafTask tk = tasks[ti];
            if (tk.type == TASK_CSR) {
                const int32_t *ptr = csr_ptr + tk.aux_off;
                const T *v = vals + tk.a_off;
                const int32_t *ci = csr_idx + (tk.a_off - csr_val_start);
                int cur = 0, end = 0;
                if (t < rows) {
                    cur = ptr[rb + t];
                    end = ptr[rb + t + 1];
                }
                for (int kb = 0; kb < tk.ncol; kb += KC) {
                    const int kcount = min(KC, tk.ncol - kb);
                    for (int e = t; e < KC * TM; e += 256) sA[e / TM][e % TM] = 0;
                    __syncthreads();
                    if (t < rows) {
                        while (cur < end && ci[cur] < kb + KC) {
                            sA[ci[cur] - kb][t] = v[cur];
                            ++cur;
                        }
                    }
                    load_b_rmajor(sB, X, (int64_t)tk.col0 + kb, kcount, ldr, r0, R, t);
                    __syncthreads();
                    tile.mma(sA, sB, lane, w);
                    __syncthreads();
                }
            } else {
                const T *A = vals + tk.a_off + rb;
                const T *Bsrc = tk.type == TASK_DENSE ? X : Tb;
                for (int kb = 0; kb < tk.ncol; kb += KC) {
                    const int kcount = min(KC, tk.ncol - kb);
                    load_a_colmajor(sA, A, tk.ld, rows, kb, kcount, t);
                    load_b_rmajor(sB, Bsrc, (int64_t)tk.col0 + kb, kcount, ldr, r0, R, t);
                    __syncthreads();
                    tile.mma(sA, sB, lane, w);
                    __syncthreads();
                }
            }
        }
        const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    int row = i * 16 + Mfma<T>::row(lk, v);
                    int col = r0 + w * 32 + j * 16 + lr;
                    if (row < rows && col < R) Y[(int64_t)(L.start + rb + row) * ldr + col] = tile.acc[i][j][v];
                }
    }
}

// col-major (original or tree order) <-> R-major tree order
template <class T>
__global__ void k_to_rmajor(const int32_t *perm, const T *src, int64_t lds, T *dst, int64_t ldr, int64_t N, int R) {
    int64_t tot = N * (int64_t)R;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t t = e / R;
        int r = (int)(e - t * R);
        int64_t row = perm ? (int64_t)perm[t] : t;
        dst[t * ldr + r] = src[row + (int64_t)r * lds];
    }
}

template <class T>
__global__ void k_from_rmajor(const int32_t *perm, const T *src, int64_t ldr, T *dst, int64_t ldd, int64_t N, int R) {
    int64_t tot = N * (int64_t)R;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t t = e / R;
        int r = (int)(e - t * R);
        int64_t row = perm ? (int64_t)perm[t] : t;
        dst[row + (int64_t)r * ldd] = src[t * ldr + r];
    }
}

// Jacobi update in R-major layout; partial[block][r] = sum over the block's facets of (Bnew - Bold)^2
template <class T>
__global__ void __launch_bounds__(256) k_jacobi_rm(const T *E, const T *rho, T rho_s, const T *FB, const T *Bold,
                                                    T *Bnew, int64_t N, int64_t ldr, int R, double *partial) {
    const int r = blockIdx.y * 256 + threadIdx.x;
    if (r >= R) return;
    const int64_t per = (N + gridDim.x - 1) / gridDim.x;
    const int64_t t0 = blockIdx.x * per, t1 = min(N, t0 + per);
    double s = 0.0;
    for (int64_t t = t0; t < t1; ++t) {
        int64_t e = t * ldr + r;
        T rh = rho ? rho[t] : rho_s;
        T b = E[e] + rh * FB[e];
        double d = (double)b - (double)Bold[e];
        s += d * d;
        Bnew[e] = b;
    }
    partial[(int64_t)blockIdx.x * R + r] = s;
}

template <class T>
__global__ void __launch_bounds__(256) k_colnorm_rm(const T *E, int64_t N, int64_t ldr, int R, double *partial) {
    const int r = blockIdx.y * 256 + threadIdx.x;
    if (r >= R) return;
    const int64_t per = (N + gridDim.x - 1) / gridDim.x;
    const int64_t t0 = blockIdx.x * per, t1 = min(N, t0 + per);
    double s = 0.0;
    for (int64_t t = t0; t < t1; ++t) {
        double v = (double)E[t * ldr + r];
        s += v * v;
    }
    partial[(int64_t)blockIdx.x * R + r] = s;
}

__global__ void k_reduce_rm(const double *partial, int nparts, int R, double *out) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s += partial[(int64_t)i * R + r];
    out[r] = s;
}

constexpr int kRmParts = 64;

template <class T>
void apply_mm_t(const rad_hmat *H, const T *X, T *Y, int64_t ldr, int R, hipStream_t s) {
    unsigned rtiles = (unsigned)((R + TN - 1) / TN);
    if (H->n_p1work > 0) {
        hipLaunchKernelGGL(k_proj_mm<T>, dim3(H->n_p1work, rtiles), dim3(256), 0, s, H->d_groups.p, H->d_p1work.p,
                           (const T *)H->d_vals.p, X, ldr, R, (T *)H->w_part.p);
        RAD_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_proj_reduce<T>, dim3(H->n_p1red, (R + 255) / 256), dim3(256), 0, s, H->d_p1red.p,
                           (const T *)H->w_part.p, ldr, R, (T *)H->w_t.p);
        RAD_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_leaf_mm<T>, dim3(H->n_leaves, rtiles), dim3(256), 0, s, H->d_leaves.p, H->d_tasks.p,
                       (const T *)H->d_vals.p, H->d_csr_ptr.p, H->d_csr_idx.p, H->csr_val_start, X,
                       (const T *)H->w_t.p, ldr, R, Y);
    RAD_HIP(hipGetLastError());
}

}  // namespace

int64_t mm_ldr(int64_t R) { return (R + 3) & ~(int64_t)3; }
int mm_part_rows() { return TM; }
size_t mm_reduction_doubles(int64_t R) { return (size_t)kRmParts * (size_t)R; }

void mm_to_rmajor(const rad_hmat *H, const void *src, int64_t lds, bool permute, void *dst, int64_t ldr, int64_t R,
                  hipStream_t s) {
    int64_t tot = H->N * R;
    unsigned blocks = (unsigned)std::min<int64_t>((tot + 255) / 256, 16384);
    const int32_t *perm = permute ? H->d_perm.p : nullptr;
    if (H->dtype == RAD_F64)
        hipLaunchKernelGGL(k_to_rmajor<double>, dim3(blocks), dim3(256), 0, s, perm, (const double *)src, lds,
                           (double *)dst, ldr, H->N, (int)R);
    else
        hipLaunchKernelGGL(k_to_rmajor<float>, dim3(blocks), dim3(256), 0, s, perm, (const float *)src, lds,
                           (float *)dst, ldr, H->N, (int)R);
    RAD_HIP(hipGetLastError());
}

void mm_from_rmajor(const rad_hmat *H, const void *src, int64_t ldr, bool permute, void *dst, int64_t ldd, int64_t R,
                    hipStream_t s) {
    int64_t tot = H->N * R;
    unsigned blocks = (unsigned)std::min<int64_t>((tot + 255) / 256, 16384);
    const int32_t *perm = permute ? H->d_perm.p : nullptr;
    if (H->dtype == RAD_F64)
        hipLaunchKernelGGL(k_from_rmajor<double>, dim3(blocks), dim3(256), 0, s, perm, (const double *)src, ldr,
                           (double *)dst, ldd, H->N, (int)R);
    else
        hipLaunchKernelGGL(k_from_rmajor<float>, dim3(blocks), dim3(256), 0, s, perm, (const float *)src, ldr,
                           (float *)dst, ldd, H->N, (int)R);
    RAD_HIP(hipGetLastError());
}

void mm_apply(const rad_hmat *H, const void *X, void *Y, int64_t ldr, int64_t R, hipStream_t s) {
    if (H->dtype == RAD_F64)
        apply_mm_t<double>(H, (const double *)X, (double *)Y, ldr, (int)R, s);
    else
        apply_mm_t<float>(H, (const float *)X, (float *)Y, ldr, (int)R, s);
}

void mm_col_norms2(const rad_hmat *H, const void *E, int64_t ldr, int64_t R, double *out, hipStream_t s) {
    dim3 grid(kRmParts, (unsigned)((R + 255) / 256));
    double *part = (double *)H->w_red.p;
    if (H->dtype == RAD_F64)
        hipLaunchKernelGGL(k_colnorm_rm<double>, grid, dim3(256), 0, s, (const double *)E, H->N, ldr, (int)R, part);
    else
        hipLaunchKernelGGL(k_colnorm_rm<float>, grid, dim3(256), 0, s, (const float *)E, H->N, ldr, (int)R, part);
    hipLaunchKernelGGL(k_reduce_rm, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, s, part, kRmParts, (int)R, out);
    RAD_HIP(hipGetLastError());
}

void mm_solve_update(const rad_hmat *H, const void *E, const void *rho, double rho_scalar, const void *FB,
                     const void *Bold, void *Bnew, int64_t ldr, int64_t R, double *norms, hipStream_t s) {
    dim3 grid(kRmParts, (unsigned)((R + 255) / 256));
    double *part = (double *)H->w_red.p;
    if (H->dtype == RAD_F64)
        hipLaunchKernelGGL(k_jacobi_rm<double>, grid, dim3(256), 0, s, (const double *)E, (const double *)rho,
                           rho_scalar, (const double *)FB, (const double *)Bold, (double *)Bnew, H->N, ldr, (int)R,
                           part);
    else
        hipLaunchKernelGGL(k_jacobi_rm<float>, grid, dim3(256), 0, s, (const float *)E, (const float *)rho,
                           (float)rho_scalar, (const float *)FB, (const float *)Bold, (float *)Bnew, H->N, ldr,
                           (int)R, part);
    hipLaunchKernelGGL(k_reduce_rm, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, s, part, kRmParts, (int)R, norms);
    RAD_HIP(hipGetLastError());
}

}  // namespace rad
