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

#include <type_traits>

#include <algorithm>
#include <cstdio>
#include <vector>

#include "rad_internal.h"
#include "mm_epilogue.h"

namespace rad {

namespace {

constexpr int TM = 64;    // output rows per workgroup; TN (64 or 128) columns is a template parameter
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

// acc[i][j]: row tile i (16 rows), column tile j (16 columns of this wave's TN / 4)
// Minimum waves per SIMD asked of the compiler: the FP32 64-column kernels
// fit six (no spills), which hides more of their memory latency; the others
// keep the compiler's choice.
template <class T, int TN>
constexpr int kWavesPerEu = (sizeof(T) == 4 && TN == 64) ? 6 : 1;

// MI row tiles of 16 (64 rows for the expansion, 128 for paired projections)
template <class T, int TN, int MI = 4>
struct Tile {
    static constexpr int NJ = TN / 64;
    typename Mfma<T>::acc_t acc[MI][NJ];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;
    }
    // one chunk of KC from LDS: sA[k][row], sB[k][col]; only the first MION row
    // tiles are computed (the others hold zero rows).  Instruction s takes
    // k = (KC / 4) lk + s in lane group lk: with row strides of 4 (mod 16)
    // values the four groups read disjoint LDS banks.
    template <int MION = MI>
    __device__ __forceinline__ void mma(const T (*sA)[MI * 16 + PADA], const T (*sB)[TN + PADB], int lane, int w) {
        const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int s = 0; s < KC / 4; ++s) {
            const int k = lk * (KC / 4) + s;
            T a[MION], b[NJ];
#pragma unroll
            for (int i = 0; i < MION; ++i) a[i] = sA[k][i * 16 + lr];
#pragma unroll
            for (int j = 0; j < NJ; ++j) b[j] = sB[k][w * (TN / 4) + j * 16 + lr];
#pragma unroll
            for (int i = 0; i < MION; ++i)
#pragma unroll
                for (int j = 0; j < NJ; ++j) acc[i][j] = Mfma<T>::run(a[i], b[j], acc[i][j]);
        }
    }
};

// B chunk: rows [brow, brow + kcount) of an R-major matrix, columns [r0, r0+TN).
// ldr and r0 are multiples of 4, so groups of four columns are loaded as one
// 16-byte (FP32) or two 16-byte (FP64) vectors.
template <class T, int TN>
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
//          kind 1 = transposed V (A[r][k] = V[k + r * ld], r < r_hi),
//          kind 2 = complete CSR rows (A[r][k] = A[rb[r] + k], r in [r_lo, r_hi)).
template <class T, int TN>
struct Stage {
    T a[KC * TM / 256];
    T b[KC * TN / 256];
    __device__ __forceinline__ void fetch(int kind, const T *A, int64_t ld, int row_off, int r_lo, int r_hi, int kb,
                                          int kcount, const T *B, int64_t brow, int64_t ldr, int r0, int R, int t,
                                          const int32_t *rb = nullptr) {
#pragma unroll
        for (int q = 0; q < KC * TM / 256; ++q) {
            int e = t + q * 256;
            T v = 0;
            if (kind == 0) {
                int k = e / TM, r = e - k * TM;
                if (k < kcount && r >= r_lo && r < r_hi) v = A[(int64_t)(row_off + r) + (int64_t)(kb + k) * ld];
            } else if (kind == 2) {
                int r = e / KC, k = e - r * KC;
                if (k < kcount && r >= r_lo && r < r_hi) v = A[(int64_t)rb[r] + kb + k];
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
template <class T, int TN>
struct PanelStage {
    T a[KC * TM / 256];
    T b[KC * TN / 256];
    // the operand-row indices this thread gathers for a chunk (loaded a chunk
    // ahead of their use, so that the dependent row loads do not wait)
    struct Rows {
        int32_t v[KC * TN / 1024];
        __device__ __forceinline__ void load(const int32_t *brc, int t) {
#pragma unroll
            for (int q = 0; q < KC * TN / 1024; ++q) v[q] = brc[(t + q * 256) / (TN / 4)];
        }
    };
    __device__ __forceinline__ void fetch(const T *pan, const Rows &rw, const T *X, const T *Tb, int64_t ldr, int r0,
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
            int32_t v = rw.v[q];
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

// Workgroups are dispatched to the 8 XCDs round-robin by linear index; this
// maps dispatch index L to a work index so that each XCD receives one
// contiguous run of work items (neighbouring tiles, which gather the same
// operand rows, then share that XCD's L2).  A bijection on [0, total).
__device__ __forceinline__ int xcd_remap(int L, int total) {
    constexpr int kXcd = 8;
    const int q = total / kXcd, rem = total % kXcd;
    const int x = L % kXcd, slot = L / kXcd;
    return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + slot;
}

// ---------------------------------------------------------------------------
// phase 1: partial projections
// ---------------------------------------------------------------------------
// Stage of the projections: 128 rows of V_J^T (A[r][k] = V[k + r ld], r < rows)
// and KC rows of X.
template <class T, int TN>
struct P1Stage {
    static constexpr int RA = 128;
    static constexpr int VW = 16 / sizeof(T);   // V values per 16-byte load
    T a[KC * RA / 256];
    T b[KC * TN / 256];
    // A: each thread loads VW consecutive k of one V column with one 16-byte
    // load (V columns start on 8-value boundaries, kb on KC boundaries)
    __device__ __forceinline__ void fetch(const T *V, int64_t ld, int rows, int kb, int kcount, const T *X,
                                          int64_t xrow, int64_t ldr, int r0, int R, int t) {
#pragma unroll
        for (int q = 0; q < KC * RA / 256 / VW; ++q) {
            const int e = t + q * 256, r = e / (KC / VW), k = (e % (KC / VW)) * VW;
            const T *p = V + (int64_t)(kb + k) + (int64_t)r * ld;
            if (r < rows && k + VW <= kcount) {
                if constexpr (sizeof(T) == 4) {
                    const float4 v = *(const float4 *)p;
                    a[VW * q] = v.x; a[VW * q + 1] = v.y; a[VW * q + 2] = v.z; a[VW * q + 3] = v.w;
                } else {
                    const double2 v = *(const double2 *)p;
                    a[VW * q] = v.x; a[VW * q + 1] = v.y;
                }
            } else {
#pragma unroll
                for (int u = 0; u < VW; ++u) a[VW * q + u] = (r < rows && k + u < kcount) ? p[u] : (T)0;
            }
        }
#pragma unroll
        for (int q = 0; q < KC * TN / 1024; ++q) {
            const int e = t + q * 256, k = e / (TN / 4), c = (e - k * (TN / 4)) * 4;
            T v0 = 0, v1 = 0, v2 = 0, v3 = 0;
            if (k < kcount) {
                const T *p = X + (xrow + k) * ldr + r0 + c;
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
    __device__ __forceinline__ void commit(T (*sA)[RA + PADA], T (*sB)[TN + PADB], int t) {
#pragma unroll
        for (int q = 0; q < KC * RA / 256 / VW; ++q) {
            const int e = t + q * 256, r = e / (KC / VW), k = (e % (KC / VW)) * VW;
#pragma unroll
            for (int u = 0; u < VW; ++u) sA[k + u][r] = a[VW * q + u];
        }
#pragma unroll
        for (int q = 0; q < KC * TN / 1024; ++q) {
            const int e = t + q * 256, k = e / (TN / 4), c = (e - k * (TN / 4)) * 4;
            sB[k][c] = b[4 * q];
            sB[k][c + 1] = b[4 * q + 1];
            sB[k][c + 2] = b[4 * q + 2];
            sB[k][c + 3] = b[4 * q + 3];
        }
    }
};

// Partial projections of up to two work items that share a facet chunk
// (consecutive 64-row slabs of V_J^T): the X chunk is staged once for 128 rows.
// A pair whose slabs have no other work item (direct[pair] = their first T
// row) writes its rows of T itself; the others write partial tiles.
template <class T, int TN>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kWavesPerEu<T, TN>, 8)))
k_proj_mm(const ProjGroup *groups, const P1Work *work, const int32_t *pairs, const int32_t *direct,
                                                  const T *vals, const T *X, int64_t ldr, int R, T *part, T *Tb,
                                                  int rtiles, const int32_t *stop) {
    if (stop && *stop) return;
    const int wi = xcd_remap(blockIdx.x, gridDim.x);
    const int p0 = pairs[2 * (wi / rtiles)], p1 = pairs[2 * (wi / rtiles) + 1];
    const int drow = direct[wi / rtiles];
    const P1Work wk = work[p0];
    const ProjGroup g = groups[wk.group];
    const int r0 = (wi % rtiles) * TN;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    __shared__ T sA[2][KC][128 + PADA];
    __shared__ T sB[2][KC][TN + PADB];
    Tile<T, TN, 8> tile;
    tile.zero();
    const int rows = min(p1 >= 0 ? 128 : TM, g.ktot - wk.krow0);
    const T *V = vals + g.v_off + (int64_t)wk.krow0 * g.ld;
    // the reduction loop for MION active row tiles (all-zero row tiles of the
    // slab are skipped): one straight-line instance per count
    auto reduce = [&](auto mion) {
        constexpr int MION = decltype(mion)::value;
        P1Stage<T, TN> st;
        int buf = 0;
        st.fetch(V, g.ld, rows, wk.jb, min(KC, wk.je - wk.jb), X, (int64_t)g.j0 + wk.jb, ldr, r0, R, t);
        for (int kb = wk.jb; kb < wk.je; kb += KC) {
            st.commit(sA[buf], sB[buf], t);
            __syncthreads();
            const int nk = kb + KC;
            if (nk < wk.je) st.fetch(V, g.ld, rows, nk, min(KC, wk.je - nk), X, (int64_t)g.j0 + nk, ldr, r0, R, t);
            tile.template mma<MION>(sA[buf], sB[buf], lane, w);
            buf ^= 1;
        }
    };
    switch ((rows + 15) / 16) {
        case 1: reduce(std::integral_constant<int, 1>{}); break;
        case 2: reduce(std::integral_constant<int, 2>{}); break;
        case 3: reduce(std::integral_constant<int, 3>{}); break;
        case 4: reduce(std::integral_constant<int, 4>{}); break;
        case 5: reduce(std::integral_constant<int, 5>{}); break;
        case 6: reduce(std::integral_constant<int, 6>{}); break;
        case 7: reduce(std::integral_constant<int, 7>{}); break;
        default: reduce(std::integral_constant<int, 8>{}); break;
    }
    const int lr = lane & 15, lk = lane >> 4;
    if (drow >= 0) {
        // rows [0, rows) are T rows drow.. (the pair's slabs are consecutive)
        T *out = Tb + (int64_t)drow * ldr;
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < TN / 64; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = i * 16 + Mfma<T>::row(lk, v);
                    const int col = r0 + w * (TN / 4) + j * 16 + lr;
                    if (row < rows && col < R) out[(int64_t)row * ldr + col] = tile.acc[i][j][v];
                }
        return;
    }
    T *out0 = part + (int64_t)wk.part * TM * ldr;
    T *out1 = p1 >= 0 ? part + (int64_t)work[p1].part * TM * ldr : nullptr;
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < TN / 64; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = i * 16 + Mfma<T>::row(lk, v);
                const int col = r0 + w * (TN / 4) + j * 16 + lr;
                T *out = row < TM ? out0 : out1;
                if (out && col < R) out[(int64_t)(row & (TM - 1)) * ldr + col] = tile.acc[i][j][v];
            }
}

// out[dst[i]] = vals[i] for entries with dst[i] >= 0
template <class T>
__global__ void k_csr_panel_scatter(const T *vals, const int64_t *dst, int64_t n, T *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = dst[i];
        if (d >= 0) out[d] = vals[i];
    }
}

dim3 reduce_grid(int32_t nred, int64_t R) { return dim3((unsigned)nred, 4, (unsigned)((R + 255) / 256)); }

// T rows = sum of the partial tiles of every split (fixed order).  Grid
// (slabs, 4, column blocks of 256): 16 rows of a slab per workgroup, four
// consecutive columns per thread (four rows at a time)
template <class T>
__global__ void __launch_bounds__(256) k_proj_reduce(const P1Red *red, const T *part, int64_t ldr, int R, T *Tb,
                                                     const int32_t *stop) {
    if (stop && *stop) return;
    typedef typename std::conditional<sizeof(T) == 4, float4, double4>::type V;
    const P1Red rd = red[blockIdx.x];
    const int c = ((int)blockIdx.z * 64 + (int)(threadIdx.x & 63)) * 4;
    if (c >= R) return;
    const int r1 = min(rd.nrows, (int)blockIdx.y * 16 + 16);
    for (int row = (int)blockIdx.y * 16 + (int)(threadIdx.x >> 6); row < r1; row += 4) {
        const V sv = ordered_sum4((const V *)(part + ((int64_t)rd.part_begin * TM + row) * ldr + c),
                                  (int64_t)TM * ldr / 4, rd.part_count);
        const T v[4] = {sv.x, sv.y, sv.z, sv.w};
        T *out = Tb + (int64_t)(rd.t_row0 + row) * ldr + c;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (c + u < R) out[u] = v[u];
    }
}

// ---------------------------------------------------------------------------
// phase 2: one workgroup per (64-row tile, 128-column tile).  With E given,
// the epilogue performs the Jacobi update B_new = E + rho * (F B_old) and
// writes the per-column partial sums of (B_new - B_old)^2 for this tile.
// ---------------------------------------------------------------------------
template <class T, int TN>
struct TileSmem {
    static constexpr int kPipe = 2 * KC * (TM + PADA) + 2 * KC * (TN + PADB);
    static constexpr int kOut = TM * (TN + PADB);
    static constexpr int kSize = kPipe > kOut ? kPipe : kOut;
    static_assert(1024 * sizeof(double) <= sizeof(T) * kSize, "partial sums fit");
};

// kMode: 0 = Y = F X; 1 = fused Jacobi update; 2 = fused, plus ||E||^2 partials
template <class T, int kMode, int TN>
__device__ __forceinline__ void tile_body(T *smem, int tile, int rt, const TileInfo *tiles, const int32_t *brow,
                                          const TileTask *ctasks, const T *vals, const int32_t *csr_ptr,
                                          const int32_t *csr_idx, int64_t csr_val_start, const CsrPanel *cpan,
                                          const T *cvals, const int32_t *cbrow, const T *X, const T *Tb,
                                          int64_t ldr, int R, int64_t N, T *Y, const T *E, const T *rho, T rho_s,
                                          double *partial, double *epartial) {
    const TileInfo ti = tiles[tile];
    const int64_t tile0 = (int64_t)tile * TM;
    const int r0 = rt * TN;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    // pipeline buffers during the reduction, the 64 x TN result tile after it
    T (*sA)[KC][TM + PADA] = (T (*)[KC][TM + PADA])smem;
    T (*sB)[KC][TN + PADB] = (T (*)[KC][TN + PADB])(smem + 2 * KC * (TM + PADA));
    Tile<T, TN> acc;
    acc.zero();
    // CSR tasks: rows expanded into dense chunks in LDS (when the schedule
    // made no compressed panels of them)
    for (int c = cpan ? ti.csr_end : ti.csr_begin; c < ti.csr_end; ++c) {
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
            load_b_rmajor<T, TN>(sB[0], X, (int64_t)tk.col0 + kb, kcount, ldr, r0, R, t);
            __syncthreads();
            acc.mma(sA[0], sB[0], lane, w);
            __syncthreads();
        }
    }
    // packed panels: the tile's compressed CSR panel (if any), then its dense
    // and low-rank panel, each through a software pipeline with two register
    // stages in flight (chunk c + 2 loads while chunk c runs on the matrix
    // cores); columns past k16 are zero padding of the 16-bit chunk width
    const CsrPanel cp = cpan ? cpan[tile] : CsrPanel{0, 0, 0, 0};
    for (int pass = cp.k16 > 0 ? 0 : 1; pass < 2; ++pass) {
        const int kend = pass == 0 ? cp.k16 : ti.k16;
        if (kend == 0) continue;
        const T *pan = pass == 0 ? cvals + cp.panel_off : vals + ti.panel_off;
        const int32_t *br = pass == 0 ? cbrow + cp.brow_off : brow + ti.brow_off;
        if (pass == 1 && cp.k16 > 0) __syncthreads();   // the first panel's last chunk is read
        PanelStage<T, TN> st0, st1;
        // row indices of the chunks st0 / st1 fetch next
        typename PanelStage<T, TN>::Rows rw0, rw1;
        auto fetch = [&](PanelStage<T, TN> &st, typename PanelStage<T, TN>::Rows &rw, int kb) {
            st.fetch(pan + (int64_t)kb * TM, rw, X, Tb, ldr, r0, R, t);
            if (kb + 2 * KC < kend) rw.load(br + kb + 2 * KC, t);
        };
        rw0.load(br, t);
        if (KC < kend) rw1.load(br + KC, t);
        fetch(st0, rw0, 0);
        if (KC < kend) fetch(st1, rw1, KC);
        for (int kb = 0; kb < kend; kb += 2 * KC) {
            st0.commit(sA[0], sB[0], t);
            __syncthreads();
            if (kb + 2 * KC < kend) fetch(st0, rw0, kb + 2 * KC);
            acc.mma(sA[0], sB[0], lane, w);
            if (kb + KC >= kend) break;
            st1.commit(sA[1], sB[1], t);
            __syncthreads();
            if (kb + 3 * KC < kend) fetch(st1, rw1, kb + 3 * KC);
            acc.mma(sA[1], sB[1], lane, w);
        }
    }
    // epilogue through LDS: the result tile is written to LDS, then every
    // thread streams 16-byte groups of whole rows (coalesced E, B_old, B_new
    // accesses).  Per-column partial sums are reduced in a fixed order.
    __syncthreads();
    T (*sC)[TN + PADB] = (T (*)[TN + PADB])smem;
    {
        const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < TN / 64; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    sC[i * 16 + Mfma<T>::row(lk, v)][w * (TN / 4) + j * 16 + lr] = acc.acc[i][j][v];
    }
    __syncthreads();
    tile_epilogue<T, kMode != 0, TM, TN, TN + PADB, kMode == 2>(sC, smem, tile, tile0, r0, ldr, R, N, Y, E, X, rho,
                                                                rho_s, partial, epartial);
}

// one workgroup per (64-row tile, TN-column tile); 1-D grid, XCD-aware order
template <class T, int kMode, int TN>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kWavesPerEu<T, TN>, 8)))
k_tile_mm(const TileInfo *tiles, const int32_t *brow, const TileTask *ctasks,
                                                  const T *vals, const int32_t *csr_ptr, const int32_t *csr_idx,
                                                  int64_t csr_val_start, const CsrPanel *cpan, const T *cvals,
                                                  const int32_t *cbrow, const T *X, const T *Tb, int64_t ldr, int R,
                                                  int64_t N, T *Y, const T *E, const T *rho, T rho_s,
                                                  double *partial, double *epartial, int rtiles, const int32_t *stop) {
    if (stop && *stop) return;
    __shared__ T smem[TileSmem<T, TN>::kSize];
    const int wi = xcd_remap(blockIdx.x, gridDim.x);
    tile_body<T, kMode, TN>(smem, wi / rtiles, wi % rtiles, tiles, brow, ctasks, vals, csr_ptr, csr_idx,
                            csr_val_start, cpan, cvals, cbrow, X, Tb, ldr, R, N, Y, E, rho, rho_s, partial, epartial);
}

// Persistent form: a fixed grid pulls work items (tiles in decreasing cost
// order, all column tiles of a tile in a row) from a counter.  Every
// workgroup leaves when the counter passes nwork; the last one to leave
// resets both counters for the next launch (no memset in captured graphs).
template <class T, int kMode, int TN>
__global__ void __launch_bounds__(256) k_tile_mm_q(const TileInfo *tiles, const int32_t *brow,
                                                    const TileTask *ctasks, const T *vals, const int32_t *csr_ptr,
                                                    const int32_t *csr_idx, int64_t csr_val_start,
                                                    const CsrPanel *cpan, const T *cvals, const int32_t *cbrow,
                                                    const T *X,
                                                    const T *Tb, int64_t ldr, int R, int64_t N, T *Y, const T *E,
                                                    const T *rho, T rho_s, double *partial, double *epartial,
                                                    const int32_t *order,
                                                    int nwork, int rtiles, int *queue, const int32_t *stop) {
    if (stop && *stop) return;   // (before the counters: they stay at zero)
    __shared__ T smem[TileSmem<T, TN>::kSize];
    __shared__ int item;
    while (true) {
        if (threadIdx.x == 0) item = atomicAdd(&queue[0], 1);
        __syncthreads();
        const int wi = item;
        __syncthreads();
        if (wi >= nwork) break;
        tile_body<T, kMode, TN>(smem, order[wi / rtiles], wi % rtiles, tiles, brow, ctasks, vals, csr_ptr, csr_idx,
                                csr_val_start, cpan, cvals, cbrow, X, Tb, ldr, R, N, Y, E, rho, rho_s, partial,
                                epartial);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&queue[1], 1) == (int)gridDim.x - 1) {
            queue[0] = 0;
            queue[1] = 0;
            __threadfence();
        }
    }
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

// out[k * R + r] = sum over parts [t0, t1) of column r, where [t0, t1) is
// [inst_tile[k], inst_tile[k + 1]) for instance k of a group, else [0, nparts).
// Sixteen part classes (i mod 16) summed in order, then the classes in order:
// the same fixed order for a matrix and for each instance of a group.  The loads
// of a class are independent of its additions, so eight are kept in flight.
__global__ void __launch_bounds__(256) k_reduce_parts(const double *partial, const int32_t *inst_tile, int nparts,
                                                      int R, double *out, const int32_t *stop) {
    if (stop && *stop) return;
    const int k = blockIdx.y;
    const int cl = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int r = blockIdx.x * 16 + cl;
    const int t0 = inst_tile ? inst_tile[k] : 0, t1 = inst_tile ? inst_tile[k + 1] : nparts;
    double s = 0.0;
    if (r < R) {
        const double *p = partial + r;
        int i = t0 + g;
        for (; i + 7 * 16 < t1; i += 8 * 16) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(i + 16 * u) * R];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; i < t1; i += 16) s += p[(int64_t)i * R];
    }
    __shared__ double red[16][17];
    red[g][cl] = s;
    __syncthreads();
    if (g == 0 && r < R) {
        double tot = 0.0;
        for (int q = 0; q < 16; ++q) tot += red[q][cl];
        out[(int64_t)k * R + r] = tot;
    }
}

// The stopping test on the sums of the reduction before it (one workgroup;
// returns at once while *stop is set, as the kernels of a skipped iteration do)
__global__ void __launch_bounds__(1024) k_conv_test(const double *out, ConvTest test) {
    if (test.mode == 1 && *test.stop) return;
    int all = 1;
    for (int c = threadIdx.x; c < test.nc; c += 1024) {
        int v;
        if (test.mode == 1) {
            const double d = out[c];
            v = test.conv[c] | (d <= test.thr[c] ? 1 : 0);
            if (test.hdn) test.hdn[c] = d;
        } else {
            const double e = out[c], d = test.dn[c];
            const double th = e > 0 ? test.rtol2 * e : test.rtol2;
            test.thr[c] = th;
            v = d <= th ? 1 : 0;
            if (test.hdn) test.hdn[c] = d;
            if (test.hen) test.hen[c] = e;
        }
        test.conv[c] = v;
        all &= v;
    }
    all = __syncthreads_and(all);
    if (threadIdx.x == 0) *test.stop = all;
}

// thr[c] = rtol2 enorm2[c] (rtol2 when 0); conv[c] and the stop flag cleared
__global__ void __launch_bounds__(256) k_conv_init(const double *enorm2, double rtol2, int nc, double *thr,
                                                   int32_t *conv, int32_t *stop) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c < nc) {
        const double e = enorm2[c];
        thr[c] = e > 0 ? rtol2 * e : rtol2;
        conv[c] = 0;
    }
    if (c == 0) *stop = 0;
}

// partial[tile * R + r] = sum over the tile's 64 facets of E^2 (R-major).
// A workgroup covers one tile and 256 columns: each thread four columns
// (16-byte loads) over 16 of the 64 rows, the
// four row quarters meeting in LDS in a fixed order.
template <class T>
__global__ void __launch_bounds__(256) k_colnorm_tiles(const T *E, int64_t N, int64_t ldr, int R, double *partial) {
    const int c4 = blockIdx.y * 256 + (threadIdx.x & 63) * 4;
    const int quarter = threadIdx.x >> 6;
    const int64_t t0 = (int64_t)blockIdx.x * 64 + quarter * 16;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int i = 0; i < 16; ++i) {
        const int64_t t = t0 + i;
        if (t < N) {
            const T *p = E + t * ldr + c4;
            if (c4 + 3 < R) {
                T v[4];
                if constexpr (sizeof(T) == 4) {
                    const float4 q = *(const float4 *)p;
                    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
                } else {
                    const double2 q0 = *(const double2 *)p, q1 = *(const double2 *)(p + 2);
                    v[0] = q0.x; v[1] = q0.y; v[2] = q1.x; v[3] = q1.y;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) s[u] += (double)v[u] * (double)v[u];
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (c4 + u < R) {
                        const double v = (double)p[u];
                        s[u] += v * v;
                    }
            }
        }
    }
    __shared__ double red[4][256];
#pragma unroll
    for (int u = 0; u < 4; ++u) red[quarter][(threadIdx.x & 63) * 4 + u] = s[u];
    __syncthreads();
    const int c = blockIdx.y * 256 + threadIdx.x;
    if (c < R)
        partial[(int64_t)blockIdx.x * R + c] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

constexpr int kRmParts = 64;

template <class T, int TN>
void proj_mm_tn(const rad_hmat *H, const T *X, int64_t ldr, int R, hipStream_t s, const int32_t *stop = nullptr) {
    unsigned rtiles = (unsigned)((R + TN - 1) / TN);
    if (H->n_p1work > 0) {
        hipLaunchKernelGGL((k_proj_mm<T, TN>), dim3(H->n_p1pairs * rtiles), dim3(256), 0, s, H->d_groups.p,
                           H->d_p1work.p, (const int32_t *)H->d_p1pairs.p, (const int32_t *)H->d_p1direct.p,
                           (const T *)H->d_vals.p, X, ldr, R, (T *)H->w_part.p, (T *)H->w_t.p, (int)rtiles, stop);
        RAD_HIP(hipGetLastError());
        if (H->n_p1red_multi > 0) {
            hipLaunchKernelGGL(k_proj_reduce<T>, reduce_grid(H->n_p1red_multi, R), dim3(256), 0, s,
                               H->d_p1red_multi.p, (const T *)H->w_part.p, ldr, R, (T *)H->w_t.p, stop);
            RAD_HIP(hipGetLastError());
        }
    }
}

template <class T, int kMode, int TN>
void tile_mm_launch(const rad_hmat *H, const MmConfig &c, const T *X, T *Y, int64_t ldr, int R, const T *E,
                    const T *rho, T rho_s, double *partial, hipStream_t s, const int32_t *stop = nullptr,
                    double *epartial = nullptr) {
    const int rtiles = (R + TN - 1) / TN;
    const CsrPanel *cpan = H->n_cpan > 0 ? H->d_cpan.p : nullptr;
    if (c.persistent) {
        const int nwork = H->n_tiles * rtiles;
        const int grid = std::max(1, std::min(nwork, H->n_cu * std::max(1, (int)c.blocks_per_cu)));
        hipLaunchKernelGGL((k_tile_mm_q<T, kMode, TN>), dim3(grid), dim3(256), 0, s, H->d_tiles.p, H->d_brow.p,
                           H->d_tile_tasks.p, (const T *)H->d_vals.p, H->d_csr_ptr.p, H->d_csr_idx.p,
                           H->csr_val_start, cpan, (const T *)H->d_cvals.p, H->d_cbrow.p, X, (const T *)H->w_t.p,
                           ldr, R, H->N, Y, E, rho, rho_s, partial,
                           epartial, (const int32_t *)H->d_tile_order.p, nwork, rtiles, H->d_queue.p, stop);
    } else {
        hipLaunchKernelGGL((k_tile_mm<T, kMode, TN>), dim3((unsigned)(H->n_tiles * rtiles)), dim3(256), 0, s,
                           H->d_tiles.p, H->d_brow.p, H->d_tile_tasks.p, (const T *)H->d_vals.p, H->d_csr_ptr.p,
                           H->d_csr_idx.p, H->csr_val_start, cpan, (const T *)H->d_cvals.p, H->d_cbrow.p, X,
                           (const T *)H->w_t.p, ldr, R, H->N, Y, E, rho, rho_s,
                           partial, epartial, rtiles, stop);
    }
    RAD_HIP(hipGetLastError());
}

// projections with at most 128-column tiles (their accumulators hold 128 rows)
template <class T, int TN>
void apply_mm_tn(const rad_hmat *H, const MmConfig &c, const T *X, T *Y, int64_t ldr, int R, const T *E, const T *rho,
                 T rho_s, double *partial, hipStream_t s, const int32_t *stop = nullptr, double *epartial = nullptr) {
    proj_mm_tn<T, (TN > 128 ? 128 : TN)>(H, X, ldr, R, s, stop);
    if (E && epartial)
        tile_mm_launch<T, 2, TN>(H, c, X, Y, ldr, R, E, rho, rho_s, partial, s, stop, epartial);
    else if (E)
        tile_mm_launch<T, 1, TN>(H, c, X, Y, ldr, R, E, rho, rho_s, partial, s, stop);
    else
        tile_mm_launch<T, 0, TN>(H, c, X, Y, ldr, R, E, rho, rho_s, partial, s, stop);
}

template <class T>
void apply_mm_cfg(const rad_hmat *H, const MmConfig &c, const T *X, T *Y, int64_t ldr, int R, const T *E,
                  const T *rho, T rho_s, double *partial, hipStream_t s, const int32_t *stop = nullptr,
                  double *epartial = nullptr) {
    if (c.tn == 64)
        apply_mm_tn<T, 64>(H, c, X, Y, ldr, R, E, rho, rho_s, partial, s, stop, epartial);
    else if (c.tn == 256 && sizeof(T) == 4)
        apply_mm_tn<T, (sizeof(T) == 4 ? 256 : 128)>(H, c, X, Y, ldr, R, E, rho, rho_s, partial, s, stop, epartial);
    else
        apply_mm_tn<T, 128>(H, c, X, Y, ldr, R, E, rho, rho_s, partial, s, stop, epartial);
}

template <class T>
void apply_mm_t(const rad_hmat *H, const T *X, T *Y, int64_t ldr, int R, const T *E, const T *rho, T rho_s,
                double *partial, hipStream_t s, const int32_t *stop = nullptr, double *epartial = nullptr) {
    apply_mm_cfg<T>(H, mm_config(H, R), X, Y, ldr, R, E, rho, rho_s, partial, s, stop, epartial);
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

void launch_csr_panel_scatter(const void *vals, const int64_t *dst, int64_t n, void *out, int32_t dtype,
                              hipStream_t s) {
    if (n <= 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    if (dtype == RAD_F64)
        hipLaunchKernelGGL(k_csr_panel_scatter<double>, dim3(grid), dim3(256), 0, s, (const double *)vals, dst, n,
                           (double *)out);
    else
        hipLaunchKernelGGL(k_csr_panel_scatter<float>, dim3(grid), dim3(256), 0, s, (const float *)vals, dst, n,
                           (float *)out);
    RAD_HIP(hipGetLastError());
}

void mm_apply(const rad_hmat *H, const void *X, void *Y, int64_t ldr, int64_t R, hipStream_t s) {
    if (H->dtype == RAD_F64)
        apply_mm_t<double>(H, (const double *)X, (double *)Y, ldr, (int)R, nullptr, nullptr, 0.0, nullptr, s);
    else
        apply_mm_t<float>(H, (const float *)X, (float *)Y, ldr, (int)R, nullptr, nullptr, 0.0f, nullptr, s);
}

// one Jacobi iteration: B_new = E + rho * (F-hat B_old), norms[r] = ||B_new - B_old||^2;
// with stop given, every kernel returns at once while *stop is set; with
// enorms given, also enorms[r] = ||E_r||^2 (from the same pass over E); with
// test given, the last reduction ends with the device-side stopping test
void mm_jacobi_step(const rad_hmat *H, const void *E, const void *rho, double rho_scalar, const void *Bold, void *Bnew,
                    int64_t ldr, int64_t R, double *norms, hipStream_t s, const int32_t *stop, double *enorms,
                    const ConvTest *test) {
    double *part = (double *)H->w_red.p;
    double *epart = enorms ? H->w_ered.p : nullptr;
    if (H->dtype == RAD_F64)
        apply_mm_t<double>(H, (const double *)Bold, (double *)Bnew, ldr, (int)R, (const double *)E,
                           (const double *)rho, rho_scalar, part, s, stop, epart);
    else
        apply_mm_t<float>(H, (const float *)Bold, (float *)Bnew, ldr, (int)R, (const float *)E, (const float *)rho,
                          (float)rho_scalar, part, s, stop, epart);
    // the stopping test rides on the last reduction of the iteration
    mm_reduce_cols(H, part, H->n_tiles, R, norms, s, stop, enorms ? nullptr : test);
    if (enorms) mm_reduce_cols(H, epart, H->n_tiles, R, enorms, s, stop, test);
    RAD_HIP(hipGetLastError());
}

template <class T>
void time_phases_t(const rad_hmat *H, int R, int nrep, hipStream_t s, double *ms) {
    const int64_t ldr = mm_ldr(R);
    const T *X = (const T *)H->w_x.p;
    T *Y = (T *)H->w_b.p;
    const T *E = (const T *)H->w_e.p;
    double *part = (double *)H->w_red.p;
    const MmConfig c = mm_config(H, R);
    hipEvent_t e0, e1;
    RAD_HIP(hipEventCreate(&e0));
    RAD_HIP(hipEventCreate(&e1));
    float t = 0;
    auto timed = [&](auto &&launch) {
        launch();   // untimed: first launches load the code object
        RAD_HIP(hipEventRecord(e0, s));
        for (int i = 0; i < nrep; ++i) launch();
        RAD_HIP(hipEventRecord(e1, s));
        RAD_HIP(hipEventSynchronize(e1));
        RAD_HIP(hipEventElapsedTime(&t, e0, e1));
        return (double)t / nrep;
    };
    ms[0] = ms[1] = ms[2] = 0.0;
    if (H->n_p1work > 0) {
        const int tn1 = c.tn == 64 ? 64 : 128;
        const unsigned rtiles = (unsigned)((R + tn1 - 1) / tn1);
        ms[0] = timed([&] {
            if (tn1 == 64)
                hipLaunchKernelGGL((k_proj_mm<T, 64>), dim3(H->n_p1pairs * rtiles), dim3(256), 0, s, H->d_groups.p,
                                   H->d_p1work.p, (const int32_t *)H->d_p1pairs.p,
                                   (const int32_t *)H->d_p1direct.p, (const T *)H->d_vals.p, X, ldr, R,
                                   (T *)H->w_part.p, (T *)H->w_t.p, (int)rtiles, nullptr);
            else
                hipLaunchKernelGGL((k_proj_mm<T, 128>), dim3(H->n_p1pairs * rtiles), dim3(256), 0, s, H->d_groups.p,
                                   H->d_p1work.p, (const int32_t *)H->d_p1pairs.p,
                                   (const int32_t *)H->d_p1direct.p, (const T *)H->d_vals.p, X, ldr, R,
                                   (T *)H->w_part.p, (T *)H->w_t.p, (int)rtiles, nullptr);
        });
        if (H->n_p1red_multi > 0)
            ms[1] = timed([&] {
                hipLaunchKernelGGL(k_proj_reduce<T>, reduce_grid(H->n_p1red_multi, R), dim3(256), 0, s,
                                   H->d_p1red_multi.p, (const T *)H->w_part.p, ldr, R, (T *)H->w_t.p, nullptr);
            });
    }
    ms[2] = timed([&] {
        if (c.tn == 64)
            tile_mm_launch<T, 1, 64>(H, c, X, Y, ldr, R, E, (const T *)nullptr, (T)0.3, part, s);
        else if (c.tn == 256 && sizeof(T) == 4)
            tile_mm_launch<T, 1, (sizeof(T) == 4 ? 256 : 128)>(H, c, X, Y, ldr, R, E, (const T *)nullptr, (T)0.3,
                                                                 part, s);
        else
            tile_mm_launch<T, 1, 128>(H, c, X, Y, ldr, R, E, (const T *)nullptr, (T)0.3, part, s);
    });
    RAD_HIP(hipGetLastError());
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

template <class T>
std::vector<std::pair<MmConfig, double>> autotune_t(rad_hmat *H, int R, int nrep, hipStream_t s) {
    const int64_t ldr = mm_ldr(R);
    const T *X = (const T *)H->w_x.p;
    T *Y = (T *)H->w_b.p;
    const T *E = (const T *)H->w_e.p;
    double *part = (double *)H->w_red.p;
    std::vector<MmConfig> cands;
    for (int tn : {64, 128, 256}) {
        if (tn == 256 && (sizeof(T) != 4 || R <= 128)) continue;
        cands.push_back(MmConfig{tn, 0, 0});
        for (int bpc : {1, 2, 4}) cands.push_back(MmConfig{tn, 1, bpc});
    }
    hipEvent_t e0, e1;
    RAD_HIP(hipEventCreate(&e0));
    RAD_HIP(hipEventCreate(&e1));
    std::vector<std::pair<MmConfig, double>> out;
    for (const MmConfig &c : cands) {
        // one Jacobi iteration's kernels: projections, their sum, fused expansion
        apply_mm_cfg<T>(H, c, X, Y, ldr, R, E, (const T *)nullptr, (T)0.3, part, s);
        float t = 0;
        RAD_HIP(hipEventRecord(e0, s));
        for (int i = 0; i < nrep; ++i) apply_mm_cfg<T>(H, c, X, Y, ldr, R, E, (const T *)nullptr, (T)0.3, part, s);
        RAD_HIP(hipEventRecord(e1, s));
        RAD_HIP(hipEventSynchronize(e1));
        RAD_HIP(hipEventElapsedTime(&t, e0, e1));
        out.push_back({c, (double)t / nrep});
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return out;
}

void mm_time_phases(const rad_hmat *H, int64_t R, int nrep, hipStream_t s, double *ms) {
    if (H->dtype == RAD_F64)
        time_phases_t<double>(H, (int)R, nrep, s, ms);
    else
        time_phases_t<float>(H, (int)R, nrep, s, ms);
}

MmConfig mm_config(const rad_hmat *H, int64_t R) {
    for (const auto &e : H->tuned)
        if (e.first == R) return e.second;
    MmConfig c;
    c.tn = R <= 64 ? 64 : 128;
    return c;
}

// tile order for the persistent kernels: decreasing reduction length
// (panel columns plus CSR columns), ties by tile index; and the zeroed counter
std::vector<std::pair<MmConfig, double>> mm_autotune(rad_hmat *H, int64_t R, int nrep, hipStream_t s) {
    auto res = H->dtype == RAD_F64 ? autotune_t<double>(H, (int)R, nrep, s) : autotune_t<float>(H, (int)R, nrep, s);
    size_t best = 0;
    for (size_t i = 1; i < res.size(); ++i)
        if (res[i].second < res[best].second) best = i;
    bool found = false;
    for (auto &e : H->tuned)
        if (e.first == R) {
            e.second = res[best].first;
            found = true;
        }
    if (!found) H->tuned.push_back({R, res[best].first});
    return res;
}

void mm_reduce_cols(const rad_hmat *H, const double *partial, int nparts, int64_t R, double *out, hipStream_t s,
                    const int32_t *stop, const ConvTest *test) {
    const bool grp = H->n_inst > 1;
    hipLaunchKernelGGL(k_reduce_parts, dim3((unsigned)((R + 15) / 16), (unsigned)H->n_inst), dim3(256), 0, s,
                       partial, grp ? (const int32_t *)H->d_inst_tile.p : nullptr, nparts, (int)R, out, stop);
    if (test) {
        RAD_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_conv_test, dim3(1), dim3(1024), 0, s, (const double *)out, *test);
    }
    RAD_HIP(hipGetLastError());
}

void conv_init(const double *enorm2, double rtol2, int64_t nc, double *thr, int32_t *conv, int32_t *stop,
               hipStream_t s) {
    hipLaunchKernelGGL(k_conv_init, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, enorm2, rtol2, (int)nc, thr,
                       conv, stop);
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
