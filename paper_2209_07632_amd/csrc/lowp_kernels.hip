// 16-bit (FP16 or BF16) copy of the compressed operator for the inner solves
// of iterative refinement: matrix-core products with FP32 accumulation.
//
// Scaling (FP16): every panel column k (a column of U' or of a dense block
// restricted to one 64-row tile) is stored as A[:, k] * c_k with c_k a power
// of two that brings max |A[:, k]| into [0.5, 1); the operand row it
// multiplies is staged as B[k, :] / c_k, so the product is unchanged.  Every
// stacked V column kk is stored as V[:, kk] * d_kk and the projection is
// divided by d_kk when the split-K partials are summed.  Powers of two make
// the scaling exact.  BF16 has the FP32 exponent range and uses unit scales,
// which lets its operand rows be converted once per product (X16, T16) and
// staged without arithmetic by the wide expansion kernel below.
//
// 16-bit panels are stored per 32-column chunk as 64 rows x 32 values with the
// reduction index contiguous (the operand layout of v_mfma_f32_16x16x32_*:
// lane l holds A[l % 16][8 (l / 16) .. 8 (l / 16) + 7]), at the same element
// offsets as the FP32 panels.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <algorithm>

#include "mm_epilogue.h"
#include "rad_internal.h"

namespace rad {

namespace {

constexpr int TM = 64, TN = 128, KC = 32, LDK = KC + 8;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <class H>
struct M16;
template <>
struct M16<_Float16> {
    typedef f16x8 vec;
    static __device__ __forceinline__ f32x4 run(vec a, vec b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};
template <>
struct M16<__bf16> {
    typedef bf16x8 vec;
    static __device__ __forceinline__ f32x4 run(vec a, vec b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

// power of two p with max_abs * p in [0.5, 1) (1 for an all-zero column)
__device__ __forceinline__ float pow2_scale(float max_abs) {
    if (!(max_abs > 0.0f)) return 1.0f;
    int e;
    frexpf(max_abs, &e);  // max_abs = m 2^e, m in [0.5, 1)
    return ldexpf(1.0f, -e);
}

// Dispatch index -> work index such that each of the 8 XCDs (which receive
// workgroups round-robin) gets one contiguous run of work items: neighbouring
// tiles gather the same operand rows and then share that XCD's L2.
__device__ __forceinline__ int xcd_remap16(int L, int total) {
    constexpr int kXcd = 8;
    const int q = total / kXcd, rem = total % kXcd;
    const int x = L % kXcd, slot = L / kXcd;
    return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + slot;
}

template <class H>
constexpr bool kUnitScale = false;
template <>
constexpr bool kUnitScale<__bf16> = true;

__device__ __forceinline__ float wave_max(float v) {
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

// ---------------------------------------------------------------------------
// conversion (build time)
// ---------------------------------------------------------------------------
template <class H>
__global__ void __launch_bounds__(256) k_lowp_panels(const float *vals, const TileInfo *tiles, H *out, float *pscale) {
    const TileInfo ti = tiles[blockIdx.x];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = w; k < ti.kpad; k += 4) {
        const float v = vals[ti.panel_off + (int64_t)k * TM + lane];
        // BF16 keeps the FP32 exponent range: unit scales (operands convert directly)
        const float c = kUnitScale<H> ? 1.0f : pow2_scale(wave_max(fabsf(v)));
        out[ti.panel_off + (int64_t)(k / KC) * TM * KC + lane * KC + (k % KC)] = (H)(v * c);
        if (lane == 0) pscale[ti.panel_off / TM + k] = c;
    }
}

// out[dst[i]] = BF16(vals[i]) for entries with dst[i] >= 0 (compressed CSR pair panels)
__global__ void k_csr_panel_scatter16(const float *vals, const int64_t *dst, int64_t n, __bf16 *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = dst[i];
        if (d >= 0) out[d] = (__bf16)vals[i];
    }
}

template <class H>
__global__ void __launch_bounds__(256) k_lowp_v(const float *vals, const ProjGroup *groups, H *out, float *tscale) {
    const ProjGroup g = groups[blockIdx.x];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int kk = blockIdx.y * 4 + w; kk < g.ktot; kk += gridDim.y * 4) {
        const float *v = vals + g.v_off + (int64_t)kk * g.ld;
        float m = 0.0f;
        for (int j = lane; j < g.n; j += 64) m = fmaxf(m, fabsf(v[j]));
        const float d = kUnitScale<H> ? 1.0f : pow2_scale(wave_max(m));
        H *o = out + g.v_off + (int64_t)kk * g.ld;
        for (int j = lane; j < g.ld; j += 64) o[j] = (H)(j < g.n ? v[j] * d : 0.0f);
        if (lane == 0) tscale[g.t_off + kk] = d;
    }
}

// ---------------------------------------------------------------------------
// products
// ---------------------------------------------------------------------------
template <class H>
struct Acc16 {
    f32x4 acc[4][2];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
    }
    __device__ __forceinline__ void mma(const H (*sA)[LDK], const H (*sB)[LDK], int lane, int w) {
        typedef typename M16<H>::vec vec;
        const int lr = lane & 15, k0 = 8 * (lane >> 4);
        vec a[4], b[2];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = *(const vec *)&sA[i * 16 + lr][k0];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = *(const vec *)&sB[w * 32 + j * 16 + lr][k0];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = M16<H>::run(a[i], b[j], acc[i][j]);
    }
};

// B chunk: 32 operand rows (FP32, R-major) times 128 columns, each row divided
// by its scale, converted and stored with the reduction index contiguous.
// Thread t takes rows 4 (t & 7) .. + 3 and columns 4 (t >> 3) .. + 3, and
// stores each column's four consecutive k as one 8-byte group: eight lanes
// fill one LDS row, and the row stride of LDK values puts the next eight
// lanes' row on the other half of the banks (no bank conflicts).
template <class H>
struct StageB16 {
    float v[4][4];   // [row 4 (t & 7) + i][column 4 (t >> 3) + u]
    __device__ __forceinline__ void fetch(const float *const *rowp, const float *inv, int r0, int R, int t) {
        const int kq = t & 7, c = (t >> 3) * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * kq + i;
            const float *p = rowp[k];
            const float s = inv[k];
            float4 x = make_float4(0, 0, 0, 0);
            if (p) {
                if (r0 + c + 3 < R) {
                    x = *(const float4 *)(p + r0 + c);
                } else {
                    if (r0 + c < R) x.x = p[r0 + c];
                    if (r0 + c + 1 < R) x.y = p[r0 + c + 1];
                    if (r0 + c + 2 < R) x.z = p[r0 + c + 2];
                }
            }
            v[i][0] = x.x * s;
            v[i][1] = x.y * s;
            v[i][2] = x.z * s;
            v[i][3] = x.w * s;
        }
    }
    __device__ __forceinline__ void commit(H (*sB)[LDK], int t) {
        const int kq = t & 7, c = (t >> 3) * 4;
        typedef H h4 __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            h4 q = {(H)v[0][u], (H)v[1][u], (H)v[2][u], (H)v[3][u]};
            *(h4 *)&sB[c + u][4 * kq] = q;
        }
    }
};

template <class H>
__global__ void __launch_bounds__(256) k_proj_mm16(const ProjGroup *groups, const P1Work *work, const H *vals16,
                                                    const float *X, int64_t ldr, int R, float *part) {
    const P1Work wk = work[blockIdx.x];
    const ProjGroup g = groups[wk.group];
    const int r0 = blockIdx.y * TN;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    __shared__ __align__(16) H sA[2][TM][LDK];
    __shared__ __align__(16) H sB[2][TN][LDK];
    __shared__ const float *rowp[2][KC];
    __shared__ float one[KC];
    if (t < KC) one[t] = 1.0f;
    Acc16<H> acc;
    acc.zero();
    const int rows = min(TM, g.ktot - wk.krow0);
    const H *V = vals16 + g.v_off + (int64_t)wk.krow0 * g.ld;
    StageB16<H> sb;
    // A: row r (a V column) x 32 consecutive facets: four 16-byte pieces per row
    auto fetchA = [&](int kb, typename M16<H>::vec &va) {
        int r = t >> 2, k8 = (t & 3) * 8;
        typename M16<H>::vec z{};
        va = z;
        if (r < rows) {
            const H *p = V + (int64_t)r * g.ld + kb + k8;
            if (kb + k8 + 7 < wk.je) {
                va = *(const typename M16<H>::vec *)p;
            } else {
                for (int u = 0; u < 8; ++u)
                    if (kb + k8 + u < wk.je) va[u] = p[u];
            }
        }
    };
    auto setrows = [&](int kb, int buf) {
        if (t < KC) rowp[buf][t] = (kb + t < wk.je) ? X + ((int64_t)g.j0 + kb + t) * ldr : nullptr;
    };
    typename M16<H>::vec va;
    int buf = 0;
    setrows(wk.jb, 0);
    __syncthreads();
    fetchA(wk.jb, va);
    sb.fetch(rowp[0], one, r0, R, t);
    for (int kb = wk.jb; kb < wk.je; kb += KC) {
        *(typename M16<H>::vec *)&sA[buf][t >> 2][(t & 3) * 8] = va;
        sb.commit(sB[buf], t);
        if (kb + KC < wk.je) setrows(kb + KC, buf ^ 1);
        __syncthreads();
        if (kb + KC < wk.je) {
            fetchA(kb + KC, va);
            sb.fetch(rowp[buf ^ 1], one, r0, R, t);
        }
        acc.mma(sA[buf], sB[buf], lane, w);
        buf ^= 1;
    }
    float *out = part + (int64_t)wk.part * TM * ldr;
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int row = i * 16 + 4 * lk + v;
                int col = r0 + w * 32 + j * 16 + lr;
                if (col < R) out[(int64_t)row * ldr + col] = acc.acc[i][j][v];
            }
}

// T rows = (sum of the split partials) / d_row
// Grid (slabs, 4, column blocks of 256): 16 rows of a slab per workgroup,
// four consecutive columns per thread (four rows at a time)
__global__ void __launch_bounds__(256) k_proj_reduce16(const P1Red *red, const float *part, const float *tscale,
                                                        int64_t ldr, int R, float *Tb, __bf16 *T16, int64_t ld16) {
    const P1Red rd = red[blockIdx.x];
    const int c = ((int)blockIdx.z * 64 + (int)(threadIdx.x & 63)) * 4;
    if (c >= R) return;
    const int r1 = min(rd.nrows, (int)blockIdx.y * 16 + 16);
    for (int row = (int)blockIdx.y * 16 + (int)(threadIdx.x >> 6); row < r1; row += 4) {
        const float4 s = ordered_sum4((const float4 *)(part + ((int64_t)rd.part_begin * TM + row) * ldr + c),
                                      (int64_t)TM * ldr / 4, rd.part_count);
        const float d = tscale[rd.t_row0 + row];
        const float v[4] = {s.x / d, s.y / d, s.z / d, s.w / d};
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (c + u < R) {
                if (Tb) Tb[(int64_t)(rd.t_row0 + row) * ldr + c + u] = v[u];
                if (T16) T16[(int64_t)(rd.t_row0 + row) * ld16 + c + u] = (__bf16)v[u];
            }
    }
}

dim3 reduce_grid(int32_t nred, int R) { return dim3((unsigned)nred, 4, (unsigned)((R + 255) / 256)); }

// X16 = bf16(X) for the R columns, zero padding up to ld16
__global__ void __launch_bounds__(256) k_to_bf16(const float *X, int64_t N, int64_t ldr, int R, __bf16 *X16,
                                                  int64_t ld16) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= N * ld16) return;
    const int64_t t = e / ld16;
    const int c = (int)(e % ld16);
    X16[e] = (__bf16)(c < R ? X[t * ldr + c] : 0.0f);
}

// ---------------------------------------------------------------------------
// BF16 wide expansion: one workgroup per 64-row tile and all R <= 256
// columns (wave w owns columns 64 w .. 64 w + 63), reduction chunks of 32
// with two register stages in flight.  Operand rows come pre-converted
// (X16, T16: facet-major, ld16 a multiple of 8); each thread loads four
// operand rows x eight columns and writes them transposed into LDS as
// 8-byte groups of four consecutive k, the operand layout of the matrix
// cores.  No CSR tasks (matrices with CSR near field use k_tile_mm16).
// ---------------------------------------------------------------------------
constexpr int WN = 256, WKC = 32, WLDK = WKC;

// LDS layout of the wide kernels' chunks: rows of 32 k (64 bytes, no
// padding); the 16-byte group c of row r sits at group c ^ wsw(r), and the
// operand row of output column R sits at row wpos(R) = R ^ ((R >> 3) & 3).
// The transposing 8-byte writes of a wave (eight lanes fill one row) then
// reach distinct banks, and so do the 16-byte reads of the matrix-core
// operands (sixteen consecutive rows, one group each).
__device__ __forceinline__ int wsw(int r) { return (((r >> 1) ^ (r >> 3)) & 1) | ((r >> 1) & 2); }
__device__ __forceinline__ int wpos(int R) { return R ^ ((R >> 3) & 3); }
// bf16 offset of (row r, 16-byte group c, 8-byte half q) in a row-swizzled chunk
__device__ __forceinline__ int wofs(int r, int c, int q) { return r * WLDK + 8 * (c ^ wsw(r)) + 4 * q; }

struct WideStage {
    bf16x8 a;          // panel: row t >> 2, k (t & 3) * 8 .. + 7
    bf16x8 b[4];       // operand rows 4 (t & 7) + i, columns 8 (t >> 3) .. + 7
    // the operand-row indices of this thread's four rows of a chunk (loaded a
    // chunk ahead of their use, so that the dependent row loads do not wait)
    struct Rows {
        int32_t v[4];
        __device__ __forceinline__ void load(const int32_t *brc, int t) {
            const int kq = t & 7;
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = brc[4 * kq + i];
        }
    };
    __device__ __forceinline__ void fetch(const __bf16 *pan, const Rows &rw, const __bf16 *X16, const __bf16 *T16,
                                          int64_t ld16, int t) {
        a = *(const bf16x8 *)(pan + t * 8);
        const int c8 = (t >> 3) * 8;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int32_t v = rw.v[i];
            const __bf16 *p = (v >= 0 ? X16 + (int64_t)v * ld16 : T16 + (int64_t)(-1 - v) * ld16) + c8;
            b[i] = c8 < ld16 ? *(const bf16x8 *)p : bf16x8{};
        }
    }
    __device__ __forceinline__ void commit(__bf16 (*sA)[WLDK], __bf16 (*sB)[WLDK], int t) {
        *(bf16x8 *)(&sA[0][0] + wofs(t >> 2, t & 3, 0)) = a;
        commit_b(sB, b, t);
    }
    __device__ __forceinline__ static void commit_b(__bf16 (*sB)[WLDK], const bf16x8 *b, int t) {
        const int kq = t & 7, c8 = (t >> 3) * 8;
        typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            bf16x4 q = {b[0][j], b[1][j], b[2][j], b[3][j]};
            *(bf16x4 *)(&sB[0][0] + wofs(wpos(c8 + j), kq >> 1, kq & 1)) = q;
        }
    }
};

// (three workgroups per CU fit its LDS; the register budget is held to match)
// (tile_list: the tiles to compute, one per workgroup; nullptr: every tile)
template <bool kFused>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) k_tile_mm16w(const TileInfo *tiles, const int32_t *tile_list, const int32_t *brow, const __bf16 *vals16,
                                                     const __bf16 *X16, const __bf16 *T16, int64_t ld16,
                                                     const float *X, int64_t ldr, int R, int64_t N, float *Y,
                                                     const float *E, const float *rho, float rho_s,
                                                     double *partial) {
    const int tile = tile_list ? tile_list[blockIdx.x] : blockIdx.x;
    const TileInfo ti = tiles[tile];
    const int64_t tile0 = (int64_t)tile * TM;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    constexpr int kPipe = (2 * TM * WLDK + 2 * WN * WLDK) * 2;
    constexpr int kOut = TM * (128 + 4) * 4;
    __shared__ __align__(16) unsigned char smem[kPipe > kOut ? kPipe : kOut];
    __bf16 (*sA)[TM][WLDK] = (__bf16 (*)[TM][WLDK])smem;
    __bf16 (*sB)[WN][WLDK] = (__bf16 (*)[WN][WLDK])(smem + 2 * TM * WLDK * sizeof(__bf16));
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
    const int lr = lane & 15, kg = lane >> 4;
    auto mma = [&](const __bf16 (*A)[WLDK], const __bf16 (*B)[WLDK]) {
        bf16x8 av[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = *(const bf16x8 *)(&A[0][0] + wofs(i * 16 + lr, kg, 0));
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[j] = *(const bf16x8 *)(&B[0][0] + wofs(wpos(w * 64 + j * 16 + lr), kg, 0));
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    };
    if (ti.kpad > 0) {
        const __bf16 *pan = vals16 + ti.panel_off;
        const int32_t *br = brow + ti.brow_off;
        WideStage s0, s1;
        WideStage::Rows rw0, rw1;   // row indices of the chunks s0 / s1 fetch next
        const int kp = ti.kpad;
        rw0.load(br, t);
        if (WKC < kp) rw1.load(br + WKC, t);
        s0.fetch(pan, rw0, X16, T16, ld16, t);
        if (2 * WKC < kp) rw0.load(br + 2 * WKC, t);
        if (WKC < kp) {
            s1.fetch(pan + (int64_t)WKC * TM, rw1, X16, T16, ld16, t);
            if (3 * WKC < kp) rw1.load(br + 3 * WKC, t);
        }
        for (int kb = 0; kb < kp; kb += 2 * WKC) {
            s0.commit(sA[0], sB[0], t);
            __syncthreads();
            if (kb + 2 * WKC < kp) {
                s0.fetch(pan + (int64_t)(kb + 2 * WKC) * TM, rw0, X16, T16, ld16, t);
                if (kb + 4 * WKC < kp) rw0.load(br + kb + 4 * WKC, t);
            }
            mma(sA[0], sB[0]);
            if (kb + WKC >= kp) break;
            s1.commit(sA[1], sB[1], t);
            __syncthreads();
            if (kb + 3 * WKC < kp) {
                s1.fetch(pan + (int64_t)(kb + 3 * WKC) * TM, rw1, X16, T16, ld16, t);
                if (kb + 5 * WKC < kp) rw1.load(br + kb + 5 * WKC, t);
            }
            mma(sA[1], sB[1]);
        }
    }
    // epilogue in two halves of 128 columns (waves 2h, 2h + 1 hold half h)
    float (*sC)[128 + 4] = (float (*)[128 + 4])smem;
    const int lk = lane >> 4;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        __syncthreads();
        if ((w >> 1) == h) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v) sC[i * 16 + 4 * lk + v][(w & 1) * 64 + j * 16 + lr] = acc[i][j][v];
        }
        __syncthreads();
        if (128 * h < R)
            tile_epilogue<float, kFused, TM, 128, 128 + 4>(sC, smem, tile, tile0, 128 * h, ldr, R, N, Y, E, X, rho,
                                                           rho_s, partial);
    }
}

// ---------------------------------------------------------------------------
// BF16 wide expansion of two consecutive 64-row tiles whose panels multiply
// the same operand rows (identical brow lists: the two halves of a 128-facet
// leaf): one workgroup computes the 128 x R block, so every gathered operand
// chunk staged in LDS feeds twice the matrix-core work of the one-tile
// kernel.  Wave w owns rows 64 (w & 1) .. + 63 and columns 128 (w >> 1) ..
// + 127.  Otherwise as k_tile_mm16w: chunks of 32 with two register stages in
// flight, epilogue per 64 x 128 quarter.
// ---------------------------------------------------------------------------
struct PairStage {
    bf16x8 a0, a1;     // panel rows t >> 2 of the first and of the second tile
    bf16x8 b[4];       // operand rows 4 (t >> 5) + i, columns 8 (t & 31) .. + 7
    __device__ __forceinline__ void fetch(const __bf16 *pa, const __bf16 *pb, const WideStage::Rows &rw,
                                          const __bf16 *X16, const __bf16 *T16, int64_t ld16, int t) {
        a0 = *(const bf16x8 *)(pa + t * 8);
        a1 = *(const bf16x8 *)(pb + t * 8);
        const int c8 = (t >> 3) * 8;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int32_t v = rw.v[i];
            const __bf16 *p = (v >= 0 ? X16 + (int64_t)v * ld16 : T16 + (int64_t)(-1 - v) * ld16) + c8;
            b[i] = c8 < ld16 ? *(const bf16x8 *)p : bf16x8{};
        }
    }
    __device__ __forceinline__ void commit(__bf16 (*sA)[WLDK], __bf16 (*sB)[WLDK], int t) {
        *(bf16x8 *)(&sA[0][0] + wofs(t >> 2, t & 3, 0)) = a0;
        *(bf16x8 *)(&sA[0][0] + wofs(TM + (t >> 2), t & 3, 0)) = a1;
        WideStage::commit_b(sB, b, t);
    }
};

// Segment kernel: work item i multiplies panel columns [k0, k1) of the two
// tiles of its pair (seg[i]: panel and row-list offsets of that range) and
// stores the 128 x 256 FP32 partial tile in slot i of wpart.  Items are
// segments of at most a fixed number of panel columns, launched longest
// first, so the uneven reductions of terrain tiles spread evenly over the
// compute units; k_pair_finish sums a pair's segments in order.
template <bool kProj = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
k_tile_mm16s(const int32_t *order, const WideSeg *segs, const int32_t *brow, const __bf16 *vals16,
             const __bf16 *X16, const __bf16 *T16, int64_t ld16, float *wpart, int64_t ldr, int R,
             const __bf16 *cvals16, const int32_t *cbrow16) {
    const int32_t item = order[blockIdx.x];
    if (item < 0) return;
    const WideSeg sg = segs[item];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    constexpr int kPipe = (2 * 2 * TM * WLDK + 2 * WN * WLDK) * 2;
    __shared__ __align__(16) unsigned char smem[kPipe];
    __bf16 (*sA)[2 * TM][WLDK] = (__bf16 (*)[2 * TM][WLDK])smem;
    __bf16 (*sB)[WN][WLDK] = (__bf16 (*)[WN][WLDK])(smem + 2 * 2 * TM * WLDK * sizeof(__bf16));
    f32x4 acc[4][8];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
    const int lr = lane & 15, kg = lane >> 4;
    const int wr = (w & 1) * TM, wc = (w >> 1) * 128;
    auto mma = [&](const __bf16 (*A)[WLDK], const __bf16 (*B)[WLDK]) {
        bf16x8 av[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = *(const bf16x8 *)(&A[0][0] + wofs(wr + i * 16 + lr, kg, 0));
#pragma unroll
        for (int jh = 0; jh < 2; ++jh) {
            bf16x8 bv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = *(const bf16x8 *)(&B[0][0] + wofs(wpos(wc + (4 * jh + j) * 16 + lr), kg, 0));
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][4 * jh + j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][4 * jh + j], 0, 0, 0);
        }
    };
    if (sg.kp > 0) {
        // (segments of a pair's compressed CSR panel read the compressed buffers)
        const __bf16 *vb = sg.pad_ ? cvals16 : vals16;
        const __bf16 *pa = vb + sg.pa, *pb = vb + sg.pb;
        const int32_t *br = (sg.pad_ ? cbrow16 : brow) + sg.br;
        PairStage s0, s1;
        WideStage::Rows rw0, rw1;
        const int kp = sg.kp;
        rw0.load(br, t);
        if (WKC < kp) rw1.load(br + WKC, t);
        s0.fetch(pa, pb, rw0, X16, T16, ld16, t);
        if (2 * WKC < kp) rw0.load(br + 2 * WKC, t);
        if (WKC < kp) {
            s1.fetch(pa + (int64_t)WKC * TM, pb + (int64_t)WKC * TM, rw1, X16, T16, ld16, t);
            if (3 * WKC < kp) rw1.load(br + 3 * WKC, t);
        }
        for (int kb = 0; kb < kp; kb += 2 * WKC) {
            s0.commit(sA[0], sB[0], t);
            __syncthreads();
            if (kb + 2 * WKC < kp) {
                s0.fetch(pa + (int64_t)(kb + 2 * WKC) * TM, pb + (int64_t)(kb + 2 * WKC) * TM, rw0, X16, T16, ld16, t);
                if (kb + 4 * WKC < kp) rw0.load(br + kb + 4 * WKC, t);
            }
            mma(sA[0], sB[0]);
            if (kb + WKC >= kp) break;
            s1.commit(sA[1], sB[1], t);
            __syncthreads();
            if (kb + 3 * WKC < kp) {
                s1.fetch(pa + (int64_t)(kb + 3 * WKC) * TM, pb + (int64_t)(kb + 3 * WKC) * TM, rw1, X16, T16, ld16, t);
                if (kb + 5 * WKC < kp) rw1.load(br + kb + 5 * WKC, t);
            }
            mma(sA[1], sB[1]);
        }
    }
    const int lk = lane >> 4;
    if constexpr (kProj) {
        // projection: rows 0..63 to partial tile `slot`, rows 64..127 to
        // `slot2` (each 64 x ldr, columns below R)
        const int32_t p = (w & 1) ? sg.slot2 : sg.slot;
        if (p < 0) return;
        float *out = wpart + (int64_t)p * TM * ldr;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int col = wc + j * 16 + lr;
                if (col < R)
#pragma unroll
                    for (int v = 0; v < 4; ++v) out[(int64_t)(i * 16 + 4 * lk + v) * ldr + col] = acc[i][j][v];
            }
    } else {
        // the partial tile, row-major 128 x 256: each lane's 16 consecutive
        // columns of a row form 64-byte runs
        float *out = wpart + (int64_t)sg.slot * (2 * TM * WN);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    __builtin_nontemporal_store(acc[i][j][v],
                                                out + (int64_t)(wr + i * 16 + 4 * lk + v) * WN + wc + j * 16 + lr);
    }
}

// Panels of the 16-bit V copy for the wide projection: slab i holds V_J
// columns krow0 .. krow0 + 63 of its group over the column node's facets,
// element (r, k) at pan + (k / 32) 2048 + 32 r + k % 32 (the packed-panel
// layout of the expansion), zero past the stacked rank and the facet count.
struct VSlab {
    int64_t pan;
    int32_t group, krow0, kpad, pad_;
};

__global__ void __launch_bounds__(256) k_vpanels(const ProjGroup *groups, const VSlab *slabs, const __bf16 *vals16,
                                                  __bf16 *out) {
    const VSlab sl = slabs[blockIdx.x];
    const ProjGroup g = groups[sl.group];
    const int64_t total = (int64_t)sl.kpad * TM;
    for (int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.y * 256) {
        const int c = (int)(e / (TM * 32)), rem = (int)(e % (TM * 32));
        const int r = rem / 32, k = c * 32 + rem % 32;
        __bf16 v = (__bf16)0.0f;
        if (sl.krow0 + r < g.ktot && k < g.n) v = vals16[g.v_off + (int64_t)(sl.krow0 + r) * g.ld + k];
        out[sl.pan + e] = v;
    }
}

// One workgroup per tile of a pair: the sum of the pair's segments (slots
// [slot, slot + nseg) of wpart, in order) for this tile's 64 rows, then the
// epilogue of the expansion (Y, or the fused Jacobi update) per 128 columns.
template <bool kFused>
__global__ void __launch_bounds__(256) k_pair_finish(const int32_t *first_tiles, const int32_t *pair_slot,
                                                      const float *wpart, const float *X, int64_t ldr, int R, int64_t N,
                                                      float *Y, const float *E, const float *rho, float rho_s,
                                                      double *partial) {
    const int pair = blockIdx.x >> 1, half = blockIdx.x & 1;
    const int tile = first_tiles[pair] + half;
    const int slot0 = pair_slot[pair], nseg = pair_slot[pair + 1] - slot0;
    if ((int64_t)tile * TM >= N) return;
    __shared__ __align__(16) float sC[TM][128 + 4];
    const int t = threadIdx.x;
    for (int h = 0; h < 2 && 128 * h < R; ++h) {
        __syncthreads();
        for (int e = t; e < TM * 128 / 4; e += 256) {
            const int r = e >> 5, c4 = (e & 31) * 4;
            const float *p = wpart + (int64_t)slot0 * (2 * TM * WN) + (int64_t)(TM * half + r) * WN + 128 * h + c4;
            f32x4 sum = {0, 0, 0, 0};
            for (int sgi = 0; sgi < nseg; ++sgi)
                sum += __builtin_nontemporal_load((const f32x4 *)(p + (int64_t)sgi * (2 * TM * WN)));
            sC[r][c4] = sum[0];
            sC[r][c4 + 1] = sum[1];
            sC[r][c4 + 2] = sum[2];
            sC[r][c4 + 3] = sum[3];
        }
        __syncthreads();
        tile_epilogue<float, kFused, TM, 128, 128 + 4>(sC, sC, tile, (int64_t)tile * TM, 128 * h, ldr, R, N, Y, E, X,
                                                       rho, rho_s, partial);
    }
}

template <class H, bool kFused>
__global__ void __launch_bounds__(256) k_tile_mm16(const TileInfo *tiles, const int32_t *brow, const TileTask *ctasks,
                                                    const H *vals16, const float *pscale, const float *vals32,
                                                    const int32_t *csr_ptr, const int32_t *csr_idx,
                                                    int64_t csr_val_start, const float *X, const float *Tb,
                                                    int64_t ldr, int R, int64_t N, float *Y, const float *E,
                                                    const float *rho, float rho_s, double *partial) {
    const int tile = blockIdx.x;
    const TileInfo ti = tiles[tile];
    const int64_t tile0 = (int64_t)tile * TM;
    const int r0 = blockIdx.y * TN;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    constexpr int kPipe = (2 * TM * LDK + 2 * TN * LDK) * 2;
    constexpr int kOut = TM * (TN + 4) * 4;
    __shared__ __align__(16) unsigned char smem[kPipe > kOut ? kPipe : kOut];
    H (*sA)[TM][LDK] = (H (*)[TM][LDK])smem;
    H (*sB)[TN][LDK] = (H (*)[TN][LDK])(smem + 2 * TM * LDK * sizeof(H));
    __shared__ const float *rowp[2][KC];
    __shared__ float inv[2][KC];
    Acc16<H> acc;
    acc.zero();
    StageB16<H> sb;
    // CSR tasks (FP32 values, unit scale), expanded to dense chunks in LDS
    for (int c = ti.csr_begin; c < ti.csr_end; ++c) {
        const TileTask tk = ctasks[c];
        const float *v = vals32 + tk.a_off;
        const int32_t *ci = csr_idx + (tk.a_off - csr_val_start);
        int cur = 0, end = 0;
        if (t >= tk.r_lo && t < tk.r_hi) {
            cur = csr_ptr[tk.aux_off + tk.row_off + t];
            end = csr_ptr[tk.aux_off + tk.row_off + t + 1];
        }
        for (int kb = 0; kb < tk.ncol; kb += KC) {
            for (int e = t; e < TM * KC; e += 256) sA[0][e / KC][e % KC] = (H)0.0f;
            if (t < KC) {
                rowp[0][t] = (kb + t < tk.ncol) ? X + ((int64_t)tk.col0 + kb + t) * ldr : nullptr;
                inv[0][t] = 1.0f;
            }
            __syncthreads();
            while (cur < end && ci[cur] < kb + KC) {
                sA[0][t][ci[cur] - kb] = (H)v[cur];
                ++cur;
            }
            sb.fetch(rowp[0], inv[0], r0, R, t);
            sb.commit(sB[0], t);
            __syncthreads();
            acc.mma(sA[0], sB[0], lane, w);
            __syncthreads();
        }
    }
    // packed panel
    if (ti.kpad > 0) {
        const H *pan = vals16 + ti.panel_off;
        const float *ps = pscale + ti.panel_off / TM;
        const int32_t *br = brow + ti.brow_off;
        auto setrows = [&](int kb, int b) {
            if (t < KC) {
                int32_t v = br[kb + t];
                rowp[b][t] = v >= 0 ? X + (int64_t)v * ldr : Tb + (int64_t)(-1 - v) * ldr;
                inv[b][t] = 1.0f / ps[kb + t];
            }
        };
        typedef typename M16<H>::vec vec;
        vec va;
        int buf = 0;
        setrows(0, 0);
        __syncthreads();
        va = *(const vec *)(pan + t * 8);
        sb.fetch(rowp[0], inv[0], r0, R, t);
        for (int kb = 0; kb < ti.kpad; kb += KC) {
            *(vec *)&sA[buf][t >> 2][(t & 3) * 8] = va;
            sb.commit(sB[buf], t);
            if (kb + KC < ti.kpad) setrows(kb + KC, buf ^ 1);
            __syncthreads();
            if (kb + KC < ti.kpad) {
                va = *(const vec *)(pan + (int64_t)(kb + KC) * TM + t * 8);
                sb.fetch(rowp[buf ^ 1], inv[buf ^ 1], r0, R, t);
            }
            acc.mma(sA[buf], sB[buf], lane, w);
            buf ^= 1;
        }
    }
    __syncthreads();
    float (*sC)[TN + 4] = (float (*)[TN + 4])smem;
    {
        const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) sC[i * 16 + 4 * lk + v][w * 32 + j * 16 + lr] = acc.acc[i][j][v];
    }
    __syncthreads();
    tile_epilogue<float, kFused, TM, TN, TN + 4>(sC, smem, tile, tile0, r0, ldr, R, N, Y, E, X, rho, rho_s, partial);
}

template <class H>
void convert_t(rad_hmat *H_, hipStream_t s) {
    H *out = (H *)H_->d_vals16.p;
    const float *vals = (const float *)H_->d_vals.p;
    if (H_->n_tiles > 0)
        hipLaunchKernelGGL(k_lowp_panels<H>, dim3(H_->n_tiles), dim3(256), 0, s, vals, H_->d_tiles.p, out,
                           H_->d_pscale.p);
    if (H_->n_groups > 0)
        hipLaunchKernelGGL(k_lowp_v<H>, dim3(H_->n_groups, 16), dim3(256), 0, s, vals, H_->d_groups.p, out,
                           H_->d_tscale.p);
    RAD_HIP(hipGetLastError());
}

// the wide BF16 kernel serves R <= 256 and matrices whose CSR slices (if
// any) all have compressed pair panels
bool wide_ok(const rad_hmat *Hm, int R) {
    return Hm->lowp == RAD_BF16 && (Hm->d_tile_tasks.n == 0 || Hm->wide_csr) && R <= WN && Hm->w_x16.p != nullptr;
}

int64_t ld16_of(int64_t R) { return (R + 7) & ~(int64_t)7; }

template <bool kFused>
void launch_wide(const rad_hmat *Hm, const float *E, const float *rho, float rho_s, const float *Bold, float *Bnew,
                 int64_t ldr, int R, double *part, hipStream_t s) {
    const int64_t ld16 = ld16_of(R);
    const __bf16 *v16 = (const __bf16 *)Hm->d_vals16.p, *x16 = (const __bf16 *)Hm->w_x16.p,
                 *t16 = (const __bf16 *)Hm->w_t16.p;
    if (Hm->n_wpairs > 0) {
        // pairs of tiles with one operand-row list: their segments longest
        // first, then each pair's sum and epilogue; then the tiles left alone
        hipLaunchKernelGGL(k_tile_mm16s<false>, dim3(Hm->n_wseg_blocks), dim3(256), 0, s, Hm->d_wseg_order.p,
                           Hm->d_wsegs.p, Hm->d_brow.p, v16, x16, t16, ld16, Hm->w_wpart.p, (int64_t)0, 0,
                           (const __bf16 *)Hm->d_cvals16.p, Hm->d_cbrow16.p);
        hipLaunchKernelGGL((k_pair_finish<kFused>), dim3(2 * Hm->n_wpairs), dim3(256), 0, s, Hm->d_wpairs.p,
                           Hm->d_wslot.p, (const float *)Hm->w_wpart.p, Bold, ldr, R, Hm->N, Bnew, E, rho, rho_s,
                           part);
        if (Hm->n_wsingles > 0)
            hipLaunchKernelGGL((k_tile_mm16w<kFused>), dim3(Hm->n_wsingles), dim3(256), 0, s, Hm->d_tiles.p,
                               Hm->d_wsingles.p, Hm->d_brow.p, v16, x16, t16, ld16, Bold, ldr, R, Hm->N, Bnew, E, rho,
                               rho_s, part);
    } else {
        hipLaunchKernelGGL((k_tile_mm16w<kFused>), dim3(Hm->n_tiles), dim3(256), 0, s, Hm->d_tiles.p,
                           (const int32_t *)nullptr, Hm->d_brow.p, v16, x16, t16, ld16, Bold, ldr, R, Hm->N, Bnew, E,
                           rho, rho_s, part);
    }
    RAD_HIP(hipGetLastError());
}

// wide BF16 projection (operands X16 already converted): the tile-pair
// segment kernel on the V panels, then the sum of each slab's partial tiles
// into T16 (the wide expansion reads only T16)
void launch_proj16w(const rad_hmat *Hm, int64_t ldr, int R, __bf16 *T16, hipStream_t s) {
    const int64_t ld16 = ld16_of(R);
    hipLaunchKernelGGL(k_tile_mm16s<true>, dim3(Hm->n_pseg_blocks), dim3(256), 0, s, Hm->d_pseg_order.p,
                       Hm->d_psegs.p, Hm->d_pbrow.p, (const __bf16 *)Hm->d_vpan16.p, (const __bf16 *)Hm->w_x16.p,
                       (const __bf16 *)nullptr, ld16, (float *)Hm->w_part.p, ldr, R, (const __bf16 *)nullptr,
                       (const int32_t *)nullptr);
    hipLaunchKernelGGL(k_proj_reduce16, reduce_grid(Hm->n_wpred, R), dim3(256), 0, s, Hm->d_wpred.p,
                       (const float *)Hm->w_part.p, Hm->d_tscale.p, ldr, R, (float *)nullptr, T16, ld16);
    RAD_HIP(hipGetLastError());
}

template <class H>
void step16_t(const rad_hmat *Hm, const float *E, const float *rho, float rho_s, const float *Bold, float *Bnew,
              int64_t ldr, int R, double *norms, hipStream_t s) {
    unsigned rtiles = (unsigned)((R + TN - 1) / TN);
    const H *v16 = (const H *)Hm->d_vals16.p;
    const bool wide = wide_ok(Hm, R);
    const int64_t ld16 = ld16_of(R);
    if (wide) {
        const int64_t n = Hm->N * ld16;
        hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Bold, Hm->N, ldr, R,
                           (__bf16 *)Hm->w_x16.p, ld16);
        RAD_HIP(hipGetLastError());
    }
    if (wide && Hm->n_psegs > 0) {
        launch_proj16w(Hm, ldr, R, (__bf16 *)Hm->w_t16.p, s);
    } else if (Hm->n_p1work > 0) {
        hipLaunchKernelGGL(k_proj_mm16<H>, dim3(Hm->n_p1work, rtiles), dim3(256), 0, s, Hm->d_groups.p,
                           Hm->d_p1work.p, v16, Bold, ldr, R, (float *)Hm->w_part.p);
        hipLaunchKernelGGL(k_proj_reduce16, reduce_grid(Hm->n_p1red, R), dim3(256), 0, s, Hm->d_p1red.p,
                           (const float *)Hm->w_part.p, Hm->d_tscale.p, ldr, R, (float *)Hm->w_t.p,
                           wide ? (__bf16 *)Hm->w_t16.p : (__bf16 *)nullptr, ld16);
        RAD_HIP(hipGetLastError());
    }
    double *part = (double *)Hm->w_red.p;
    if (wide) {
        if (E)
            launch_wide<true>(Hm, E, rho, rho_s, Bold, Bnew, ldr, R, part, s);
        else
            launch_wide<false>(Hm, E, rho, rho_s, Bold, Bnew, ldr, R, part, s);
        if (E) mm_reduce_cols(Hm, part, Hm->n_tiles, R, norms, s);
        return;
    }
    if (E)
        hipLaunchKernelGGL((k_tile_mm16<H, true>), dim3(Hm->n_tiles, rtiles), dim3(256), 0, s, Hm->d_tiles.p,
                           Hm->d_brow.p, Hm->d_tile_tasks.p, v16, Hm->d_pscale.p, (const float *)Hm->d_vals.p,
                           Hm->d_csr_ptr.p, Hm->d_csr_idx.p, Hm->csr_val_start, Bold, (const float *)Hm->w_t.p, ldr,
                           R, Hm->N, Bnew, E, rho, rho_s, part);
    else
        hipLaunchKernelGGL((k_tile_mm16<H, false>), dim3(Hm->n_tiles, rtiles), dim3(256), 0, s, Hm->d_tiles.p,
                           Hm->d_brow.p, Hm->d_tile_tasks.p, v16, Hm->d_pscale.p, (const float *)Hm->d_vals.p,
                           Hm->d_csr_ptr.p, Hm->d_csr_idx.p, Hm->csr_val_start, Bold, (const float *)Hm->w_t.p, ldr,
                           R, Hm->N, Bnew, E, rho, rho_s, part);
    RAD_HIP(hipGetLastError());
    if (E) mm_reduce_cols(Hm, part, Hm->n_tiles, R, norms, s);
}

// r = E - B + rho (F B) in FP64 (stored FP32); partial[tile * R + c] = sum of r^2
__global__ void __launch_bounds__(256) k_ir_resid(const float *E, const double *B64, const float *FB, const float *rho,
                                                   double rho_s, float *r, int64_t N, int64_t ldr, int R,
                                                   double *partial) {
    const int c = blockIdx.y * 256 + threadIdx.x;
    if (c >= R) return;
    const int64_t t0 = (int64_t)blockIdx.x * TM, t1 = min(N, t0 + TM);
    double s = 0.0;
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t e = t * ldr + c;
        const double rh = rho ? (double)rho[t] : rho_s;
        const double v = (double)E[e] - B64[e] + rh * (double)FB[e];
        r[e] = (float)v;
        s += v * v;
    }
    partial[(int64_t)blockIdx.x * R + c] = s;
}

// B64 += d; B32 = (float) B64
__global__ void __launch_bounds__(256) k_ir_update(double *B64, const float *d, float *B32, int64_t N, int64_t ldr,
                                                    int R) {
    const int c = blockIdx.y * 256 + threadIdx.x;
    if (c >= R) return;
    const int64_t t0 = (int64_t)blockIdx.x * TM, t1 = min(N, t0 + TM);
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t e = t * ldr + c;
        const double b = B64[e] + (double)d[e];
        B64[e] = b;
        B32[e] = (float)b;
    }
}

template <class H>
void time16_t(const rad_hmat *Hm, int R, int nrep, hipStream_t s, double *ms) {
    const int64_t ldr = (R + 3) & ~3;
    const float *X = (const float *)Hm->w_x.p;
    const float *E = (const float *)Hm->w_e.p;
    float *Y = (float *)Hm->w_b.p;
    const H *v16 = (const H *)Hm->d_vals16.p;
    double *part = (double *)Hm->w_red.p;
    unsigned rtiles = (unsigned)((R + TN - 1) / TN);
    hipEvent_t e0, e1;
    RAD_HIP(hipEventCreate(&e0));
    RAD_HIP(hipEventCreate(&e1));
    float t = 0;
    ms[0] = ms[1] = ms[2] = 0.0;
    auto timed = [&](auto &&launch) {
        launch();   // untimed: first launches load the code object
        RAD_HIP(hipEventRecord(e0, s));
        for (int i = 0; i < nrep; ++i) launch();
        RAD_HIP(hipEventRecord(e1, s));
        RAD_HIP(hipEventSynchronize(e1));
        RAD_HIP(hipEventElapsedTime(&t, e0, e1));
        return (double)t / nrep;
    };
    const bool wide = wide_ok(Hm, R);
    const int64_t ld16 = ld16_of(R);
    if (wide) {
        // operand rows need finite values: convert the (zeroed) workspace once
        const int64_t n = Hm->N * ld16;
        hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, Hm->N, ldr, R,
                           (__bf16 *)Hm->w_x16.p, ld16);
        RAD_HIP(hipMemsetAsync(Hm->w_t16.p, 0, Hm->w_t16.bytes(), s));
    }
    if (wide && Hm->n_psegs > 0) {
        ms[0] = timed([&] {
            hipLaunchKernelGGL(k_tile_mm16s<true>, dim3(Hm->n_pseg_blocks), dim3(256), 0, s, Hm->d_pseg_order.p,
                               Hm->d_psegs.p, Hm->d_pbrow.p, (const __bf16 *)Hm->d_vpan16.p,
                               (const __bf16 *)Hm->w_x16.p, (const __bf16 *)nullptr, ld16, (float *)Hm->w_part.p,
                               ldr, R, (const __bf16 *)nullptr, (const int32_t *)nullptr);
        });
        ms[1] = timed([&] {
            hipLaunchKernelGGL(k_proj_reduce16, reduce_grid(Hm->n_wpred, R), dim3(256), 0, s,
                               Hm->d_wpred.p, (const float *)Hm->w_part.p, Hm->d_tscale.p, ldr, R, (float *)nullptr,
                               (__bf16 *)Hm->w_t16.p, ld16);
        });
    } else if (Hm->n_p1work > 0) {
        ms[0] = timed([&] {
            hipLaunchKernelGGL(k_proj_mm16<H>, dim3(Hm->n_p1work, rtiles), dim3(256), 0, s, Hm->d_groups.p,
                               Hm->d_p1work.p, v16, X, ldr, R, (float *)Hm->w_part.p);
        });
        ms[1] = timed([&] {
            hipLaunchKernelGGL(k_proj_reduce16, reduce_grid(Hm->n_p1red, R), dim3(256), 0, s,
                               Hm->d_p1red.p, (const float *)Hm->w_part.p, Hm->d_tscale.p, ldr, R, (float *)Hm->w_t.p,
                               (__bf16 *)nullptr, (int64_t)0);
        });
    }
    if (wide) {
        ms[2] = timed([&] { launch_wide<true>(Hm, E, nullptr, 0.3f, X, Y, ldr, R, part, s); });
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return;
    }
    ms[2] = timed([&] {
        hipLaunchKernelGGL((k_tile_mm16<H, true>), dim3(Hm->n_tiles, rtiles), dim3(256), 0, s, Hm->d_tiles.p,
                           Hm->d_brow.p, Hm->d_tile_tasks.p, v16, Hm->d_pscale.p, (const float *)Hm->d_vals.p,
                           Hm->d_csr_ptr.p, Hm->d_csr_idx.p, Hm->csr_val_start, X, (const float *)Hm->w_t.p, ldr, R,
                           Hm->N, Y, E, (const float *)nullptr, 0.3f, part);
    });
    RAD_HIP(hipGetLastError());
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

// columns with flag 0 restart from B = 0, r = E
__global__ void __launch_bounds__(256) k_ir_select(double *B64, float *B32, float *r, const float *E,
                                                    const int32_t *flag, int64_t N, int64_t ldr, int R) {
    const int c = blockIdx.y * 256 + threadIdx.x;
    if (c >= R || flag[c]) return;
    const int64_t t0 = (int64_t)blockIdx.x * TM, t1 = min(N, t0 + TM);
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t e = t * ldr + c;
        B64[e] = 0.0;
        B32[e] = 0.0f;
        r[e] = E[e];
    }
}

// B64 = B32 = B0
__global__ void __launch_bounds__(256) k_ir_load(double *B64, float *B32, const float *B0, int64_t N, int64_t ldr,
                                                  int R) {
    const int c = blockIdx.y * 256 + threadIdx.x;
    if (c >= R) return;
    const int64_t t0 = (int64_t)blockIdx.x * TM, t1 = min(N, t0 + TM);
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t e = t * ldr + c;
        B64[e] = (double)B0[e];
        B32[e] = B0[e];
    }
}

}  // namespace

void ir_select(const rad_hmat *H, double *B64, float *B32, float *r, const float *E, const int32_t *flag, int64_t ldr,
               int64_t R, hipStream_t s) {
    dim3 grid((unsigned)H->n_tiles, (unsigned)((R + 255) / 256));
    hipLaunchKernelGGL(k_ir_select, grid, dim3(256), 0, s, B64, B32, r, E, flag, H->N, ldr, (int)R);
    RAD_HIP(hipGetLastError());
}

void ir_load(const rad_hmat *H, double *B64, float *B32, const float *B0, int64_t ldr, int64_t R, hipStream_t s) {
    dim3 grid((unsigned)H->n_tiles, (unsigned)((R + 255) / 256));
    hipLaunchKernelGGL(k_ir_load, grid, dim3(256), 0, s, B64, B32, B0, H->N, ldr, (int)R);
    RAD_HIP(hipGetLastError());
}

void lowp_time_phases(const rad_hmat *H, int64_t R, int nrep, hipStream_t s, double *ms) {
    if (H->lowp == RAD_F16)
        time16_t<_Float16>(H, (int)R, nrep, s, ms);
    else
        time16_t<__bf16>(H, (int)R, nrep, s, ms);
}

void ir_residual(const rad_hmat *H, const float *E, const double *B64, const float *FB, const float *rho, double rho_s,
                 float *r, int64_t ldr, int64_t R, double *norms, hipStream_t s) {
    double *part = (double *)H->w_red.p;
    dim3 grid((unsigned)H->n_tiles, (unsigned)((R + 255) / 256));
    hipLaunchKernelGGL(k_ir_resid, grid, dim3(256), 0, s, E, B64, FB, rho, rho_s, r, H->N, ldr, (int)R, part);
    RAD_HIP(hipGetLastError());
    mm_reduce_cols(H, part, H->n_tiles, R, norms, s);
}

void ir_update(const rad_hmat *H, double *B64, const float *d, float *B32, int64_t ldr, int64_t R, hipStream_t s) {
    dim3 grid((unsigned)H->n_tiles, (unsigned)((R + 255) / 256));
    hipLaunchKernelGGL(k_ir_update, grid, dim3(256), 0, s, B64, d, B32, H->N, ldr, (int)R);
    RAD_HIP(hipGetLastError());
}

// Wide BF16 projection schedule.  Items pair the 64-row slabs of each
// stacked V_J^T and cut the column node's facets into runs of kw (whole
// 32-facet chunks; kw a power of two from 512, the largest that still gives at
// least eight items per compute unit, so that long column nodes leave few
// partial tiles to sum).  A slab's partial tiles are numbered in facet order
// (the fixed order of the sum).  The items of one facet run share their
// operand rows and are launched on one XCD (xcd_launch_order).
void lowp_prepare_proj(rad_hmat *H) {
    H->n_psegs = H->n_pseg_blocks = H->n_wpred = 0;
    if (H->lowp != RAD_BF16 || (H->d_tile_tasks.n != 0 && !H->wide_csr) || H->h_groups.empty() ||
        H->max_rhs < kMfmaMinRhs)
        return;
    const std::vector<ProjGroup> &gs = H->h_groups;
    auto items_for = [&](int64_t kw) {
        int64_t c = 0;
        for (const ProjGroup &g : gs) c += (int64_t)((g.ktot + 127) / 128) * ((g.n + kw - 1) / kw);
        return c;
    };
    int32_t kw = 512;
    while (kw < (1 << 16) && items_for(2 * kw) >= 8 * (int64_t)H->n_cu) kw *= 2;
    std::vector<VSlab> slabs;
    std::vector<int32_t> pbrow;
    std::vector<WideSeg> segs;
    std::vector<std::vector<int32_t>> share;   // items of one facet run of one column node
    std::vector<P1Red> red;
    int64_t pan = 0;
    int32_t part = 0;
    for (int32_t gi = 0; gi < (int32_t)gs.size(); ++gi) {
        const ProjGroup &g = gs[gi];
        if (g.n <= 0 || g.ktot <= 0) continue;
        const int32_t kpad = (g.n + 31) / 32 * 32, nseg = (g.n + kw - 1) / kw;
        const int64_t br0 = (int64_t)pbrow.size();
        for (int32_t k = 0; k < kpad; ++k) pbrow.push_back(g.j0 + std::min(k, g.n - 1));
        const size_t share0 = share.size();
        share.resize(share0 + nseg);
        for (int32_t k0 = 0; k0 < g.ktot; k0 += 128) {
            const bool two = k0 + TM < g.ktot;
            const int64_t pa = pan, pb = two ? pan + (int64_t)kpad * TM : pan;
            slabs.push_back(VSlab{pa, gi, k0, kpad, 0});
            if (two) slabs.push_back(VSlab{pb, gi, k0 + TM, kpad, 0});
            pan += (two ? 2 : 1) * (int64_t)kpad * TM;
            const int32_t b0 = part, b1 = two ? part + nseg : -1;
            red.push_back(P1Red{g.t_off + k0, std::min(TM, g.ktot - k0), b0, nseg});
            if (two) red.push_back(P1Red{g.t_off + k0 + TM, std::min(TM, g.ktot - k0 - TM), b1, nseg});
            part += two ? 2 * nseg : nseg;
            for (int32_t sg = 0; sg < nseg; ++sg) {
                const int32_t jb = sg * kw, je = std::min(kpad, (sg + 1) * kw);
                WideSeg w{};
                w.pa = pa + (int64_t)jb * TM;
                w.pb = pb + (int64_t)jb * TM;
                w.br = br0 + jb;
                w.kp = je - jb;
                w.slot = b0 + sg;
                w.slot2 = two ? b1 + sg : -1;
                share[share0 + sg].push_back((int32_t)segs.size());
                segs.push_back(w);
            }
        }
    }
    if (part > H->n_parts) throw Error(RAD_EUNSUP, "wide projection needs more partial tiles than the workspace holds");
    std::vector<int64_t> cost(segs.size());
    for (size_t i = 0; i < segs.size(); ++i) cost[i] = segs[i].kp;
    const std::vector<int32_t> order = xcd_launch_order(share, cost);
    H->d_vpan16.alloc((size_t)std::max<int64_t>(pan, 1));
    H->d_pbrow.upload(pbrow);
    H->d_psegs.upload(segs);
    H->d_pseg_order.upload(order);
    H->n_pseg_blocks = (int32_t)order.size();
    H->d_wpred.upload(red);
    DevBuf<VSlab> d_slabs;
    d_slabs.upload(slabs);
    hipLaunchKernelGGL(k_vpanels, dim3((unsigned)slabs.size(), 16), dim3(256), 0, 0, H->d_groups.p, d_slabs.p,
                       (const __bf16 *)H->d_vals16.p, (__bf16 *)H->d_vpan16.p);
    RAD_HIP(hipGetLastError());
    RAD_HIP(hipStreamSynchronize(0));
    H->n_psegs = (int32_t)segs.size();
    H->n_wpred = (int32_t)red.size();
}

void launch_csr_panel_scatter16(const float *vals, const int64_t *dst, int64_t n, uint16_t *out, hipStream_t s) {
    if (n <= 0) return;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_csr_panel_scatter16, dim3(grid), dim3(256), 0, s, vals, dst, n, (__bf16 *)out);
    RAD_HIP(hipGetLastError());
}

void lowp_convert(rad_hmat *H, hipStream_t s) {
    if (H->lowp == RAD_F16)
        convert_t<_Float16>(H, s);
    else
        convert_t<__bf16>(H, s);
}

// One product (E == nullptr: Bnew = F16 Bold) or fused Jacobi step with the 16-bit operator.
void lowp_step(const rad_hmat *H, const void *E, const void *rho, double rho_s, const void *Bold, void *Bnew,
               int64_t ldr, int64_t R, double *norms, hipStream_t s) {
    if (H->lowp == RAD_F16)
        step16_t<_Float16>(H, (const float *)E, (const float *)rho, (float)rho_s, (const float *)Bold, (float *)Bnew,
                           ldr, (int)R, norms, s);
    else
        step16_t<__bf16>(H, (const float *)E, (const float *)rho, (float)rho_s, (const float *)Bold, (float *)Bnew,
                         ldr, (int)R, norms, s);
}

}  // namespace rad
