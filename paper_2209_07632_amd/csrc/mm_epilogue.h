// Shared epilogue of the multi-RHS expansion kernels (included by the
// FP32/FP64 and the 16-bit kernels).  The 64 x TN (TN = 64 or 128) result tile
// sits in LDS (sC); every thread streams 16-byte groups of whole rows: Y = tile, or
// with the fused Jacobi update B_new = E + rho * tile, writing the per-column
// partial sums of (B_new - B_old)^2 of this tile.  Reductions use a fixed order.
// E, B_old and the output are streamed once per launch: their accesses are
// non-temporal, which leaves the caches to the operator panels and T rows that
// every column tile of a row tile re-reads.
#pragma once

#include <hip/hip_runtime.h>

namespace rad {

typedef float epi_f4 __attribute__((ext_vector_type(4)));
typedef double epi_d2 __attribute__((ext_vector_type(2)));

// E and B_old values of one group of four rows of this thread's epilogue
// share (rows rsub + RS (4 g + q), columns col .. col + 3)
// p[0] + p[stride] + ... + p[(n - 1) stride], added in index order from
// zero, with the loads of eight terms in flight at a time (the split-K sums
// of partial tiles; the result is that of the plain sequential loop)
template <class T>
__device__ __forceinline__ T ordered_sum(const T *p, int64_t stride, int n) {
    T s = 0;
    int i = 0;
    for (; i + 8 <= n; i += 8) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(i + u) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; i < n; ++i) s += p[(int64_t)i * stride];
    return s;
}

// the same for four consecutive columns at once (V: float4 or double4),
// component by component in index order
template <class V>
__device__ __forceinline__ V ordered_sum4(const V *p, int64_t stride, int n) {
    V s;
    s.x = s.y = s.z = s.w = 0;
    int i = 0;
    for (; i + 8 <= n; i += 8) {
        V v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(i + u) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            s.x += v[u].x;
            s.y += v[u].y;
            s.z += v[u].z;
            s.w += v[u].w;
        }
    }
    for (; i < n; ++i) {
        const V v = p[(int64_t)i * stride];
        s.x += v.x;
        s.y += v.y;
        s.z += v.z;
        s.w += v.w;
    }
    return s;
}

template <class T, int TM, int TN>
struct EpiRegs {
    static constexpr int CT = TN / 4, RS = 256 / CT;
    T ev[4][4], bo[4][4];
    __device__ __forceinline__ void load(int grp, int64_t tile0, int r0, int64_t ldr, int R, int64_t N, const T *E,
                                         const T *X) {
        const int t = threadIdx.x;
        const int rows = (int)min((int64_t)TM, N - tile0);
        const int rsub = t / CT, col = r0 + (t % CT) * 4;
        const bool full = col + 3 < R;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const int row = rsub + RS * (4 * grp + qq);
            const int64_t e = (tile0 + row) * ldr + col;
            // values first, then unconditional register writes (keeps the
            // arrays in registers)
            T a[4] = {0, 0, 0, 0}, o[4] = {0, 0, 0, 0};
            if (row < rows && full) {
                if constexpr (sizeof(T) == 4) {
                    const epi_f4 av = __builtin_nontemporal_load((const epi_f4 *)(E + e));
                    const epi_f4 ov = __builtin_nontemporal_load((const epi_f4 *)(X + e));
                    a[0] = av.x; a[1] = av.y; a[2] = av.z; a[3] = av.w;
                    o[0] = ov.x; o[1] = ov.y; o[2] = ov.z; o[3] = ov.w;
                } else {
                    const epi_d2 a0 = __builtin_nontemporal_load((const epi_d2 *)(E + e));
                    const epi_d2 a1 = __builtin_nontemporal_load((const epi_d2 *)(E + e + 2));
                    const epi_d2 o0 = __builtin_nontemporal_load((const epi_d2 *)(X + e));
                    const epi_d2 o1 = __builtin_nontemporal_load((const epi_d2 *)(X + e + 2));
                    a[0] = a0.x; a[1] = a0.y; a[2] = a1.x; a[3] = a1.y;
                    o[0] = o0.x; o[1] = o0.y; o[2] = o1.x; o[3] = o1.y;
                }
            } else if (row < rows) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (col + u < R) {
                        a[u] = E[e + u];
                        o[u] = X[e + u];
                    }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ev[qq][u] = a[u];
                bo[qq][u] = o[u];
            }
        }
    }
};

// kNormE (with kFused): also the per-column partial sums of E^2 into epartial
template <class T, bool kFused, int TM, int TN, int LDC, bool kNormE = false>
__device__ __forceinline__ void tile_epilogue(const T (*sC)[LDC], void *smem, int tile, int64_t tile0, int r0,
                                              int64_t ldr, int R, int64_t N, T *Y, const T *E, const T *X,
                                              const T *rho, T rho_s, double *partial, double *epartial = nullptr) {
    constexpr int CT = TN / 4;            // threads per row, four columns each
    constexpr int RS = 256 / CT;          // row groups
    constexpr int NQ = TM / RS;           // rows per thread
    static_assert(NQ % 4 == 0 && RS * CT == 256, "tile shape");
    const int t = threadIdx.x;
    const int rows = (int)min((int64_t)TM, N - tile0);
    const int c4 = (t % CT) * 4;          // this thread's four columns
    const int rsub = t / CT;              // rows rsub, rsub + RS, ...
    const int col = r0 + c4;
    double d2[4] = {0.0, 0.0, 0.0, 0.0};
    double e2[4] = {0.0, 0.0, 0.0, 0.0};
    const bool full = col + 3 < R;
    // rows rsub + RS q in groups of four: all loads of a group first, then
    // the arithmetic and the stores
#pragma unroll
    for (int half = 0; half < NQ / 4; ++half) {
        EpiRegs<T, TM, TN> cur;
        if constexpr (kFused) cur.load(half, tile0, r0, ldr, R, N, E, X);
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            const int row = rsub + RS * (4 * half + qq);
            if (row < rows) {
                const int64_t e = (tile0 + row) * ldr + col;
                T y[4] = {sC[row][c4], sC[row][c4 + 1], sC[row][c4 + 2], sC[row][c4 + 3]};
                if constexpr (kFused) {
                    T rh = rho ? rho[tile0 + row] : rho_s;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        T bn = cur.ev[qq][u] + rh * y[u];
                        double d = (double)bn - (double)cur.bo[qq][u];
                        if (col + u < R) d2[u] += d * d;
                        if constexpr (kNormE) e2[u] += (double)cur.ev[qq][u] * (double)cur.ev[qq][u];
                        y[u] = bn;
                    }
                }
                if (full) {
                    if constexpr (sizeof(T) == 4) {
                        const epi_f4 yv = {y[0], y[1], y[2], y[3]};
                        __builtin_nontemporal_store(yv, (epi_f4 *)(Y + e));
                    } else {
                        const epi_d2 y0 = {y[0], y[1]}, y1 = {y[2], y[3]};
                        __builtin_nontemporal_store(y0, (epi_d2 *)(Y + e));
                        __builtin_nontemporal_store(y1, (epi_d2 *)(Y + e + 2));
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (col + u < R) Y[e + u] = y[u];
                }
            }
        }
    }
    if constexpr (kFused) {
        __syncthreads();
        double *red = (double *)smem;   // RS x TN partial sums (1024 doubles; fit in the LDS tile)
#pragma unroll
        for (int u = 0; u < 4; ++u) red[rsub * TN + c4 + u] = d2[u];
        __syncthreads();
        if (t < TN) {
            double sum = 0.0;
            for (int q = 0; q < RS; ++q) sum += red[q * TN + t];
            if (r0 + t < R) partial[(int64_t)tile * R + r0 + t] = sum;
        }
        if constexpr (kNormE) {
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 4; ++u) red[rsub * TN + c4 + u] = e2[u];
            __syncthreads();
            if (t < TN) {
                double sum = 0.0;
                for (int q = 0; q < RS; ++q) sum += red[q * TN + t];
                if (r0 + t < R) epartial[(int64_t)tile * R + r0 + t] = sum;
            }
        }
    }
}

}  // namespace rad
