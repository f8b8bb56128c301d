// Shared epilogue of the multi-RHS expansion kernels (included by the
// FP32/FP64 and the 16-bit kernels).  The 64 x TN (TN = 64 or 128) result tile
// sits in LDS (sC); every thread streams 16-byte groups of whole rows: Y = tile, or
// with the fused Jacobi update B_new = E + rho * tile, writing the per-column
// partial sums of (B_new - B_old)^2 of this tile.  Reductions use a fixed order.
#pragma once

#include <hip/hip_runtime.h>

namespace rad {

template <class T, bool kFused, int TM, int TN, int LDC>
__device__ __forceinline__ void tile_epilogue(const T (*sC)[LDC], void *smem, int tile, int64_t tile0, int r0,
                                              int64_t ldr, int R, int64_t N, T *Y, const T *E, const T *X,
                                              const T *rho, T rho_s, double *partial) {
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
    const bool full = col + 3 < R;
    // rows rsub + RS q in groups of four: all loads of a group first, then
    // the arithmetic and the stores
#pragma unroll
    for (int half = 0; half < NQ / 4; ++half) {
        T ev[4][4], bo[4][4];
        if constexpr (kFused) {
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const int row = rsub + RS * (4 * half + qq);
                const int64_t e = (tile0 + row) * ldr + col;
                if (row < rows && full) {
                    if constexpr (sizeof(T) == 4) {
                        float4 a = *(const float4 *)(E + e), o = *(const float4 *)(X + e);
                        ev[qq][0] = a.x; ev[qq][1] = a.y; ev[qq][2] = a.z; ev[qq][3] = a.w;
                        bo[qq][0] = o.x; bo[qq][1] = o.y; bo[qq][2] = o.z; bo[qq][3] = o.w;
                    } else {
                        double2 a0 = *(const double2 *)(E + e), a1 = *(const double2 *)(E + e + 2);
                        double2 o0 = *(const double2 *)(X + e), o1 = *(const double2 *)(X + e + 2);
                        ev[qq][0] = a0.x; ev[qq][1] = a0.y; ev[qq][2] = a1.x; ev[qq][3] = a1.y;
                        bo[qq][0] = o0.x; bo[qq][1] = o0.y; bo[qq][2] = o1.x; bo[qq][3] = o1.y;
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        bool ok = row < rows && col + u < R;
                        ev[qq][u] = ok ? E[e + u] : (T)0;
                        bo[qq][u] = ok ? X[e + u] : (T)0;
                    }
                }
            }
        }
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
                        T bn = ev[qq][u] + rh * y[u];
                        double d = (double)bn - (double)bo[qq][u];
                        if (col + u < R) d2[u] += d * d;
                        y[u] = bn;
                    }
                }
                if (full) {
                    if constexpr (sizeof(T) == 4) {
                        *(float4 *)(Y + e) = make_float4(y[0], y[1], y[2], y[3]);
                    } else {
                        *(double2 *)(Y + e) = make_double2(y[0], y[1]);
                        *(double2 *)(Y + e + 2) = make_double2(y[2], y[3]);
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
    }
}

}  // namespace rad
