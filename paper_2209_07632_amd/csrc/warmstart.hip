// Warm start for the radiosity solve: POD basis by the method of snapshots
// (FP64 Gram matrix and re-orthonormalisation) and a tanh perceptron with
// forward, backward and Adam kernels (FP32 products, or BF16 operands on the
// matrix cores with FP32 accumulation).
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>

#include "rad_internal.h"
#include "rad_warmstart.h"

namespace rad {
namespace {

__device__ __forceinline__ double wave_sum_d(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// POD
// ---------------------------------------------------------------------------
constexpr int AT = 64, AROWS = 16;

// Partial tiles of A^T (B - Bsub) over one chunk of facets, FP64 accumulation.
// A: N x p, B and Bsub: N x q (facet-major).  part tile (chunk, bi, bj) is
// 64 x 64 doubles, row-major.
__global__ void __launch_bounds__(256) k_atb_part(const float *A, int64_t lda, int p, const float *B, const float *Bsub,
                                                   int64_t ldb, int q, int64_t N, int64_t rows_per_chunk,
                                                   double *part) {
    const int bi = blockIdx.x, bj = blockIdx.y, ch = blockIdx.z;
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    __shared__ double sA[AROWS][AT + 1];
    __shared__ double sB[AROWS][AT + 1];
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    const int64_t r0 = (int64_t)ch * rows_per_chunk, r1 = min(N, r0 + rows_per_chunk);
    for (int64_t rb = r0; rb < r1; rb += AROWS) {
        for (int e = t; e < AROWS * AT; e += 256) {
            const int r = e / AT, c = e % AT;
            const int64_t row = rb + r;
            const int ca = bi * AT + c, cb = bj * AT + c;
            double a = 0.0, b = 0.0;
            if (row < r1) {
                if (ca < p) a = (double)A[row * lda + ca];
                if (cb < q) {
                    b = (double)B[row * ldb + cb];
                    if (Bsub) b -= (double)Bsub[row * ldb + cb];
                }
            }
            sA[r][c] = a;
            sB[r][c] = b;
        }
        __syncthreads();
#pragma unroll 4
        for (int r = 0; r < AROWS; ++r) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = sA[r][ty * 4 + u];
                b[u] = sB[r][tx * 4 + u];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
    double *out = part + (((int64_t)ch * gridDim.x + bi) * gridDim.y + bj) * (AT * AT);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) out[(ty * 4 + i) * AT + tx * 4 + j] = acc[i][j];
}

// Sum of the chunk partials in chunk order: G[i q + j] (FP64) and/or
// C[j p + i] = scale_i * sum (FP32, transposed).
__global__ void __launch_bounds__(256) k_atb_reduce(const double *part, int nch, int ntp, int ntq, int p, int q,
                                                     double *G, float *C, const float *scale) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)p * q) return;
    const int i = (int)(e / q), j = (int)(e % q);
    const int bi = i / AT, bj = j / AT, li = i % AT, lj = j % AT;
    double s = 0.0;
    for (int ch = 0; ch < nch; ++ch) s += part[(((int64_t)ch * ntp + bi) * ntq + bj) * (AT * AT) + li * AT + lj];
    if (G) G[(int64_t)i * q + j] = s;
    if (C) C[(int64_t)j * p + i] = (float)(scale ? s * (double)scale[i] : s);
}

// out (N x m, column-major FP64, ld N) = S (N x M facet-major FP32) Cm (M x m row-major FP64)
__global__ void __launch_bounds__(256) k_s_times_c(const float *S, int64_t lds, int64_t N, int M, const double *Cm,
                                                    int m, double *out) {
    const int64_t r0 = (int64_t)blockIdx.x * AT;
    const int c0 = blockIdx.y * AT;
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    __shared__ double sS[AT][AROWS + 1];
    __shared__ double sC[AROWS][AT + 1];
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int k0 = 0; k0 < M; k0 += AROWS) {
        for (int e = t; e < AT * AROWS; e += 256) {
            const int r = e / AROWS, k = e % AROWS;
            const int64_t row = r0 + r;
            sS[r][k] = (row < N && k0 + k < M) ? (double)S[row * lds + k0 + k] : 0.0;
            const int kk = e / AT, c = e % AT;
            sC[kk][c] = (k0 + kk < M && c0 + c < m) ? Cm[(int64_t)(k0 + kk) * m + c0 + c] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < AROWS; ++k) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = sS[ty * 4 + u][k];
                b[u] = sC[k][tx * 4 + u];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t row = r0 + ty * 4 + i;
            const int c = c0 + tx * 4 + j;
            if (row < N && c < m) out[(int64_t)c * N + row] = acc[i][j];
        }
}

__global__ void __launch_bounds__(256) k_to_phi32(const double *Q, int64_t N, int m, float *Phi, int64_t ldp) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= N * m) return;
    const int64_t row = e / m;
    const int c = (int)(e % m);
    Phi[row * ldp + c] = (float)Q[(int64_t)c * N + row];
}

__global__ void __launch_bounds__(256) k_nonfinite(const float *S, int64_t lds, int64_t N, int M, int *flag) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= N * M) return;
    const float v = S[(e / M) * lds + e % M];
    if (!isfinite(v)) flag[0] = 1;
}

// B[t, c] = E[t, c] + sum_j Phi[t, j] scale_j C[c m + j]
__global__ void __launch_bounds__(256) k_pod_expand(const float *Phi, int64_t ldp, int64_t N, int m, const float *C,
                                                     const float *scale, const float *E, int64_t ldb, int R,
                                                     float *B) {
    const int64_t r0 = (int64_t)blockIdx.x * AT;
    const int c0 = blockIdx.y * AT;
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    __shared__ float sP[AT][AROWS + 1];
    __shared__ float sC[AROWS][AT + 1];
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0f;
    for (int k0 = 0; k0 < m; k0 += AROWS) {
        for (int e = t; e < AT * AROWS; e += 256) {
            const int r = e / AROWS, k = e % AROWS;
            const int64_t row = r0 + r;
            sP[r][k] = (row < N && k0 + k < m) ? Phi[row * ldp + k0 + k] : 0.0f;
            const int kk = e % AROWS, c = e / AROWS;   // k fastest: C rows are contiguous in j
            float v = 0.0f;
            if (k0 + kk < m && c0 + c < R) {
                v = C[(int64_t)(c0 + c) * m + k0 + kk];
                if (scale) v *= scale[k0 + kk];
            }
            sC[kk][c] = v;
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < AROWS; ++k) {
            float a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = sP[ty * 4 + u][k];
                b[u] = sC[k][tx * 4 + u];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t row = r0 + ty * 4 + i;
            const int c = c0 + tx * 4 + j;
            if (row < N && c < R) {
                const int64_t e = row * ldb + c;
                B[e] = (E ? E[e] : 0.0f) + acc[i][j];
            }
        }
}

// ---------------------------------------------------------------------------
// perceptron
// ---------------------------------------------------------------------------
enum Epi : int { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_TANH = 2, EPI_TANH_GRAD = 3 };

// C = op(A) op(B): A(i, k) = A[i sai + k sak], B(k, j) = B[k sbk + j sbj],
// C(i, j) = C[i ldc + j]; epilogue per Epi (aux(i, j) = aux[i ldaux + j]).
struct GemmArgs {
    const float *A;
    int64_t sai, sak;
    const float *B;
    int64_t sbk, sbj;
    float *C;
    int64_t ldc;
    const float *bias;
    const float *aux;
    int64_t ldaux;
    int M, N, K, epi;
};

__device__ __forceinline__ void gemm_store(const GemmArgs &g, int i, int j, float v) {
    if (i >= g.M || j >= g.N) return;
    if (g.epi == EPI_BIAS) {
        v += g.bias[j];
    } else if (g.epi == EPI_BIAS_TANH) {
        v = tanhf(v + g.bias[j]);
    } else if (g.epi == EPI_TANH_GRAD) {
        const float h = g.aux[(int64_t)i * g.ldaux + j];
        v *= 1.0f - h * h;
    }
    g.C[(int64_t)i * g.ldc + j] = v;
}

// FP32: 64 x 64 tile, 4 x 4 outputs per thread
__global__ void __launch_bounds__(256) k_gemm_f32(GemmArgs g) {
    constexpr int T = 64, KC = 16;
    __shared__ float sA[KC][T + 4];
    __shared__ float sB[KC][T + 4];
    const int i0 = blockIdx.x * T, j0 = blockIdx.y * T;
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0f;
    for (int k0 = 0; k0 < g.K; k0 += KC) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + 256 * q;
            int i, k;
            if (g.sak == 1) {
                k = e % KC;
                i = e / KC;
            } else {
                i = e % T;
                k = e / T;
            }
            int gi = i0 + i, gk = k0 + k;
            sA[k][i] = (gi < g.M && gk < g.K) ? g.A[(int64_t)gi * g.sai + (int64_t)gk * g.sak] : 0.0f;
            int j;
            if (g.sbk == 1) {
                k = e % KC;
                j = e / KC;
            } else {
                j = e % T;
                k = e / T;
            }
            const int gj = j0 + j;
            gk = k0 + k;
            sB[k][j] = (gj < g.N && gk < g.K) ? g.B[(int64_t)gk * g.sbk + (int64_t)gj * g.sbj] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            float a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = sA[k][ty * 4 + u];
                b[u] = sB[k][tx * 4 + u];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) gemm_store(g, i0 + ty * 4 + i, j0 + tx * 4 + j, acc[i][j]);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// BF16 operands on v_mfma_f32_16x16x32_bf16 (lane l: A[l % 16][8 (l / 16) ..],
// B[8 (l / 16) ..][l % 16]; result row 4 (l / 16) + v, column l % 16), FP32
// accumulation.  64 x 64 tile: wave w owns rows 16 w .. 16 w + 15.
__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
    constexpr int T = 64, KC = 32, LD = KC + 8;
    __shared__ __align__(16) __bf16 sA[T][LD];
    __shared__ __align__(16) __bf16 sB[T][LD];
    const int i0 = blockIdx.x * T, j0 = blockIdx.y * T;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int lr = lane & 15, k8 = 8 * (lane >> 4);
    f32x4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < g.K; k0 += KC) {
        if (g.sak == 1) {
            const int i = t >> 2, k = (t & 3) * 8, gi = i0 + i;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int gk = k0 + k + u;
                sA[i][k + u] = (__bf16)((gi < g.M && gk < g.K) ? g.A[(int64_t)gi * g.sai + gk] : 0.0f);
            }
        } else {
            const int k = t >> 3, i = (t & 7) * 8, gk = k0 + k;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int gi = i0 + i + u;
                sA[i + u][k] =
                    (__bf16)((gi < g.M && gk < g.K) ? g.A[(int64_t)gi * g.sai + (int64_t)gk * g.sak] : 0.0f);
            }
        }
        if (g.sbk == 1) {
            const int j = t >> 2, k = (t & 3) * 8, gj = j0 + j;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int gk = k0 + k + u;
                sB[j][k + u] = (__bf16)((gj < g.N && gk < g.K) ? g.B[gk + (int64_t)gj * g.sbj] : 0.0f);
            }
        } else {
            const int k = t >> 3, j = (t & 7) * 8, gk = k0 + k;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int gj = j0 + j + u;
                sB[j + u][k] =
                    (__bf16)((gj < g.N && gk < g.K) ? g.B[(int64_t)gk * g.sbk + (int64_t)gj * g.sbj] : 0.0f);
            }
        }
        __syncthreads();
        const bf16x8 a = *(const bf16x8 *)&sA[w * 16 + lr][k8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bf16x8 b = *(const bf16x8 *)&sB[j * 16 + lr][k8];
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) gemm_store(g, i0 + w * 16 + 4 * (lane >> 4) + v, j0 + j * 16 + lr, acc[j][v]);
}

// delta = w_j (y - t) / B; part[block] = sum of w_j (y - t)^2 over the block's elements
__global__ void __launch_bounds__(256) k_out_delta(const float *Y, const float *T, const float *w, int64_t n, int nout,
                                                    float invB, float *delta, double *part) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double s = 0.0;
    if (e < n) {
        const int j = (int)(e % nout);
        const float d = Y[e] - T[e];
        delta[e] = w[j] * d * invB;
        s = (double)w[j] * (double)d * (double)d;
    }
    __shared__ double red[4];
    s = wave_sum_d(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// loss = scale * sum(part) in a fixed order, written to hist[*counter] (hist[0] without a counter)
__global__ void __launch_bounds__(256) k_loss_final(const double *part, int np, double scale, double *hist,
                                                     const int *counter) {
    double s = 0.0;
    for (int p = threadIdx.x; p < np; p += 256) s += part[p];
    __shared__ double red[4];
    s = wave_sum_d(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) hist[counter ? counter[0] : 0] = scale * ((red[0] + red[1]) + (red[2] + red[3]));
}

__global__ void __launch_bounds__(256) k_colsum(const float *D, int64_t B, int n, float *out) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    float s = 0.0f;
    for (int64_t b = 0; b < B; ++b) s += D[b * n + j];
    out[j] = s;
}

__global__ void __launch_bounds__(256) k_adam(float *th, const float *g, float *m, float *v, int64_t P, float lr,
                                               float b1, float b2, float eps, const int *counter) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= P) return;
    const int t = counter[0] + 1;
    const float c1 = (float)(1.0 - pow((double)b1, (double)t));
    const float c2 = (float)(1.0 - pow((double)b2, (double)t));
    const float ge = g[e];
    const float mm = b1 * m[e] + (1.0f - b1) * ge;
    const float vv = b2 * v[e] + (1.0f - b2) * ge * ge;
    m[e] = mm;
    v[e] = vv;
    th[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

__global__ void k_tick(int *counter) {
    if (threadIdx.x == 0) counter[0] = counter[0] + 1;
}

}  // namespace

// launch helpers shared by the entry points below
static void gemm(int compute, const GemmArgs &g, hipStream_t s) {
    dim3 grid((unsigned)((g.M + 63) / 64), (unsigned)((g.N + 63) / 64));
    if (compute == RAD_BF16)
        hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL(k_gemm_f32, grid, dim3(256), 0, s, g);
    RAD_HIP(hipGetLastError());
}

// A^T (B - Bsub) with FP64 accumulation over the facet dimension
static void atb(const float *A, int64_t lda, int p, const float *B, const float *Bsub, int64_t ldb, int q, int64_t N,
                double *G, float *C, const float *scale, hipStream_t s) {
    const int ntp = (p + AT - 1) / AT, ntq = (q + AT - 1) / AT;
    int64_t nch = std::min<int64_t>(64, (N + 2047) / 2048);
    nch = std::max<int64_t>(nch, 1);
    int64_t rows = (N + nch - 1) / nch;
    rows = (rows + AROWS - 1) / AROWS * AROWS;
    nch = (N + rows - 1) / rows;
    DevBuf<double> part((size_t)nch * ntp * ntq * AT * AT);
    hipLaunchKernelGGL(k_atb_part, dim3(ntp, ntq, (unsigned)nch), dim3(256), 0, s, A, lda, p, B, Bsub, ldb, q, N, rows,
                       part.p);
    const int64_t n = (int64_t)p * q;
    hipLaunchKernelGGL(k_atb_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (const double *)part.p,
                       (int)nch, ntp, ntq, p, q, G, C, scale);
    RAD_HIP(hipGetLastError());
    RAD_HIP(hipStreamSynchronize(s));  // part is released on return
}

}  // namespace rad

// ---------------------------------------------------------------------------
// perceptron state
// ---------------------------------------------------------------------------
struct rad_mlp {
    int device = 0;
    int compute = RAD_F32;
    std::vector<int> sizes;
    int64_t P = 0;
    int max_batch = 0;
    std::vector<int64_t> w_off, b_off, h_off;
    rad::DevBuf<float> params, grad, m, v, act, delta;
    rad::DevBuf<double> part, loss1;
    rad::DevBuf<int> counter;
    int64_t delta_stride = 0;
    hipStream_t cap_stream = nullptr;
    ~rad_mlp() {
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
    int layers() const { return (int)sizes.size() - 1; }
    float *hidden(int l) { return act.p + h_off[l]; }          // output of layer l (l < layers - 1)
    float *output() { return act.p + h_off[layers() - 1]; }    // training-time network output
};

namespace rad {

static void mlp_forward(rad_mlp *net, const float *X, int64_t B, float *Y, hipStream_t s) {
    const int L = net->layers();
    const float *h = X;
    for (int l = 0; l < L; ++l) {
        const int fi = net->sizes[l], fo = net->sizes[l + 1];
        float *out = l < L - 1 ? net->hidden(l) : Y;
        GemmArgs g{h, fi, 1, net->params.p + net->w_off[l], 1, fi, out, fo, net->params.p + net->b_off[l], nullptr,
                   0, (int)B, fo, fi, l < L - 1 ? EPI_BIAS_TANH : EPI_BIAS};
        gemm(net->compute, g, s);
        h = out;
    }
}

// loss partials, loss into hist (indexed by the step counter when counter != NULL), gradient
static void mlp_loss_grad(rad_mlp *net, const float *X, const float *T, const float *w, int64_t B, double *hist,
                          const int *counter, hipStream_t s) {
    const int L = net->layers();
    mlp_forward(net, X, B, net->output(), s);
    const int nout = net->sizes[L];
    const int64_t n = B * nout;
    const unsigned nb = (unsigned)((n + 255) / 256);
    float *d0 = net->delta.p, *d1 = net->delta.p + net->delta_stride;
    hipLaunchKernelGGL(k_out_delta, dim3(nb), dim3(256), 0, s, (const float *)net->output(), T, w, n, nout,
                       (float)(1.0 / (double)B), d0, net->part.p);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, (const double *)net->part.p, (int)nb,
                       0.5 / (double)B, hist, counter);
    RAD_HIP(hipGetLastError());
    for (int l = L - 1; l >= 0; --l) {
        const int fi = net->sizes[l], fo = net->sizes[l + 1];
        const float *hin = l == 0 ? X : net->hidden(l - 1);
        GemmArgs gw{d0, 1, fo, hin, fi, 1, net->grad.p + net->w_off[l], fi, nullptr, nullptr, 0, fo, fi, (int)B,
                    EPI_STORE};
        gemm(net->compute, gw, s);
        hipLaunchKernelGGL(k_colsum, dim3((unsigned)((fo + 255) / 256)), dim3(256), 0, s, (const float *)d0, B, fo,
                           net->grad.p + net->b_off[l]);
        RAD_HIP(hipGetLastError());
        if (l > 0) {
            GemmArgs gd{d0, fo, 1, net->params.p + net->w_off[l], fi, 1, d1, fi, nullptr, hin, fi, (int)B, fi, fo,
                        EPI_TANH_GRAD};
            gemm(net->compute, gd, s);
            std::swap(d0, d1);
        }
    }
}

static void mlp_adam(rad_mlp *net, double lr, double b1, double b2, double eps, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((net->P + 255) / 256)), dim3(256), 0, s, net->params.p,
                       (const float *)net->grad.p, net->m.p, net->v.p, net->P, (float)lr, (float)b1, (float)b2,
                       (float)eps, (const int *)net->counter.p);
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, s, net->counter.p);
    RAD_HIP(hipGetLastError());
}

static void reset_state(rad_mlp *net) {
    std::vector<float> z((size_t)net->P, 0.0f);
    RAD_HIP(hipMemcpy(net->m.p, z.data(), z.size() * sizeof(float), hipMemcpyHostToDevice));
    RAD_HIP(hipMemcpy(net->v.p, z.data(), z.size() * sizeof(float), hipMemcpyHostToDevice));
    RAD_HIP(hipMemcpy(net->grad.p, z.data(), z.size() * sizeof(float), hipMemcpyHostToDevice));
    int zero = 0;
    RAD_HIP(hipMemcpy(net->counter.p, &zero, sizeof(int), hipMemcpyHostToDevice));
}

static void check_net(const rad_mlp *net) { RAD_REQUIRE(net != nullptr, "null network handle"); }

static void check_batch(const rad_mlp *net, int64_t B) {
    RAD_REQUIRE(B >= 1 && B <= net->max_batch, "batch size must be in [1, max_batch]");
}

}  // namespace rad

using namespace rad;

extern "C" {

rad_status rad_pod_build(const float *S, int64_t N, int64_t M, int64_t lds, int32_t m, float *Phi, int64_t ldp,
                         double *sigma, int32_t device, void *hip_stream) {
    return guard([&] {
        RAD_REQUIRE(S && Phi && sigma, "null S, Phi or sigma");
        RAD_REQUIRE(N >= 1 && M >= 1 && M <= 1024, "need N >= 1 and 1 <= M <= 1024");
        RAD_REQUIRE(m >= 1 && m <= M && m <= N, "need 1 <= m <= min(M, N)");
        RAD_REQUIRE(lds >= M && ldp >= m, "leading dimension too small");
        RAD_HIP(hipSetDevice(device));
        hipStream_t s = (hipStream_t)hip_stream;
        DevBuf<int> flag(1);
        int zero = 0;
        RAD_HIP(hipMemcpyAsync(flag.p, &zero, sizeof(int), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)((N * M + 255) / 256)), dim3(256), 0, s, S, lds, N, (int)M,
                           flag.p);
        RAD_HIP(hipGetLastError());
        int bad = 0;
        RAD_HIP(hipMemcpyAsync(&bad, flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
        RAD_HIP(hipStreamSynchronize(s));
        RAD_REQUIRE(!bad, "snapshots contain non-finite values");
        // Gram matrix G = S^T S (FP64), eigenpairs on the host
        DevBuf<double> dG((size_t)M * M);
        atb(S, lds, (int)M, S, nullptr, lds, (int)M, N, dG.p, nullptr, nullptr, s);
        std::vector<double> G = dG.download((size_t)M * M);
        std::vector<double> A(G), W, lam;
        jacobi_svd((int)M, A, W, lam);   // G symmetric positive semi-definite: singular values are its eigenvalues
        RAD_REQUIRE(lam[0] > 0.0, "snapshots are all zero");
        RAD_REQUIRE(lam[m - 1] > lam[0] * 1e-14 * (double)M, "snapshots have rank below m");
        // Cm = W[:, :m] Lambda^{-1/2}, row-major M x m
        std::vector<double> Cm((size_t)M * m);
        for (int j = 0; j < m; ++j) {
            const double inv = 1.0 / std::sqrt(lam[j]);
            for (int64_t k = 0; k < M; ++k) Cm[(size_t)k * m + j] = W[(size_t)j * M + k] * inv;
            sigma[j] = std::sqrt(lam[j]);
        }
        DevBuf<double> dC;
        dC.upload(Cm);
        DevBuf<double> Q((size_t)N * m);
        hipLaunchKernelGGL(k_s_times_c, dim3((unsigned)((N + AT - 1) / AT), (unsigned)((m + AT - 1) / AT)), dim3(256),
                           0, s, S, lds, N, (int)M, (const double *)dC.p, (int)m, Q.p);
        RAD_HIP(hipGetLastError());
        // re-orthonormalise the modes (CGS2, FP64)
        SketchBlock b{};
        b.i0 = 0;
        b.m = (int32_t)N;
        b.ell = m;
        b.y_off = 0;
        std::vector<SketchBlock> hb{b};
        DevBuf<SketchBlock> db;
        db.upload(hb);
        if (N >= 4096) {
            const int64_t nch = (N + 2047) / 2048;
            DevBuf<double> part((size_t)nch * (m + 1)), normpart((size_t)nch);
            launch_cgs2_tall(Q.p, db.p, 1, 0, nullptr, nullptr, (int32_t)N, m, part.p, normpart.p, nullptr, s);
            RAD_HIP(hipStreamSynchronize(s));
        } else {
            launch_cgs2(Q.p, db.p, 1, 0, nullptr, nullptr, s);
        }
        hipLaunchKernelGGL(k_to_phi32, dim3((unsigned)((N * m + 255) / 256)), dim3(256), 0, s, (const double *)Q.p, N,
                           (int)m, Phi, ldp);
        RAD_HIP(hipGetLastError());
        RAD_HIP(hipStreamSynchronize(s));
    });
}

rad_status rad_pod_project(const float *Phi, int64_t N, int32_t m, int64_t ldp, const float *B, const float *E,
                           int64_t R, int64_t ldb, const float *scale, float *C, void *hip_stream) {
    return guard([&] {
        RAD_REQUIRE(Phi && B && C, "null Phi, B or C");
        RAD_REQUIRE(N >= 1 && m >= 1 && R >= 1 && m <= 4096 && R <= (1 << 20), "bad sizes");
        RAD_REQUIRE(ldp >= m && ldb >= R, "leading dimension too small");
        atb(Phi, ldp, m, B, E, ldb, (int)R, N, nullptr, C, scale, (hipStream_t)hip_stream);
    });
}

rad_status rad_pod_expand(const float *Phi, int64_t N, int32_t m, int64_t ldp, const float *C, const float *scale,
                          const float *E, int64_t R, int64_t ldb, float *B, void *hip_stream) {
    return guard([&] {
        RAD_REQUIRE(Phi && B && C, "null Phi, B or C");
        RAD_REQUIRE(N >= 1 && m >= 1 && R >= 1 && R <= (1 << 20), "bad sizes");
        RAD_REQUIRE(ldp >= m && ldb >= R, "leading dimension too small");
        dim3 grid((unsigned)((N + AT - 1) / AT), (unsigned)((R + AT - 1) / AT));
        hipLaunchKernelGGL(k_pod_expand, grid, dim3(256), 0, (hipStream_t)hip_stream, Phi, ldp, N, (int)m, C, scale, E,
                           ldb, (int)R, B);
        RAD_HIP(hipGetLastError());
    });
}

rad_status rad_mlp_create(const int32_t *sizes, int32_t nsizes, const float *params, int32_t compute,
                          int32_t max_batch, int32_t device, rad_mlp **out) {
    if (out) *out = nullptr;
    return guard([&] {
        RAD_REQUIRE(out && sizes && params, "null sizes, params or out");
        RAD_REQUIRE(nsizes >= 2 && nsizes <= 8, "need 2 <= nsizes <= 8");
        RAD_REQUIRE(compute == RAD_F32 || compute == RAD_BF16, "compute must be RAD_F32 or RAD_BF16");
        RAD_REQUIRE(max_batch >= 1 && max_batch <= (1 << 20), "max_batch must be in [1, 2^20]");
        for (int i = 0; i < nsizes; ++i) RAD_REQUIRE(sizes[i] >= 1 && sizes[i] <= 1024, "layer widths must be 1..1024");
        RAD_HIP(hipSetDevice(device));
        auto net = std::make_unique<rad_mlp>();
        net->device = device;
        net->compute = compute;
        net->sizes.assign(sizes, sizes + nsizes);
        net->max_batch = max_batch;
        const int L = nsizes - 1;
        int64_t off = 0, hoff = 0;
        int maxw = 1;
        for (int l = 0; l < L; ++l) {
            net->w_off.push_back(off);
            off += (int64_t)sizes[l + 1] * sizes[l];
            net->b_off.push_back(off);
            off += sizes[l + 1];
            net->h_off.push_back(hoff);
            hoff += (int64_t)max_batch * sizes[l + 1];
            maxw = std::max(maxw, (int)sizes[l + 1]);
        }
        net->P = off;
        for (int64_t i = 0; i < net->P; ++i) RAD_REQUIRE(std::isfinite(params[i]), "non-finite parameter");
        net->params.alloc((size_t)net->P);
        net->grad.alloc((size_t)net->P);
        net->m.alloc((size_t)net->P);
        net->v.alloc((size_t)net->P);
        net->act.alloc((size_t)hoff);
        net->delta_stride = (int64_t)max_batch * maxw;
        net->delta.alloc((size_t)(2 * net->delta_stride));
        net->part.alloc((size_t)(((int64_t)max_batch * sizes[L] + 255) / 256));
        net->loss1.alloc(1);
        net->counter.alloc(1);
        RAD_HIP(hipMemcpy(net->params.p, params, (size_t)net->P * sizeof(float), hipMemcpyHostToDevice));
        reset_state(net.get());
        RAD_HIP(hipStreamCreateWithFlags(&net->cap_stream, hipStreamNonBlocking));
        *out = net.release();
    });
}

int64_t rad_mlp_param_count(const rad_mlp *net) { return net ? net->P : -1; }

rad_status rad_mlp_get_params(const rad_mlp *net, float *params) {
    return guard([&] {
        check_net(net);
        RAD_REQUIRE(params, "null params");
        RAD_HIP(hipSetDevice(net->device));
        RAD_HIP(hipDeviceSynchronize());
        RAD_HIP(hipMemcpy(params, net->params.p, (size_t)net->P * sizeof(float), hipMemcpyDeviceToHost));
    });
}

rad_status rad_mlp_set_params(rad_mlp *net, const float *params) {
    return guard([&] {
        check_net(net);
        RAD_REQUIRE(params, "null params");
        for (int64_t i = 0; i < net->P; ++i) RAD_REQUIRE(std::isfinite(params[i]), "non-finite parameter");
        RAD_HIP(hipSetDevice(net->device));
        RAD_HIP(hipDeviceSynchronize());
        RAD_HIP(hipMemcpy(net->params.p, params, (size_t)net->P * sizeof(float), hipMemcpyHostToDevice));
        reset_state(net);
    });
}

rad_status rad_mlp_forward(rad_mlp *net, const float *X, int64_t B, float *Y, void *hip_stream) {
    return guard([&] {
        check_net(net);
        RAD_REQUIRE(X && Y, "null X or Y");
        check_batch(net, B);
        RAD_HIP(hipSetDevice(net->device));
        mlp_forward(net, X, B, Y, (hipStream_t)hip_stream);
    });
}

rad_status rad_mlp_loss_grad(rad_mlp *net, const float *X, const float *T, const float *w, int64_t B, double *loss,
                             float *grad, void *hip_stream) {
    return guard([&] {
        check_net(net);
        RAD_REQUIRE(X && T && w, "null X, T or w");
        check_batch(net, B);
        RAD_HIP(hipSetDevice(net->device));
        hipStream_t s = (hipStream_t)hip_stream;
        mlp_loss_grad(net, X, T, w, B, net->loss1.p, nullptr, s);
        if (loss) RAD_HIP(hipMemcpyAsync(loss, net->loss1.p, sizeof(double), hipMemcpyDeviceToHost, s));
        if (grad) RAD_HIP(hipMemcpyAsync(grad, net->grad.p, (size_t)net->P * sizeof(float), hipMemcpyDeviceToHost, s));
        if (loss || grad) RAD_HIP(hipStreamSynchronize(s));
    });
}

rad_status rad_mlp_adam_step(rad_mlp *net, double lr, double beta1, double beta2, double eps, void *hip_stream) {
    return guard([&] {
        check_net(net);
        RAD_REQUIRE(lr > 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0, "bad Adam parameters");
        RAD_HIP(hipSetDevice(net->device));
        mlp_adam(net, lr, beta1, beta2, eps, (hipStream_t)hip_stream);
    });
}

rad_status rad_mlp_train(rad_mlp *net, const float *X, const float *T, const float *w, int64_t B, int32_t steps,
                         double lr, double beta1, double beta2, double eps, double *loss_hist, void *hip_stream) {
    return guard([&] {
        check_net(net);
        RAD_REQUIRE(X && T && w, "null X, T or w");
        check_batch(net, B);
        RAD_REQUIRE(steps >= 1, "steps must be >= 1");
        RAD_REQUIRE(lr > 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0, "bad Adam parameters");
        RAD_HIP(hipSetDevice(net->device));
        hipStream_t s = (hipStream_t)hip_stream;
        // loss history indexed by the step counter: counter values from its
        // current value on; the device buffer covers them all
        int c0 = 0;
        RAD_HIP(hipStreamSynchronize(s));
        RAD_HIP(hipMemcpy(&c0, net->counter.p, sizeof(int), hipMemcpyDeviceToHost));
        DevBuf<double> hist((size_t)c0 + (size_t)steps);
        // one step captured as a graph (no memory-set nodes), replayed steps times
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        RAD_HIP(hipStreamBeginCapture(net->cap_stream, hipStreamCaptureModeThreadLocal));
        try {
            mlp_loss_grad(net, X, T, w, B, hist.p, net->counter.p, net->cap_stream);
            mlp_adam(net, lr, beta1, beta2, eps, net->cap_stream);
        } catch (...) {
            hipGraph_t tmp = nullptr;
            (void)hipStreamEndCapture(net->cap_stream, &tmp);
            if (tmp) (void)hipGraphDestroy(tmp);
            throw;
        }
        RAD_HIP(hipStreamEndCapture(net->cap_stream, &graph));
        hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            RAD_HIP(e);
        }
        hipError_t err = hipSuccess;
        for (int i = 0; i < steps && err == hipSuccess; ++i) err = hipGraphLaunch(exec, s);
        if (err == hipSuccess) err = hipStreamSynchronize(s);
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        RAD_HIP(err);
        if (loss_hist)
            RAD_HIP(hipMemcpy(loss_hist, hist.p + c0, (size_t)steps * sizeof(double), hipMemcpyDeviceToHost));
    });
}

void rad_mlp_free(rad_mlp *net) {
    if (!net) return;
    (void)hipSetDevice(net->device);
    (void)hipDeviceSynchronize();
    delete net;
}

}  // extern "C"
