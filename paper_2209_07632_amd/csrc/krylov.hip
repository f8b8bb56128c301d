// Elementwise and reduction kernels of the accelerated solves of
// (I - rho F-hat) B = E: Chebyshev acceleration and GMRES.  Neither is in the
// paper, which relaxes with Jacobi; they serve systems whose spectral radius
// rho(F) approaches one (closed or deep bodies in the infrared band, rho = 1),
// where Jacobi needs many products.
//
// Every kernel works on blocks of R columns in the solver's working layout:
// R-major (element (t, c) at t ld + c, ld a multiple of 4) on the matrix-core
// path, or column-major (c ld + t) on the single-RHS path.  Column sums are
// taken per 64-row tile (rows in order, then a fixed-order sum over tiles,
// k_reduce_parts), so every result is deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rad_internal.h"

namespace rad {

namespace {

// Work split of a (tile, column chunk) pair.  R-major: 256 threads, lane =
// column (64 per chunk), wave = a quarter of the tile's rows, so a wave reads
// 64 consecutive values of a row.  Column-major: 64 threads per (tile,
// column), lane = row.
struct Geo {
    int64_t N, ld;
    int R;
    int rmajor;
};

__device__ __forceinline__ int64_t at(const Geo &g, int64_t t, int c) { return g.rmajor ? t * g.ld + c : c * g.ld + t; }

// Sums the per-thread values of one column over the tile in a fixed order and
// stores the tile's sum at out[tile * R + c].
__device__ __forceinline__ void tile_sum(const Geo &g, double v, int c, int tile, double *out) {
    if (g.rmajor) {
        __shared__ double red[4][64];
        red[threadIdx.x >> 6][threadIdx.x & 63] = v;
        __syncthreads();
        if (threadIdx.x < 64 && c < g.R)
            out[(int64_t)tile * g.R + c] = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
    } else {
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (threadIdx.x == 0) out[(int64_t)tile * g.R + c] = v;
    }
}

// Iterates f(t) over this thread's rows of the tile, for column c.
template <class F>
__device__ __forceinline__ void rows_of(const Geo &g, int tile, F &&f) {
    if (g.rmajor) {
        const int64_t t0 = (int64_t)tile * 64 + (threadIdx.x >> 6) * 16;
        for (int i = 0; i < 16; ++i)
            if (t0 + i < g.N) f(t0 + i);
    } else {
        const int64_t t = (int64_t)tile * 64 + threadIdx.x;
        if (t < g.N) f(t);
    }
}

__device__ __forceinline__ int column(const Geo &g) {
    return g.rmajor ? blockIdx.y * 64 + (threadIdx.x & 63) : blockIdx.y;
}

// Chebyshev start: r = rho Y (Y = F-hat E, i.e. r = E - (I - rho F) E),
// d = r / theta; tile sums of r^2.
template <class T>
__global__ void k_cheb_init(Geo g, double rho, double inv_theta, const T *Y, T *r, T *d, double *part) {
    const int c = column(g);
    double s = 0.0;
    if (c < g.R)
        rows_of(g, blockIdx.x, [&](int64_t t) {
            const int64_t k = at(g, t, c);
            const T rv = (T)(rho * (double)Y[k]);
            r[k] = rv;
            d[k] = (T)((double)rv * inv_theta);
            s += (double)rv * (double)rv;
        });
    tile_sum(g, s, c, blockIdx.x, part);
}

// One Chebyshev step after Y = F-hat d:  B += d;  r -= d - rho Y;
// d = a d + b r (the next direction, with the updated r); tile sums of r^2.
template <class T>
__global__ void k_cheb_step(Geo g, double rho, double a, double b, const T *Y, T *B, T *r, T *d, double *part) {
    const int c = column(g);
    double s = 0.0;
    if (c < g.R)
        rows_of(g, blockIdx.x, [&](int64_t t) {
            const int64_t k = at(g, t, c);
            const T dv = d[k];
            B[k] = B[k] + dv;
            const T rv = r[k] - (dv - (T)(rho * (double)Y[k]));
            r[k] = rv;
            d[k] = (T)(a * (double)dv + b * (double)rv);
            s += (double)rv * (double)rv;
        });
    tile_sum(g, s, c, blockIdx.x, part);
}

// w = e - (v - rho Y): the residual of (I - rho F-hat) v = e with Y = F-hat v;
// with e = nullptr, w = v - rho Y (the operator applied to v)
// (rho per facet from rhov when given, tree order)
template <class T>
__global__ void k_apply_a(Geo g, double rho, const T *rhov, const T *e, const T *v, const T *Y, T *w) {
    const int c = column(g);
    if (c < g.R) rows_of(g, blockIdx.x, [&](int64_t t) {
        const int64_t k = at(g, t, c);
        const double av = (double)v[k] - (rhov ? (double)rhov[t] : rho) * (double)Y[k];
        w[k] = (T)(e ? (double)e[k] - av : av);
    });
}

// tile sums of the products V_i w, i = 0 .. nv-1 (V_i at V + i vstride):
// part[(i n_tiles + tile) R + c]
template <class T>
__global__ void k_dots(Geo g, const T *V, int64_t vstride, int nv, const T *w, double *part, int n_tiles) {
    const int c = column(g);
    for (int i = 0; i < nv; ++i) {
        double s = 0.0;
        if (c < g.R)
            rows_of(g, blockIdx.x, [&](int64_t t) {
                const int64_t k = at(g, t, c);
                s += (double)V[i * vstride + k] * (double)w[k];
            });
        tile_sum(g, s, c, blockIdx.x, part + (int64_t)i * n_tiles * g.R);
        __syncthreads();
    }
}

// w += sign sum_i h[i R + c] V_i (FP64 coefficients)
template <class T>
__global__ void k_combine(Geo g, const T *V, int64_t vstride, int nv, const double *h, double sign, T *w) {
    const int c = column(g);
    if (c < g.R) rows_of(g, blockIdx.x, [&](int64_t t) {
        const int64_t k = at(g, t, c);
        double acc = (double)w[k];
        for (int i = 0; i < nv; ++i) acc += sign * h[(int64_t)i * g.R + c] * (double)V[i * vstride + k];
        w[k] = (T)acc;
    });
}

// v = w / sqrt(nrm2[c]) (0 where nrm2[c] is 0)
template <class T>
__global__ void k_scale_cols(Geo g, const T *w, const double *nrm2, T *v) {
    const int c = column(g);
    if (c < g.R) rows_of(g, blockIdx.x, [&](int64_t t) {
        const int64_t k = at(g, t, c);
        const double s = nrm2[c] > 0.0 ? 1.0 / sqrt(nrm2[c]) : 0.0;
        v[k] = (T)((double)w[k] * s);
    });
}

// out[i R + c] = sum over tiles of part[(i n_tiles + tile) R + c], tiles in order
__global__ void k_reduce_many(const double *part, int n_tiles, int R, int nv, double *out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nv * R) return;
    const int i = (int)(e / R), c = (int)(e % R);
    const double *p = part + (int64_t)i * n_tiles * R + c;
    double s = 0.0;
    for (int tl = 0; tl < n_tiles; ++tl) s += p[(int64_t)tl * R];
    out[e] = s;
}

dim3 grid_of(const rad_hmat *H, int64_t R, bool rmajor) {
    return dim3((unsigned)((H->N + 63) / 64), (unsigned)(rmajor ? (R + 63) / 64 : R));
}
dim3 block_of(bool rmajor) { return dim3(rmajor ? 256 : 64); }

}  // namespace

void krylov_cheb_init(const rad_hmat *H, bool rmajor, int64_t ld, int64_t R, double rho, double theta, const void *Y,
                      void *r, void *d, double *part, hipStream_t s) {
    const dim3 gr = grid_of(H, R, rmajor), bl = block_of(rmajor);
    const Geo g{H->N, ld, (int)R, rmajor ? 1 : 0};
    if (H->dtype == RAD_F64)
        hipLaunchKernelGGL(k_cheb_init<double>, gr, bl, 0, s, g, rho, 1.0 / theta, (const double *)Y, (double *)r,
                           (double *)d, part);
    else
        hipLaunchKernelGGL(k_cheb_init<float>, gr, bl, 0, s, g, rho, 1.0 / theta, (const float *)Y, (float *)r,
                           (float *)d, part);
    RAD_HIP(hipGetLastError());
}

void krylov_cheb_step(const rad_hmat *H, bool rmajor, int64_t ld, int64_t R, double rho, double a, double b,
                      const void *Y, void *B, void *r, void *d, double *part, hipStream_t s) {
    const dim3 gr = grid_of(H, R, rmajor), bl = block_of(rmajor);
    const Geo g{H->N, ld, (int)R, rmajor ? 1 : 0};
    if (H->dtype == RAD_F64)
        hipLaunchKernelGGL(k_cheb_step<double>, gr, bl, 0, s, g, rho, a, b, (const double *)Y, (double *)B,
                           (double *)r, (double *)d, part);
    else
        hipLaunchKernelGGL(k_cheb_step<float>, gr, bl, 0, s, g, rho, a, b, (const float *)Y, (float *)B, (float *)r,
                           (float *)d, part);
    RAD_HIP(hipGetLastError());
}

void krylov_apply_a(const rad_hmat *H, bool rmajor, int64_t ld, int64_t R, double rho, const void *rhov, const void *e,
                    const void *v, const void *Y, void *w, hipStream_t s) {
    const dim3 gr = grid_of(H, R, rmajor), bl = block_of(rmajor);
    const Geo g{H->N, ld, (int)R, rmajor ? 1 : 0};
    if (H->dtype == RAD_F64)
        hipLaunchKernelGGL(k_apply_a<double>, gr, bl, 0, s, g, rho, (const double *)rhov, (const double *)e,
                           (const double *)v, (const double *)Y, (double *)w);
    else
        hipLaunchKernelGGL(k_apply_a<float>, gr, bl, 0, s, g, rho, (const float *)rhov, (const float *)e,
                           (const float *)v, (const float *)Y, (float *)w);
    RAD_HIP(hipGetLastError());
}

void krylov_dots(const rad_hmat *H, bool rmajor, int64_t ld, int64_t R, const void *V, int64_t vstride, int nv,
                 const void *w, double *part, double *out, hipStream_t s) {
    const dim3 gr = grid_of(H, R, rmajor), bl = block_of(rmajor);
    const Geo g{H->N, ld, (int)R, rmajor ? 1 : 0};
    const int n_tiles = (int)gr.x;
    if (H->dtype == RAD_F64)
        hipLaunchKernelGGL(k_dots<double>, gr, bl, 0, s, g, (const double *)V, vstride, nv, (const double *)w, part,
                           n_tiles);
    else
        hipLaunchKernelGGL(k_dots<float>, gr, bl, 0, s, g, (const float *)V, vstride, nv, (const float *)w, part,
                           n_tiles);
    const int64_t tot = (int64_t)nv * R;
    hipLaunchKernelGGL(k_reduce_many, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, (const double *)part,
                       n_tiles, (int)R, nv, out);
    RAD_HIP(hipGetLastError());
}

void krylov_combine(const rad_hmat *H, bool rmajor, int64_t ld, int64_t R, const void *V, int64_t vstride, int nv,
                    const double *h, double sign, void *w, hipStream_t s) {
    const dim3 gr = grid_of(H, R, rmajor), bl = block_of(rmajor);
    const Geo g{H->N, ld, (int)R, rmajor ? 1 : 0};
    if (H->dtype == RAD_F64)
        hipLaunchKernelGGL(k_combine<double>, gr, bl, 0, s, g, (const double *)V, vstride, nv, h, sign, (double *)w);
    else
        hipLaunchKernelGGL(k_combine<float>, gr, bl, 0, s, g, (const float *)V, vstride, nv, h, sign, (float *)w);
    RAD_HIP(hipGetLastError());
}

void krylov_scale(const rad_hmat *H, bool rmajor, int64_t ld, int64_t R, const void *w, const double *nrm2, void *v,
                  hipStream_t s) {
    const dim3 gr = grid_of(H, R, rmajor), bl = block_of(rmajor);
    const Geo g{H->N, ld, (int)R, rmajor ? 1 : 0};
    if (H->dtype == RAD_F64)
        hipLaunchKernelGGL(k_scale_cols<double>, gr, bl, 0, s, g, (const double *)w, nrm2, (double *)v);
    else
        hipLaunchKernelGGL(k_scale_cols<float>, gr, bl, 0, s, g, (const float *)w, nrm2, (float *)v);
    RAD_HIP(hipGetLastError());
}

}  // namespace rad
