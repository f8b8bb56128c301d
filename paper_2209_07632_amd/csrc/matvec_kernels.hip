// H-matvec Y = F-hat X (Algorithm 5) and the Jacobi update of the radiosity
// solve, on the device layout written by the builder.
//
// Two phases per product, both owner-computes (no atomics, deterministic):
//   phase 1: for every column node J with low-rank blocks, T_J = V_J^T X_J
//            (V_J = the V factors of all those blocks stacked side by side);
//   phase 2: for every quadtree leaf L (rows I_L):
//            Y_L = sum_dense A_LJ X_J + sum_csr A_LJ X_J + sum_lowrank U'_L T_b.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "rad_internal.h"

namespace rad {

namespace {

template <class T>
__device__ __forceinline__ T wsum(T v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <class T>
__global__ void k_gather(const int32_t *perm, const T *src, int64_t lds, T *dst, int64_t ldd, int64_t N, int64_t R) {
    int64_t tot = N * R;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = e / N, t = e - r * N;
        dst[t + r * ldd] = src[(int64_t)perm[t] + r * lds];
    }
}

template <class T>
__global__ void k_scatter(const int32_t *perm, const T *src, int64_t lds, T *dst, int64_t ldd, int64_t N, int64_t R) {
    int64_t tot = N * R;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = e / N, t = e - r * N;
        dst[(int64_t)perm[t] + r * ldd] = src[t + r * lds];
    }
}

// phase 1 for column nodes below kProjWideN facets: one wave per stacked V
// column, from a list of (group, column) items, four items per workgroup.
// Lanes take VW consecutive facets with one 16-byte load of V (columns start
// on 8-value boundaries), up to four loads in flight; X_J, which starts at
// any facet, is read value by value (the waves of one node share it in
// cache).  Lane sums meet by a fixed butterfly.
template <class T>
__global__ void __launch_bounds__(256) k_proj_cols(const int32_t *items, int32_t n_items, const ProjGroup *groups,
                                                    const T *vals, const T *X, int64_t ldx, T *Tb, int32_t t_ld,
                                                    const int32_t *stop) {
    if (stop && *stop) return;
    constexpr int VW = 16 / sizeof(T);
    typedef typename std::conditional<sizeof(T) == 4, float4, double2>::type vec_t;
    const int it = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (it >= n_items) return;
    const int lane = threadIdx.x & 63;
    const ProjGroup g = groups[items[2 * it]];
    const int kk = items[2 * it + 1];
    const int64_t r = blockIdx.z;
    const T *x = X + g.j0 + r * ldx;
    const T *v = vals + g.v_off + (int64_t)kk * g.ld;
    constexpr int STEP = 64 * VW;
    T acc = 0;
    int j = VW * lane;
    for (; j + 3 * STEP + VW <= g.n; j += 4 * STEP) {
        vec_t a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = *(const vec_t *)(v + j + q * STEP);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const T *av = (const T *)&a[q];
#pragma unroll
            for (int u = 0; u < VW; ++u) acc += av[u] * x[j + q * STEP + u];
        }
    }
    for (; j + VW <= g.n; j += STEP) {
        const vec_t a = *(const vec_t *)(v + j);
        const T *av = (const T *)&a;
#pragma unroll
        for (int u = 0; u < VW; ++u) acc += av[u] * x[j + u];
    }
    for (int u = 0; j + u < g.n && u < VW; ++u) acc += v[j + u] * x[j + u];
    acc = wsum(acc);
    if (lane == 0) Tb[g.t_off + kk + r * t_ld] = acc;
}

// phase 2: one workgroup per (64-row tile, right-hand side).  The packed panel
// (64 x K, column-major) is streamed with 16-byte loads: a wave reads VW
// consecutive columns per step, lane l holding rows VW (l % (64/VW)) .. + VW-1
// of column VW g + l / (64/VW); wave w takes column groups w, w+4, ... and
// keeps four groups in flight.  CSR tasks are split over the waves by task.
// Partial row sums meet in LDS in a fixed order.
// kMode 0: Y = F-hat X.  kMode 1: one Jacobi iteration with X = B_old,
// Y = B_new = E + rho (F-hat B_old), and partial[tile R + r] = the tile's
// sum of (B_new - B_old)^2 (FP64, rows in order).  kMode 2: also
// epartial[tile R + r] = the tile's sum of E^2.  With stop given, the kernel
// returns at once while *stop is set.
// phase 1 for column nodes of many facets: one workgroup per stacked V
// column (item = (group, column)); its 256 threads stride the facets with
// 16-byte loads of V, four loads in flight, and meet in LDS in a fixed order.
template <class T>
__global__ void __launch_bounds__(256) k_proj_wide(const int32_t *items, const ProjGroup *groups, const T *vals,
                                                    const T *X, int64_t ldx, T *Tb, int32_t t_ld,
                                                    const int32_t *stop) {
    if (stop && *stop) return;
    constexpr int VW = 16 / sizeof(T);
    typedef typename std::conditional<sizeof(T) == 4, float4, double2>::type vec_t;
    const ProjGroup g = groups[items[2 * blockIdx.x]];
    const int kk = items[2 * blockIdx.x + 1];
    const int64_t r = blockIdx.z;
    const T *x = X + g.j0 + r * ldx;
    const T *v = vals + g.v_off + (int64_t)kk * g.ld;   // 16-byte aligned (v_off, ld multiples of 8)
    const int t = threadIdx.x;
    T acc = 0;
    constexpr int STEP = 256 * VW;
    int j = VW * t;
    for (; j + 3 * STEP + VW <= g.n; j += 4 * STEP) {
        vec_t a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = *(const vec_t *)(v + j + q * STEP);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const T *av = (const T *)&a[q];
#pragma unroll
            for (int u = 0; u < VW; ++u) acc += av[u] * x[j + q * STEP + u];
        }
    }
    for (; j < g.n; j += STEP)
        for (int u = 0; u < VW && j + u < g.n; ++u) acc += v[j + u] * x[j + u];
    acc = wsum(acc);
    __shared__ T red[4];
    if ((t & 63) == 0) red[t >> 6] = acc;
    __syncthreads();
    if (t == 0) Tb[g.t_off + kk + r * t_ld] = (red[0] + red[1]) + (red[2] + red[3]);
}

// The end of a single-RHS product for one 64-row tile and right-hand side r,
// run by one wave (lane = row): y (this row's value of F-hat X, valid for
// row < N) is stored, or turned into the Jacobi update with its partial sums
// (kMode as k_tile_gemv).
template <class T, int kMode>
__device__ __forceinline__ void gemv_epilogue(int tile, int64_t r, int lane, T y, int64_t N, const T *x, T *Y,
                                              int64_t ldy, const T *E, const T *rho, T rho_s, double *partial,
                                              double *epartial, int R) {
    const int64_t row = (int64_t)tile * 64 + lane;
    double d2 = 0.0, e2 = 0.0;
    if (row < N) {
        if (kMode == 0) {
            Y[row + r * ldy] = y;
        } else {
            const T e = E[row + r * ldy];
            const T b = e + (rho ? rho[row] : rho_s) * y;
            const double d = (double)b - (double)x[row];
            d2 = d * d;
            e2 = (double)e * (double)e;
            Y[row + r * ldy] = b;
        }
    }
    if (kMode != 0) {
        d2 = wsum(d2);
        if (kMode == 2) e2 = wsum(e2);
        if (lane == 0) {
            partial[(int64_t)tile * R + r] = d2;
            if (kMode == 2) epartial[(int64_t)tile * R + r] = e2;
        }
    }
}

// The column groups of a tile are those of its panel followed by those of
// its compressed CSR panel (when cpan is given; the CSR tasks are then not
// walked row by row).  With segs given, blockIdx.x is a segment of them
// (column groups [g0, g1), the tile's CSR tasks when csr is set): its 64 row
// sums go to spart[(slot R + r) 64 + row] and k_gemv_finish completes the tile.
template <class T, int kMode>
__global__ void __launch_bounds__(256) k_tile_gemv(const TileInfo *tiles, const int32_t *brow, const TileTask *ctasks,
                                                    const T *vals, const int32_t *csr_ptr, const int32_t *csr_idx,
                                                    int64_t csr_val_start, const CsrPanel *cpan, const T *cvals,
                                                    const int32_t *cbrow, const T *X, int64_t ldx, const T *Tb,
                                                    int32_t t_ld, int64_t N, T *Y, int64_t ldy, const T *E,
                                                    const T *rho, T rho_s, double *partial, double *epartial,
                                                    const int32_t *stop, const GemvSeg *segs, T *spart) {
    if (stop && *stop) return;
    constexpr int VW = 16 / sizeof(T);      // values per 16-byte load
    constexpr int LPC = 64 / VW;            // lanes per panel column
    typedef typename std::conditional<sizeof(T) == 4, float4, double2>::type vec_t;
    const GemvSeg sg = segs ? segs[blockIdx.x] : GemvSeg{(int32_t)blockIdx.x, 0, -1, 1, 0};
    const int tile = sg.tile;
    const TileInfo ti = tiles[tile];
    const int64_t r = blockIdx.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int sub = lane / LPC, r0 = VW * (lane % LPC);
    const T *x = X + r * ldx;
    const T *tb = Tb + r * t_ld;
    T acc[VW];
#pragma unroll
    for (int u = 0; u < VW; ++u) acc[u] = 0;
    auto fma_col = [&](const vec_t &a, T xv) {
        const T *av = (const T *)&a;
#pragma unroll
        for (int u = 0; u < VW; ++u) acc[u] += av[u] * xv;
    };
    auto value = [&](int32_t b) -> T { return b >= 0 ? x[b] : tb[-1 - b]; };
    const CsrPanel cp = cpan ? cpan[tile] : CsrPanel{0, 0, 0, 0};
    const int ngm = ti.k16 / VW, ngc = cp.k16 / VW;
    // column groups [g0, gend) of this workgroup (all columns that hold
    // values, a multiple of 16, or a segment of them), the panel's first
    const int gend = sg.g1 < 0 ? ngm + ngc : sg.g1;
    for (int part = 0; part < 2; ++part) {
        const int base = part == 0 ? 0 : ngm;
        const int ngroups = min(gend, part == 0 ? ngm : ngm + ngc) - base;
        int g = max(sg.g0, base) - base + w;
        if (g - w >= ngroups) continue;
        const T *panel = part == 0 ? vals + ti.panel_off + r0 : cvals + cp.panel_off + r0;
        const int32_t *br = part == 0 ? brow + ti.brow_off : cbrow + cp.brow_off;
        // the operand-row indices of an iteration are loaded one iteration
        // ahead of the gathers that use them
        int32_t bi[4] = {0, 0, 0, 0};
        if (g + 12 < ngroups)
#pragma unroll
            for (int q = 0; q < 4; ++q) bi[q] = br[VW * g + sub + 4 * VW * q];
        for (; g + 12 < ngroups; g += 16) {
            const int k0 = VW * g + sub, k1 = k0 + 4 * VW, k2 = k0 + 8 * VW, k3 = k0 + 12 * VW;
            const vec_t a0 = *(const vec_t *)(panel + (int64_t)k0 * 64);
            const vec_t a1 = *(const vec_t *)(panel + (int64_t)k1 * 64);
            const vec_t a2 = *(const vec_t *)(panel + (int64_t)k2 * 64);
            const vec_t a3 = *(const vec_t *)(panel + (int64_t)k3 * 64);
            const T x0 = value(bi[0]), x1 = value(bi[1]), x2 = value(bi[2]), x3 = value(bi[3]);
            if (g + 28 < ngroups)
#pragma unroll
                for (int q = 0; q < 4; ++q) bi[q] = br[k0 + 16 * VW + 4 * VW * q];
            fma_col(a0, x0);
            fma_col(a1, x1);
            fma_col(a2, x2);
            fma_col(a3, x3);
        }
        for (; g < ngroups; g += 4) {
            const int k0 = VW * g + sub;
            const vec_t a0 = *(const vec_t *)(panel + (int64_t)k0 * 64);
            fma_col(a0, value(br[k0]));
        }
    }
    __shared__ T red[4][VW][64];
#pragma unroll
    for (int u = 0; u < VW; ++u) red[w][sub][r0 + u] = acc[u];
    // CSR tasks: lane = row, wave w takes tasks w, w+4, ...
    T cacc = 0;
    for (int c = ti.csr_begin + w; sg.csr && !cpan && c < ti.csr_end; c += 4) {
        const TileTask tk = ctasks[c];
        if (lane >= tk.r_lo && lane < tk.r_hi) {
            const int32_t *ptr = csr_ptr + tk.aux_off + tk.row_off + lane;
            const T *v = vals + tk.a_off;
            const int32_t *ci = csr_idx + (tk.a_off - csr_val_start);
            const T *xc = x + tk.col0;
            for (int e = ptr[0]; e < ptr[1]; ++e) cacc += v[e] * xc[ci[e]];
        }
    }
    __shared__ T cred[4][64];
    cred[w][lane] = cacc;
    __syncthreads();
    if (w != 0) return;
    T s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int u = 0; u < VW; ++u) s += red[q][u][lane];
    const T y = s + ((cred[0][lane] + cred[1][lane]) + (cred[2][lane] + cred[3][lane]));
    if (segs) {
        spart[((int64_t)sg.slot * gridDim.y + r) * 64 + lane] = y;
        return;
    }
    gemv_epilogue<T, kMode>(tile, r, lane, y, N, x, Y, ldy, E, rho, rho_s, partial, epartial, (int)gridDim.y);
}

// The tiles of a segmented single-RHS product: one wave per (tile, right-hand
// side) sums the tile's segments (slots [tseg[tile], tseg[tile + 1]), in
// order) and runs the epilogue of k_tile_gemv.
template <class T, int kMode>
__global__ void __launch_bounds__(64) k_gemv_finish(const int32_t *tseg, const T *spart, int64_t N, const T *X,
                                                     int64_t ldx, T *Y, int64_t ldy, const T *E, const T *rho, T rho_s,
                                                     double *partial, double *epartial, const int32_t *stop) {
    if (stop && *stop) return;
    const int tile = blockIdx.x;
    const int64_t r = blockIdx.y;
    const int lane = threadIdx.x;
    const int R = (int)gridDim.y;
    T y = 0;
    for (int sl = tseg[tile]; sl < tseg[tile + 1]; ++sl) y += spart[((int64_t)sl * R + r) * 64 + lane];
    gemv_epilogue<T, kMode>(tile, r, lane, y, N, X + r * ldx, Y, ldy, E, rho, rho_s, partial, epartial, R);
}

template <class T>
__global__ void __launch_bounds__(256) k_colnorm2(const T *E, int64_t N, int64_t ld, double *partial) {
    const int64_t r = blockIdx.y;
    double s = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N; t += (int64_t)gridDim.x * blockDim.x) {
        double v = (double)E[t + r * ld];
        s += v * v;
    }
    s = wsum(s);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x + r * gridDim.x] = red[0] + red[1] + red[2] + red[3];
}

// deterministic per-column sum of the partials
__global__ void k_reduce_cols(const double *partial, int nparts, int64_t R, double *out) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s += partial[i + r * nparts];
    out[r] = s;
}

// Y = F-hat X (E == nullptr), or one fused Jacobi iteration (X = B_old,
// Y = B_new, E with leading dimension ldy == ldx; per-tile partial sums of the
// squared change, and of E^2 when epartial is given)
template <class T>
void apply_t(const rad_hmat *H, const T *X, int64_t ldx, T *Y, int64_t ldy, int64_t R, T *Tb, hipStream_t s,
             const T *E = nullptr, const T *rho = nullptr, T rho_s = 0, double *partial = nullptr,
             double *epartial = nullptr, const int32_t *stop = nullptr, bool segmented = true) {
    if (H->n_groups > 0) {
        if (H->n_pcols > 0)
            hipLaunchKernelGGL(k_proj_cols<T>, dim3((unsigned)((H->n_pcols + 3) / 4), 1, (unsigned)R), dim3(256), 0,
                               s, H->d_pcols.p, H->n_pcols, H->d_groups.p, (const T *)H->d_vals.p, X, ldx, Tb,
                               H->t_ld, stop);
        if (H->n_pwide > 0)
            hipLaunchKernelGGL(k_proj_wide<T>, dim3(H->n_pwide, 1, (unsigned)R), dim3(256), 0, s, H->d_pwide.p,
                               H->d_groups.p, (const T *)H->d_vals.p, X, ldx, Tb, H->t_ld, stop);
        RAD_HIP(hipGetLastError());
    }
    // long panels (terrain near field) are cut into segments that run as
    // separate workgroups, longest first, and are summed per tile in order;
    // otherwise one workgroup per tile (also the allocation-free product,
    // which passes its own T buffer and uses no segment workspace)
    const bool seg = segmented && H->n_gsegs > 0 && (int64_t)H->w_gpart.n >= (int64_t)H->n_gsegs * 64 * R * sizeof(T);
    T *spart = seg ? (T *)H->w_gpart.p : nullptr;
    const GemvSeg *segs = seg ? H->d_gsegs.p : nullptr;
    dim3 grid2(seg ? H->n_gsegs : H->n_tiles, (unsigned)R);
    auto tile_kernel = [&](auto mode) {
        constexpr int M = decltype(mode)::value;
        hipLaunchKernelGGL((k_tile_gemv<T, M>), grid2, dim3(256), 0, s, H->d_tiles.p, H->d_brow.p,
                           H->d_tile_tasks.p, (const T *)H->d_vals.p, H->d_csr_ptr.p, H->d_csr_idx.p,
                           H->csr_val_start, H->n_cpan > 0 ? H->d_cpan.p : nullptr, (const T *)H->d_cvals.p,
                           H->d_cbrow.p, X, ldx, (const T *)Tb, H->t_ld, H->N, Y, ldy, E, rho, rho_s, partial,
                           epartial, stop, segs, spart);
        if (seg)
            hipLaunchKernelGGL((k_gemv_finish<T, M>), dim3(H->n_tiles, (unsigned)R), dim3(64), 0, s,
                               H->d_gseg_of_tile.p, (const T *)spart, H->N, X, ldx, Y, ldy, E, rho, rho_s, partial,
                               epartial, stop);
    };
    if (!E)
        tile_kernel(std::integral_constant<int, 0>{});
    else if (!epartial)
        tile_kernel(std::integral_constant<int, 1>{});
    else
        tile_kernel(std::integral_constant<int, 2>{});
    RAD_HIP(hipGetLastError());
}

constexpr int kRedParts = 128;

}  // namespace

void mv_gather(const rad_hmat *H, const void *src, int64_t lds, void *dst, int64_t ldd, int64_t R, hipStream_t s) {
    int64_t tot = H->N * R;
    unsigned blocks = (unsigned)std::min<int64_t>((tot + 255) / 256, 8192);
    if (H->dtype == RAD_F64)
        hipLaunchKernelGGL(k_gather<double>, dim3(blocks), dim3(256), 0, s, H->d_perm.p, (const double *)src, lds,
                           (double *)dst, ldd, H->N, R);
    else
        hipLaunchKernelGGL(k_gather<float>, dim3(blocks), dim3(256), 0, s, H->d_perm.p, (const float *)src, lds,
                           (float *)dst, ldd, H->N, R);
    RAD_HIP(hipGetLastError());
}

void mv_scatter(const rad_hmat *H, const void *src, int64_t lds, void *dst, int64_t ldd, int64_t R, hipStream_t s) {
    int64_t tot = H->N * R;
    unsigned blocks = (unsigned)std::min<int64_t>((tot + 255) / 256, 8192);
    if (H->dtype == RAD_F64)
        hipLaunchKernelGGL(k_scatter<double>, dim3(blocks), dim3(256), 0, s, H->d_perm.p, (const double *)src, lds,
                           (double *)dst, ldd, H->N, R);
    else
        hipLaunchKernelGGL(k_scatter<float>, dim3(blocks), dim3(256), 0, s, H->d_perm.p, (const float *)src, lds,
                           (float *)dst, ldd, H->N, R);
    RAD_HIP(hipGetLastError());
}

void mv_apply(const rad_hmat *H, const void *X, int64_t ldx, void *Y, int64_t ldy, int64_t R, hipStream_t s) {
    if (H->dtype == RAD_F64)
        apply_t<double>(H, (const double *)X, ldx, (double *)Y, ldy, R, (double *)H->w_t.p, s);
    else
        apply_t<float>(H, (const float *)X, ldx, (float *)Y, ldy, R, (float *)H->w_t.p, s);
}

void mv_apply_ws(const rad_hmat *H, const void *X, int64_t ldx, void *Y, int64_t ldy, int64_t R, void *Tb,
                 hipStream_t s) {
    // (one workgroup per tile: no workspace of the matrix is used)
    if (H->dtype == RAD_F64)
        apply_t<double>(H, (const double *)X, ldx, (double *)Y, ldy, R, (double *)Tb, s, nullptr, nullptr, 0.0,
                        nullptr, nullptr, nullptr, false);
    else
        apply_t<float>(H, (const float *)X, ldx, (float *)Y, ldy, R, (float *)Tb, s, nullptr, nullptr, 0.0f,
                       nullptr, nullptr, nullptr, false);
}

// ----------------------------------------------------------------------------
// Static scratch of the allocation-free product.  Every device that loads
// this code object holds its own copy of the array until the process ends.
// In host code the array's name is only a stand-in for the symbol: its
// device address comes from hipGetSymbolAddress, taken once per device with
// that device current, and only that address is ever passed to kernels.
// ----------------------------------------------------------------------------
namespace {
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_addr[kMaxDevices] = {};
}  // namespace

void *static_scratch(int device) {
    RAD_REQUIRE(device >= 0 && device < kMaxDevices, "device ordinal out of range for the static scratch");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_addr[device]) {
        int cur = -1;
        RAD_HIP(hipGetDevice(&cur));
        RAD_REQUIRE(cur == device, "the static scratch is looked up with its device current");
        void *ptr = nullptr;
        RAD_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        RAD_REQUIRE(ptr != nullptr, "hipGetSymbolAddress returned no address for the static scratch");
        g_scratch_addr[device] = ptr;
    }
    return g_scratch_addr[device];
}

void col_norms2(const rad_hmat *H, const void *E, int64_t ld, int64_t R, double *out, hipStream_t s) {
    dim3 grid(kRedParts, (unsigned)R);
    double *part = (double *)H->w_red.p;
    if (H->dtype == RAD_F64)
        hipLaunchKernelGGL(k_colnorm2<double>, grid, dim3(256), 0, s, (const double *)E, H->N, ld, part);
    else
        hipLaunchKernelGGL(k_colnorm2<float>, grid, dim3(256), 0, s, (const float *)E, H->N, ld, part);
    hipLaunchKernelGGL(k_reduce_cols, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, s, part, kRedParts, R, out);
    RAD_HIP(hipGetLastError());
}

size_t reduction_doubles(int64_t R) { return (size_t)kRedParts * (size_t)R; }

void mv_jacobi_step(const rad_hmat *H, const void *E, const void *rho, double rho_scalar, const void *Bold, void *Bnew,
                    int64_t ld, int64_t R, double *norms, hipStream_t s, const int32_t *stop, double *enorms,
                    const ConvTest *test) {
    double *part = (double *)H->w_red.p;
    double *epart = enorms ? H->w_ered.p : nullptr;
    if (H->dtype == RAD_F64)
        apply_t<double>(H, (const double *)Bold, ld, (double *)Bnew, ld, R, (double *)H->w_t.p, s, (const double *)E,
                        (const double *)rho, rho_scalar, part, epart, stop);
    else
        apply_t<float>(H, (const float *)Bold, ld, (float *)Bnew, ld, R, (float *)H->w_t.p, s, (const float *)E,
                       (const float *)rho, (float)rho_scalar, part, epart, stop);
    // per-column sums in a fixed order; the stopping test rides on the last one
    mm_reduce_cols(H, part, H->n_tiles, R, norms, s, stop, enorms ? nullptr : test);
    if (enorms) mm_reduce_cols(H, epart, H->n_tiles, R, enorms, s, stop, test);
}

namespace {
template <class T>
__global__ void k_elementwise(int32_t op, double a, double b, double c, const T *x, const T *y, T *z, int64_t N,
                              int64_t R, int64_t ld, int rmajor) {
    const int64_t tot = N * R;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t i, r;
        if (rmajor) {
            i = e / R;
            r = e - i * R;
        } else {
            r = e / N;
            i = e - r * N;
        }
        const int64_t k = rmajor ? i * ld + r : i + r * ld;
        if (op == EW_SCALE) {
            z[k] = (T)(a * (double)x[k]);
        } else if (op == EW_ADD) {
            z[k] = x[k] + y[k];
        } else {
            double f = a * (double)x[k] + b * (double)y[k];
            z[k] = (T)sqrt(sqrt((f > 0.0 ? f : 0.0) / c));
        }
    }
}
}  // namespace

void launch_elementwise(const rad_hmat *H, int32_t op, double a, double b, double c, const void *x, const void *y,
                        void *z, int64_t R, int64_t ld, bool rmajor, hipStream_t s) {
    int64_t tot = H->N * R;
    unsigned blocks = (unsigned)std::min<int64_t>((tot + 255) / 256, 16384);
    if (H->dtype == RAD_F64)
        hipLaunchKernelGGL(k_elementwise<double>, dim3(blocks), dim3(256), 0, s, op, a, b, c, (const double *)x,
                           (const double *)y, (double *)z, H->N, R, ld, (int)rmajor);
    else
        hipLaunchKernelGGL(k_elementwise<float>, dim3(blocks), dim3(256), 0, s, op, a, b, c, (const float *)x,
                           (const float *)y, (float *)z, H->N, R, ld, (int)rmajor);
    RAD_HIP(hipGetLastError());
}

namespace {
// out[:, c] = flag[c] ? a[:, c] : b[:, c] (R-major: element (t, c) at t ld + c; else c ld + t)
template <class T>
__global__ void k_select_cols(const T *a, const T *b, const int32_t *flag, T *out, int64_t N, int64_t R, int64_t ld,
                              int rmajor) {
    const int64_t tot = N * R;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = rmajor ? e / R : e % N, c = rmajor ? e % R : e / N;
        const int64_t k = rmajor ? i * ld + c : i + c * ld;
        out[k] = flag[c] ? a[k] : b[k];
    }
}
}  // namespace

void select_columns(const rad_hmat *H, const void *a, const void *b, const int32_t *flag, void *out, int64_t ld,
                    int64_t R, bool rmajor, hipStream_t s) {
    const int64_t tot = H->N * R;
    const unsigned blocks = (unsigned)std::min<int64_t>((tot + 255) / 256, 65536);
    if (H->dtype == RAD_F64)
        hipLaunchKernelGGL(k_select_cols<double>, dim3(blocks), dim3(256), 0, s, (const double *)a, (const double *)b,
                           flag, (double *)out, H->N, R, ld, (int)rmajor);
    else
        hipLaunchKernelGGL(k_select_cols<float>, dim3(blocks), dim3(256), 0, s, (const float *)a, (const float *)b,
                           flag, (float *)out, H->N, R, ld, (int)rmajor);
    RAD_HIP(hipGetLastError());
}

}  // namespace rad
