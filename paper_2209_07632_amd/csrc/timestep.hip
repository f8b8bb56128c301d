// Time stepping with subsurface heat storage (section 5.2, Algorithm 6):
// C-ABI of include/rad_timestep.h and its kernels.
//
// State layout (tree order, scenario fastest): element (t, r) of a per-facet
// field at i = t R + r; the column nodes in blocks of 64 columns, node j of
// column i at ((i / 64) (M + 1) + j) 64 + i % 64, so that the threads of a
// wave (64 consecutive columns) read and write one contiguous run of
// (M + 1) x 512 bytes (FP64) per step instead of M + 1 runs far apart.  The
// 2R-column operand X and product Y of the terrain multiply hold band 1
// (reflected sunlight) in columns [0, R) and band 2 (infrared) in [R, 2R):
// R-major with ld = 2R rounded to 4 when 2R >= 16 (the matrix-core path),
// else column-major with ld = N.
#include <algorithm>
#include <cmath>
#include <vector>

#include "rad_internal.h"
#include "rad_timestep.h"

namespace {

constexpr int kMaxLayers = 127;
constexpr int kColThreads = 64;          // threads per workgroup of the column kernel
constexpr double kSigmaSB = 5.670374419e-8;  // Stefan-Boltzmann constant, W m^-2 K^-4

// Offset of element (t, r) of a caller block in the given rad_order.
__device__ inline int64_t user_index(int order, int64_t t, int64_t r, int64_t ld, const int32_t *perm) {
    if (order == RAD_ORDER_TREE_RMAJOR) return t * ld + r;
    if (order == RAD_ORDER_TREE) return r * ld + t;
    return r * ld + (int64_t)perm[t];
}

// Position of node j of column i in the column state (blocks of 64 columns).
__device__ inline int64_t node_at(int j, int64_t i, int M) {
    return ((i >> 6) * (M + 1) + j) * 64 + (i & 63);
}

// Position of (t, column c) in X / Y.
// Surface temperature at the new level from the radiation boundary condition
// (section 2), the surface holding no heat: with node 1 eliminated as
// T_1' = d - e_1 T_0', the condition is the quartic
//   f(u) = es u^4 + c u - b = 0,  c = g_1 (1 + e_1) > 0,  b = Q_abs' + g_1 d,
// increasing and convex for u > 0.  A Newton step from any point lands at or
// above the root, and from above Newton descends to it without overshoot.
// The first step is taken from the old surface temperature and capped by the
// smaller of two bounds above the root, (b / es)^(1/4) and b / c (after a
// jump in Q_abs a step from far below would overshoot far above); `newton`
// more steps follow.
__device__ inline double balanced_surface(double t0, double qa_new, double g1, double d, double e1, double es,
                                          int newton) {
    const double c = g1 * (1.0 + e1), b = qa_new + g1 * d, bp = fmax(b, 0.0);
    const double bound = fmin(sqrt(sqrt(bp / es)), bp / c);
    double u = t0;
    for (int it = 0; it <= newton; ++it) {
        const double u3 = u * u * u;
        u = (3.0 * es * u3 * u + b) / (c + 4.0 * es * u3);
        if (it == 0) u = fmin(u, bound);
    }
    return u;
}

__device__ inline int64_t op_index(bool rmajor, int64_t t, int64_t c, int64_t ldx, int64_t N) {
    return rmajor ? t * ldx + c : c * N + t;
}

template <class T>
__global__ void k_ts_init(int M, int64_t N, int64_t R, const double *T0, int64_t ldt, int64_t blk, const T *qd0,
                          int64_t ldq, int order, const int32_t *perm, double h0, double albedo, double *Ts,
                          double *qabs, double *qrad, T *Y, int64_t ldx, int rmajor) {
    const int64_t NR = N * R;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < NR; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = i / R, r = i - t * R;
        const int64_t u = user_index(order, t, r, ldt, perm);
        for (int j = 0; j <= M; ++j) Ts[node_at(j, i, M)] = T0[(int64_t)j * blk + u];
        const double qa = (1.0 - albedo) * (double)qd0[user_index(order, t, r, ldq, perm)] + h0;
        qabs[i] = qa;
        qrad[i] = qa;
        Y[op_index(rmajor, t, r, ldx, N)] = T(0);
        Y[op_index(rmajor, t, R + r, ldx, N)] = T(0);
    }
}

// Operand of the next multiply from the state: band 1 albedo (Q_dir' + Q_refl),
// band 2 Q_rad + (1 - emiss) Q_IR (Q_refl, Q_IR: the last product).
template <class T>
__global__ void k_ts_operand(int64_t N, int64_t R, const double *qrad, const T *Y, T *X, int64_t ldx, int rmajor,
                             const T *qd, int64_t ldq, int order, const int32_t *perm, double albedo, double emiss) {
    const int64_t NR = N * R;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < NR; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = i / R, r = i - t * R;
        const int64_t y1 = op_index(rmajor, t, r, ldx, N), y2 = op_index(rmajor, t, R + r, ldx, N);
        const double qrefl = (double)Y[y1], qir = (double)Y[y2];
        const double q = (double)qd[user_index(order, t, r, ldq, perm)];
        X[y1] = (T)(albedo * (q + qrefl));
        X[y2] = (T)(qrad[i] + (1.0 - emiss) * qir);
    }
}

// One step of every column.  coef holds, per node j, cap_j = rho c V_j / dt,
// g_j = k / (z_j - z_{j-1}), ib_j = 1 / beta_j and e_j = l_j / beta_j of the
// bottom-up elimination (T_j = d_j - e_j T_{j-1}), four runs of M + 1 values.
// The d_j of a thread wait in LDS for the downward substitution.  Rows 1..M
// are the same in both surface readings; only the surface row differs:
//   half layer (newton < 0): half a layer of heat capacity at the surface,
//     Q_abs averaged over the two levels, the emission averaged with its new
//     value linearised about T_0^n;
//   balanced (newton >= 0): no heat capacity at the surface, which meets the
//     radiation boundary condition of section 2 at the new level,
//     Q_abs' + g_1 (T_1' - T_0') = emiss sigma T_0'^4, with the emission
//     linearised about T_0^n and then newton more times about the latest T_0'
//     (Newton's method on the one nonlinear row; T_1' = d_1 - e_1 T_0' from
//     the elimination below, which does not depend on the surface row).
template <class T>
__global__ void __launch_bounds__(kColThreads) k_ts_column(int M, int64_t N, int64_t R, const double *coef,
                                                           const double *Tin, double *Tout, double *qabs,
                                                           double *qrad, const T *Y, T *X, int64_t ldx, int rmajor,
                                                           const T *qd, const T *qd_next, int64_t ldq, int order,
                                                           const int32_t *perm, double albedo, double emiss,
                                                           double hb, int newton) {
    extern __shared__ double d_lds[];   // M x kColThreads
    const double *cap = coef, *g = coef + (M + 1), *ib = coef + 2 * (M + 1), *e = coef + 3 * (M + 1);
    double *dl = d_lds + threadIdx.x;
    const int64_t NR = N * R;
    const double es = emiss * kSigmaSB;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < NR; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = i / R, r = i - t * R;
        const int64_t y1 = op_index(rmajor, t, r, ldx, N), y2 = op_index(rmajor, t, R + r, ldx, N);
        const double qrefl = (double)Y[y1], qir = (double)Y[y2];
        const double qdir = (double)qd[user_index(order, t, r, ldq, perm)];
        const double qa_new = (1.0 - albedo) * (qdir + qrefl) + emiss * qir;
        const double qa_old = qabs[i];
        // bottom-up: r_j (explicit half of the step), d_j = (r_j - u_j d_{j+1}) / beta_j
        double t_below = 0.0, t_here = Tin[node_at(M, i, M)], d = 0.0;
        for (int j = M; j >= 1; --j) {
            const double t_above = Tin[node_at(j - 1, i, M)];
            double rj = cap[j] * t_here + 0.5 * g[j] * (t_above - t_here);
            if (j < M)
                rj += 0.5 * g[j + 1] * (t_below - t_here) + 0.5 * g[j + 1] * d;
            else
                rj += hb;
            d = rj * ib[j];
            dl[(j - 1) * kColThreads] = d;
            t_below = t_here;
            t_here = t_above;
        }
        const double t0 = t_here, t1 = t_below, g1 = g[1];
        double tn;
        if (newton < 0) {
            // half layer: conduction, the averaged absorbed flux and the
            // emission linearised about the old surface temperature
            const double t03 = t0 * t0 * t0;
            const double drad = 2.0 * es * t03;
            const double r0 =
                cap[0] * t0 + 0.5 * g1 * (t1 - t0) + 0.5 * (qa_old + qa_new) - es * t03 * t0 + drad * t0;
            tn = (r0 + 0.5 * g1 * d) / (cap[0] + 0.5 * g1 + drad + 0.5 * g1 * e[1]);
        } else {
            tn = balanced_surface(t0, qa_new, g1, d, e[1], es, newton);
        }
        Tout[node_at(0, i, M)] = tn;
        const double ts = tn;
        for (int j = 1; j <= M; ++j) {
            tn = dl[(j - 1) * kColThreads] - e[j] * tn;
            Tout[node_at(j, i, M)] = tn;
        }
        qabs[i] = qa_new;
        const double qr = es * ts * ts * ts * ts;
        qrad[i] = qr;
        if (qd_next) {
            const double q2 = (double)qd_next[user_index(order, t, r, ldq, perm)];
            X[y1] = (T)(albedo * (q2 + qrefl));
            X[y2] = (T)(qr + (1.0 - emiss) * qir);
        }
    }
}

// The same step with the column in registers, for columns of at most kMax
// layers: the thread issues the loads of all M + 1 levels of its column at
// once (the elimination above waits on them one by one) and keeps the
// pivoted right-hand sides d_j in registers.  Same arithmetic, same order.
constexpr int kRegLayers = 32;
constexpr int kRegThreads = 256;

template <class T, int kMax>
__global__ void __launch_bounds__(kRegThreads) k_ts_column_r(int M, int64_t N, int64_t R, const double *coef,
                                                             const double *Tin, double *Tout, double *qabs,
                                                             double *qrad, const T *Y, T *X, int64_t ldx, int rmajor,
                                                             const T *qd, const T *qd_next, int64_t ldq, int order,
                                                             const int32_t *perm, double albedo, double emiss,
                                                             double hb, int newton) {
    const double *cap = coef, *g = coef + (M + 1), *ib = coef + 2 * (M + 1), *e = coef + 3 * (M + 1);
    const int64_t NR = N * R;
    const double es = emiss * kSigmaSB;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < NR; i += (int64_t)gridDim.x * blockDim.x) {
        // tv[j]: node j; the elimination below stores level j's reduced
        // right-hand side in tv[j + 1], whose node value it no longer needs
        double tv[kMax + 2];
#pragma unroll
        for (int j = 0; j <= kMax; ++j)
            if (j <= M) tv[j] = __builtin_nontemporal_load(Tin + node_at(j, i, M));
        const int64_t t = i / R, r = i - t * R;
        const int64_t y1 = op_index(rmajor, t, r, ldx, N), y2 = op_index(rmajor, t, R + r, ldx, N);
        const double qrefl = (double)Y[y1], qir = (double)Y[y2];
        const double qdir = (double)qd[user_index(order, t, r, ldq, perm)];
        const double qa_new = (1.0 - albedo) * (qdir + qrefl) + emiss * qir;
        const double qa_old = qabs[i];
        double d = 0.0;
#pragma unroll
        for (int j = kMax; j >= 1; --j) {
            if (j <= M) {
                const double t_here = tv[j], t_above = tv[j - 1];
                double rj = cap[j] * t_here + 0.5 * g[j] * (t_above - t_here);
                if (j < M)
                    rj += 0.5 * g[j + 1] * (tv[j + 1] - t_here) + 0.5 * g[j + 1] * d;
                else
                    rj += hb;
                d = rj * ib[j];
                tv[j + 1] = d;
            }
        }
        const double t0 = tv[0], t1 = tv[1], g1 = g[1];
        double tn;
        if (newton < 0) {
            const double t03 = t0 * t0 * t0;
            const double drad = 2.0 * es * t03;
            const double r0 =
                cap[0] * t0 + 0.5 * g1 * (t1 - t0) + 0.5 * (qa_old + qa_new) - es * t03 * t0 + drad * t0;
            tn = (r0 + 0.5 * g1 * d) / (cap[0] + 0.5 * g1 + drad + 0.5 * g1 * e[1]);
        } else {
            tn = balanced_surface(t0, qa_new, g1, d, e[1], es, newton);
        }
        __builtin_nontemporal_store(tn, Tout + node_at(0, i, M));
        const double ts = tn;
#pragma unroll
        for (int j = 1; j <= kMax; ++j) {
            if (j <= M) {
                tn = tv[j + 1] - e[j] * tn;
                __builtin_nontemporal_store(tn, Tout + node_at(j, i, M));
            }
        }
        qabs[i] = qa_new;
        const double qr = es * ts * ts * ts * ts;
        qrad[i] = qr;
        if (qd_next) {
            const double q2 = (double)qd_next[user_index(order, t, r, ldq, perm)];
            X[y1] = (T)(albedo * (q2 + qrefl));
            X[y2] = (T)(qr + (1.0 - emiss) * qir);
        }
    }
}

template <class T>
__global__ void k_ts_read(int field, int M, int64_t N, int64_t R, const double *Ts, const double *qabs,
                          const double *qrad, const T *Y, int64_t ldx, int rmajor, double *out, int64_t ld,
                          int64_t blk, int order, const int32_t *perm) {
    const int64_t NR = N * R;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < NR; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = i / R, r = i - t * R;
        const int64_t u = user_index(order, t, r, ld, perm);
        switch (field) {
            case RAD_TS_T:
                for (int j = 0; j <= M; ++j) out[(int64_t)j * blk + u] = Ts[node_at(j, i, M)];
                break;
            case RAD_TS_QABS: out[u] = qabs[i]; break;
            case RAD_TS_QRAD: out[u] = qrad[i]; break;
            case RAD_TS_QREFL: out[u] = (double)Y[op_index(rmajor, t, r, ldx, N)]; break;
            default: out[u] = (double)Y[op_index(rmajor, t, R + r, ldx, N)]; break;
        }
    }
}

unsigned grid_for(int64_t n, int threads) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + threads - 1) / threads, 1 << 20));
}

// one step of every column: the register form (its smallest instance that
// holds M layers) for up to kRegLayers layers
template <class T>
void launch_column(int M, int64_t N, int64_t R, const double *coef, const double *Tin, double *Tout, double *qabs,
                   double *qrad, const T *Y, T *X, int64_t ldx, int rmajor, const T *qd, const T *qd_next,
                   int64_t ldq, int order, const int32_t *perm, double albedo, double emiss, double hb, int newton,
                   hipStream_t s) {
    const int64_t NR = N * R;
    auto reg = [&](auto kmax) {
        hipLaunchKernelGGL((k_ts_column_r<T, decltype(kmax)::value>), dim3(grid_for(NR, kRegThreads)),
                           dim3(kRegThreads), 0, s, M, N, R, coef, Tin, Tout, qabs, qrad, Y, X, ldx, rmajor, qd,
                           qd_next, ldq, order, perm, albedo, emiss, hb, newton);
    };
    if (M <= 16)
        reg(std::integral_constant<int, 16>{});
    else if (M <= 24)
        reg(std::integral_constant<int, 24>{});
    else if (M <= kRegLayers)
        reg(std::integral_constant<int, kRegLayers>{});
    else
        hipLaunchKernelGGL(k_ts_column<T>, dim3(grid_for(NR, kColThreads)), dim3(kColThreads),
                           sizeof(double) * (size_t)M * kColThreads, s, M, N, R, coef, Tin, Tout, qabs, qrad, Y, X,
                           ldx, rmajor, qd, qd_next, ldq, order, perm, albedo, emiss, hb, newton);
    RAD_HIP(hipGetLastError());
}

}  // namespace

struct rad_ts {
    const rad_hmat *H = nullptr;
    int64_t N = 0, R = 0;
    int32_t M = 0;
    double albedo = 0, emiss = 1, hb = 0;
    int32_t newton = -1;   // -1: half-layer surface; >= 0: balanced surface with this many repeats
    bool rmajor = false;   // X / Y on the matrix-core path (2R >= 16)
    int64_t ldx = 0;
    int64_t level = -1;
    int cur = 0;           // T[cur] holds the current level
    rad::DevBuf<double> coef, T[2], qabs, qrad;
    rad::DevBuf<unsigned char> X, Y;
};

using namespace rad;

namespace {

void check_order(const rad_ts *S, int32_t order, int64_t ld, const char *name) {
    RAD_REQUIRE(order == RAD_ORDER_ORIGINAL || order == RAD_ORDER_TREE || order == RAD_ORDER_TREE_RMAJOR, "bad order");
    if (order == RAD_ORDER_TREE_RMAJOR)
        RAD_REQUIRE(ld == mm_ldr(S->R), std::string(name) + ": R-major leading dimension must be R rounded up to 4");
    else
        RAD_REQUIRE(ld >= S->N, std::string(name) + ": leading dimension smaller than N");
}

int64_t block_extent(const rad_ts *S, int32_t order, int64_t ld) {
    return order == RAD_ORDER_TREE_RMAJOR ? S->N * ld : S->R * ld;
}

// Per-node constants of the column scheme and of its bottom-up elimination.
std::vector<double> column_coefficients(const rad_ts_params &p) {
    const int M = p.n_layers;
    std::vector<double> c(4 * (size_t)(M + 1), 0.0);
    double *cap = c.data(), *g = cap + (M + 1), *ib = cap + 2 * (M + 1), *e = cap + 3 * (M + 1);
    const double *z = p.z;
    for (int j = 1; j <= M; ++j) g[j] = p.conductivity / (z[j] - z[j - 1]);
    for (int j = 0; j <= M; ++j) {
        const double lo = j > 0 ? z[j] - z[j - 1] : 0.0, hi = j < M ? z[j + 1] - z[j] : 0.0;
        cap[j] = p.heat_capacity * 0.5 * (lo + hi) / p.dt;
    }
    // row j: -g_j/2 T_{j-1} + b_j T_j - g_{j+1}/2 T_{j+1}; beta_M = b_M,
    // beta_j = b_j + g_{j+1}/2 e_{j+1}, e_j = -g_j/2 / beta_j
    for (int j = M; j >= 1; --j) {
        double beta = cap[j] + 0.5 * g[j];
        if (j < M) beta += 0.5 * g[j + 1] + 0.5 * g[j + 1] * e[j + 1];
        ib[j] = 1.0 / beta;
        e[j] = -0.5 * g[j] / beta;
    }
    return c;
}

template <class T>
void enqueue_steps(rad_ts *S, int64_t n_steps, const void *Qdir, int64_t ldq, int64_t stride, int32_t order,
                   hipStream_t s) {
    const rad_hmat *H = S->H;
    const int64_t NR = S->N * S->R;
    const T *qd0 = (const T *)Qdir;
    const int32_t *perm = H->d_perm.p;
    const int rm = S->rmajor ? 1 : 0;
    hipLaunchKernelGGL(k_ts_operand<T>, dim3(grid_for(NR, 256)), dim3(256), 0, s, S->N, S->R, S->qrad.p,
                       (const T *)S->Y.p, (T *)S->X.p, S->ldx, rm, qd0, ldq, (int)order, perm, S->albedo, S->emiss);
    RAD_HIP(hipGetLastError());
    for (int64_t k = 0; k < n_steps; ++k) {
        if (S->rmajor)
            mm_apply(H, S->X.p, S->Y.p, S->ldx, 2 * S->R, s);
        else
            mv_apply(H, S->X.p, S->N, S->Y.p, S->N, 2 * S->R, s);
        const T *qd = qd0 + k * stride;
        const T *qn = k + 1 < n_steps ? qd0 + (k + 1) * stride : nullptr;
        launch_column<T>(S->M, S->N, S->R, S->coef.p, S->T[S->cur].p, S->T[S->cur ^ 1].p, S->qabs.p, S->qrad.p,
                         (const T *)S->Y.p, (T *)S->X.p, S->ldx, rm, qd, qn, ldq, (int)order, perm, S->albedo,
                         S->emiss, S->hb, S->newton, s);
        S->cur ^= 1;
        ++S->level;
    }
}

}  // namespace

extern "C" {

rad_status rad_ts_create(const rad_hmat *H, const rad_ts_params *p, int64_t R, rad_ts **out) {
    if (out) *out = nullptr;
    rad_ts *S = nullptr;
    rad_status st = guard([&] {
        RAD_REQUIRE(out != nullptr && H != nullptr && p != nullptr, "null argument");
        if (H->n_inst > 1) throw Error(RAD_EUNSUP, "the time stepper runs per instance, not on a group");
        RAD_REQUIRE(H->dtype == RAD_F64 || H->dtype == RAD_F32, "the matrix must be stored in FP64 or FP32");
        RAD_REQUIRE(R >= 1 && 2 * R <= H->max_rhs, "need 1 <= R and 2 R <= max_rhs of the matrix");
        const int M = p->n_layers;
        RAD_REQUIRE(M >= 1 && M <= kMaxLayers, "n_layers must be in [1, 127]");
        RAD_REQUIRE(p->z != nullptr, "null z");
        RAD_REQUIRE(p->z[0] == 0.0, "z[0] must be 0 (the surface)");
        for (int j = 1; j <= M; ++j)
            RAD_REQUIRE(std::isfinite(p->z[j]) && p->z[j] > p->z[j - 1], "z must be finite and strictly increasing");
        RAD_REQUIRE(std::isfinite(p->conductivity) && p->conductivity > 0, "conductivity must be > 0");
        RAD_REQUIRE(std::isfinite(p->heat_capacity) && p->heat_capacity > 0, "heat_capacity must be > 0");
        RAD_REQUIRE(std::isfinite(p->dt) && p->dt > 0, "dt must be > 0");
        RAD_REQUIRE(p->albedo >= 0.0 && p->albedo < 1.0, "albedo must be in [0, 1)");
        RAD_REQUIRE(p->emissivity > 0.0 && p->emissivity <= 1.0, "emissivity must be in (0, 1]");
        RAD_REQUIRE(std::isfinite(p->bottom_flux), "bottom_flux must be finite");
        RAD_REQUIRE(p->surface == RAD_TS_SURFACE_HALF_LAYER || p->surface == RAD_TS_SURFACE_BALANCED,
                    "surface must be RAD_TS_SURFACE_HALF_LAYER or RAD_TS_SURFACE_BALANCED");
        RAD_REQUIRE(p->surface == RAD_TS_SURFACE_HALF_LAYER || (p->newton >= 0 && p->newton <= 16),
                    "newton must be in [0, 16] for the balanced surface");
        RAD_HIP(hipSetDevice(H->device));
        S = new rad_ts();
        S->H = H;
        S->N = H->N;
        S->R = R;
        S->M = M;
        S->albedo = p->albedo;
        S->emiss = p->emissivity;
        S->hb = p->bottom_flux;
        S->newton = p->surface == RAD_TS_SURFACE_BALANCED ? p->newton : -1;
        S->rmajor = 2 * R >= kMfmaMinRhs;
        S->ldx = S->rmajor ? mm_ldr(2 * R) : S->N;
        const size_t es = H->dtype == RAD_F64 ? 8 : 4;
        const size_t nr = (size_t)S->N * (size_t)R;
        S->coef.upload(column_coefficients(*p));
        const size_t nr64 = (nr + 63) / 64 * 64;   // the column state in whole blocks of 64 columns
        S->T[0].alloc((size_t)(M + 1) * nr64);
        S->T[1].alloc((size_t)(M + 1) * nr64);
        S->qabs.alloc(nr);
        S->qrad.alloc(nr);
        const size_t opbytes = (size_t)S->N * (size_t)(S->rmajor ? S->ldx : 2 * R) * es;
        S->X.alloc(opbytes);
        S->Y.alloc(opbytes);
        // padding columns of the R-major operand are multiplied too: keep them zero
        RAD_HIP(hipMemset(S->X.p, 0, opbytes));
        RAD_HIP(hipMemset(S->Y.p, 0, opbytes));
    });
    if (st != RAD_OK) {
        delete S;
        return st;
    }
    *out = S;
    return RAD_OK;
}

rad_status rad_ts_init(rad_ts *S, const double *T0, int64_t ldt, const void *Qdir0, int64_t ldq, double H0,
                       int32_t order, void *hip_stream) {
    return guard([&] {
        RAD_REQUIRE(S != nullptr, "null stepper");
        RAD_REQUIRE(T0 && Qdir0, "null T0 or Qdir0");
        RAD_REQUIRE(std::isfinite(H0), "H0 must be finite");
        check_order(S, order, ldt, "T0");
        check_order(S, order, ldq, "Qdir0");
        RAD_HIP(hipSetDevice(S->H->device));
        hipStream_t s = (hipStream_t)hip_stream;
        const int64_t NR = S->N * S->R;
        const int rm = S->rmajor ? 1 : 0;
        const int64_t blk = block_extent(S, order, ldt);
        if (S->H->dtype == RAD_F64)
            hipLaunchKernelGGL(k_ts_init<double>, dim3(grid_for(NR, 256)), dim3(256), 0, s, S->M, S->N, S->R, T0, ldt,
                               blk, (const double *)Qdir0, ldq, (int)order, S->H->d_perm.p, H0, S->albedo,
                               S->T[0].p, S->qabs.p, S->qrad.p, (double *)S->Y.p, S->ldx, rm);
        else
            hipLaunchKernelGGL(k_ts_init<float>, dim3(grid_for(NR, 256)), dim3(256), 0, s, S->M, S->N, S->R, T0, ldt,
                               blk, (const float *)Qdir0, ldq, (int)order, S->H->d_perm.p, H0, S->albedo,
                               S->T[0].p, S->qabs.p, S->qrad.p, (float *)S->Y.p, S->ldx, rm);
        RAD_HIP(hipGetLastError());
        S->cur = 0;
        S->level = 0;
    });
}

rad_status rad_ts_step(rad_ts *S, int64_t n_steps, const void *Qdir, int64_t ldq, int64_t level_stride,
                       int32_t order, void *hip_stream) {
    return guard([&] {
        RAD_REQUIRE(S != nullptr, "null stepper");
        RAD_REQUIRE(S->level >= 0, "rad_ts_init has not been called");
        RAD_REQUIRE(Qdir != nullptr, "null Qdir");
        RAD_REQUIRE(n_steps >= 1, "n_steps must be >= 1");
        check_order(S, order, ldq, "Qdir");
        RAD_REQUIRE(n_steps == 1 || level_stride >= block_extent(S, order, ldq),
                    "level_stride smaller than one level's block");
        RAD_HIP(hipSetDevice(S->H->device));
        hipStream_t s = (hipStream_t)hip_stream;
        if (S->H->dtype == RAD_F64)
            enqueue_steps<double>(S, n_steps, Qdir, ldq, level_stride, order, s);
        else
            enqueue_steps<float>(S, n_steps, Qdir, ldq, level_stride, order, s);
    });
}

rad_status rad_ts_read(const rad_ts *S, int32_t field, double *out, int64_t ld, int32_t order, void *hip_stream) {
    return guard([&] {
        RAD_REQUIRE(S != nullptr, "null stepper");
        RAD_REQUIRE(S->level >= 0, "rad_ts_init has not been called");
        RAD_REQUIRE(out != nullptr, "null out");
        RAD_REQUIRE(field >= RAD_TS_T && field <= RAD_TS_QRAD, "bad field");
        check_order(S, order, ld, "out");
        RAD_HIP(hipSetDevice(S->H->device));
        hipStream_t s = (hipStream_t)hip_stream;
        const int64_t NR = S->N * S->R;
        const int rm = S->rmajor ? 1 : 0;
        const int64_t blk = block_extent(S, order, ld);
        if (S->H->dtype == RAD_F64)
            hipLaunchKernelGGL(k_ts_read<double>, dim3(grid_for(NR, 256)), dim3(256), 0, s, (int)field, S->M, S->N,
                               S->R, S->T[S->cur].p, S->qabs.p, S->qrad.p, (const double *)S->Y.p, S->ldx, rm, out,
                               ld, blk, (int)order, S->H->d_perm.p);
        else
            hipLaunchKernelGGL(k_ts_read<float>, dim3(grid_for(NR, 256)), dim3(256), 0, s, (int)field, S->M, S->N,
                               S->R, S->T[S->cur].p, S->qabs.p, S->qrad.p, (const float *)S->Y.p, S->ldx, rm, out,
                               ld, blk, (int)order, S->H->d_perm.p);
        RAD_HIP(hipGetLastError());
    });
}

rad_status rad_ts_time_column(rad_ts *S, int32_t nrep, void *hip_stream, double *ms) {
    return guard([&] {
        RAD_REQUIRE(S != nullptr && ms != nullptr, "null argument");
        RAD_REQUIRE(S->level >= 0, "rad_ts_init has not been called");
        RAD_REQUIRE(nrep >= 1, "nrep must be >= 1");
        RAD_HIP(hipSetDevice(S->H->device));
        hipStream_t s = (hipStream_t)hip_stream;
        const int rm = S->rmajor ? 1 : 0;
        // the operand buffer X stands in for Q_dir: read as an N x R block in
        // X's own layout (R-major with ld ldx, or column-major with ld N)
        const int qorder = rm ? (int)RAD_ORDER_TREE_RMAJOR : (int)RAD_ORDER_TREE;
        const int64_t ldq = rm ? S->ldx : S->N;
        hipEvent_t e0, e1;
        RAD_HIP(hipEventCreate(&e0));
        RAD_HIP(hipEventCreate(&e1));
        auto launch = [&] {
            // the current level's product stands in for the next level's and
            // the operand for Q_dir (the state is advanced from level n into
            // the spare column buffer every time: the same work per launch)
            if (S->H->dtype == RAD_F64)
                launch_column<double>(S->M, S->N, S->R, S->coef.p, S->T[S->cur].p, S->T[S->cur ^ 1].p, S->qabs.p,
                                      S->qrad.p, (const double *)S->Y.p, (double *)S->X.p, S->ldx, rm,
                                      (const double *)S->X.p, (const double *)nullptr, ldq, qorder, S->H->d_perm.p,
                                      S->albedo, S->emiss, S->hb, S->newton, s);
            else
                launch_column<float>(S->M, S->N, S->R, S->coef.p, S->T[S->cur].p, S->T[S->cur ^ 1].p, S->qabs.p,
                                     S->qrad.p, (const float *)S->Y.p, (float *)S->X.p, S->ldx, rm,
                                     (const float *)S->X.p, (const float *)nullptr, ldq, qorder, S->H->d_perm.p,
                                     S->albedo, S->emiss, S->hb, S->newton, s);
        };
        launch();
        RAD_HIP(hipEventRecord(e0, s));
        for (int i = 0; i < nrep; ++i) launch();
        RAD_HIP(hipEventRecord(e1, s));
        RAD_HIP(hipGetLastError());
        RAD_HIP(hipEventSynchronize(e1));
        float t = 0.0f;
        RAD_HIP(hipEventElapsedTime(&t, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *ms = (double)t / nrep;
    });
}

int64_t rad_ts_level(const rad_ts *S) { return S ? S->level : -1; }

void rad_ts_free(rad_ts *S) {
    if (!S) return;
    (void)hipSetDevice(S->H->device);
    delete S;
}

}  // extern "C"
