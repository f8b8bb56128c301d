// C-ABI of librad: argument checks, error translation, workspace, solve loop.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "rad_internal.h"

namespace rad {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

static int dsize(int32_t dt) { return dt == RAD_F64 ? 8 : dt == RAD_F32 ? 4 : 2; }

void alloc_workspace(rad_hmat *H) {
    size_t s = (size_t)dsize(H->dtype);
    size_t ldr = (size_t)mm_ldr(H->max_rhs);
    size_t nr = (size_t)H->N * ldr;
    H->w_x.alloc(nr * s);
    H->w_y.alloc(nr * s);
    H->w_b.alloc(nr * s);
    H->w_e.alloc(nr * s);
    H->w_t.alloc((size_t)std::max(H->t_ld, 4) * ldr * s);
    H->w_rho.alloc((size_t)H->N * s);
    H->w_red.alloc(std::max(reduction_doubles(H->max_rhs), mm_reduction_doubles_for(H, H->max_rhs)) * sizeof(double));
    const size_t nc = (size_t)H->max_rhs * (size_t)H->n_inst;  // per-column norms (per instance in a group)
    H->w_norms.alloc(3 * nc);
    H->w_flags.alloc(nc);
    H->w_thr.alloc(nc);
    H->w_conv.alloc(nc + 1);   // per-column flags, then the stop flag
    RAD_HIP(hipMemset(H->w_conv.p, 0, (nc + 1) * sizeof(int32_t)));
    if (H->max_rhs >= kMfmaMinRhs && H->n_tiles > 0) H->w_ered.alloc((size_t)H->n_tiles * (size_t)H->max_rhs);
    if (H->max_rhs >= kMfmaMinRhs && H->n_parts > 0)
        H->w_part.alloc((size_t)H->n_parts * mm_part_rows() * ldr * s);
    H->w_q1.alloc(nr * s);
    H->w_q2.alloc(nr * s);
    if (H->lowp) H->w_b64.alloc(nr);
    if (H->lowp == RAD_BF16 && H->max_rhs >= kMfmaMinRhs) {
        const size_t ld16 = (size_t)((H->max_rhs + 7) & ~7);
        H->w_x16.alloc((size_t)H->N * ld16);
        H->w_t16.alloc((size_t)std::max(H->t_ld, 4) * ld16);
    }
    RAD_HIP(hipHostMalloc((void **)&H->h_norms, sizeof(double) * 3 * nc, hipHostMallocMapped));
    RAD_HIP(hipHostGetDevicePointer((void **)&H->d_hnorms, H->h_norms, 0));
    for (auto &e : H->ev) RAD_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    RAD_HIP(hipStreamCreateWithFlags(&H->cap_stream, hipStreamNonBlocking));
    if (H->n_tiles > 0) mm_prepare_schedule(H);
}

// One Jacobi iteration, enqueued on stream s: B_new = E + rho (F-hat B_old),
// the squared column changes in w_norms[max_rhs...], copied to pinned memory
// (hn, else the first slot).  With stop set (multi-RHS path only) every kernel
// returns at once while the device flag is set, and the iteration ends with
// the device-side stopping test, which itself writes the changes to the
// pinned slot.  first (multi-RHS, B_old = E): the same pass also sums
// ||E||^2 per column (to w_norms and the pinned slot after the two change
// slots), and the test starts from thresholds rtol2 ||E||^2.
struct IterArgs {
    bool mm;
    bool lowp;
    int64_t R, ld;
    const void *E, *rho, *Bold;
    void *Bnew;
    double rho_s;
    double *hn = nullptr;
    const int32_t *stop = nullptr;
    bool first = false;
    double rtol2 = 0.0;
};

static void enqueue_iteration(const rad_hmat *H, const IterArgs &a, hipStream_t s) {
    double *dn = H->w_norms.p + (int64_t)H->max_rhs * H->n_inst;
    if (a.lowp) {
        lowp_step(H, a.E, a.rho, a.rho_s, a.Bold, a.Bnew, a.ld, a.R, dn, s);
    } else if (a.mm) {
        const int64_t nc = a.R * H->n_inst, nc_all = (int64_t)H->max_rhs * H->n_inst;
        double *en = a.first ? H->w_norms.p : nullptr;
        int32_t *conv = H->w_conv.p;
        if (a.first || a.stop) {
            // the stopping test also hands the norms to the host (mapped pinned memory)
            double *hn = a.hn ? a.hn : H->h_norms;
            ConvTest test{a.first ? 2 : 1, (int)nc, dn, H->w_thr.p, a.rtol2, conv, conv + nc_all};
            test.hdn = H->d_hnorms + (hn - H->h_norms);
            if (a.first) test.hen = H->d_hnorms + 2 * nc_all;
            mm_jacobi_step(H, a.E, a.rho, a.rho_s, a.Bold, a.Bnew, a.ld, a.R, dn, s, a.stop, en, &test);
            return;
        }
        mm_jacobi_step(H, a.E, a.rho, a.rho_s, a.Bold, a.Bnew, a.ld, a.R, dn, s, nullptr, en, nullptr);
    } else {
        mv_apply(H, a.Bold, a.ld, H->w_y.p, a.ld, a.R, s);
        solve_update(H, a.E, a.rho, a.rho_s, H->w_y.p, a.Bold, a.Bnew, a.ld, a.R, dn, s);
    }
    RAD_HIP(hipMemcpyAsync(a.hn ? a.hn : H->h_norms, dn, sizeof(double) * a.R * H->n_inst, hipMemcpyDeviceToHost,
                           s));
}

// Cached graph of one iteration (captured on the library's own stream,
// launched on the caller's); the cache is keyed by every captured argument.
static hipGraphExec_t iteration_graph(rad_hmat *H, const IterArgs &a) {
    for (auto &g : H->graphs)
        if (g.path == (int)a.mm + 2 * (int)a.lowp && g.R == a.R && g.Bold == a.Bold && g.Bnew == a.Bnew && g.E == a.E &&
            g.rho == a.rho && g.rho_s == a.rho_s && g.hn == a.hn && g.stop == a.stop && g.first == a.first &&
            g.rtol2 == a.rtol2)
            return g.ex;
    if (H->graphs.size() >= 24) {
        for (auto &g : H->graphs) {
            (void)hipGraphExecDestroy(g.ex);
            (void)hipGraphDestroy(g.g);
        }
        H->graphs.clear();
    }
    rad_hmat::GraphEntry e{};
    e.path = (int)a.mm + 2 * (int)a.lowp;
    e.R = a.R;
    e.Bold = a.Bold;
    e.Bnew = a.Bnew;
    e.E = a.E;
    e.rho = a.rho;
    e.rho_s = a.rho_s;
    e.hn = a.hn;
    e.stop = a.stop;
    e.first = a.first;
    e.rtol2 = a.rtol2;
    RAD_HIP(hipStreamBeginCapture(H->cap_stream, hipStreamCaptureModeThreadLocal));
    try {
        enqueue_iteration(H, a, H->cap_stream);
    } catch (...) {
        hipGraph_t tmp = nullptr;
        (void)hipStreamEndCapture(H->cap_stream, &tmp);
        if (tmp) (void)hipGraphDestroy(tmp);
        throw;
    }
    RAD_HIP(hipStreamEndCapture(H->cap_stream, &e.g));
    RAD_HIP(hipGraphInstantiate(&e.ex, e.g, nullptr, nullptr, 0));
    H->graphs.push_back(e);
    return e.ex;
}


static void check_hmat(const rad_hmat *H) { RAD_REQUIRE(H != nullptr, "null matrix handle"); }

// Waits for e by polling: the solve waits for every iteration's norms, and a
// poll returns as soon as they have landed (no wake-up of a blocked thread).
static void wait_event(hipEvent_t e) {
    for (;;) {
        const hipError_t r = hipEventQuery(e);
        if (r == hipSuccess) return;
        if (r != hipErrorNotReady) RAD_HIP(r);
    }
}

}  // namespace rad

rad_hmat::~rad_hmat() {
    for (auto &g : graphs) {
        (void)hipGraphExecDestroy(g.ex);
        (void)hipGraphDestroy(g.g);
    }
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (auto e : ev)
        if (e) (void)hipEventDestroy(e);
    if (h_norms) (void)hipHostFree(h_norms);
}

using namespace rad;

extern "C" {

void rad_build_opts_default(rad_build_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-3;
    o->leaf_size = 64;
    o->max_depth = 0;
    o->nearfield = RAD_NEAR_AUTO;
    o->visibility = RAD_VIS_BACKFACE;
    o->storage = RAD_F64;
    o->oversample = 8;
    o->power_iters = 1;
    o->max_rhs = 1;
    o->device = 0;
    o->seed = 0x5eed;
    o->verbose = 0;
}

void rad_solve_opts_default(rad_solve_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->rtol = 1e-3;
    o->max_iter = 100;
    o->order = RAD_ORDER_ORIGINAL;
    o->check_every = 1;
    o->use_graph = 1;
    o->refine = 0;
    o->inner_iters = 3;
    o->warm = 0;
}

const char *rad_last_error(void) { return g_last_error.c_str(); }

rad_status rad_hmat_build_tree(const double *verts, int64_t nv, const int32_t *faces, int64_t nf,
                               const rad_build_opts *opts, int32_t tree_dims, rad_hmat **out) {
    if (out) *out = nullptr;
    rad_hmat *H = nullptr;
    rad_status st = guard([&] {
        RAD_REQUIRE(out != nullptr, "null output pointer");
        rad_build_opts o;
        if (opts)
            o = *opts;
        else
            rad_build_opts_default(&o);
        H = new rad_hmat();
        build_hmat(H, verts, nv, faces, nf, o, tree_dims);
        alloc_workspace(H);
    });
    if (st != RAD_OK) {
        delete H;
        return st;
    }
    *out = H;
    return RAD_OK;
}

rad_status rad_hmat_build(const double *verts, int64_t nv, const int32_t *faces, int64_t nf,
                          const rad_build_opts *opts, rad_hmat **out) {
    return rad_hmat_build_tree(verts, nv, faces, nf, opts, 2, out);
}

void rad_hmat_free(rad_hmat *H) {
    if (!H) return;
    (void)hipSetDevice(H->device);
    delete H;
}

int64_t rad_hmat_n(const rad_hmat *H) { return H ? H->N : -1; }
int32_t rad_hmat_dtype(const rad_hmat *H) { return H ? H->dtype : -1; }

rad_status rad_hmat_info(const rad_hmat *H, rad_hmat_stats *s) {
    return guard([&] {
        check_hmat(H);
        RAD_REQUIRE(s != nullptr, "null stats pointer");
        *s = H->stats;
    });
}

rad_status rad_hmat_perm(const rad_hmat *H, int32_t *perm) {
    return guard([&] {
        check_hmat(H);
        RAD_REQUIRE(perm != nullptr, "null perm pointer");
        std::copy(H->perm.begin(), H->perm.end(), perm);
    });
}

static void check_layout(const rad_hmat *H, int32_t order, int64_t R, int64_t ld, const char *name) {
    RAD_REQUIRE(order == RAD_ORDER_ORIGINAL || order == RAD_ORDER_TREE || order == RAD_ORDER_TREE_RMAJOR, "bad order");
    if (order == RAD_ORDER_TREE_RMAJOR)
        RAD_REQUIRE(ld == mm_ldr(R), std::string(name) + ": R-major leading dimension must be R rounded up to 4");
    else
        RAD_REQUIRE(ld >= H->N, std::string(name) + ": leading dimension smaller than N");
}

rad_status rad_hmat_matvec(const rad_hmat *H, int64_t R, int32_t dtype, const void *X, int64_t ldx, void *Y,
                           int64_t ldy, int32_t order, void *hip_stream) {
    return guard([&] {
        check_hmat(H);
        RAD_REQUIRE(X && Y, "null X or Y");
        const bool lowp = H->lowp != 0 && dtype == H->lowp;
        RAD_REQUIRE(dtype == H->dtype || lowp, "dtype does not match the matrix");
        RAD_REQUIRE(R >= 1 && R <= H->max_rhs, "R must be in [1, max_rhs]");
        RAD_REQUIRE(!lowp || R >= kMfmaMinRhs, "the 16-bit operator needs R >= 16");
        RAD_REQUIRE(H->n_inst == 1 || (order == RAD_ORDER_TREE_RMAJOR && R >= kMfmaMinRhs),
                    "a group multiplies in RAD_ORDER_TREE_RMAJOR with R >= 16");
        check_layout(H, order, R, ldx, "X");
        check_layout(H, order, R, ldy, "Y");
        RAD_HIP(hipSetDevice(H->device));
        hipStream_t s = (hipStream_t)hip_stream;
        const int64_t N = H->N;
        if (R >= kMfmaMinRhs) {
            int64_t ldr = mm_ldr(R);
            auto apply = [&](const void *x, void *y) {
                if (lowp)
                    lowp_step(H, nullptr, nullptr, 0.0, x, y, ldr, R, nullptr, s);
                else
                    mm_apply(H, x, y, ldr, R, s);
            };
            if (order == RAD_ORDER_TREE_RMAJOR) {
                apply(X, Y);
            } else {
                bool perm = order == RAD_ORDER_ORIGINAL;
                mm_to_rmajor(H, X, ldx, perm, H->w_x.p, ldr, R, s);
                apply(H->w_x.p, H->w_y.p);
                mm_from_rmajor(H, H->w_y.p, ldr, perm, Y, ldy, R, s);
            }
        } else if (order == RAD_ORDER_TREE) {
            mv_apply(H, X, ldx, Y, ldy, R, s);
        } else if (order == RAD_ORDER_TREE_RMAJOR) {
            mm_from_rmajor(H, X, ldx, false, H->w_x.p, N, R, s);
            mv_apply(H, H->w_x.p, N, H->w_y.p, N, R, s);
            mm_to_rmajor(H, H->w_y.p, N, false, Y, ldy, R, s);
        } else {
            mv_gather(H, X, ldx, H->w_x.p, N, R, s);
            mv_apply(H, H->w_x.p, N, H->w_y.p, N, R, s);
            mv_scatter(H, H->w_y.p, N, Y, ldy, R, s);
        }
    });
}

size_t rad_noalloc_scratch_bytes(void) { return kStaticScratchBytes; }

rad_status rad_hmat_matvec_noalloc(const rad_hmat *H, int64_t R, int32_t dtype, const void *X, int64_t ldx, void *Y,
                                   int64_t ldy, int32_t order, void *hip_stream) {
    return guard([&] {
        check_hmat(H);
        RAD_REQUIRE(X && Y, "null X or Y");
        RAD_REQUIRE(dtype == H->dtype, "dtype does not match the matrix");
        RAD_REQUIRE(R >= 1 && R < kMfmaMinRhs, "R must be in [1, 15] for the allocation-free product");
        RAD_REQUIRE(H->n_inst == 1, "the allocation-free product takes a single matrix, not a group");
        check_layout(H, order, R, ldx, "X");
        check_layout(H, order, R, ldy, "Y");
        // scratch: projections T (t_ld x R), then, unless X and Y are already
        // column-major in tree order, X and Y in that layout (N x R each)
        const size_t es = (size_t)dsize(H->dtype);
        auto round256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
        const size_t t_bytes = round256((size_t)std::max(H->t_ld, 1) * (size_t)R * es);
        const size_t v_bytes = round256((size_t)H->N * (size_t)R * es);
        const size_t need = t_bytes + (order == RAD_ORDER_TREE ? 0 : 2 * v_bytes);
        RAD_REQUIRE(need <= kStaticScratchBytes,
                    "the allocation-free product needs " + std::to_string(need) + " bytes of scratch, more than its " +
                        std::to_string(kStaticScratchBytes) + "-byte static array");
        RAD_HIP(hipSetDevice(H->device));
        unsigned char *base = (unsigned char *)static_scratch(H->device);
        void *Tb = base, *Xt = base + t_bytes, *Yt = base + t_bytes + v_bytes;
        hipStream_t s = (hipStream_t)hip_stream;
        const int64_t N = H->N;
        if (order == RAD_ORDER_TREE) {
            mv_apply_ws(H, X, ldx, Y, ldy, R, Tb, s);
        } else if (order == RAD_ORDER_TREE_RMAJOR) {
            mm_from_rmajor(H, X, ldx, false, Xt, N, R, s);
            mv_apply_ws(H, Xt, N, Yt, N, R, Tb, s);
            mm_to_rmajor(H, Yt, N, false, Y, ldy, R, s);
        } else {
            mv_gather(H, X, ldx, Xt, N, R, s);
            mv_apply_ws(H, Xt, N, Yt, N, R, Tb, s);
            mv_scatter(H, Yt, N, Y, ldy, R, s);
        }
    });
}

rad_status rad_solve(const rad_hmat *H, const void *rho, double rho_scalar, int64_t R, int32_t dtype, const void *E,
                     int64_t lde, void *B, int64_t ldb, const rad_solve_opts *opts, rad_solve_info *info,
                     void *hip_stream) {
    rad_status conv = RAD_OK;
    rad_status st = guard([&] {
        check_hmat(H);
        RAD_REQUIRE(E && B, "null E or B");
        RAD_REQUIRE(dtype == H->dtype, "dtype does not match the matrix");
        RAD_REQUIRE(R >= 1 && R <= H->max_rhs, "R must be in [1, max_rhs]");
        RAD_REQUIRE(std::isfinite(rho_scalar), "rho_scalar must be finite");
        rad_solve_opts o;
        if (opts)
            o = *opts;
        else
            rad_solve_opts_default(&o);
        RAD_REQUIRE(o.rtol > 0 && o.max_iter >= 1 && o.check_every >= 1, "bad solve options");
        RAD_REQUIRE(H->n_inst == 1 || (o.order == RAD_ORDER_TREE_RMAJOR && R >= kMfmaMinRhs && !o.warm),
                    "a group solves in RAD_ORDER_TREE_RMAJOR with R >= 16 and without a warm start");
        const int64_t NC = R * H->n_inst;  // convergence is tracked per (instance, column)
        check_layout(H, o.order, R, lde, "E");
        check_layout(H, o.order, R, ldb, "B");
        RAD_HIP(hipSetDevice(H->device));
        rad_hmat *Hm = const_cast<rad_hmat *>(H);  // graph cache only
        hipStream_t s = (hipStream_t)hip_stream;
        const int64_t N = H->N;
        const size_t es = (size_t)dsize(H->dtype);
        const bool mm = R >= kMfmaMinRhs;
        const bool rmaj = o.order == RAD_ORDER_TREE_RMAJOR;
        const int64_t ld = mm ? mm_ldr(R) : N;
        // E in the working layout, ping-pong buffers P[0], P[1]
        const void *Ein;
        void *P[2];
        if (mm && rmaj) {
            Ein = E;
            P[0] = B;
        } else {
            if (mm)
                mm_to_rmajor(H, E, lde, o.order == RAD_ORDER_ORIGINAL, H->w_e.p, ld, R, s);
            else if (rmaj)
                mm_from_rmajor(H, E, lde, false, H->w_e.p, N, R, s);
            else if (o.order == RAD_ORDER_TREE)
                RAD_HIP(hipMemcpy2DAsync(H->w_e.p, N * es, E, lde * es, N * es, R, hipMemcpyDeviceToDevice, s));
            else
                mv_gather(H, E, lde, H->w_e.p, N, R, s);
            Ein = H->w_e.p;
            P[0] = H->w_x.p;
        }
        P[1] = H->w_b.p;
        const void *rho_t = nullptr;
        if (rho) {
            if (o.order == RAD_ORDER_ORIGINAL)
                mv_gather(H, rho, N, H->w_rho.p, N, 1, s);
            else
                RAD_HIP(hipMemcpyAsync(H->w_rho.p, rho, N * es, hipMemcpyDeviceToDevice, s));
            rho_t = H->w_rho.p;
        }
        double *enorm_d = H->w_norms.p;
        // Multi-RHS Jacobi tested every iteration runs one iteration ahead of
        // the host; the device skips that iteration once every column has met
        // rtol (the same test in the same arithmetic as the host's below).
        // The first iteration (from E, or from the warm guess) also sums ||E||^2.
        const bool ahead = mm && !o.refine && o.check_every == 1;
        const bool fused_en = ahead;
        if (!fused_en) {
            if (mm)
                mm_col_norms2(H, Ein, ld, R, enorm_d, s);
            else
                col_norms2(H, Ein, N, R, enorm_d, s);
        }
        const int64_t nc_all = (int64_t)H->max_rhs * H->n_inst;
        double *h_en = H->h_norms + 2 * nc_all;
        int32_t *conv_d = H->w_conv.p, *stop_d = H->w_conv.p + nc_all;
        const double rtol2 = o.rtol * o.rtol;
        if (ahead && !fused_en) conv_init(enorm_d, rtol2, NC, H->w_thr.p, conv_d, stop_d, s);
        if (!fused_en) RAD_HIP(hipMemcpyAsync(h_en, enorm_d, NC * sizeof(double), hipMemcpyDeviceToHost, s));
        // column c has met rtol when its squared change (or residual) is <= thr[c]
        std::vector<double> enorm(NC), thr(NC), dn(NC);
        bool have_en = false;
        auto take_enorm = [&] {   // after a synchronisation
            if (have_en) return;
            for (int64_t c = 0; c < NC; ++c) {
                const double e2 = h_en[c];
                if (!std::isfinite(e2)) {
                    (void)hipStreamSynchronize(s);
                    RAD_REQUIRE(false, "E contains non-finite values");
                }
                enorm[c] = std::sqrt(e2);
                thr[c] = e2 > 0 ? rtol2 * e2 : rtol2;
            }
            have_en = true;
        };
        if (!fused_en) {
            RAD_HIP(hipStreamSynchronize(s));
            take_enorm();
        }
        std::vector<int32_t> iters(NC, -1);
        std::vector<double> rel(NC, 0.0);
        int k = 0;
        bool done = false;
        if (o.refine) {
            // iterative refinement: FP64 accumulator, FP64 residual with the FP32
            // operator, inner Jacobi with the 16-bit copy
            RAD_REQUIRE(H->lowp != 0, "refine needs a matrix built with lowp");
            RAD_REQUIRE(mm, "refine needs R >= 16");
            RAD_REQUIRE(o.inner_iters >= 1, "inner_iters must be >= 1");
            double *B64 = H->w_b64.p;
            float *B32 = (float *)H->w_x.p, *FB = (float *)H->w_y.p, *r = (float *)H->w_q1.p;
            float *D[2] = {(float *)H->w_q2.p, (float *)H->w_b.p};
            double *dn_d = H->w_norms.p + (int64_t)H->max_rhs * H->n_inst;
            int inner_total = 0;
            int warm_cols = 0;
            if (o.warm) {
                // guess G into the working layout (w_q2), residual with the FP32
                // operator, judged against ||rho F16 E|| (one 16-bit Jacobi step from E)
                // (an R-major B is read in place: it is only written at the end)
                const float *G = rmaj ? (const float *)B : (const float *)H->w_q2.p;
                if (!rmaj) mm_to_rmajor(H, B, ldb, o.order == RAD_ORDER_ORIGINAL, H->w_q2.p, ld, R, s);
                ir_load(H, B64, B32, G, ld, R, s);
                mm_apply(H, B32, FB, ld, R, s);
                ir_residual(H, (const float *)Ein, B64, FB, (const float *)rho_t, rho_scalar, r, ld, R, dn_d, s);
                std::vector<double> nw(R), nc(R, 0.0);
                RAD_HIP(hipMemcpyAsync(nw.data(), dn_d, R * sizeof(double), hipMemcpyDeviceToHost, s));
                RAD_HIP(hipStreamSynchronize(s));
                // a guess that already meets rtol is kept without the comparison
                std::vector<char> met(R);
                bool all_met = true;
                for (int64_t c = 0; c < R; ++c) {
                    RAD_REQUIRE(std::isfinite(nw[c]), "starting guess gives a non-finite residual");
                    met[c] = nw[c] <= thr[c];
                    all_met = all_met && met[c];
                }
                if (!all_met) {
                    lowp_step(H, Ein, rho_t, rho_scalar, Ein, D[1], ld, R, dn_d, s);
                    RAD_HIP(hipMemcpyAsync(nc.data(), dn_d, R * sizeof(double), hipMemcpyDeviceToHost, s));
                    RAD_HIP(hipStreamSynchronize(s));
                }
                std::vector<int32_t> flag(R);
                done = true;
                for (int64_t c = 0; c < R; ++c) {
                    flag[c] = met[c] || nw[c] <= nc[c];
                    warm_cols += flag[c];
                    const double d2 = flag[c] ? nw[c] : h_en[c];
                    rel[c] = enorm[c] > 0 ? std::sqrt(d2) / enorm[c] : std::sqrt(d2);
                    if (d2 <= thr[c]) iters[c] = 0;
                    if (iters[c] < 0) done = false;
                }
                RAD_HIP(hipMemcpyAsync(H->w_flags.p, flag.data(), R * sizeof(int32_t), hipMemcpyHostToDevice, s));
                ir_select(H, B64, B32, r, (const float *)Ein, H->w_flags.p, ld, R, s);
                RAD_HIP(hipStreamSynchronize(s));
            } else {
                RAD_HIP(hipMemsetAsync(B64, 0, (size_t)N * ld * sizeof(double), s));
                RAD_HIP(hipMemsetAsync(B32, 0, (size_t)N * ld * sizeof(float), s));
            }
            while (!done) {
                const float *rp = o.warm ? r : (const float *)Ein;
                if (k > 0) {
                    mm_apply(H, B32, FB, ld, R, s);
                    ir_residual(H, (const float *)Ein, B64, FB, (const float *)rho_t, rho_scalar, r, ld, R, dn_d, s);
                    RAD_HIP(hipMemcpyAsync(dn.data(), dn_d, NC * sizeof(double), hipMemcpyDeviceToHost, s));
                    RAD_HIP(hipStreamSynchronize(s));
                    rp = r;
                    done = true;
                    for (int64_t c = 0; c < NC; ++c) {
                        double d = std::sqrt(dn[c]);
                        rel[c] = enorm[c] > 0 ? d / enorm[c] : d;
                        RAD_REQUIRE(std::isfinite(rel[c]), "solve produced non-finite values");
                        if (iters[c] < 0 && dn[c] <= thr[c]) iters[c] = k;
                        if (iters[c] < 0) done = false;
                    }
                    if (done || k >= o.max_iter) break;
                }
                // inner: d^0 = r, d^{i} = r + rho F16 d^{i-1}
                const void *prev = rp;
                for (int it = 1; it <= o.inner_iters; ++it) {
                    IterArgs a{true, true, R, ld, rp, rho_t, prev, D[(it - 1) % 2], rho_scalar};
                    if (o.use_graph)
                        RAD_HIP(hipGraphLaunch(iteration_graph(Hm, a), s));
                    else
                        enqueue_iteration(H, a, s);
                    prev = D[(it - 1) % 2];
                }
                inner_total += o.inner_iters;
                ir_update(H, B64, (const float *)prev, B32, ld, R, s);
                ++k;
            }
            void *Bk = B32;
            if (rmaj)
                RAD_HIP(hipMemcpyAsync(B, Bk, (size_t)N * ld * es, hipMemcpyDeviceToDevice, s));
            else
                mm_from_rmajor(H, Bk, ld, o.order == RAD_ORDER_ORIGINAL, B, ldb, R, s);
            RAD_HIP(hipStreamSynchronize(s));
            if (info) {
                if (info->iters) std::copy(iters.begin(), iters.end(), info->iters);
                if (info->rel_change) std::copy(rel.begin(), rel.end(), info->rel_change);
                info->total_iters = k;
                info->inner_iters = inner_total;
                info->warm_columns = warm_cols;
            }
            if (!done) {
                conv = RAD_ENOCONV;
                set_error("refinement reached max_iter before rtol");
            }
            return;
        }
        int warm_cols = 0;
        if (o.warm) {
            // guess G into the working layout (w_q2); one iteration from G into
            // P[1] and one from E into w_q1; per column the smaller change wins
            // and its iterate becomes B^1 in P[0]
            // (an R-major B on the multi-RHS path is read in place)
            void *G = (mm && rmaj) ? B : H->w_q2.p, *C1 = H->w_q1.p;
            if (mm && rmaj) {
                // read in place
            } else if (mm)
                mm_to_rmajor(H, B, ldb, o.order == RAD_ORDER_ORIGINAL, G, ld, R, s);
            else if (rmaj)
                mm_from_rmajor(H, B, ldb, false, G, N, R, s);
            else if (o.order == RAD_ORDER_TREE)
                RAD_HIP(hipMemcpy2DAsync(G, N * es, B, ldb * es, N * es, R, hipMemcpyDeviceToDevice, s));
            else
                mv_gather(H, B, ldb, G, N, R, s);
            std::vector<double> nw(R), nc(R, 0.0);
            IterArgs aw{mm, false, R, ld, Ein, rho_t, G, P[1], rho_scalar, nullptr, nullptr, fused_en, rtol2};
            enqueue_iteration(H, aw, s);
            RAD_HIP(hipStreamSynchronize(s));
            take_enorm();
            std::copy(H->h_norms, H->h_norms + R, nw.begin());
            // a guess whose first change already meets rtol is kept without the
            // comparison; otherwise one iteration from E decides
            std::vector<char> met(R);
            bool all_met = true;
            for (int64_t c = 0; c < R; ++c) {
                RAD_REQUIRE(std::isfinite(nw[c]), "starting guess gives a non-finite residual");
                met[c] = nw[c] <= thr[c];
                all_met = all_met && met[c];
            }
            if (!all_met) {
                IterArgs ac{mm, false, R, ld, Ein, rho_t, Ein, C1, rho_scalar};
                enqueue_iteration(H, ac, s);
                RAD_HIP(hipStreamSynchronize(s));
                std::copy(H->h_norms, H->h_norms + R, nc.begin());
            }
            std::vector<int32_t> flag(R);
            k = 1;
            done = true;
            for (int64_t c = 0; c < R; ++c) {
                flag[c] = met[c] || nw[c] <= nc[c];
                warm_cols += flag[c];
                const double d2 = flag[c] ? nw[c] : nc[c];
                rel[c] = enorm[c] > 0 ? std::sqrt(d2) / enorm[c] : std::sqrt(d2);
                RAD_REQUIRE(std::isfinite(rel[c]), "solve produced non-finite values");
                if (d2 <= thr[c]) iters[c] = 1;
                if (iters[c] < 0) done = false;
            }
            RAD_HIP(hipMemcpyAsync(H->w_flags.p, flag.data(), R * sizeof(int32_t), hipMemcpyHostToDevice, s));
            select_columns(H, P[1], C1, H->w_flags.p, P[0], ld, R, mm, s);
        }
        if (ahead) {
            if (o.warm) {   // columns already met by the warm start
                std::vector<int32_t> cv(NC);
                for (int64_t c = 0; c < NC; ++c) cv[c] = iters[c] >= 0;
                RAD_HIP(hipMemcpyAsync(conv_d, cv.data(), NC * sizeof(int32_t), hipMemcpyHostToDevice, s));
            }
            double *slot[2] = {H->h_norms, H->h_norms + nc_all};
            auto enqueue = [&](int kk) {
                // (the first iteration of a cold start is never skipped)
                const bool first = kk == 1 && fused_en;
                IterArgs a{mm, false, R, ld, Ein, rho_t, kk == 1 ? Ein : P[kk % 2], P[(kk - 1) % 2], rho_scalar,
                           slot[kk % 2], first ? nullptr : stop_d, first, rtol2};
                if (o.use_graph)
                    RAD_HIP(hipGraphLaunch(iteration_graph(Hm, a), s));
                else
                    enqueue_iteration(H, a, s);
                RAD_HIP(hipEventRecord(H->ev[kk % 2], s));
            };
            // Iteration k + 1 is normally queued behind the one in flight.  When
            // every open column's ratio q = |dB|^2 / thr, extrapolated
            // geometrically from its last two iterations, is predicted to fall
            // below 1/4 in the iteration in flight, nothing is queued behind it
            // (a wrong guess costs one host round trip, never a result).
            int queued = k;
            bool predicted = false;
            std::vector<double> q_prev(NC, 0.0);
            while (!done && k < o.max_iter) {
                while (queued < std::min(k + 2, o.max_iter) && !(queued == k + 1 && predicted)) enqueue(++queued);
                wait_event(H->ev[(k + 1) % 2]);
                ++k;
                take_enorm();
                const double *d2 = slot[k % 2];
                done = true;
                predicted = k >= 2;
                for (int64_t c = 0; c < NC; ++c) {
                    const double d = std::sqrt(d2[c]);
                    rel[c] = enorm[c] > 0 ? d / enorm[c] : d;
                    if (!std::isfinite(rel[c])) {
                        (void)hipStreamSynchronize(s);
                        RAD_REQUIRE(false, "solve produced non-finite values");
                    }
                    if (iters[c] < 0 && d2[c] <= thr[c]) iters[c] = k;
                    if (iters[c] < 0) {
                        done = false;
                        const double q = d2[c] / thr[c];
                        if (!(q_prev[c] > 0 && q * q <= 0.25 * q_prev[c])) predicted = false;
                    }
                    q_prev[c] = d2[c] / thr[c];
                }
            }
        }
        while (!ahead && k < o.max_iter && !done) {
            ++k;
            IterArgs a{mm, false, R, ld, Ein, rho_t, k == 1 ? Ein : P[k % 2], P[(k - 1) % 2], rho_scalar};
            if (o.use_graph)
                RAD_HIP(hipGraphLaunch(iteration_graph(Hm, a), s));
            else
                enqueue_iteration(H, a, s);
            if (k % o.check_every == 0 || k == o.max_iter) {
                RAD_HIP(hipStreamSynchronize(s));
                std::copy(H->h_norms, H->h_norms + NC, dn.begin());
                done = true;
                for (int64_t c = 0; c < NC; ++c) {
                    double d = std::sqrt(dn[c]);
                    rel[c] = enorm[c] > 0 ? d / enorm[c] : d;
                    RAD_REQUIRE(std::isfinite(rel[c]), "solve produced non-finite values");
                    if (iters[c] < 0 && dn[c] <= thr[c]) iters[c] = k;
                    if (iters[c] < 0) done = false;
                }
            }
        }
        void *Bk = P[(k - 1) % 2];
        if (mm && rmaj) {
            if (Bk != B) RAD_HIP(hipMemcpyAsync(B, Bk, (size_t)N * ld * es, hipMemcpyDeviceToDevice, s));
        } else if (mm) {
            mm_from_rmajor(H, Bk, ld, o.order == RAD_ORDER_ORIGINAL, B, ldb, R, s);
        } else if (rmaj) {
            mm_to_rmajor(H, Bk, N, false, B, ldb, R, s);
        } else if (o.order == RAD_ORDER_TREE) {
            RAD_HIP(hipMemcpy2DAsync(B, ldb * es, Bk, N * es, N * es, R, hipMemcpyDeviceToDevice, s));
        } else {
            mv_scatter(H, Bk, N, B, ldb, R, s);
        }
        RAD_HIP(hipStreamSynchronize(s));
        if (info) {
            if (info->iters) std::copy(iters.begin(), iters.end(), info->iters);
            if (info->rel_change) std::copy(rel.begin(), rel.end(), info->rel_change);
            info->total_iters = k;
            info->inner_iters = 0;
            info->warm_columns = warm_cols;
        }
        if (!done) {
            conv = RAD_ENOCONV;
            set_error("Jacobi reached max_iter before rtol");
        }
    });
    return st != RAD_OK ? st : conv;
}

rad_status rad_equilibrium(const rad_hmat *H, int64_t R, int32_t dtype, const void *Qdir, int64_t ld, double albedo,
                           double emissivity, void *T, void *Qvis, void *Qir, const rad_solve_opts *opts,
                           rad_solve_info *info_sw, rad_solve_info *info_ir, void *hip_stream) {
    rad_status conv = RAD_OK;
    rad_status st = guard([&] {
        check_hmat(H);
        RAD_REQUIRE(Qdir && T, "null Qdir or T");
        if (H->n_inst > 1) throw Error(RAD_EUNSUP, "equilibrium runs per instance, not on a group");
        RAD_REQUIRE(dtype == H->dtype, "dtype does not match the matrix");
        RAD_REQUIRE(R >= 1 && R <= H->max_rhs, "R must be in [1, max_rhs]");
        RAD_REQUIRE(albedo >= 0.0 && albedo < 1.0, "albedo must be in [0, 1)");
        RAD_REQUIRE(emissivity > 0.0 && emissivity <= 1.0, "emissivity must be in (0, 1]");
        rad_solve_opts o;
        if (opts)
            o = *opts;
        else
            rad_solve_opts_default(&o);
        o.refine = 0;  // the bands run plain Jacobi from B^0 = E (their inputs live in the refinement workspace)
        o.warm = 0;
        check_layout(H, o.order, R, ld, "Qdir");
        const bool rmaj = o.order == RAD_ORDER_TREE_RMAJOR;
        RAD_REQUIRE(rmaj || ld == H->N, "column-major layouts need ld == N here");
        RAD_HIP(hipSetDevice(H->device));
        hipStream_t s = (hipStream_t)hip_stream;
        void *q1 = H->w_q1.p, *q2 = H->w_q2.p;
        auto ew = [&](int32_t op, double a, double b, double c, const void *x, const void *y, void *z) {
            launch_elementwise(H, op, a, b, c, x, y, z, R, ld, rmaj, s);
        };
        auto band = [&](double rho, const void *E, rad_solve_info *info) {
            rad_status r = rad_solve(H, nullptr, rho, R, dtype, E, ld, T, ld, &o, info, hip_stream);
            if (r == RAD_ENOCONV)
                conv = RAD_ENOCONV;
            else if (r != RAD_OK)
                throw Error(r, rad_last_error());
        };
        auto product = [&](const void *X, void *Y) {
            rad_status r = rad_hmat_matvec(H, R, dtype, X, ld, Y, ld, o.order, hip_stream);
            if (r != RAD_OK) throw Error(r, rad_last_error());
        };
        // short wave: T holds B_s, q1 ends as Q_vis
        ew(EW_SCALE, albedo, 0, 0, Qdir, nullptr, q1);
        band(albedo, q1, info_sw);
        product(T, q1);
        ew(EW_ADD, 0, 0, 0, Qdir, q1, q1);
        // long wave: T holds B_IR, q2 ends as Q_IR
        ew(EW_SCALE, 1.0 - albedo, 0, 0, q1, nullptr, q2);
        band(1.0, q2, info_ir);
        product(T, q2);
        ew(EW_TEMP, 1.0 - albedo, emissivity, emissivity * 5.670374419e-8, q1, q2, T);
        const size_t bytes = (size_t)H->N * (size_t)(rmaj ? ld : R) * dsize(H->dtype);
        if (Qvis) RAD_HIP(hipMemcpyAsync(Qvis, q1, bytes, hipMemcpyDeviceToDevice, s));
        if (Qir) RAD_HIP(hipMemcpyAsync(Qir, q2, bytes, hipMemcpyDeviceToDevice, s));
        RAD_HIP(hipStreamSynchronize(s));
        if (conv != RAD_OK) set_error("a band's Jacobi solve reached max_iter before rtol");
    });
    return st != RAD_OK ? st : conv;
}

rad_status rad_insolation(const rad_hmat *H, int64_t R, const double *suns, double flux, int32_t dtype, void *Q,
                          int64_t ldq, int32_t order, void *hip_stream) {
    return guard([&] {
        check_hmat(H);
        RAD_REQUIRE(suns && Q, "null suns or Q");
        if (H->n_inst > 1) throw Error(RAD_EUNSUP, "insolation runs per instance, not on a group");
        RAD_REQUIRE(R >= 1, "R must be >= 1");
        RAD_REQUIRE(dtype == H->dtype, "dtype does not match the matrix");
        RAD_REQUIRE(std::isfinite(flux), "flux must be finite");
        check_layout(H, order, R, ldq, "Q");
        for (int64_t r = 0; r < R; ++r) {
            double n2 = suns[3 * r] * suns[3 * r] + suns[3 * r + 1] * suns[3 * r + 1] + suns[3 * r + 2] * suns[3 * r + 2];
            RAD_REQUIRE(std::isfinite(n2) && n2 > 0.0, "sun direction must be finite and non-zero");
        }
        RAD_HIP(hipSetDevice(H->device));
        hipStream_t s = (hipStream_t)hip_stream;
        DevBuf<double> d_s((size_t)3 * R);
        RAD_HIP(hipMemcpy(d_s.p, suns, sizeof(double) * 3 * R, hipMemcpyHostToDevice));
        launch_insolation(H, d_s.p, R, flux, H->dtype, Q, ldq, order, s);
        RAD_HIP(hipStreamSynchronize(s));
    });
}

rad_status rad_hmat_time_phases(const rad_hmat *H, int64_t R, int32_t dtype, int32_t nrep, void *hip_stream,
                                double *ms) {
    return guard([&] {
        check_hmat(H);
        RAD_REQUIRE(ms != nullptr, "null ms pointer");
        const bool lowp = H->lowp != 0 && dtype == H->lowp;
        RAD_REQUIRE(dtype == H->dtype || lowp, "dtype does not match the matrix");
        RAD_REQUIRE(R >= kMfmaMinRhs && R <= H->max_rhs, "R must be in [16, max_rhs]");
        RAD_REQUIRE(nrep >= 1, "nrep must be >= 1");
        RAD_HIP(hipSetDevice(H->device));
        hipStream_t s = (hipStream_t)hip_stream;
        size_t es = (size_t)dsize(H->dtype);
        size_t n = (size_t)H->N * (size_t)mm_ldr(R) * es;
        RAD_HIP(hipMemsetAsync(H->w_x.p, 0, n, s));
        RAD_HIP(hipMemsetAsync(H->w_e.p, 0, n, s));
        if (lowp)
            lowp_time_phases(H, R, nrep, s, ms);
        else
            mm_time_phases(H, R, nrep, s, ms);
    });
}

}  // extern "C"
