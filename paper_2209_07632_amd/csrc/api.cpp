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
    if (H->n_tiles > 0) H->w_ered.alloc((size_t)H->n_tiles * (size_t)H->max_rhs);
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
    RAD_HIP(hipHostMalloc((void **)&H->h_norms, sizeof(double) * (rad_hmat::kNormSlots + 1) * nc,
                          hipHostMallocMapped));
    RAD_HIP(hipHostGetDevicePointer((void **)&H->d_hnorms, H->h_norms, 0));
    for (auto &e : H->ev) RAD_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    RAD_HIP(hipStreamCreateWithFlags(&H->cap_stream, hipStreamNonBlocking));
    if (H->n_tiles > 0) mm_prepare_schedule(H);
    // partial row sums of the segmented single-RHS product (R < 16)
    if (H->n_gsegs > 0)
        H->w_gpart.alloc((size_t)H->n_gsegs * 64 * (size_t)std::min<int64_t>(H->max_rhs, kMfmaMinRhs - 1) * s);
    // partial tiles of the split reductions of the wide 16-bit expansion
    if (H->n_wsegs > 0 && H->max_rhs >= kMfmaMinRhs) H->w_wpart.alloc((size_t)H->n_wsegs * 128 * 256);
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
    } else {
        // multi-RHS (matrix cores) or single-RHS kernels, Jacobi update fused
        // into the tile kernel either way
        auto step = a.mm ? mm_jacobi_step : mv_jacobi_step;
        const int64_t nc = a.R * H->n_inst, nc_all = (int64_t)H->max_rhs * H->n_inst;
        double *en = a.first ? H->w_norms.p : nullptr;
        int32_t *conv = H->w_conv.p;
        if (a.first || a.stop) {
            // the stopping test also hands the norms to the host (mapped pinned memory)
            double *hn = a.hn ? a.hn : H->h_norms;
            ConvTest test{a.first ? 2 : 1, (int)nc, dn, H->w_thr.p, a.rtol2, conv, conv + nc_all};
            test.hdn = H->d_hnorms + (hn - H->h_norms);
            if (a.first) test.hen = H->d_hnorms + rad_hmat::kNormSlots * nc_all;
            step(H, a.E, a.rho, a.rho_s, a.Bold, a.Bnew, a.ld, a.R, dn, s, a.stop, en, &test);
            return;
        }
        step(H, a.E, a.rho, a.rho_s, a.Bold, a.Bnew, a.ld, a.R, dn, s, nullptr, en, nullptr);
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

// Y = F-hat X on the working layout of a solve
static void product_ws(const rad_hmat *H, bool mm, int64_t ld, int64_t R, const void *X, void *Y, hipStream_t s) {
    if (mm)
        mm_apply(H, X, Y, ld, R, s);
    else
        mv_apply(H, X, ld, Y, ld, R, s);
}

// max_i (F-hat 1)_i, the largest row sum: one single-RHS product
static double max_row_sum(const rad_hmat *H, hipStream_t s) {
    const int64_t N = H->N;
    std::vector<double> y(N);
    if (H->dtype == RAD_F64) {
        std::vector<double> ones(N, 1.0);
        RAD_HIP(hipMemcpyAsync(H->w_q2.p, ones.data(), N * 8, hipMemcpyHostToDevice, s));
        mv_apply(H, H->w_q2.p, N, H->w_q1.p, N, 1, s);
        RAD_HIP(hipMemcpyAsync(y.data(), H->w_q1.p, N * 8, hipMemcpyDeviceToHost, s));
        RAD_HIP(hipStreamSynchronize(s));
    } else {
        std::vector<float> ones(N, 1.0f), yf(N);
        RAD_HIP(hipMemcpyAsync(H->w_q2.p, ones.data(), N * 4, hipMemcpyHostToDevice, s));
        mv_apply(H, H->w_q2.p, N, H->w_q1.p, N, 1, s);
        RAD_HIP(hipMemcpyAsync(yf.data(), H->w_q1.p, N * 4, hipMemcpyDeviceToHost, s));
        RAD_HIP(hipStreamSynchronize(s));
        std::copy(yf.begin(), yf.end(), y.begin());
    }
    double m = 0.0;
    for (double v : y) {
        RAD_REQUIRE(std::isfinite(v), "the operator gives non-finite row sums");
        m = std::max(m, v);
    }
    return m;
}

// Chebyshev iteration for (I - rho F-hat) B = E from B^0 = E (three-term
// recurrence of Saad, section 12.1), in the working layout: E in Ein, B in Bw.
// Returns whether every column met rtol; iters, rel and k as rad_solve_info.
bool solve_chebyshev(const rad_hmat *H, const rad_solve_opts &o, bool mm, int64_t ld, int64_t R, double rho,
                     const void *Ein, void *Bw, std::vector<int32_t> &iters, std::vector<double> &rel, int &k,
                     hipStream_t s) {
    const int64_t N = H->N;
    const size_t es = (size_t)dsize(H->dtype);
    double lam_lo = o.lam_lo, lam_hi = o.lam_hi;
    RAD_REQUIRE(std::isfinite(lam_lo) && std::isfinite(lam_hi) && lam_lo <= lam_hi, "bad spectral interval");
    if (lam_lo == 0.0 && lam_hi == 0.0) {
        // F-hat is F up to the compression error, and F >= 0 has its spectrum
        // in [-rho(F), rho(F)] with rho(F) <= the largest row sum
        const double sm = 1.01 * max_row_sum(H, s);
        lam_lo = -sm;
        lam_hi = sm;
    }
    const double a1 = 1.0 - rho * lam_hi, a2 = 1.0 - rho * lam_lo;
    const double lo = std::min(a1, a2), hi = std::max(a1, a2);
    RAD_REQUIRE(lo > 0.0, "the Chebyshev interval of I - rho F-hat must lie in (0, inf): need rho lam < 1");
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
    void *r = H->w_q1.p, *d = H->w_q2.p, *Y = H->w_y.p;
    double *part = (double *)H->w_red.p;
    double *en_d = H->w_norms.p, *dn_d = H->w_norms.p + R;
    // (a block of R columns holds N ld values R-major, ld R column-major)
    const size_t blk = (size_t)(mm ? N * ld : ld * R) * es;
    RAD_HIP(hipMemcpyAsync(Bw, Ein, blk, hipMemcpyDeviceToDevice, s));
    krylov_dots(H, mm, ld, R, Ein, 0, 1, Ein, part, en_d, s);
    product_ws(H, mm, ld, R, Ein, Y, s);
    krylov_cheb_init(H, mm, ld, R, rho, theta, Y, r, d, part, s);
    mm_reduce_cols(H, part, H->n_tiles, R, dn_d, s);
    std::vector<double> e2(R), d2(R), thr(R);
    RAD_HIP(hipMemcpyAsync(e2.data(), en_d, R * sizeof(double), hipMemcpyDeviceToHost, s));
    RAD_HIP(hipMemcpyAsync(d2.data(), dn_d, R * sizeof(double), hipMemcpyDeviceToHost, s));
    RAD_HIP(hipStreamSynchronize(s));
    const double rtol2 = o.rtol * o.rtol;
    bool done = true;
    auto take = [&](int kk) {
        done = true;
        for (int64_t c = 0; c < R; ++c) {
            RAD_REQUIRE(std::isfinite(d2[c]), "solve produced non-finite values");
            rel[c] = e2[c] > 0 ? std::sqrt(d2[c] / e2[c]) : std::sqrt(d2[c]);
            if (iters[c] < 0 && d2[c] <= thr[c]) iters[c] = kk;
            if (iters[c] < 0) done = false;
        }
    };
    for (int64_t c = 0; c < R; ++c) {
        RAD_REQUIRE(std::isfinite(e2[c]), "E contains non-finite values");
        thr[c] = e2[c] > 0 ? rtol2 * e2[c] : rtol2;
    }
    take(0);
    k = 0;
    if (delta == 0.0) {
        // a single point: B = E + r / theta (= E + d) is exact
        std::vector<double> one(R, 1.0);
        RAD_HIP(hipMemcpyAsync(en_d, one.data(), R * sizeof(double), hipMemcpyHostToDevice, s));
        krylov_combine(H, mm, ld, R, d, 0, 1, en_d, 1.0, Bw, s);
        for (auto &it : iters) it = std::max(it, 1);
        k = 1;
        return true;
    }
    const double sigma = theta / delta;
    double rk = 1.0 / sigma;
    while (!done && k < o.max_iter) {
        ++k;
        product_ws(H, mm, ld, R, d, Y, s);
        const double rk1 = 1.0 / (2.0 * sigma - rk);
        krylov_cheb_step(H, mm, ld, R, rho, rk1 * rk, 2.0 * rk1 / delta, Y, Bw, r, d, part, s);
        mm_reduce_cols(H, part, H->n_tiles, R, dn_d, s);
        RAD_HIP(hipMemcpyAsync(d2.data(), dn_d, R * sizeof(double), hipMemcpyDeviceToHost, s));
        RAD_HIP(hipStreamSynchronize(s));
        take(k);
        rk = rk1;
    }
    return done;
}

// Restarted GMRES, all columns advancing together (see rad_solve_method).
bool solve_gmres(const rad_hmat *H, const rad_solve_opts &o, bool mm, int64_t ld, int64_t R, double rho,
                 const void *rhov, const void *Ein, void *x, std::vector<int32_t> &iters, std::vector<double> &rel,
                 int &k, hipStream_t s) {
    const int64_t N = H->N;
    const size_t es = (size_t)dsize(H->dtype);
    const int m = o.restart;
    // elements of one block of R columns (R-major N ld, column-major ld R):
    // the stride between basis vectors
    const int64_t vstride = mm ? N * ld : ld * R;
    const int n_tiles = (int)((N + 63) / 64);
    AllocScope scope(H->hook(), H->device);
    DevBuf<unsigned char> Vb((size_t)(m + 1) * (size_t)vstride * es);
    DevBuf<double> part((size_t)(m + 1) * n_tiles * R), h1((size_t)(m + 1) * R), h2((size_t)(m + 1) * R), nrm(R),
        yd((size_t)m * R);
    unsigned char *V = Vb.p;
    void *w = H->w_q1.p, *r = H->w_q2.p, *Y = H->w_y.p;
    auto Vj = [&](int j) { return (void *)(V + (size_t)j * vstride * es); };
    RAD_HIP(hipMemsetAsync(x, 0, (size_t)vstride * es, s));
    std::vector<double> e2(R), thr(R), beta(R);
    krylov_dots(H, mm, ld, R, Ein, 0, 1, Ein, part.p, nrm.p, s);
    RAD_HIP(hipMemcpyAsync(e2.data(), nrm.p, R * sizeof(double), hipMemcpyDeviceToHost, s));
    RAD_HIP(hipStreamSynchronize(s));
    for (int64_t c = 0; c < R; ++c) {
        RAD_REQUIRE(std::isfinite(e2[c]), "E contains non-finite values");
        thr[c] = o.rtol * (e2[c] > 0 ? std::sqrt(e2[c]) : 1.0);
    }
    std::vector<int32_t> steps(R, 0);
    std::vector<char> done(R, 0);
    // per column: Hessenberg ((m + 1) x m, column-major), rotations, rhs g
    std::vector<double> Hh((size_t)R * (m + 1) * m), cs((size_t)R * m), sn((size_t)R * m), g((size_t)R * (m + 1));
    std::vector<double> h1h((size_t)(m + 1) * R), h2h((size_t)(m + 1) * R), n2h(R), yh((size_t)m * R);
    bool first = true;
    for (;;) {
        // true residual r = E - (I - rho F) x (x = 0 at the start: r = E)
        if (first) {
            RAD_HIP(hipMemcpyAsync(r, Ein, (size_t)vstride * es, hipMemcpyDeviceToDevice, s));
        } else {
            product_ws(H, mm, ld, R, x, Y, s);
            krylov_apply_a(H, mm, ld, R, rho, rhov, Ein, x, Y, r, s);
        }
        krylov_dots(H, mm, ld, R, r, 0, 1, r, part.p, nrm.p, s);
        RAD_HIP(hipMemcpyAsync(n2h.data(), nrm.p, R * sizeof(double), hipMemcpyDeviceToHost, s));
        RAD_HIP(hipStreamSynchronize(s));
        bool any = false;
        for (int64_t c = 0; c < R; ++c) {
            RAD_REQUIRE(std::isfinite(n2h[c]), "solve produced non-finite values");
            beta[c] = std::sqrt(n2h[c]);
            rel[c] = e2[c] > 0 ? beta[c] / std::sqrt(e2[c]) : beta[c];
            if (!done[c] && beta[c] <= thr[c]) {
                done[c] = 1;
                iters[c] = steps[c];
            }
            if (!done[c] && steps[c] < o.max_iter) any = true;
        }
        if (!any) break;
        first = false;
        krylov_scale(H, mm, ld, R, r, nrm.p, Vj(0), s);
        // one cycle
        std::vector<char> in(R, 0);
        std::vector<int> mc(R, 0), jc(R, 0);
        for (int64_t c = 0; c < R; ++c) {
            if (done[c] || steps[c] >= o.max_iter) continue;
            in[c] = 1;
            mc[c] = std::min(m, o.max_iter - steps[c]);
            std::fill(g.begin() + c * (m + 1), g.begin() + (c + 1) * (m + 1), 0.0);
            g[c * (m + 1)] = beta[c];
        }
        for (int j = 0; j < m; ++j) {
            bool open = false;
            for (int64_t c = 0; c < R; ++c) open = open || in[c];
            if (!open) break;
            // w = (I - rho F) V_j, orthogonalised against V_0..V_j twice
            product_ws(H, mm, ld, R, Vj(j), Y, s);
            krylov_apply_a(H, mm, ld, R, rho, rhov, nullptr, Vj(j), Y, w, s);
            krylov_dots(H, mm, ld, R, V, vstride, j + 1, w, part.p, h1.p, s);
            krylov_combine(H, mm, ld, R, V, vstride, j + 1, h1.p, -1.0, w, s);
            krylov_dots(H, mm, ld, R, V, vstride, j + 1, w, part.p, h2.p, s);
            krylov_combine(H, mm, ld, R, V, vstride, j + 1, h2.p, -1.0, w, s);
            krylov_dots(H, mm, ld, R, w, 0, 1, w, part.p, nrm.p, s);
            krylov_scale(H, mm, ld, R, w, nrm.p, Vj(j + 1), s);
            RAD_HIP(hipMemcpyAsync(h1h.data(), h1.p, (size_t)(j + 1) * R * sizeof(double), hipMemcpyDeviceToHost, s));
            RAD_HIP(hipMemcpyAsync(h2h.data(), h2.p, (size_t)(j + 1) * R * sizeof(double), hipMemcpyDeviceToHost, s));
            RAD_HIP(hipMemcpyAsync(n2h.data(), nrm.p, R * sizeof(double), hipMemcpyDeviceToHost, s));
            RAD_HIP(hipStreamSynchronize(s));
            for (int64_t c = 0; c < R; ++c) {
                if (!in[c]) continue;
                double *Hc = Hh.data() + (size_t)c * (m + 1) * m + (size_t)j * (m + 1);  // column j
                double *csc = cs.data() + c * m, *snc = sn.data() + c * m, *gc = g.data() + c * (m + 1);
                for (int i = 0; i <= j; ++i) Hc[i] = h1h[(size_t)i * R + c] + h2h[(size_t)i * R + c];
                Hc[j + 1] = std::sqrt(n2h[c]);
                for (int i = 0; i < j; ++i) {   // earlier rotations on the new column
                    const double t = csc[i] * Hc[i] + snc[i] * Hc[i + 1];
                    Hc[i + 1] = -snc[i] * Hc[i] + csc[i] * Hc[i + 1];
                    Hc[i] = t;
                }
                const double dd = std::hypot(Hc[j], Hc[j + 1]);
                csc[j] = dd > 0 ? Hc[j] / dd : 1.0;
                snc[j] = dd > 0 ? Hc[j + 1] / dd : 0.0;
                Hc[j] = dd;
                Hc[j + 1] = 0.0;
                gc[j + 1] = -snc[j] * gc[j];
                gc[j] = csc[j] * gc[j];
                ++steps[c];
                jc[c] = j + 1;
                RAD_REQUIRE(std::isfinite(gc[j + 1]), "solve produced non-finite values");
                if (std::fabs(gc[j + 1]) <= thr[c] || Hc[j] == 0.0 || j + 1 >= mc[c]) in[c] = 0;
            }
        }
        // x += V y with H y = g (upper triangular, per column)
        int jmax = 0;
        std::fill(yh.begin(), yh.end(), 0.0);
        for (int64_t c = 0; c < R; ++c) {
            const int n = jc[c];
            jmax = std::max(jmax, n);
            const double *Hc = Hh.data() + (size_t)c * (m + 1) * m, *gc = g.data() + c * (m + 1);
            for (int i = n - 1; i >= 0; --i) {
                double t = gc[i];
                for (int l = i + 1; l < n; ++l) t -= Hc[(size_t)l * (m + 1) + i] * yh[(size_t)l * R + c];
                const double piv = Hc[(size_t)i * (m + 1) + i];
                yh[(size_t)i * R + c] = piv != 0.0 ? t / piv : 0.0;
            }
        }
        if (jmax > 0) {
            RAD_HIP(hipMemcpyAsync(yd.p, yh.data(), (size_t)jmax * R * sizeof(double), hipMemcpyHostToDevice, s));
            krylov_combine(H, mm, ld, R, V, vstride, jmax, yd.p, 1.0, x, s);
        }
    }
    k = 0;
    bool all = true;
    for (int64_t c = 0; c < R; ++c) {
        k = std::max(k, steps[c]);
        if (!done[c]) {
            iters[c] = -1;
            all = false;
        }
    }
    return all;
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
    o->allocator = nullptr;
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
    o->method = RAD_SOLVE_JACOBI;
    o->lam_lo = 0.0;
    o->lam_hi = 0.0;
    o->restart = 30;
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
        if (o.allocator) H->allocator = *o.allocator;
        AllocScope scope(H->hook(), o.device);
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

rad_status rad_hmat_build_facets(const double *x, const double *n, const double *area, int64_t N,
                                 const double *tri_verts, const rad_build_opts *opts, int32_t tree_dims,
                                 rad_hmat **out) {
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
        if (o.allocator) H->allocator = *o.allocator;
        AllocScope scope(H->hook(), o.device);
        build_hmat_facets(H, x, n, area, N, tri_verts, o, tree_dims);
        alloc_workspace(H);
    });
    if (st != RAD_OK) {
        delete H;
        return st;
    }
    *out = H;
    return RAD_OK;
}

rad_status rad_hmat_convert(const rad_hmat *H, int32_t dtype, int32_t max_rhs, rad_hmat **out) {
    if (out) *out = nullptr;
    rad_hmat *G = nullptr;
    rad_status st = guard([&] {
        RAD_REQUIRE(out != nullptr, "null output pointer");
        check_hmat(H);
        RAD_REQUIRE(max_rhs >= 0, "max_rhs must be >= 0");
        G = new rad_hmat();
        G->allocator = H->allocator;
        AllocScope scope(G->hook(), H->device);
        convert_hmat(G, H, dtype, max_rhs);
        alloc_workspace(G);
    });
    if (st != RAD_OK) {
        delete G;
        return st;
    }
    *out = G;
    return RAD_OK;
}

rad_status rad_hmat_export(const rad_hmat *H, const char *path) {
    return guard([&] {
        check_hmat(H);
        export_blocks(H, path);
    });
}

rad_status rad_hmat_save(const rad_hmat *H, const char *path) {
    return guard([&] {
        check_hmat(H);
        save_hmat(H, path);
    });
}

rad_status rad_hmat_load(const char *path, int32_t device, int32_t max_rhs, const rad_allocator *allocator,
                         rad_hmat **out) {
    if (out) *out = nullptr;
    rad_hmat *H = nullptr;
    rad_status st = guard([&] {
        RAD_REQUIRE(out != nullptr, "null output pointer");
        RAD_REQUIRE(device >= 0 && max_rhs >= 0, "bad device or max_rhs");
        H = new rad_hmat();
        if (allocator) H->allocator = *allocator;
        AllocScope scope(H->hook(), device);
        load_hmat(H, path, device, max_rhs);
        RAD_REQUIRE(H->n_inst == 1 || H->max_rhs >= kMfmaMinRhs, "a group needs max_rhs >= 16");
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
int32_t rad_hmat_lowp(const rad_hmat *H) { return H ? H->lowp : -1; }
int32_t rad_hmat_max_rhs(const rad_hmat *H) { return H ? H->max_rhs : -1; }

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
        RAD_REQUIRE(o.method == RAD_SOLVE_JACOBI || o.method == RAD_SOLVE_CHEBYSHEV || o.method == RAD_SOLVE_GMRES,
                    "method must be RAD_SOLVE_JACOBI, RAD_SOLVE_CHEBYSHEV or RAD_SOLVE_GMRES");
        RAD_REQUIRE(o.method == RAD_SOLVE_JACOBI || (!o.refine && !o.warm && H->n_inst == 1),
                    "Chebyshev and GMRES solves take no refinement, no warm start and no group");
        RAD_REQUIRE(o.method != RAD_SOLVE_CHEBYSHEV || rho == nullptr, "the Chebyshev solve needs a scalar rho");
        RAD_REQUIRE(o.method != RAD_SOLVE_GMRES || (o.restart >= 1 && o.restart <= 500),
                    "restart must be in [1, 500]");
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
        // B (working layout, in the buffer bk) back to the caller's layout
        auto copy_out = [&](void *Bk) {
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
        };
        if (o.method != RAD_SOLVE_JACOBI) {
            std::vector<int32_t> iters(R, -1);
            std::vector<double> rel(R, 0.0);
            int k = 0;
            const bool ok = o.method == RAD_SOLVE_CHEBYSHEV
                                ? solve_chebyshev(H, o, mm, ld, R, rho_scalar, Ein, P[0], iters, rel, k, s)
                                : solve_gmres(H, o, mm, ld, R, rho_scalar, rho_t, Ein, P[0], iters, rel, k, s);
            copy_out(P[0]);
            if (info) {
                if (info->iters) std::copy(iters.begin(), iters.end(), info->iters);
                if (info->rel_change) std::copy(rel.begin(), rel.end(), info->rel_change);
                info->total_iters = k;
                info->inner_iters = 0;
                info->warm_columns = 0;
            }
            if (!ok) {
                conv = RAD_ENOCONV;
                set_error(o.method == RAD_SOLVE_CHEBYSHEV ? "Chebyshev reached max_iter before rtol"
                                                          : "GMRES reached max_iter before rtol");
            }
            return;
        }
        double *enorm_d = H->w_norms.p;
        // Jacobi tested every iteration runs one iteration ahead of the host;
        // the device skips that iteration once every column has met rtol (the
        // same test in the same arithmetic as the host's below).  The first
        // iteration (from E, or from the warm guess) also sums ||E||^2.
        const bool ahead = !o.refine && o.check_every == 1;
        const bool fused_en = ahead;
        if (!fused_en) {
            if (mm)
                mm_col_norms2(H, Ein, ld, R, enorm_d, s);
            else
                col_norms2(H, Ein, N, R, enorm_d, s);
        }
        const int64_t nc_all = (int64_t)H->max_rhs * H->n_inst;
        double *h_en = H->h_norms + rad_hmat::kNormSlots * nc_all;
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
            constexpr int S = rad_hmat::kNormSlots;
            auto slot = [&](int kk) { return H->h_norms + (int64_t)(kk % S) * nc_all; };
            auto enqueue = [&](int kk) {
                // (the first iteration of a cold start is never skipped)
                const bool first = kk == 1 && fused_en;
                IterArgs a{mm, false, R, ld, Ein, rho_t, kk == 1 ? Ein : P[kk % 2], P[(kk - 1) % 2], rho_scalar,
                           slot(kk), first ? nullptr : stop_d, first, rtol2};
                if (o.use_graph)
                    RAD_HIP(hipGraphLaunch(iteration_graph(Hm, a), s));
                else
                    enqueue_iteration(H, a, s);
                RAD_HIP(hipEventRecord(H->ev[kk % S], s));
            };
            // Up to `depth` iterations are queued behind the one the host waits
            // for: one on the matrix cores (an iteration there outlasts the
            // host's test), S - 1 on the single-RHS kernels (whose iterations
            // are short against a host round trip; those queued past
            // convergence cost only their launches).  When every open column's
            // ratio q = |dB|^2 / thr, extrapolated geometrically from its last
            // two iterations, is predicted to fall below 1/4 in the iteration
            // in flight, nothing is queued behind it (a wrong guess costs one
            // host round trip, never a result).  Iteration kk writes its
            // changes to slot kk mod S, which the host has read before kk is
            // queued (queued <= k + depth + 1 <= k + S).
            const int depth = mm ? 1 : S - 1;
            int queued = k;
            bool predicted = false;
            std::vector<double> q_prev(NC, 0.0);
            while (!done && k < o.max_iter) {
                while (queued < std::min(k + depth + 1, o.max_iter) && !(queued >= k + 1 && predicted))
                    enqueue(++queued);
                wait_event(H->ev[(k + 1) % S]);
                ++k;
                take_enorm();
                const double *d2 = slot(k);
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
        copy_out(P[(k - 1) % 2]);
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
        AllocScope scope(H->hook(), H->device);
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
