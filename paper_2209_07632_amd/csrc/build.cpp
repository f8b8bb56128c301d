// Builder of the compressed view-factor matrix (host orchestration).
//
// Steps (Potter et al., arXiv 2209.07632):
//   geometry of every facet ............................. section 3
//   quadtree on centroids ............................... Algorithm 2
//   block pairs from the first level below the root ..... Algorithm 4 (closing remark)
//   non-zero counts of leaf blocks (Algorithm 1 entries) . GPU kernel
//   numerical rank with a doubling sketch width ......... Algorithm 3
//   bottom-up choice of the fewest-bytes form ........... Algorithm 4
//   device layout for the product ....................... Algorithm 5
//
// The rank search replaces ARPACK's truncated SVD by a randomized range
// finder on the GPU (FP64 products computed from the geometry without
// storing F, FP64 Gram-Schmidt) followed by a small FP64 Jacobi SVD on the
// host; the doubling of k and the acceptance test are the paper's.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <numeric>

#include "rad_internal.h"

namespace rad {

namespace {

int dtype_size(int32_t dt) {
    switch (dt) {
    case RAD_F64: return 8;
    case RAD_F32: return 4;
    case RAD_F16: case RAD_BF16: return 2;
    default: return 0;
    }
}

inline int32_t round4(int32_t v) { return (v + 3) & ~3; }

// ---------------------------------------------------------------------------
// Section 3: centroid, unit normal, area
// ---------------------------------------------------------------------------
void facet_geometry(const double *V, int64_t nv, const int32_t *Fc, int64_t nf, std::vector<double> &x,
                    std::vector<double> &n, std::vector<double> &A) {
    x.resize(3 * nf);
    n.resize(3 * nf);
    A.resize(nf);
    for (int64_t i = 0; i < 3 * nv; ++i)
        RAD_REQUIRE(std::isfinite(V[i]), "non-finite vertex coordinate");
    for (int64_t f = 0; f < nf; ++f) {
        int32_t ia = Fc[3 * f], ib = Fc[3 * f + 1], ic = Fc[3 * f + 2];
        RAD_REQUIRE(ia >= 0 && ia < nv && ib >= 0 && ib < nv && ic >= 0 && ic < nv,
                    "face " + std::to_string(f) + " has a vertex index outside [0, nv)");
        const double *a = V + 3 * ia, *b = V + 3 * ib, *c = V + 3 * ic;
        double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                        e1[0] * e2[1] - e1[1] * e2[0]};
        double len = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        RAD_REQUIRE(len > 0.0, "face " + std::to_string(f) + " has zero area");
        for (int k = 0; k < 3; ++k) {
            x[3 * f + k] = (a[k] + b[k] + c[k]) / 3.0;
            n[3 * f + k] = cr[k] / len;
        }
        A[f] = 0.5 * len;
    }
}

// ---------------------------------------------------------------------------
// Algorithm 2: quadtree.  Split at the midpoint of the node's own bounding
// box; children in the printed order (x<,y<), (x<,y>=), (x>=,y<), (x>=,y>=);
// stop at leaf_size points, at max_depth, or when all centroids coincide.
// Leaves in depth-first order define the tree permutation.
// With dims = 3 the same split runs on (x, y, z): the octree of section 4.1
// for closed bodies, each of the four children above split again at the z
// midpoint (z< first), so x is the most significant side, then y, then z.
// ---------------------------------------------------------------------------
struct QuadBuilder {
    const double *x;
    int leaf_size, max_depth;
    int dims = 2;
    std::vector<TreeNode> nodes;
    std::vector<int32_t> perm;
    int32_t nleaves = 0;

    void split(int32_t node, std::vector<int32_t> idx, int32_t depth) {
        nodes[node].start = (int32_t)perm.size();
        nodes[node].size = (int32_t)idx.size();
        nodes[node].depth = depth;
        bool leaf = (int)idx.size() <= leaf_size || (max_depth > 0 && depth >= max_depth);
        double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
        double zmin = INFINITY, zmax = -INFINITY;
        if (!leaf) {
            for (int32_t i : idx) {
                xmin = std::min(xmin, x[3 * i]);
                xmax = std::max(xmax, x[3 * i]);
                ymin = std::min(ymin, x[3 * i + 1]);
                ymax = std::max(ymax, x[3 * i + 1]);
                if (dims == 3) {
                    zmin = std::min(zmin, x[3 * i + 2]);
                    zmax = std::max(zmax, x[3 * i + 2]);
                }
            }
            if (xmin == xmax && ymin == ymax && (dims == 2 || zmin == zmax)) leaf = true;
        }
        if (leaf) {
            nodes[node].first_child = -1;
            nodes[node].nchild = 0;
            nodes[node].leaf_index = nleaves;
            nodes[node].leaf_first = nleaves;
            nodes[node].leaf_count = 1;
            ++nleaves;
            perm.insert(perm.end(), idx.begin(), idx.end());
            return;
        }
        double xmid = 0.5 * (xmin + xmax), ymid = 0.5 * (ymin + ymax), zmid = 0.5 * (zmin + zmax);
        std::vector<int32_t> part[8];   // quadtree: parts 0..3 only
        for (int32_t i : idx) {
            bool lx = x[3 * i] < xmid, ly = x[3 * i + 1] < ymid;
            int q = lx ? (ly ? 0 : 1) : (ly ? 2 : 3);
            if (dims == 3) q = 2 * q + (x[3 * i + 2] < zmid ? 0 : 1);
            part[q].push_back(i);
        }
        idx.clear();
        idx.shrink_to_fit();
        int nch = 0;
        for (auto &p : part) nch += !p.empty();
        int32_t first = (int32_t)nodes.size();
        nodes.resize(nodes.size() + nch);
        nodes[node].first_child = first;
        nodes[node].nchild = nch;
        nodes[node].leaf_index = -1;
        int k = 0;
        for (auto &p : part)
            if (!p.empty()) split(first + k++, std::move(p), depth + 1);
        nodes[node].leaf_first = nodes[first].leaf_first;
        int32_t cnt = 0;
        for (int c = 0; c < nch; ++c) cnt += nodes[first + c].leaf_count;
        nodes[node].leaf_count = cnt;
    }
};

}  // namespace

// One-sided Jacobi SVD (Hestenes) of the l x l matrix A (column-major), in
// place: on return the columns of A are U*Sigma (sorted by decreasing norm)
// and V holds the right singular vectors.  sv gets the column norms.
void jacobi_svd(int l, std::vector<double> &A, std::vector<double> &V, std::vector<double> &sv) {
    V.assign((size_t)l * l, 0.0);
    for (int i = 0; i < l; ++i) V[(size_t)i * l + i] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < l - 1; ++p) {
            for (int q = p + 1; q < l; ++q) {
                double *ap = &A[(size_t)p * l], *aq = &A[(size_t)q * l];
                double alpha = 0, beta = 0, gamma = 0;
                for (int r = 0; r < l; ++r) {
                    alpha += ap[r] * ap[r];
                    beta += aq[r] * aq[r];
                    gamma += ap[r] * aq[r];
                }
                if (gamma == 0.0) continue;
                double conv = std::fabs(gamma) / std::sqrt(alpha * beta);
                if (!(conv > 1e-15)) continue;
                off = std::max(off, conv);
                double zeta = (beta - alpha) / (2.0 * gamma);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
                for (int r = 0; r < l; ++r) {
                    double u = ap[r], w = aq[r];
                    ap[r] = c * u - s * w;
                    aq[r] = s * u + c * w;
                }
                double *vp = &V[(size_t)p * l], *vq = &V[(size_t)q * l];
                for (int r = 0; r < l; ++r) {
                    double u = vp[r], w = vq[r];
                    vp[r] = c * u - s * w;
                    vq[r] = s * u + c * w;
                }
            }
        }
        if (off <= 1e-15) break;
    }
    sv.resize(l);
    for (int i = 0; i < l; ++i) {
        double s2 = 0;
        for (int r = 0; r < l; ++r) s2 += A[(size_t)i * l + r] * A[(size_t)i * l + r];
        sv[i] = std::sqrt(s2);
    }
    std::vector<int> ord(l);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return sv[a] > sv[b]; });
    std::vector<double> A2(A.size()), V2(V.size()), s2(l);
    for (int i = 0; i < l; ++i) {
        std::copy_n(&A[(size_t)ord[i] * l], l, &A2[(size_t)i * l]);
        std::copy_n(&V[(size_t)ord[i] * l], l, &V2[(size_t)i * l]);
        s2[i] = sv[ord[i]];
    }
    A.swap(A2);
    V.swap(V2);
    sv.swap(s2);
}

namespace {

// verbose progress: one flushed line per stage with the elapsed time
struct StageLog {
    bool on = false;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    void operator()(const char *what, const std::string &extra = std::string()) const {
        if (!on) return;
        double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        std::fprintf(stderr, "[rad build %7.2fs] %s %s\n", dt, what, extra.c_str());
        std::fflush(stderr);
    }
};

// Row count from which CGS2 runs on many workgroups per block (the
// environment variable RAD_CGS2_TALL_ROWS overrides it, for tests).
int32_t cgs2_tall_rows() {
    const char *e = std::getenv("RAD_CGS2_TALL_ROWS");
    return e ? std::max(1, std::atoi(e)) : 4096;
}

struct Builder {
    StageLog log;
    rad_hmat *H;
    rad_build_opts o;
    int s;  // bytes per stored value
    std::vector<double> xt, nt, at;  // tree-ordered geometry
    DevBuf<uint32_t> d_vis;
    DevGeom geom{};
    std::vector<BlockPair> bp;
    std::vector<DevBuf<double>> pools;  // candidate factors per level
    std::vector<int64_t> pool_fill;
    hipStream_t st = nullptr;

    const TreeNode &node(int32_t i) const { return H->nodes[i]; }

    int64_t dense_bytes(int64_t m, int64_t n) const { return m * n * s; }
    int64_t csr_bytes(int64_t m, int64_t nnz) const { return 4 * (m + 1) + nnz * (4 + s); }
    int64_t svd_bytes(int64_t m, int64_t n, int64_t q) const { return (m + n) * q * s + q * s; }

    bool is_leaf_pair(int32_t I, int32_t J) const {
        const TreeNode &a = node(I), &b = node(J);
        return (a.nchild == 0 && b.nchild == 0) ||
               (int64_t)a.size * b.size <= (int64_t)o.leaf_size * o.leaf_size;
    }

    void enumerate_pairs() {
        const TreeNode &root = node(0);
        if (root.nchild == 0) {
            bp.push_back(BlockPair{0, 0, 0, -1, 0, 0, 0, 0, 0, -1, -1, -1});
            return;
        }
        for (int a = 0; a < root.nchild; ++a)
            for (int b = 0; b < root.nchild; ++b)
                bp.push_back(BlockPair{root.first_child + a, root.first_child + b, 0, -1, 0, 0, 0, 0, 0,
                                       -1, -1, -1});
        for (size_t p = 0; p < bp.size(); ++p) {
            int32_t I = bp[p].I, J = bp[p].J;
            if (is_leaf_pair(I, J)) continue;
            const TreeNode &a = node(I), &b = node(J);
            int na = a.nchild ? a.nchild : 1, nb = b.nchild ? b.nchild : 1;
            int32_t first = (int32_t)bp.size();
            int32_t lvl = bp[p].level + 1;
            for (int u = 0; u < na; ++u)
                for (int v = 0; v < nb; ++v) {
                    int32_t ci = a.nchild ? a.first_child + u : I;
                    int32_t cj = b.nchild ? b.first_child + v : J;
                    bp.push_back(BlockPair{ci, cj, lvl, -1, 0, 0, 0, 0, 0, -1, -1, -1});
                }
            bp[p].first_child = first;
            bp[p].nchild = na * nb;
        }
    }

    void count_nnz() {
        std::vector<int32_t> pairs;
        std::vector<int64_t> ids;
        for (size_t p = 0; p < bp.size(); ++p) {
            if (bp[p].first_child >= 0) continue;
            const TreeNode &a = node(bp[p].I), &b = node(bp[p].J);
            pairs.insert(pairs.end(), {a.start, a.size, b.start, b.size});
            ids.push_back((int64_t)p);
        }
        DevBuf<int32_t> d_pairs;
        d_pairs.upload(pairs);
        DevBuf<int64_t> d_nnz(ids.size());
        launch_leaf_nnz(geom, d_pairs.p, (int64_t)ids.size(), d_nnz.p, st);
        RAD_HIP(hipStreamSynchronize(st));
        std::vector<int64_t> nnz = d_nnz.download(ids.size());
        for (size_t k = 0; k < ids.size(); ++k) bp[ids[k]].nnz = nnz[k];
        for (size_t p = bp.size(); p-- > 0;) {
            if (bp[p].first_child < 0) continue;
            int64_t t = 0;
            for (int c = 0; c < bp[p].nchild; ++c) t += bp[bp[p].first_child + c].nnz;
            bp[p].nnz = t;
        }
    }

    // Algorithm 3 for every internal block of one level, batched on the GPU.
    void rank_search(int32_t level, const std::vector<int64_t> &ids) {
        struct State {
            int64_t p;
            int32_t k;
            int32_t qlim;
        };
        std::vector<State> active;
        for (int64_t p : ids) {
            const TreeNode &a = node(bp[p].I), &b = node(bp[p].J);
            int64_t m = a.size, n = b.size;
            int64_t cb = csr_bytes(m, bp[p].nnz);
            int64_t per = (m + n + 1) * (int64_t)s;
            // Algorithm 3 accepts q only if its bytes are below the CSR bytes.
            int64_t qlim = (cb + per - 1) / per - 1;
            // Algorithm 4 then keeps the SVD only if it also beats the other
            // forms: below dense/CSR (when allowed) and not above the children,
            // which are already decided.  Ranks beyond that cannot change the
            // result, so the doubling stops there.
            int64_t hb = 0;
            for (int k = 0; k < bp[p].nchild; ++k) hb += bp[bp[p].first_child + k].best_bytes;
            qlim = std::min<int64_t>(qlim, hb / per);
            if (o.nearfield != RAD_NEAR_CSR) qlim = std::min<int64_t>(qlim, (dense_bytes(m, n) - 1) / per);
            if (o.max_rank > 0) qlim = std::min<int64_t>(qlim, o.max_rank);
            qlim = std::min<int64_t>(qlim, std::min(m, n));
            if (qlim < 1) continue;
            active.push_back(State{p, 8, (int32_t)qlim});
        }
        if (pools.size() <= (size_t)level) {
            pools.resize(level + 1);
            pool_fill.resize(level + 1, 0);
        }
        // accepted candidates of this level: (p, q, U-small, V-small, Q/Q2 location)
        std::vector<std::pair<int64_t, int32_t>> accepted_meta;
        int round = 0;
        while (!active.empty()) {
            ++round;
            // chunk by workspace budget
            const int64_t budget = (int64_t)1 << 28;  // doubles per workspace (2 GiB)
            size_t pos = 0;
            std::vector<State> next;
            while (pos < active.size()) {
                std::vector<SketchBlock> sb;
                std::vector<State> chunk;
                int64_t yfill = 0, zfill = 0;
                int32_t max_rows = 0, max_ell = 0;
                while (pos < active.size()) {
                    const State &stt = active[pos];
                    const TreeNode &a = node(bp[stt.p].I), &b = node(bp[stt.p].J);
                    int32_t mn = std::min(a.size, b.size);
                    int32_t ell = std::min(stt.k + o.oversample, mn);
                    int64_t ny = (int64_t)a.size * ell, nz = (int64_t)b.size * ell;
                    if (!sb.empty() && (yfill + ny > budget || zfill + nz > budget || sb.size() >= 32768)) break;
                    SketchBlock k{};
                    k.i0 = a.start;
                    k.m = a.size;
                    k.j0 = b.start;
                    k.n = b.size;
                    k.ell = ell;
                    k.y_off = yfill;
                    k.z_off = zfill;
                    k.seed = o.seed * 0x9E3779B97F4A7C15ull + (uint64_t)stt.p * 0x632BE59BD9B4E019ull +
                             (uint64_t)round;
                    yfill += ny;
                    zfill += nz;
                    max_rows = std::max({max_rows, a.size, b.size});
                    max_ell = std::max(max_ell, ell);
                    sb.push_back(k);
                    chunk.push_back(stt);
                    ++pos;
                }
                process_chunk(level, sb, chunk.size(), yfill, zfill, max_rows, max_ell,
                              [&](size_t c, bool resolved) {
                                  if (!resolved) {
                                      // doubling, capped at the first width that
                                      // decides every rank up to the limit
                                      State nx = chunk[c];
                                      nx.k = std::min(2 * nx.k, nx.qlim + 1);
                                      next.push_back(nx);
                                  }
                              },
                              chunk);
            }
            log("  rank round", "L=" + std::to_string(level) + " round=" + std::to_string(round) +
                                    " blocks=" + std::to_string(active.size()) + " unresolved=" +
                                    std::to_string(next.size()));
            active.swap(next);
        }
    }

    template <class Cb, class StateVec>
    void process_chunk(int32_t level, std::vector<SketchBlock> &sb, size_t nb, int64_t yfill, int64_t zfill,
                       int32_t max_rows, int32_t max_ell, Cb on_done, const StateVec &chunk) {
        DevBuf<SketchBlock> d_sb;
        d_sb.upload(sb);
        DevBuf<double> Y(yfill), Z(zfill);
        int64_t rfill = 0;
        std::vector<int64_t> roff(nb);
        for (size_t c = 0; c < nb; ++c) {
            roff[c] = rfill;
            rfill += (int64_t)sb[c].ell * sb[c].ell;
        }
        DevBuf<double> Rbuf(rfill);
        DevBuf<int64_t> d_roff;
        d_roff.upload(roff);
        // tall blocks are orthonormalised by many workgroups per block
        const bool tall = max_rows >= cgs2_tall_rows();
        DevBuf<double> part, normpart;
        if (tall) {
            int64_t nch = (max_rows + 2047) / 2048;
            part.alloc((size_t)nb * nch * (max_ell + 1));
            normpart.alloc((size_t)nb * nch);
        }
        auto orth = [&](double *base, int use_z, double *R) {
            if (tall)
                launch_cgs2_tall(base, d_sb.p, (int32_t)nb, use_z, R, d_roff.p, max_rows, max_ell, part.p, normpart.p,
                                 nullptr, st);
            else
                launch_cgs2(base, d_sb.p, (int32_t)nb, use_z, R, d_roff.p, st);
        };
        // Y = F Omega (Omega: random signs written into Z), then subspace iterations.
        launch_fill_rademacher(Z.p, d_sb.p, (int32_t)nb, st);
        launch_sketch_apply(geom, d_sb.p, (int32_t)nb, 0, Z.p, Y.p, max_rows, max_ell, st);
        orth(Y.p, 0, nullptr);
        for (int it = 0; it < o.power_iters; ++it) {
            launch_sketch_apply(geom, d_sb.p, (int32_t)nb, 1, Y.p, Z.p, max_rows, max_ell, st);
            orth(Z.p, 1, nullptr);
            launch_sketch_apply(geom, d_sb.p, (int32_t)nb, 0, Z.p, Y.p, max_rows, max_ell, st);
            orth(Y.p, 0, nullptr);
        }
        // Z = F^T Q = Q2 R
        launch_sketch_apply(geom, d_sb.p, (int32_t)nb, 1, Y.p, Z.p, max_rows, max_ell, st);
        orth(Z.p, 1, Rbuf.p);
        RAD_HIP(hipStreamSynchronize(st));
        std::vector<double> Rh = Rbuf.download(rfill);

        // host: SVD of R^T per block, rank rule, acceptance
        std::vector<int32_t> qsel(nb, 0);
        std::vector<int8_t> resolved(nb, 0);
        std::vector<std::vector<double>> smallU(nb), smallV(nb);
#pragma omp parallel for schedule(dynamic, 1)
        for (long c = 0; c < (long)nb; ++c) {
            int l = sb[c].ell;
            std::vector<double> A((size_t)l * l), V, sv;
            // A = R^T (R stored column-major, upper triangular)
            for (int i = 0; i < l; ++i)
                for (int j = 0; j < l; ++j) A[(size_t)j * l + i] = Rh[roff[c] + (size_t)i * l + j];
            jacobi_svd(l, A, V, sv);
            const BlockPair &pp = bp[chunk[c].p];
            int32_t mn = std::min(sb[c].m, sb[c].n);
            bool exact = (l == mn);
            int32_t keff = exact ? l : l - o.oversample;
            int32_t q = 0;
            if (sv[0] > 0.0) {
                for (int32_t qq = 1; qq <= keff; ++qq) {
                    double nxt = (qq < l) ? sv[qq] : 0.0;
                    if (qq < keff || exact) {
                        if (qq == keff && !exact) break;
                        if (nxt / sv[0] < o.tol) {
                            q = qq;
                            break;
                        }
                    }
                }
            }
            (void)pp;
            if (q > 0) {
                resolved[c] = 1;
                if (q <= chunk[c].qlim) {
                    qsel[c] = q;
                    smallU[c].assign(A.begin(), A.begin() + (size_t)l * q);
                    smallV[c].assign(V.begin(), V.begin() + (size_t)l * q);
                }
            } else if (exact || keff >= chunk[c].qlim + 1) {
                resolved[c] = 1;  // no rank below the byte limit: Algorithm 3 fails
            }
        }
        // factors of accepted blocks: U' = Q (U_r Sigma)_q, V = Q2 (W_r)_q
        std::vector<int64_t> soff, ooff_u, ooff_v;
        std::vector<int32_t> qk;
        std::vector<double> small;
        std::vector<SketchBlock> acc_sb;
        std::vector<size_t> acc_c;
        int64_t need = 0;
        for (size_t c = 0; c < nb; ++c)
            if (qsel[c] > 0) need += (int64_t)(sb[c].m + sb[c].n) * qsel[c];
        if (need > 0) {
            DevBuf<double> &pool = pools[level];
            int64_t base = pool_fill[level];
            if ((int64_t)pool.n < base + need) {
                // grow: keep existing candidates
                int64_t cap = std::max<int64_t>(base + need, (int64_t)pool.n * 2);
                DevBuf<double> np(cap);
                if (base > 0) RAD_HIP(hipMemcpy(np.p, pool.p, base * sizeof(double), hipMemcpyDeviceToDevice));
                pool = std::move(np);
            }
            int64_t fill = base;
            for (size_t c = 0; c < nb; ++c) {
                if (qsel[c] == 0) continue;
                BlockPair &pp = bp[chunk[c].p];
                pp.rank = qsel[c];
                pp.svd_bytes = svd_bytes(sb[c].m, sb[c].n, qsel[c]);
                pp.cand_off = fill;
                pp.cand_level = level;
                acc_sb.push_back(sb[c]);
                acc_c.push_back(c);
                qk.push_back(qsel[c]);
                soff.push_back((int64_t)small.size());
                small.insert(small.end(), smallU[c].begin(), smallU[c].end());
                ooff_u.push_back(fill);
                fill += (int64_t)sb[c].m * qsel[c];
                ooff_v.push_back(fill);
                fill += (int64_t)sb[c].n * qsel[c];
            }
            pool_fill[level] = fill;
            // second half of small: V parts
            std::vector<int64_t> soff_v;
            for (size_t t = 0; t < acc_c.size(); ++t) {
                soff_v.push_back((int64_t)small.size());
                small.insert(small.end(), smallV[acc_c[t]].begin(), smallV[acc_c[t]].end());
            }
            // The sketch offsets in acc_sb still point into Y/Z of this chunk.
            DevBuf<SketchBlock> d_acc;
            d_acc.upload(acc_sb);
            DevBuf<double> d_small;
            d_small.upload(small);
            DevBuf<int64_t> d_soff, d_soffv, d_ou, d_ov;
            DevBuf<int32_t> d_qk;
            d_soff.upload(soff);
            d_soffv.upload(soff_v);
            d_ou.upload(ooff_u);
            d_ov.upload(ooff_v);
            d_qk.upload(qk);
            launch_small_gemm(Y.p, d_acc.p, d_soff.p, d_small.p, d_qk.p, d_ou.p, pools[level].p,
                              (int32_t)acc_sb.size(), 0, max_rows, st);
            launch_small_gemm(Z.p, d_acc.p, d_soffv.p, d_small.p, d_qk.p, d_ov.p, pools[level].p,
                              (int32_t)acc_sb.size(), 1, max_rows, st);
            RAD_HIP(hipStreamSynchronize(st));
        }
        for (size_t c = 0; c < nb; ++c) on_done(c, resolved[c] != 0);
    }

    void decide(int64_t p) {
        BlockPair &b = bp[p];
        const TreeNode &a = node(b.I), &c = node(b.J);
        int64_t m = a.size, n = c.size;
        bool allow_dense = o.nearfield != RAD_NEAR_CSR;
        bool allow_csr = o.nearfield != RAD_NEAR_DENSE;
        if (b.nnz == 0) {
            b.kind = BK_ZERO;
            b.best_bytes = 0;
            return;
        }
        int64_t db = dense_bytes(m, n), cb = csr_bytes(m, b.nnz);
        struct Cand {
            int8_t kind;
            int64_t bytes;
        };
        std::vector<Cand> cands;
        if (allow_dense) cands.push_back({BK_DENSE, db});
        if (allow_csr) cands.push_back({BK_CSR, cb});
        if (b.first_child >= 0) {
            if (b.rank > 0) cands.push_back({BK_LOWRANK, b.svd_bytes});
            int64_t hb = 0;
            for (int k = 0; k < b.nchild; ++k) hb += bp[b.first_child + k].best_bytes;
            cands.push_back({BK_HIER, hb});
        }
        Cand best = cands[0];
        for (const Cand &cd : cands)
            if (cd.bytes < best.bytes || (cd.bytes == best.bytes && cd.kind < best.kind)) best = cd;
        b.kind = best.kind;
        b.best_bytes = best.bytes;
        if (b.kind == BK_HIER) {  // Algorithm 4, coalescing: merge uniform children
            bool all_dense = true, all_sparse = true, any_csr = false;
            for (int k = 0; k < b.nchild; ++k) {
                int8_t ck = bp[b.first_child + k].kind;
                all_dense &= ck == BK_DENSE;
                all_sparse &= (ck == BK_CSR || ck == BK_ZERO);
                any_csr |= ck == BK_CSR;
            }
            if (all_dense) {
                b.kind = BK_DENSE;
                b.best_bytes = db;
            } else if (all_sparse && any_csr) {
                b.kind = BK_CSR;
                b.best_bytes = cb;
            }
        }
    }

    void run_dp() {
        int32_t max_level = 0;
        for (auto &b : bp) max_level = std::max(max_level, b.level);
        std::vector<std::vector<int64_t>> by_level(max_level + 1);
        for (size_t p = 0; p < bp.size(); ++p) by_level[bp[p].level].push_back((int64_t)p);
        for (int32_t L = max_level; L >= 0; --L) {
            std::vector<int64_t> internal;
            for (int64_t p : by_level[L])
                if (bp[p].first_child >= 0 && bp[p].nnz > 0) internal.push_back(p);
            if (!internal.empty()) rank_search(L, internal);
            for (int64_t p : by_level[L]) decide(p);
            log("level decided", "L=" + std::to_string(L) + " pairs=" + std::to_string(by_level[L].size()) +
                                     " internal=" + std::to_string(internal.size()));
        }
    }

    // ---------------------------------------------------------------------
    // device layout
    // ---------------------------------------------------------------------
    void layout() {
        // final (non-hierarchical, non-zero) blocks of the chosen partition
        std::vector<int64_t> finals;
        std::vector<int64_t> stack;
        for (size_t p = 0; p < bp.size() && bp[p].level == 0; ++p) stack.push_back((int64_t)p);
        while (!stack.empty()) {
            int64_t p = stack.back();
            stack.pop_back();
            if (bp[p].kind == BK_HIER) {
                for (int k = 0; k < bp[p].nchild; ++k) stack.push_back(bp[p].first_child + k);
            } else if (bp[p].kind != BK_ZERO) {
                finals.push_back(p);
            } else {
                H->stats.n_zero++;
            }
        }
        std::sort(finals.begin(), finals.end());
        // the block table kept for rad_hmat_export
        std::vector<int32_t> blk_of(bp.size(), -1);
        H->blocks.clear();
        H->pieces.clear();
        for (size_t b = 0; b < finals.size(); ++b) {
            const BlockPair &q = bp[finals[b]];
            blk_of[finals[b]] = (int32_t)b;
            BlockRec r{};
            r.kind = q.kind;
            r.i0 = H->nodes[q.I].start;
            r.m = H->nodes[q.I].size;
            r.j0 = H->nodes[q.J].start;
            r.n = H->nodes[q.J].size;
            r.rank = q.kind == BK_LOWRANK ? q.rank : 0;
            r.nnz = q.nnz;
            r.group = -1;
            H->blocks.push_back(r);
        }

        struct Copy {
            int64_t src_off;  // candidate pool (doubles)
            int32_t level;
            int32_t rows, cols, lds;
            int64_t dst_off;
            int32_t ldd;
        };
        std::vector<Copy> copies;
        int64_t vfill = 0;

        // phase 1 groups: V factors of the low-rank blocks, stacked per column node
        std::vector<std::vector<int64_t>> by_col(H->nodes.size());
        for (int64_t p : finals)
            if (bp[p].kind == BK_LOWRANK) by_col[bp[p].J].push_back(p);
        std::vector<ProjGroup> groups;
        std::vector<std::pair<int64_t, int32_t>> t_rows;  // (block, first row in T)
        int32_t t_fill = 0;
        for (size_t J = 0; J < by_col.size(); ++J) {
            if (by_col[J].empty()) continue;
            const TreeNode &cn = H->nodes[J];
            ProjGroup g{};
            g.j0 = cn.start;
            g.n = cn.size;
            g.ld = (cn.size + 7) / 8 * 8;  // 16-byte rows for the 16-bit copy too
            vfill = (vfill + 7) / 8 * 8;
            g.t_off = t_fill;
            int32_t ktot = 0;
            for (int64_t p : by_col[J]) ktot += bp[p].rank;
            g.ktot = ktot;
            g.v_off = vfill;
            int32_t col = 0;
            for (int64_t p : by_col[J]) {
                const BlockPair &b = bp[p];
                const TreeNode &rn = H->nodes[b.I];
                H->blocks[blk_of[p]].group = (int32_t)groups.size();
                H->blocks[blk_of[p]].vcol = col;
                copies.push_back(Copy{b.cand_off + (int64_t)rn.size * b.rank, b.cand_level, cn.size, b.rank,
                                      cn.size, vfill + (int64_t)col * g.ld, g.ld});
                t_rows.push_back({p, t_fill + col});
                col += b.rank;
            }
            vfill += (int64_t)g.ld * ktot;
            t_fill += ktot;
            groups.push_back(g);
            H->stats.n_lowrank += (int64_t)by_col[J].size();
        }
        std::sort(t_rows.begin(), t_rows.end());
        auto t_find = [&](int64_t p) {
            auto it = std::lower_bound(t_rows.begin(), t_rows.end(), std::make_pair(p, INT32_MIN));
            return it->second;
        };

        // Row tiles of 64 facets (tree order).  Dense and low-rank blocks are
        // stored per tile as one packed panel: 64 x K_tile, column-major
        // (ld 64), holding the dense rows and U' rows of every block that
        // touches the tile, with brow[] naming the operand row of each panel
        // column (X row >= 0, T row -1-t < 0).  CSR blocks keep their own
        // per-block storage and per-tile task entries.
        const int32_t n_tiles = (int32_t)((H->N + 63) / 64);
        struct PT {
            int32_t type;
            int64_t p;
            int32_t ncol, r_lo, r_hi, row_off, src_row0;
        };
        std::vector<std::vector<PT>> tp(n_tiles);
        std::vector<std::vector<TileTask>> tcsr(n_tiles);
        std::vector<int32_t> csr_tiles;
        std::vector<int64_t> csr_row_offs;
        std::vector<std::pair<int64_t, int64_t>> csr_ptr_of;  // (p, ptr_off)
        int64_t ptr_fill = 0;
        for (int64_t p : finals) {
            const BlockPair &b = bp[p];
            const TreeNode &rn = H->nodes[b.I], &cn = H->nodes[b.J];
            int64_t ptr_off = 0;
            if (b.kind == BK_CSR) H->blocks[blk_of[p]].ptr_off = ptr_fill;
            if (b.kind == BK_DENSE) {
                H->stats.n_dense++;
                H->stats.bytes_dense += dense_bytes(rn.size, cn.size);
                H->stats.nnz_near += (int64_t)rn.size * cn.size;
            } else if (b.kind == BK_CSR) {
                ptr_off = ptr_fill;
                csr_tiles.insert(csr_tiles.end(), {rn.start, rn.size, cn.start, cn.size, 0, 0});
                csr_row_offs.push_back(ptr_fill);
                csr_ptr_of.push_back({p, ptr_fill});
                ptr_fill += rn.size + 1;
                H->stats.n_csr++;
                H->stats.bytes_csr += csr_bytes(rn.size, b.nnz);
                H->stats.nnz_near += b.nnz;
            } else {
                H->stats.bytes_lowrank += svd_bytes(rn.size, cn.size, b.rank);
                H->stats.sum_rank += b.rank;
                H->stats.lowrank_elems += (int64_t)(rn.size + cn.size) * b.rank;
                H->stats.lowrank_row_elems += (int64_t)rn.size * b.rank;
                H->stats.lowrank_col_elems += (int64_t)cn.size * b.rank;
                H->stats.max_rank = std::max(H->stats.max_rank, b.rank);
            }
            for (int32_t tile = rn.start / 64; (int64_t)tile * 64 < (int64_t)rn.start + rn.size; ++tile) {
                int32_t tile0 = tile * 64;
                int32_t r_lo = std::max(0, rn.start - tile0);
                int32_t r_hi = std::min(64, rn.start + rn.size - tile0);
                int32_t row_off = tile0 - rn.start;
                if (b.kind == BK_CSR) {
                    TileTask t{};
                    t.type = TASK_CSR;
                    t.ncol = cn.size;
                    t.col0 = cn.start;
                    t.aux_off = ptr_off;
                    t.a_off = p;  // replaced by the value base once CSR sizes are known
                    t.row_off = row_off;
                    t.r_lo = r_lo;
                    t.r_hi = r_hi;
                    tcsr[tile].push_back(t);
                } else {
                    int32_t type = b.kind == BK_DENSE ? TASK_DENSE : TASK_LOWRANK;
                    int32_t ncol = b.kind == BK_DENSE ? cn.size : b.rank;
                    int32_t src = b.kind == BK_DENSE ? cn.start : t_find(p);
                    tp[tile].push_back(PT{type, p, ncol, r_lo, r_hi, row_off, src});
                }
            }
        }

        // CSR: count per row on the GPU, scan on the host
        int64_t ntile_csr = (int64_t)csr_tiles.size() / 6;
        std::vector<int32_t> h_ptr;
        int64_t csr_nnz_total = 0;
        std::vector<int64_t> csr_val_base(ntile_csr);
        DevBuf<int32_t> d_ctiles;
        DevBuf<int64_t> d_crow;
        if (ntile_csr > 0) {
            d_ctiles.upload(csr_tiles);
            d_crow.upload(csr_row_offs);
            DevBuf<int32_t> d_cnt(ptr_fill);
            RAD_HIP(hipMemsetAsync(d_cnt.p, 0, ptr_fill * sizeof(int32_t), st));
            launch_csr_count(geom, d_ctiles.p, ntile_csr, d_cnt.p, d_crow.p, st);
            RAD_HIP(hipStreamSynchronize(st));
            std::vector<int32_t> cnt = d_cnt.download(ptr_fill);
            h_ptr.assign(ptr_fill, 0);
            for (int64_t t = 0; t < ntile_csr; ++t) {
                int32_t m = csr_tiles[6 * t + 1];
                int64_t ro = csr_row_offs[t];
                int32_t acc = 0;
                for (int32_t r = 0; r < m; ++r) {
                    h_ptr[ro + r] = acc;
                    acc += cnt[ro + r];
                }
                h_ptr[ro + m] = acc;
                csr_val_base[t] = csr_nnz_total;
                csr_nnz_total += acc;
            }
            // (csr_ptr_of lists the CSR blocks in the order of csr_tiles)
            for (int64_t t = 0; t < ntile_csr; ++t) H->blocks[blk_of[csr_ptr_of[t].first]].val_base = csr_val_base[t];
        }

        // panels (16-byte vector loads need panel_off aligned to 64 elements)
        vfill = (vfill + 63) / 64 * 64;
        std::vector<TileInfo> tinfo(n_tiles);
        std::vector<int32_t> brow;
        std::vector<int32_t> dense_desc;  // i0, m, j0, n, ld, pad
        std::vector<int64_t> dense_offs;
        std::vector<CopyDesc> lr_copies;
        std::vector<TileTask> ttasks;
        std::sort(csr_ptr_of.begin(), csr_ptr_of.end());
        for (int32_t tl = 0; tl < n_tiles; ++tl) {
            auto &v = tp[tl];
            std::stable_sort(v.begin(), v.end(), [](const PT &a, const PT &b) { return a.type < b.type; });
            int64_t K = 0;
            for (const PT &pt : v) K += pt.ncol;
            H->stats.max_panel_cols = std::max<int64_t>(H->stats.max_panel_cols, K);
            int64_t kpad = (K + 31) / 32 * 32;
            TileInfo ti{};
            ti.panel_off = vfill;
            ti.kpad = (int32_t)kpad;
            ti.k16 = (int32_t)((K + 15) / 16 * 16);
            ti.brow_off = (int64_t)brow.size();
            int64_t col = 0;
            for (const PT &pt : v) {
                const BlockPair &b = bp[pt.p];
                int64_t dst = vfill + col * 64 + pt.r_lo;
                H->pieces.push_back(BlockPiece{blk_of[pt.p], tl, (int32_t)col, pt.r_lo, pt.r_hi});
                if (pt.type == TASK_DENSE) {
                    dense_desc.insert(dense_desc.end(), {tl * 64 + pt.r_lo, pt.r_hi - pt.r_lo, pt.src_row0, pt.ncol, 64, 0});
                    dense_offs.push_back(dst);
                    for (int32_t k = 0; k < pt.ncol; ++k) brow.push_back(pt.src_row0 + k);
                } else {
                    const TreeNode &rn = H->nodes[b.I];
                    CopyDesc c{};
                    c.src = pools[b.cand_level].p + b.cand_off + (pt.row_off + pt.r_lo);
                    c.rows = pt.r_hi - pt.r_lo;
                    c.cols = pt.ncol;
                    c.lds = rn.size;
                    c.dst_off = dst;
                    c.ldd = 64;
                    lr_copies.push_back(c);
                    for (int32_t k = 0; k < pt.ncol; ++k) brow.push_back(-(pt.src_row0 + k) - 1);
                }
                col += pt.ncol;
            }
            for (int64_t k = K; k < kpad; ++k) brow.push_back(0);
            vfill += 64 * kpad;
            ti.csr_begin = (int32_t)ttasks.size();
            for (TileTask t : tcsr[tl]) {
                auto it = std::lower_bound(csr_ptr_of.begin(), csr_ptr_of.end(), std::make_pair(t.a_off, (int64_t)INT64_MIN));
                int64_t ci = it - csr_ptr_of.begin();
                t.a_off = csr_val_base[ci];  // relative; made absolute below
                ttasks.push_back(t);
            }
            ti.csr_end = (int32_t)ttasks.size();
            tinfo[tl] = ti;
        }
        const int64_t csr_val_start = vfill;
        vfill += csr_nnz_total;
        for (TileTask &t : ttasks) {
            t.a_off += csr_val_start;
            // rows that hold every column of the block: their values form a
            // row-major dense slab the expansion kernel stages without indices
            t.full = 1;
            for (int32_t r = t.r_lo; r < t.r_hi && t.full; ++r) {
                const int64_t q = t.aux_off + t.row_off + r;
                if (h_ptr[q + 1] - h_ptr[q] != t.ncol) t.full = 0;
            }
        }

        // allocate the value pool and fill it
        H->d_vals.alloc((size_t)std::max<int64_t>(vfill, 1) * s);
        RAD_HIP(hipMemsetAsync(H->d_vals.p, 0, (size_t)std::max<int64_t>(vfill, 1) * s, st));
        int64_t n_dense_desc = (int64_t)dense_desc.size() / 6;
        if (n_dense_desc > 0) {
            DevBuf<int32_t> d_t;
            d_t.upload(dense_desc);
            DevBuf<int64_t> d_o;
            d_o.upload(dense_offs);
            launch_dense_fill(geom, d_t.p, d_o.p, n_dense_desc, H->d_vals.p, H->dtype, st);
            RAD_HIP(hipStreamSynchronize(st));
        }
        if (ntile_csr > 0) {
            H->d_csr_ptr.upload(h_ptr);
            H->d_csr_idx.alloc((size_t)std::max<int64_t>(csr_nnz_total, 1));
            DevBuf<int64_t> d_vb;
            d_vb.upload(csr_val_base);
            // values at csr_val_start + base; column indices at base
            char *vals_csr = (char *)H->d_vals.p + (size_t)csr_val_start * s;
            launch_csr_fill(geom, d_ctiles.p, ntile_csr, H->d_csr_ptr.p, d_crow.p, d_vb.p, vals_csr,
                            H->d_csr_idx.p, H->dtype, st);
            RAD_HIP(hipStreamSynchronize(st));
        }
        for (const Copy &c : copies) {  // stacked V factors
            CopyDesc d{};
            d.src = pools[c.level].p + c.src_off;
            d.rows = c.rows;
            d.cols = c.cols;
            d.lds = c.lds;
            d.dst_off = c.dst_off;
            d.ldd = c.ldd;
            lr_copies.push_back(d);
        }
        if (!lr_copies.empty()) {
            DevBuf<CopyDesc> d_c;
            d_c.upload(lr_copies);
            launch_copy_batched(d_c.p, (int64_t)lr_copies.size(), H->d_vals.p, H->dtype, st);
            RAD_HIP(hipStreamSynchronize(st));
        }
        H->csr_val_start = csr_val_start;

        H->h_groups = groups;
        H->d_groups.upload(groups);
        H->d_tiles.upload(tinfo);
        H->d_brow.upload(brow);
        H->d_tile_tasks.upload(ttasks);
        H->n_tiles = n_tiles;
        H->n_groups = (int32_t)groups.size();
        // split-K work lists of the multi-RHS projections
        {
            const int32_t kSplit = 512;
            std::vector<P1Work> work;
            std::vector<P1Red> red;
            int32_t part = 0;
            for (int32_t gi = 0; gi < (int32_t)groups.size(); ++gi) {
                const ProjGroup &g = groups[gi];
                for (int32_t k0 = 0; k0 < g.ktot; k0 += 64) {
                    P1Red rd{g.t_off + k0, std::min(64, g.ktot - k0), part, 0};
                    for (int32_t jb = 0; jb < g.n; jb += kSplit) {
                        work.push_back(P1Work{gi, k0, jb, std::min(g.n, jb + kSplit), part++, 0});
                        rd.part_count++;
                    }
                    red.push_back(rd);
                }
            }
            // launch order: the row tiles of one facet chunk next to each other,
            // so that workgroups sharing an X chunk run together (same L2)
            std::stable_sort(work.begin(), work.end(), [](const P1Work &a, const P1Work &b) {
                if (a.group != b.group) return a.group < b.group;
                if (a.jb != b.jb) return a.jb < b.jb;
                return a.krow0 < b.krow0;
            });
            H->d_p1work.upload(work);
            H->d_p1red.upload(red);
            H->n_p1work = (int32_t)work.size();
            H->n_p1red = (int32_t)red.size();
            H->n_parts = part;
        }
        H->t_rows = t_fill;
        H->t_ld = std::max<int32_t>(round4(t_fill), 4);

        H->stats.bytes_total = (int64_t)H->d_vals.bytes() + (int64_t)H->d_csr_idx.bytes() +
                               (int64_t)H->d_csr_ptr.bytes() + (int64_t)H->d_tiles.bytes() +
                               (int64_t)H->d_brow.bytes() + (int64_t)H->d_groups.bytes() +
                               (int64_t)H->d_tile_tasks.bytes() + (int64_t)H->d_perm.bytes();
        H->stats.flops_per_rhs = 2.0 * ((double)H->stats.lowrank_elems + (double)H->stats.nnz_near);
        if (o.lowp) {
            H->lowp = o.lowp;
            H->d_vals16.alloc((size_t)std::max<int64_t>(vfill, 1));
            RAD_HIP(hipMemsetAsync(H->d_vals16.p, 0, (size_t)std::max<int64_t>(vfill, 1) * 2, st));
            H->d_pscale.alloc((size_t)std::max<int64_t>(csr_val_start / 64 + 1, 1));
            H->d_tscale.alloc((size_t)std::max<int32_t>(t_fill, 1));
            lowp_convert(H, st);
            RAD_HIP(hipStreamSynchronize(st));
            H->stats.bytes_total += (int64_t)H->d_vals16.bytes() + (int64_t)H->d_pscale.bytes() +
                                    (int64_t)H->d_tscale.bytes();
        }
    }
};

}  // namespace

namespace {

void check_opts(const rad_build_opts &o, int tree_dims) {
    RAD_REQUIRE(tree_dims == 2 || tree_dims == 3, "tree_dims must be 2 (quadtree) or 3 (octree)");
    RAD_REQUIRE(o.tol > 0.0 && std::isfinite(o.tol), "tol must be positive");
    RAD_REQUIRE(o.leaf_size >= 1 && o.leaf_size <= 4096, "leaf_size must be in [1, 4096]");
    RAD_REQUIRE(o.storage == RAD_F64 || o.storage == RAD_F32, "storage must be RAD_F64 or RAD_F32");
    RAD_REQUIRE(o.nearfield >= RAD_NEAR_AUTO && o.nearfield <= RAD_NEAR_CSR, "bad nearfield option");
    RAD_REQUIRE(o.visibility == RAD_VIS_BACKFACE || o.visibility == RAD_VIS_RAYCAST, "bad visibility option");
    RAD_REQUIRE(o.oversample >= 2 && o.oversample <= 64, "oversample must be in [2, 64]");
    RAD_REQUIRE(o.power_iters >= 0 && o.power_iters <= 4, "power_iters must be in [0, 4]");
    RAD_REQUIRE(o.max_rhs >= 1, "max_rhs must be >= 1");
    RAD_REQUIRE(o.lowp == 0 || ((o.lowp == RAD_F16 || o.lowp == RAD_BF16) && o.storage == RAD_F32),
                "lowp must be 0, RAD_F16 or RAD_BF16, with storage RAD_F32");
}

// Everything after the facet geometry: x, n (nf x 3) and A (nf) in the
// caller's facet order; tri (nf x 9, the facets' own triangles, same order)
// for ray casting and shadows, or empty (no occluders).
void build_from_geometry(rad_hmat *H, std::vector<double> &x, std::vector<double> &n, std::vector<double> &A,
                         const std::vector<double> &tri_orig, int64_t nf, const rad_build_opts &o, int tree_dims,
                         std::chrono::steady_clock::time_point t0) {
    Builder B;
    B.log.on = o.verbose != 0;
    B.H = H;
    B.o = o;
    B.s = dtype_size(o.storage);
    H->device = o.device;
    H->N = nf;
    H->dtype = o.storage;
    H->max_rhs = o.max_rhs;
    H->leaf_size = o.leaf_size;

    RAD_HIP(hipSetDevice(o.device));

    QuadBuilder qb;
    qb.x = x.data();
    qb.leaf_size = o.leaf_size;
    qb.max_depth = o.max_depth;
    qb.dims = tree_dims;
    qb.nodes.resize(1);
    std::vector<int32_t> all(nf);
    std::iota(all.begin(), all.end(), 0);
    qb.split(0, std::move(all), 0);
    B.log(tree_dims == 3 ? "octree" : "quadtree", "leaves=" + std::to_string(qb.nleaves));
    H->nodes = std::move(qb.nodes);
    H->perm = std::move(qb.perm);
    H->n_leaves = qb.nleaves;
    int32_t depth = 0;
    for (auto &t : H->nodes) depth = std::max(depth, t.depth);
    H->stats.n = nf;
    H->stats.n_leaves = H->n_leaves;
    H->stats.depth = depth;
    H->stats.dtype = o.storage;

    B.xt.resize(3 * nf);
    B.nt.resize(3 * nf);
    B.at.resize(nf);
    for (int64_t t = 0; t < nf; ++t) {
        int32_t i = H->perm[t];
        for (int k = 0; k < 3; ++k) {
            B.xt[3 * t + k] = x[3 * i + k];
            B.nt[3 * t + k] = n[3 * i + k];
        }
        B.at[t] = A[i];
    }
    H->d_x.upload(B.xt);
    H->d_n.upload(B.nt);
    H->d_a.upload(B.at);
    H->d_perm.upload(H->perm);
    B.geom.x = H->d_x.p;
    B.geom.n = H->d_n.p;
    B.geom.a = H->d_a.p;
    B.geom.vis = nullptr;
    {
        std::vector<double> tri(tri_orig.size());
        if (!tri.empty())
            for (int64_t t = 0; t < nf; ++t) {
                int32_t f = H->perm[t];
                std::copy(tri_orig.begin() + 9 * (int64_t)f, tri_orig.begin() + 9 * (int64_t)f + 9,
                          tri.begin() + 9 * t);
            }
        build_grid(H, tri);
    }
    B.log("grid");
    if (o.visibility == RAD_VIS_RAYCAST) {
        int64_t wpr = (nf + 31) / 32;
        B.d_vis.alloc((size_t)wpr * nf);
        B.geom.vis = B.d_vis.p;
        B.geom.vis_words_per_row = wpr;
        // in row chunks of about 2^31 facet pairs, each reported when done
        const int64_t chunk = std::max<int64_t>(1, ((int64_t)1 << 26) / wpr);
        for (int64_t r0 = 0; r0 < nf; r0 += chunk) {
            launch_vis_grid(H, B.d_vis.p, wpr, r0, std::min<int64_t>(chunk, nf - r0), B.st);
            RAD_HIP(hipStreamSynchronize(B.st));
            if (nf > chunk) B.log("  visibility rows", std::to_string(std::min<int64_t>(nf, r0 + chunk)));
        }
        B.log("visibility bitmap");
    }

    B.enumerate_pairs();
    B.log("block pairs", std::to_string(B.bp.size()));
    B.count_nnz();
    B.log("leaf non-zeros");
    B.run_dp();
    B.log("rank search and choice");
    B.layout();
    B.log("layout");

    auto t1 = std::chrono::steady_clock::now();
    H->stats.build_seconds = std::chrono::duration<double>(t1 - t0).count();
    if (o.verbose) {
        const rad_hmat_stats &s = H->stats;
        std::fprintf(stderr,
                     "[rad] N=%lld leaves=%lld depth=%d pairs=%zu dense=%lld csr=%lld lowrank=%lld zero=%lld "
                     "bytes=%lld (dense %lld csr %lld lr %lld) sum_rank=%lld max_rank=%d build=%.2fs\n",
                     (long long)s.n, (long long)s.n_leaves, s.depth, B.bp.size(), (long long)s.n_dense,
                     (long long)s.n_csr, (long long)s.n_lowrank, (long long)s.n_zero, (long long)s.bytes_total,
                     (long long)s.bytes_dense, (long long)s.bytes_csr, (long long)s.bytes_lowrank,
                     (long long)s.sum_rank, s.max_rank, s.build_seconds);
    }
}

}  // namespace

void build_hmat(rad_hmat *H, const double *verts, int64_t nv, const int32_t *faces, int64_t nf,
                const rad_build_opts &o, int tree_dims) {
    auto t0 = std::chrono::steady_clock::now();
    RAD_REQUIRE(verts && faces, "null mesh pointer");
    RAD_REQUIRE(nv >= 3 && nf >= 1, "mesh needs nv >= 3 and nf >= 1");
    RAD_REQUIRE(nf < (int64_t)1 << 31, "too many faces");
    check_opts(o, tree_dims);
    // all host-side validation happens before the first HIP call
    std::vector<double> x, n, A;
    facet_geometry(verts, nv, faces, nf, x, n, A);
    std::vector<double> tri(9 * nf);
    for (int64_t f = 0; f < nf; ++f)
        for (int v = 0; v < 3; ++v)
            for (int k = 0; k < 3; ++k) tri[9 * f + 3 * v + k] = verts[3 * (int64_t)faces[3 * f + v] + k];
    build_from_geometry(H, x, n, A, tri, nf, o, tree_dims, t0);
}

void build_hmat_facets(rad_hmat *H, const double *xc, const double *nc, const double *area, int64_t N,
                       const double *tri_verts, const rad_build_opts &o, int tree_dims) {
    auto t0 = std::chrono::steady_clock::now();
    RAD_REQUIRE(xc && nc && area, "null facet array");
    RAD_REQUIRE(N >= 1 && N < (int64_t)1 << 31, "N must be in [1, 2^31)");
    check_opts(o, tree_dims);
    RAD_REQUIRE(tri_verts || o.visibility == RAD_VIS_BACKFACE,
                "ray-cast visibility needs the facets' triangles (tri_verts)");
    std::vector<double> x(xc, xc + 3 * N), n(nc, nc + 3 * N), A(area, area + N), tri;
    for (int64_t i = 0; i < N; ++i) {
        for (int k = 0; k < 3; ++k)
            RAD_REQUIRE(std::isfinite(x[3 * i + k]) && std::isfinite(n[3 * i + k]),
                        "facet " + std::to_string(i) + " has a non-finite centroid or normal");
        const double len = std::sqrt(n[3 * i] * n[3 * i] + n[3 * i + 1] * n[3 * i + 1] + n[3 * i + 2] * n[3 * i + 2]);
        RAD_REQUIRE(std::fabs(len - 1.0) <= 1e-6, "facet " + std::to_string(i) + " has a normal that is not unit length");
        RAD_REQUIRE(std::isfinite(A[i]) && A[i] > 0.0, "facet " + std::to_string(i) + " has a non-positive area");
    }
    if (tri_verts) {
        tri.assign(tri_verts, tri_verts + 9 * N);
        for (double v : tri) RAD_REQUIRE(std::isfinite(v), "non-finite triangle vertex");
    }
    build_from_geometry(H, x, n, A, tri, N, o, tree_dims, t0);
}

}  // namespace rad
