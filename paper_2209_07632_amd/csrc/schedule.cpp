// Host-side launch schedules of the product kernels, prepared once per
// matrix (after the build, a load, a precision conversion or a grouping):
// the tile order of the persistent expansion, the pairs of projection slabs,
// the single-RHS projection items of long column nodes and the segments of
// long single-RHS tile reductions, the tile pairs and reduction segments of
// the wide BF16 expansion, and the launch tables that place work items that
// read the same operand rows on one XCD.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <vector>

#include "rad_internal.h"

namespace rad {

std::vector<int32_t> xcd_launch_order(const std::vector<std::vector<int32_t>> &groups,
                                      const std::vector<int64_t> &cost) {
    constexpr int kXcd = 8;
    std::vector<int64_t> gmax(groups.size(), 0), gsum(groups.size(), 0);
    for (size_t g = 0; g < groups.size(); ++g)
        for (int32_t i : groups[g]) {
            gmax[g] = std::max(gmax[g], cost[i]);
            gsum[g] += cost[i];
        }
    std::vector<int32_t> gi(groups.size());
    for (size_t g = 0; g < gi.size(); ++g) gi[g] = (int32_t)g;
    std::stable_sort(gi.begin(), gi.end(), [&](int32_t a, int32_t b) { return gmax[a] > gmax[b]; });
    std::vector<std::vector<int32_t>> q(kXcd);
    std::vector<int64_t> load(kXcd, 0);
    for (int32_t g : gi) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        q[x].insert(q[x].end(), groups[g].begin(), groups[g].end());
        load[x] += gsum[g];
    }
    size_t len = 0;
    for (const auto &v : q) len = std::max(len, v.size());
    std::vector<int32_t> order(kXcd * len, -1);
    for (int x = 0; x < kXcd; ++x)
        for (size_t sl = 0; sl < q[x].size(); ++sl) order[kXcd * sl + x] = q[x][sl];
    return order;
}

std::vector<int32_t> xcd_region_order(const std::vector<std::vector<int32_t>> &groups,
                                      const std::vector<int64_t> &cost) {
    constexpr int kXcd = 8;
    std::vector<int64_t> gsum(groups.size(), 0);
    int64_t total = 0;
    for (size_t g = 0; g < groups.size(); ++g) {
        for (int32_t i : groups[g]) gsum[g] += cost[i];
        total += gsum[g];
    }
    std::vector<std::vector<int32_t>> q(kXcd);
    int64_t before = 0;
    for (size_t g = 0; g < groups.size(); ++g) {
        // the XCD whose share of the total cost holds this group's midpoint
        const int64_t mid = 2 * before + gsum[g];
        const int x = total > 0 ? (int)std::min<int64_t>(kXcd - 1, mid * kXcd / (2 * total)) : 0;
        q[x].insert(q[x].end(), groups[g].begin(), groups[g].end());
        before += gsum[g];
    }
    size_t len = 0;
    for (const auto &v : q) len = std::max(len, v.size());
    std::vector<int32_t> order(kXcd * len, -1);
    for (int x = 0; x < kXcd; ++x)
        for (size_t sl = 0; sl < q[x].size(); ++sl) order[kXcd * sl + x] = q[x][sl];
    return order;
}

namespace {

// The CSR structure on the host (row pointers and column indices).
struct CsrHost {
    std::vector<int32_t> ptr, idx;
};

// f(row of the tile, X row, entry index) for every CSR entry of tile i
template <class F>
void for_each_csr_entry(const rad_hmat *H, const CsrHost &c, const std::vector<TileInfo> &ti,
                        const std::vector<TileTask> &tk, int32_t i, F &&f) {
    for (int32_t ct = ti[i].csr_begin; ct < ti[i].csr_end; ++ct) {
        const TileTask &t = tk[ct];
        const int64_t g0 = t.a_off - H->csr_val_start;
        for (int32_t r = t.r_lo; r < t.r_hi; ++r)
            for (int32_t q = c.ptr[t.aux_off + t.row_off + r]; q < c.ptr[t.aux_off + t.row_off + r + 1]; ++q)
                f(r, t.col0 + c.idx[g0 + q], g0 + q);
    }
}

// The CSR slices of each tile as one compressed panel (FP32 / FP64
// products, single- and multi-RHS): the panel's columns are the sorted union
// of the X rows where any of the tile's rows has an entry, so the slices run
// through the same streamed panel loops as dense and low-rank columns, with
// the zeros of that union as the only extra work.  Returns each tile's
// compressed width.
std::vector<int32_t> prepare_csr_panels(rad_hmat *H, const CsrHost &c, const std::vector<TileInfo> &ti,
                                        const std::vector<TileTask> &tk) {
    const int32_t n = H->n_tiles;
    std::vector<int32_t> width(n, 0);
    H->n_cpan = 0;
    H->cpan_elems = 0;
    if (tk.empty() || c.idx.empty()) return width;
    std::vector<int64_t> dst(c.idx.size(), -1);   // per CSR entry: its element of the compressed panels
    std::vector<CsrPanel> cp(n, CsrPanel{0, 0, 0, 0});
    std::vector<int32_t> cbrow, cols;
    int64_t vfill = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (ti[i].csr_begin >= ti[i].csr_end) continue;
        cols.clear();
        for_each_csr_entry(H, c, ti, tk, i, [&](int32_t, int32_t col, int64_t) { cols.push_back(col); });
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        if (cols.empty()) continue;
        const int32_t k16 = (int32_t)((cols.size() + 15) / 16 * 16);
        cp[i] = CsrPanel{vfill, (int64_t)cbrow.size(), k16, 0};
        cbrow.insert(cbrow.end(), cols.begin(), cols.end());
        cbrow.insert(cbrow.end(), (size_t)k16 - cols.size(), cols.back());   // padding columns (zero values)
        for_each_csr_entry(H, c, ti, tk, i, [&](int32_t r, int32_t col, int64_t g) {
            const int64_t pos = std::lower_bound(cols.begin(), cols.end(), col) - cols.begin();
            dst[g] = vfill + pos * 64 + r;
        });
        width[i] = k16;
        vfill += (int64_t)64 * k16;
    }
    if (vfill == 0) return width;
    const size_t s = H->dtype == RAD_F64 ? sizeof(double) : sizeof(float);
    H->d_cvals.alloc((size_t)vfill * s);
    RAD_HIP(hipMemset(H->d_cvals.p, 0, (size_t)vfill * s));
    {
        DevBuf<int64_t> d_dst;
        d_dst.upload(dst);
        launch_csr_panel_scatter((const char *)H->d_vals.p + (size_t)H->csr_val_start * s, d_dst.p,
                                 (int64_t)dst.size(), H->d_cvals.p, H->dtype, nullptr);
        RAD_HIP(hipStreamSynchronize(nullptr));
    }
    H->d_cpan.upload(cp);
    H->d_cbrow.upload(cbrow);
    H->n_cpan = n;
    H->cpan_elems = vfill;
    return width;
}

// A tile pair's compressed CSR panel for the wide BF16 expansion: offset of
// its values (the pair's first tile; the second follows 64 x k32 values
// later) and of its X-row list, and its width k32 (a multiple of 32; 0: none).
struct PairCsr {
    int64_t off, br;
    int32_t k32;
};

// One compressed panel per tile pair (wp: the pairs' first tiles) over the
// union of both tiles' nonzero columns, in the 16-bit chunk layout
// [k / 32][row][32] of each tile, so that the pair's two tiles share one
// operand-row list as the wide kernel needs.
std::vector<PairCsr> prepare_pair_csr(rad_hmat *H, const CsrHost &c, const std::vector<TileInfo> &ti,
                                      const std::vector<TileTask> &tk, const std::vector<int32_t> &wp) {
    std::vector<PairCsr> out(wp.size(), PairCsr{0, 0, 0});
    std::vector<int64_t> dst(c.idx.size(), -1);
    std::vector<int32_t> cb, cols;
    int64_t fill = 0;
    for (size_t p = 0; p < wp.size(); ++p) {
        cols.clear();
        for (int32_t h = 0; h < 2; ++h)
            for_each_csr_entry(H, c, ti, tk, wp[p] + h, [&](int32_t, int32_t col, int64_t) { cols.push_back(col); });
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        if (cols.empty()) continue;
        const int32_t k32 = (int32_t)((cols.size() + 31) / 32 * 32);
        out[p] = PairCsr{fill, (int64_t)cb.size(), k32};
        cb.insert(cb.end(), cols.begin(), cols.end());
        cb.insert(cb.end(), (size_t)k32 - cols.size(), cols.back());   // padding columns (zero values)
        for (int32_t h = 0; h < 2; ++h)
            for_each_csr_entry(H, c, ti, tk, wp[p] + h, [&](int32_t r, int32_t col, int64_t g) {
                const int64_t k = std::lower_bound(cols.begin(), cols.end(), col) - cols.begin();
                dst[g] = fill + (int64_t)h * 64 * k32 + (k / 32) * 64 * 32 + (int64_t)r * 32 + k % 32;
            });
        fill += (int64_t)2 * 64 * k32;
    }
    if (fill == 0) return out;
    H->d_cvals16.alloc((size_t)fill);
    RAD_HIP(hipMemset(H->d_cvals16.p, 0, (size_t)fill * sizeof(uint16_t)));
    {
        DevBuf<int64_t> d_dst;
        d_dst.upload(dst);
        launch_csr_panel_scatter16((const float *)H->d_vals.p + H->csr_val_start, d_dst.p, (int64_t)dst.size(),
                                   H->d_cvals16.p, nullptr);
        RAD_HIP(hipStreamSynchronize(nullptr));
    }
    H->d_cbrow16.upload(cb);
    return out;
}

}  // namespace

void mm_prepare_schedule(rad_hmat *H) {
    const int32_t n = H->n_tiles;
    std::vector<TileInfo> ti = H->d_tiles.download((size_t)n);
    std::vector<TileTask> tk = H->d_tile_tasks.download(H->d_tile_tasks.n);
    CsrHost csr;
    if (!tk.empty()) {
        csr.ptr = H->d_csr_ptr.download(H->d_csr_ptr.n);
        csr.idx = H->d_csr_idx.download(H->d_csr_idx.n);
    }
    H->d_cvals16.release();
    H->d_cbrow16.release();
    const std::vector<int32_t> cwidth = prepare_csr_panels(H, csr, ti, tk);
    std::vector<int64_t> cost(n, 0);
    for (int32_t i = 0; i < n; ++i) {
        cost[i] = ti[i].k16;
        if (H->n_cpan > 0)
            cost[i] += cwidth[i];
        else
            for (int32_t c = ti[i].csr_begin; c < ti[i].csr_end; ++c) cost[i] += tk[c].ncol;
    }
    std::vector<int32_t> order(n);
    for (int32_t i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    H->d_tile_order.upload(order);
    std::vector<int32_t> zero(2, 0);
    H->d_queue.upload(zero);
    // phase-1 pairs: consecutive work items of one group and facet chunk whose
    // V slabs follow each other (the list is ordered by group, chunk, slab)
    std::vector<P1Work> wl = H->d_p1work.download((size_t)H->n_p1work);
    std::vector<int32_t> pairs;
    for (int32_t i = 0; i < H->n_p1work;) {
        const bool pair = i + 1 < H->n_p1work && wl[i + 1].group == wl[i].group && wl[i + 1].jb == wl[i].jb &&
                          wl[i + 1].krow0 == wl[i].krow0 + mm_part_rows();
        pairs.push_back(i);
        pairs.push_back(pair ? i + 1 : -1);
        i += pair ? 2 : 1;
    }
    H->n_p1pairs = (int32_t)(pairs.size() / 2);
    H->d_p1pairs.upload(pairs);
    // slabs that one work item reduces alone are written straight into T by
    // it (both slabs of a pair, or neither); the split-K sum takes the rest
    {
        std::vector<P1Red> rl = H->d_p1red.download((size_t)H->n_p1red);
        std::vector<int32_t> lone_row(std::max(H->n_parts, 1), -1);  // T row of a part alone in its slab
        for (const P1Red &r : rl)
            if (r.part_count == 1) lone_row[r.part_begin] = r.t_row0;
        std::vector<char> direct_part(std::max(H->n_parts, 1), 0);
        std::vector<int32_t> direct(H->n_p1pairs, -1);
        for (int32_t q = 0; q < H->n_p1pairs; ++q) {
            const int32_t p0 = pairs[2 * q], p1 = pairs[2 * q + 1];
            const int32_t d0 = lone_row[wl[p0].part];
            if (d0 < 0) continue;
            if (p1 >= 0 && lone_row[wl[p1].part] != d0 + mm_part_rows()) continue;
            direct[q] = d0;
            direct_part[wl[p0].part] = 1;
            if (p1 >= 0) direct_part[wl[p1].part] = 1;
        }
        std::vector<P1Red> multi;
        for (const P1Red &r : rl)
            if (!(r.part_count == 1 && direct_part[r.part_begin])) multi.push_back(r);
        H->d_p1direct.upload(direct);
        H->n_p1red_multi = (int32_t)multi.size();
        if (!multi.empty()) H->d_p1red_multi.upload(multi);
    }
    // single-RHS projections: one workgroup per V column of long column
    // nodes, one wave per V column of the others (a node's columns adjacent)
    {
        std::vector<int32_t> items, cols;
        for (int32_t gi = 0; gi < (int32_t)H->h_groups.size(); ++gi)
            for (int32_t kk = 0; kk < H->h_groups[gi].ktot; ++kk) {
                std::vector<int32_t> &dst = H->h_groups[gi].n >= kProjWideN ? items : cols;
                dst.push_back(gi);
                dst.push_back(kk);
            }
        H->n_pwide = (int32_t)(items.size() / 2);
        H->d_pwide.upload(items);
        H->n_pcols = (int32_t)(cols.size() / 2);
        H->d_pcols.upload(cols);
    }
    // segments of the single-RHS tile product: panels longer than kGSeg
    // columns (1 MB of values) are cut into near-equal runs of whole 16-column
    // chunks, so one long tile no longer holds the product back
    {
        const int32_t vw = H->dtype == RAD_F64 ? 2 : 4;            // values per 16-byte load
        const int32_t kGSeg = H->dtype == RAD_F64 ? 2048 : 4096;
        int32_t kmax = 0;
        for (int32_t i = 0; i < n; ++i) kmax = std::max(kmax, ti[i].k16 + cwidth[i]);
        H->n_gsegs = 0;
        if (kmax > kGSeg) {
            std::vector<GemvSeg> segs;
            std::vector<int32_t> tseg(1, 0);
            for (int32_t i = 0; i < n; ++i) {
                const int32_t chunks = (ti[i].k16 + cwidth[i]) / 16;   // the panel, then the CSR panel
                const int32_t nseg = std::max(1, (ti[i].k16 + cwidth[i] + kGSeg - 1) / kGSeg);
                for (int32_t sg = 0; sg < nseg; ++sg) {
                    const int64_t c0 = (int64_t)chunks * sg / nseg, c1 = (int64_t)chunks * (sg + 1) / nseg;
                    segs.push_back(GemvSeg{i, (int32_t)(16 * c0 / vw), (int32_t)(16 * c1 / vw), sg == 0 ? 1 : 0,
                                           (int32_t)segs.size()});
                }
                tseg.push_back((int32_t)segs.size());
            }
            std::stable_sort(segs.begin(), segs.end(),
                             [](const GemvSeg &a, const GemvSeg &b) { return a.g1 - a.g0 > b.g1 - b.g0; });
            H->n_gsegs = (int32_t)segs.size();
            H->d_gsegs.upload(segs);
            H->d_gseg_of_tile.upload(tseg);
        }
    }
    // tile pairs of the wide BF16 expansion: consecutive tiles (the halves of
    // a 128-facet leaf) whose panels multiply the same operand rows
    H->n_wpairs = H->n_wsingles = H->n_wsegs = H->n_wseg_blocks = 0;
    H->wide_csr = 0;
    if (H->lowp == RAD_BF16 && n > 1) {
        std::vector<int32_t> br = H->d_brow.download(H->d_brow.n);
        std::vector<int32_t> wp, ws;
        for (int32_t i = 0; i < n;) {
            // (two tiles with empty panels pair too: their CSR slices, if
            // any, get one compressed panel over both)
            bool same = i + 1 < n && ti[i].kpad == ti[i + 1].kpad;
            if (same)
                same = std::equal(br.begin() + ti[i].brow_off, br.begin() + ti[i].brow_off + ti[i].kpad,
                                  br.begin() + ti[i + 1].brow_off);
            if (same) {
                wp.push_back(i);
                i += 2;
            } else {
                ws.push_back(i);
                i += 1;
            }
        }
        // CSR slices: one compressed panel per pair, when no lone tile has any
        // (the wide kernels do not walk CSR rows; otherwise the matrix keeps
        // the 16-bit tile kernel, which does)
        std::vector<PairCsr> pc;
        if (!tk.empty()) {
            bool lone = false;
            for (int32_t i : ws) lone = lone || ti[i].csr_begin < ti[i].csr_end;
            if (!lone && H->max_rhs >= kMfmaMinRhs) {
                pc = prepare_pair_csr(H, csr, ti, tk, wp);
                H->wide_csr = 1;
            }
        }
        if (!tk.empty() && !H->wide_csr) {
            wp.clear();
            ws.clear();
        }
        H->n_wpairs = (int32_t)wp.size();
        H->n_wsingles = (int32_t)ws.size();
        H->d_wpairs.upload(wp);
        H->d_wsingles.upload(ws);
        // segments: a pair's reduction is cut into near-equal runs of at most
        // kSeg panel columns (whole 32-column chunks of the 16-bit layout,
        // 64 x 32 values each); a pair's segments take consecutive partial
        // slots in order
        constexpr int32_t kSeg = 12288;
        std::vector<WideSeg> bySlot;
        std::vector<int32_t> pslot(1, 0);
        // share groups: segment sg of consecutive pairs with one operand-row
        // list (the tiles of one leaf) reads the same operand rows
        std::vector<std::vector<int32_t>> share;
        int32_t first_of_run = 0;
        for (int32_t p = 0; p < (int32_t)wp.size(); ++p) {
            const TileInfo &a = ti[wp[p]], &b = ti[wp[p] + 1];
            bool same_rows = false;
            if (p > 0) {
                const TileInfo &q = ti[wp[p - 1]];
                same_rows = q.kpad == a.kpad && std::equal(br.begin() + a.brow_off, br.begin() + a.brow_off + a.kpad,
                                                           br.begin() + q.brow_off);
            }
            const int32_t chunks = a.kpad / 32;
            const int32_t nseg = std::max(1, (a.kpad + kSeg - 1) / kSeg);
            if (!same_rows) first_of_run = (int32_t)share.size();
            for (int32_t sg = 0; sg < nseg; ++sg) {
                const int64_t c0 = (int64_t)chunks * sg / nseg, c1 = (int64_t)chunks * (sg + 1) / nseg;
                WideSeg w{};
                w.pa = a.panel_off + c0 * 32 * 64;
                w.pb = b.panel_off + c0 * 32 * 64;
                w.br = a.brow_off + c0 * 32;
                w.kp = (int32_t)(32 * (c1 - c0));
                w.slot = (int32_t)bySlot.size();
                w.slot2 = -1;
                if (same_rows)
                    share[first_of_run + sg].push_back(w.slot);
                else
                    share.push_back({w.slot});
                bySlot.push_back(w);
            }
            // then the segments of the pair's compressed CSR panel (own share groups)
            const int32_t ck = pc.empty() ? 0 : pc[p].k32;
            const int32_t cch = ck / 32, cns = std::max(1, (ck + kSeg - 1) / kSeg);
            for (int32_t sg = 0; ck > 0 && sg < cns; ++sg) {
                const int64_t c0 = (int64_t)cch * sg / cns, c1 = (int64_t)cch * (sg + 1) / cns;
                WideSeg w{};
                w.pa = pc[p].off + c0 * 32 * 64;
                w.pb = pc[p].off + (int64_t)64 * ck + c0 * 32 * 64;
                w.br = pc[p].br + c0 * 32;
                w.kp = (int32_t)(32 * (c1 - c0));
                w.slot = (int32_t)bySlot.size();
                w.slot2 = -1;
                w.pad_ = 1;
                share.push_back({w.slot});
                bySlot.push_back(w);
            }
            pslot.push_back((int32_t)bySlot.size());
        }
        // neighbouring leaves multiply mostly the same operand rows: the pairs,
        // in tree order, go to the XCDs as 8 runs of near-equal work, so that
        // the workgroups an XCD runs at one time share those rows in its L2
        std::vector<int64_t> cost(bySlot.size());
        for (size_t i = 0; i < bySlot.size(); ++i) cost[i] = bySlot[i].kp;
        const std::vector<int32_t> order = xcd_region_order(share, cost);
        H->n_wsegs = (int32_t)bySlot.size();
        H->d_wsegs.upload(bySlot);
        H->n_wseg_blocks = (int32_t)order.size();
        H->d_wseg_order.upload(order);
        H->d_wslot.upload(pslot);
    }
    {
        const int64_t cb = (H->n_cpan > 0 ? (int64_t)(H->d_cvals.n + H->d_cbrow.n * sizeof(int32_t) +
                                                      H->d_cpan.n * sizeof(CsrPanel))
                                          : 0) +
                           (int64_t)(H->d_cvals16.n * sizeof(uint16_t) + H->d_cbrow16.n * sizeof(int32_t));
        H->stats.bytes_total += cb - H->stats.bytes_csr_panels;
        H->stats.bytes_csr_panels = cb;
    }
    int ncu = 0;
    RAD_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, H->device));
    H->n_cu = std::max(1, ncu);
    lowp_prepare_proj(H);
    // signature: FNV-1a over the log2 histogram of tile costs and the shape counts
    std::vector<int64_t> hist(40, 0);
    for (int64_t c : cost) {
        int b = 0;
        while (b < 39 && ((int64_t)1 << b) <= c) ++b;
        hist[b]++;
    }
    hist.push_back(H->n_p1work);
    hist.push_back(H->n_p1red);
    hist.push_back(H->n_inst);
    uint64_t h = 1469598103934665603ull;
    for (int64_t v : hist)
        for (int byte = 0; byte < 8; ++byte) {
            h ^= (uint64_t)((v >> (8 * byte)) & 0xff);
            h *= 1099511628211ull;
        }
    char buf[128];
    std::snprintf(buf, sizeof buf, "dt%d_tiles%d_cu%d_h%016llx", (int)H->dtype, (int)n, H->n_cu,
                  (unsigned long long)h);
    H->sched_sig = buf;
}

}  // namespace rad
