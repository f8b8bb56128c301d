// Groups of independent compressed matrices behind one operator.
//
// A group is the block-diagonal union of K built matrices: instance k's
// facets occupy rows [off_k, off_k + N_k) of the group's tree-ordered,
// right-hand-side-minor layout, with off_k a multiple of 64 so that every
// 64-row tile belongs to one instance.  All tile, panel, projection and CSR
// tables are concatenated with their offsets remapped, so one launch of each
// multi-RHS kernel covers every block of every instance (uneven ranks and
// sizes included).  The value pool keeps the single-matrix layout: the
// panels and stacked V factors of all instances first (each instance's
// region starting on a 64-element boundary), then all CSR values, parallel
// to the concatenated CSR column indices.
#include <algorithm>
#include <cstring>

#include "rad_internal.h"

namespace rad {

namespace {

int64_t round64(int64_t v) { return (v + 63) / 64 * 64; }

int dsize(int32_t dt) { return dt == RAD_F64 ? 8 : dt == RAD_F32 ? 4 : 2; }

}  // namespace

}  // namespace rad

using namespace rad;

extern "C" rad_status rad_hmat_group(const rad_hmat *const *parts, int32_t count, int32_t max_rhs, rad_hmat **out) {
    if (out) *out = nullptr;
    rad_hmat *G = nullptr;
    rad_status st = guard([&] {
        RAD_REQUIRE(out && parts, "null parts or out");
        RAD_REQUIRE(count >= 1, "count must be >= 1");
        RAD_REQUIRE(max_rhs >= kMfmaMinRhs, "a group needs max_rhs >= 16");
        for (int k = 0; k < count; ++k) {
            RAD_REQUIRE(parts[k] != nullptr, "null matrix in parts");
            RAD_REQUIRE(parts[k]->n_inst == 1, "parts must not be groups");
            RAD_REQUIRE(parts[k]->device == parts[0]->device, "parts must live on one device");
            RAD_REQUIRE(parts[k]->dtype == parts[0]->dtype, "parts must share the dtype");
            RAD_REQUIRE(parts[k]->lowp == parts[0]->lowp, "parts must share the 16-bit copy setting");
        }
        const rad_hmat &P0 = *parts[0];
        RAD_HIP(hipSetDevice(P0.device));
        const size_t es = (size_t)dsize(P0.dtype);
        G = new rad_hmat();
        G->allocator = P0.allocator;   // the parts' hook (if any) also serves the group
        AllocScope scope(G->hook(), P0.device);
        G->device = P0.device;
        G->dtype = P0.dtype;
        G->lowp = P0.lowp;
        G->max_rhs = max_rhs;
        G->n_inst = count;

        // offsets of every table, per instance
        int64_t rows = 0, pre = 0, csr = 0, brow = 0, ptr = 0;
        int32_t tiles = 0, tasks = 0, groups = 0, work = 0, red = 0, partn = 0, trows = 0;
        struct Off {
            int64_t row, pre, csr, brow, ptr;
            int32_t tile, task, group, work, red, part, trow;
        };
        std::vector<Off> off(count);
        for (int k = 0; k < count; ++k) {
            const rad_hmat &P = *parts[k];
            off[k] = {rows, pre, csr, brow, ptr, tiles, tasks, groups, work, red, partn, trows};
            G->inst_off.push_back(rows);
            G->inst_n.push_back(P.N);
            G->inst_tile.push_back(tiles);
            rows += round64(P.N);
            pre += round64(P.csr_val_start);
            csr += (int64_t)(P.d_vals.bytes() / es) - P.csr_val_start;
            brow += (int64_t)P.d_brow.n;
            ptr += (int64_t)P.d_csr_ptr.n;
            tiles += P.n_tiles;
            tasks += (int32_t)P.d_tile_tasks.n;
            groups += P.n_groups;
            work += P.n_p1work;
            red += P.n_p1red;
            partn += P.n_parts;
            trows += P.t_rows;
        }
        G->inst_tile.push_back(tiles);
        RAD_REQUIRE(rows < ((int64_t)1 << 31), "group exceeds 2^31 rows");
        G->N = rows;
        G->n_tiles = tiles;
        G->n_groups = groups;
        G->n_p1work = work;
        G->n_p1red = red;
        G->n_parts = partn;
        G->t_rows = trows;
        G->t_ld = std::max<int32_t>((trows + 3) & ~3, 4);
        G->csr_val_start = pre;

        // value pool, CSR indices and row pointers, 16-bit copy
        G->d_vals.alloc((size_t)std::max<int64_t>(pre + csr, 1) * es);
        RAD_HIP(hipMemset(G->d_vals.p, 0, G->d_vals.bytes()));
        G->d_csr_idx.alloc((size_t)std::max<int64_t>(csr, 1));
        if (ptr > 0) G->d_csr_ptr.alloc((size_t)ptr);
        if (G->lowp) {
            G->d_vals16.alloc((size_t)std::max<int64_t>(pre + csr, 1));
            RAD_HIP(hipMemset(G->d_vals16.p, 0, G->d_vals16.bytes()));
            G->d_pscale.alloc((size_t)std::max<int64_t>(pre / 64 + 1, 1));
            G->d_tscale.alloc((size_t)std::max<int32_t>(trows, 1));
        }
        for (int k = 0; k < count; ++k) {
            const rad_hmat &P = *parts[k];
            const int64_t ncsr = (int64_t)(P.d_vals.bytes() / es) - P.csr_val_start;
            if (P.csr_val_start > 0)
                RAD_HIP(hipMemcpy((char *)G->d_vals.p + off[k].pre * es, P.d_vals.p, P.csr_val_start * es,
                                  hipMemcpyDeviceToDevice));
            if (ncsr > 0) {
                RAD_HIP(hipMemcpy((char *)G->d_vals.p + (pre + off[k].csr) * es,
                                  (const char *)P.d_vals.p + P.csr_val_start * es, ncsr * es,
                                  hipMemcpyDeviceToDevice));
                RAD_HIP(hipMemcpy(G->d_csr_idx.p + off[k].csr, P.d_csr_idx.p, ncsr * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice));
            }
            if (P.d_csr_ptr.n > 0)
                RAD_HIP(hipMemcpy(G->d_csr_ptr.p + off[k].ptr, P.d_csr_ptr.p, P.d_csr_ptr.bytes(),
                                  hipMemcpyDeviceToDevice));
            if (G->lowp) {
                if (P.csr_val_start > 0) {
                    RAD_HIP(hipMemcpy(G->d_vals16.p + off[k].pre, P.d_vals16.p, P.csr_val_start * sizeof(uint16_t),
                                      hipMemcpyDeviceToDevice));
                    RAD_HIP(hipMemcpy(G->d_pscale.p + off[k].pre / 64, P.d_pscale.p,
                                      (size_t)(P.csr_val_start / 64) * sizeof(float), hipMemcpyDeviceToDevice));
                }
                if (P.t_rows > 0)
                    RAD_HIP(hipMemcpy(G->d_tscale.p + off[k].trow, P.d_tscale.p, (size_t)P.t_rows * sizeof(float),
                                      hipMemcpyDeviceToDevice));
            }
        }

        // tables, remapped
        std::vector<ProjGroup> vg;
        std::vector<TileInfo> vt;
        std::vector<int32_t> vb;
        std::vector<TileTask> vk;
        std::vector<P1Work> vw;
        std::vector<P1Red> vr;
        std::vector<int32_t> perm;
        for (int k = 0; k < count; ++k) {
            const rad_hmat &P = *parts[k];
            const Off &o = off[k];
            auto map_val = [&](int64_t v) {
                return v < P.csr_val_start ? o.pre + v : pre + o.csr + (v - P.csr_val_start);
            };
            for (ProjGroup g : P.h_groups) {
                g.j0 += (int32_t)o.row;
                g.v_off = map_val(g.v_off);
                g.t_off += o.trow;
                vg.push_back(g);
            }
            for (TileInfo t : P.d_tiles.download(P.n_tiles)) {
                if (t.kpad > 0) t.panel_off = map_val(t.panel_off);
                t.brow_off += o.brow;
                t.csr_begin += o.task;
                t.csr_end += o.task;
                vt.push_back(t);
            }
            for (int32_t v : P.d_brow.download(P.d_brow.n))
                vb.push_back(v >= 0 ? v + (int32_t)o.row : -1 - ((-1 - v) + o.trow));
            for (TileTask t : P.d_tile_tasks.download(P.d_tile_tasks.n)) {
                t.col0 += (int32_t)o.row;
                t.a_off = map_val(t.a_off);
                t.aux_off += o.ptr;
                vk.push_back(t);
            }
            for (P1Work w : P.d_p1work.download(P.n_p1work)) {
                w.group += o.group;
                w.part += o.part;
                vw.push_back(w);
            }
            for (P1Red r : P.d_p1red.download(P.n_p1red)) {
                r.t_row0 += o.trow;
                r.part_begin += o.part;
                vr.push_back(r);
            }
            for (int64_t t = 0; t < round64(P.N); ++t)
                perm.push_back((int32_t)(o.row + (t < P.N ? P.perm[t] : t)));
        }
        G->h_groups = vg;
        G->d_groups.upload(vg);
        G->d_tiles.upload(vt);
        G->d_brow.upload(vb);
        G->d_tile_tasks.upload(vk);
        G->d_p1work.upload(vw);
        G->d_p1red.upload(vr);
        G->perm = perm;
        G->d_perm.upload(perm);
        G->d_inst_tile.upload(G->inst_tile);

        // statistics: sums over the instances
        rad_hmat_stats &S = G->stats;
        S.dtype = G->dtype;
        for (int k = 0; k < count; ++k) {
            const rad_hmat_stats &p = parts[k]->stats;
            S.n += p.n;
            S.n_leaves += p.n_leaves;
            S.depth = std::max(S.depth, p.depth);
            S.n_dense += p.n_dense;
            S.n_csr += p.n_csr;
            S.n_lowrank += p.n_lowrank;
            S.n_zero += p.n_zero;
            S.bytes_dense += p.bytes_dense;
            S.bytes_csr += p.bytes_csr;
            S.bytes_lowrank += p.bytes_lowrank;
            S.nnz_near += p.nnz_near;
            S.sum_rank += p.sum_rank;
            S.lowrank_elems += p.lowrank_elems;
            S.max_rank = std::max(S.max_rank, p.max_rank);
            S.build_seconds += p.build_seconds;
            S.flops_per_rhs += p.flops_per_rhs;
            S.lowrank_row_elems += p.lowrank_row_elems;
            S.lowrank_col_elems += p.lowrank_col_elems;
            S.max_panel_cols = std::max(S.max_panel_cols, p.max_panel_cols);
        }
        S.bytes_total = (int64_t)(G->d_vals.bytes() + G->d_csr_idx.bytes() + G->d_csr_ptr.bytes() +
                                  G->d_tiles.bytes() + G->d_brow.bytes() + G->d_tile_tasks.bytes() +
                                  G->d_groups.bytes() + G->d_p1work.bytes() + G->d_p1red.bytes() +
                                  G->d_vals16.bytes() + G->d_pscale.bytes() + G->d_tscale.bytes());
        alloc_workspace(G);
    });
    if (st != RAD_OK) {
        delete G;
        return st;
    }
    *out = G;
    return RAD_OK;
}

extern "C" rad_status rad_hmat_group_layout(const rad_hmat *G, int64_t *offsets, int64_t *sizes) {
    return guard([&] {
        RAD_REQUIRE(G != nullptr, "null matrix handle");
        for (int k = 0; k < G->n_inst; ++k) {
            if (offsets) offsets[k] = G->n_inst > 1 ? G->inst_off[k] : 0;
            if (sizes) sizes[k] = G->n_inst > 1 ? G->inst_n[k] : G->N;
        }
    });
}

extern "C" int32_t rad_hmat_instances(const rad_hmat *H) { return H ? H->n_inst : -1; }
