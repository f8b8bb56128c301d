"""Benchmark: sun-RHS radiosity solves/s on one MI355X.

Workload (default): spherical-cap crater, depth/diameter 0.2, rim radius
1 km, ~40,000 facets (seeded jittered grid, lower convex hull); compressed
view-factor matrix at tol 1e-3 with near-field leaves stored as CSR; 1,024
sun directions (elevation U[5, 30] deg, azimuth U[0, 360) deg, seed 1);
E = albedo * Q_dir with albedo 0.3 (insolation with shadows computed on the
GPU, outside the timed region).  One step = the Jacobi solve of
(I - 0.3 F-hat) B = E for all 1,024 right-hand sides to a per-column
relative change of 1e-3.

Prints one JSON line.  Its roofline object covers the dominant kernel (the
fused phase-2 tile product): algorithmic bytes per launch (E and B_old read,
B_new written; the U' rows, near-field values and projected rows T read once)
over the launch time measured with HIP events on the kernel's own stream.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
# the metric's accuracy: relative L2 error per sun column against the FP64 oracle
ACCURACY_TOL = 1e-3


def spread_columns(suns, count):
    """Indices of `count` sun columns spread evenly over the elevation range,
    the lowest and the highest sun included."""
    elev = np.arcsin(np.clip(suns[:, 2], -1.0, 1.0))
    order = np.argsort(elev, kind="stable")
    pick = np.round(np.linspace(0, len(order) - 1, count)).astype(int)
    return sorted(set(int(order[i]) for i in pick))


def roofline(flops, bytes_, ms, peak_tflops, kernel):
    """Roofline record of one kernel launch (or one whole product): the bound
    is the one its arithmetic intensity selects against the chip's peaks."""
    tf = flops / (ms * 1e-3) / 1e12
    gbs = bytes_ / (ms * 1e-3) / 1e9
    intensity = flops / bytes_
    ridge = peak_tflops * 1e12 / (HBM_PEAK_GBS * 1e9)
    if intensity < ridge:
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
    else:
        roof = {"bound": "mfma", "achieved": tf, "peak": peak_tflops, "unit": "TFLOP/s", "frac": tf / peak_tflops}
    roof.update({"traffic": None, "kernel": kernel, "ms_per_launch": ms, "flops_per_launch": flops,
                 "bytes_per_launch": bytes_, "intensity_flop_per_byte": intensity, "ridge_flop_per_byte": ridge,
                 "tflops": tf, "gbs": gbs})
    return roof


def block_counts(st):
    """The compressed operator's structure, so that its shape is visible."""
    return {k: st[k] for k in ("n_leaves", "depth", "n_dense", "n_csr", "n_lowrank", "n_zero", "sum_rank",
                               "max_rank", "nnz_near", "bytes_dense", "bytes_csr", "bytes_lowrank", "bytes_total")}


def single_rhs_leg(G, cols, albedo, rtol):
    """The plain FP64 single-RHS form: the given suns solved one at a time
    (Jacobi, same tolerance and stopping rule), timed; its product kernels
    (k_proj_cols, k_proj_wide, k_tile_gemv, one column) timed on their own;
    and each set against HBM: one iteration must at least read the operator
    and the column vectors (E, B_old read, B_new written: 3 N 8 bytes)."""
    import torch
    N = G.N
    Bt = torch.zeros(N, dtype=torch.float64, device="cuda:0")
    for e in cols[:2]:
        G.solve(e, rho=albedo, rtol=rtol, out=Bt, order="tree")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for e in cols:
        _, inf = G.solve(e, rho=albedo, rtol=rtol, out=Bt, order="tree")
        its.append(int(inf["total_iters"]))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    y = torch.empty_like(Bt)
    for _ in range(3):
        G.matvec(cols[0], out=y, order="tree")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(20):
        G.matvec(cols[0], out=y, order="tree")
    ev1.record()
    torch.cuda.synchronize()
    mv_ms = ev0.elapsed_time(ev1) / 20
    op_bytes = G.stats()["bytes_total"]
    it_bytes = op_bytes + 3 * N * 8
    hbm_ms = sum(its) * it_bytes / (HBM_PEAK_GBS * 1e9) * 1e3 / len(cols)
    solve_ms = 1e3 * dt / len(cols)
    return {"solves_per_s": len(cols) / dt, "iterations": its, "ms_per_solve": solve_ms,
            "hbm_ms_per_solve": hbm_ms, "solve_vs_hbm": solve_ms / hbm_ms,
            "product_ms": mv_ms, "product_gbs": (op_bytes + 2 * N * 8) / (mv_ms * 1e-3) / 1e9,
            "product_frac_hbm": (op_bytes + 2 * N * 8) / (mv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "operator_bytes": op_bytes}


def expansion_bytes(st, N, R, s_bytes):
    """Algorithmic bytes of one launch of the expansion kernel over R columns:
    E, B_old read and B_new written (3 N R s), the U' rows and near-field values
    once, T read once (sum_rank x R)."""
    return (3.0 * N * R * s_bytes + st["lowrank_row_elems"] * s_bytes + st["bytes_dense"] + st["bytes_csr"]
            + st["sum_rank"] * R * s_bytes)


def calib_copy():
    """A plain device copy of known size (1 GiB read, 1 GiB written, three
    times), for scaling hardware byte counters taken in the same run."""
    import torch

    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("calibration copy: 3 x 1 GiB read + 1 GiB written")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measured_traffic(dtype, R, tn):
    """HBM bytes per launch of the dominant kernel from the committed counter
    runs, or None when the kernel's sources (the files holding its device
    code) changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha1()
    for rel in rec["sources"]:
        src = os.path.join(ROOT, rel)
        if not os.path.exists(src):
            return None
        h.update(open(src, "rb").read())
    if h.hexdigest() != rec["sources_sha1"]:
        return None
    if rec["dtype"] != dtype or rec["rhs"] != R or rec.get("tn") != tn:
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_baseline(verts, faces, suns, albedo, B_gpu_cols, cols, S):
    """Time the FP64 CPU reference on a bounded sample: the listed sun columns,
    full mesh, insolation + matrix-free Jacobi to 1e-10."""
    from oracle import reference as ref
    t0 = time.perf_counter()
    fac = ref.Facets(verts, faces)
    Q = ref.insolation(fac, suns[cols], S=S)
    E = albedo * Q
    B, iters = ref.jacobi(lambda X: ref.matvec_free(fac, X), albedo, E, tol=1e-10)
    dt = time.perf_counter() - t0
    return {"value": len(cols) / dt, "unit": "solves/s", "cores": ref.num_threads(), "kind": "oracle",
            "sample": f"{len(cols)} sun columns of the full workload (insolation + FP64 matrix-free "
                      f"Jacobi to 1e-10), {dt:.1f} s"}, col_err(B_gpu_cols, B), B


def col_err(B_gpu, B_ref):
    """Largest relative L2 error over the columns."""
    return max(float(np.linalg.norm(B_gpu[:, k] - B_ref[:, k]) / np.linalg.norm(B_ref[:, k]))
               for k in range(B_ref.shape[1]))


def sampled_row_residual(verts, faces, B_orig, E_orig, rho, rows):
    """Relative residual of the sampled rows of (I - rho F) B = E, with the exact
    FP64 view-factor rows (ray-cast visibility) from the CPU reference."""
    from oracle import reference as ref
    fac = ref.Facets(verts, faces)
    Fr = ref.view_factor_rows(fac, rows, "raycast")
    res = B_orig[rows] - E_orig[rows] - rho * (Fr @ B_orig)
    return float(np.linalg.norm(res) / np.linalg.norm(B_orig[rows]))


def terrain_measure(steps, tol=1e-3, lowp="bf16", rtol=1e-4, inner=3, cpu_rows=6, fp64=True, csr=True):
    """Polar terrain: 256 x 256 DEM (131,072 facets), sun at 1.5 deg elevation
    stepping through 2,880 azimuths (0.125 deg), right-hand sides in batches of
    256; FP32 operator with a 16-bit copy.  Times the sweep of all suns by
    refined 16-bit solves to rtol, by plain FP32 Jacobi, and (fp64) by the
    plain FP64 single-RHS form on the same compressed operator converted to
    FP64; the single-RHS FP32 product on the multi-GB operator; the kernels of
    one iteration; and (csr) the same terrain with CSR near field.  Returns a
    dict."""
    import torch
    from paper_2209_07632_amd import HMatrix
    from synth import DEM_256, dem_mesh, sun_grid_azimuth

    S, albedo, Rb = 1365.0, 0.3, 256
    verts, faces = dem_mesh(DEM_256)
    N = faces.shape[0]
    suns = sun_grid_azimuth(1.5, 2880, 0.125)
    log(f"DEM N={N}; building F-hat tol={tol} f32 + {lowp} copy, near field dense, leaf 128")
    t0 = time.perf_counter()
    H = HMatrix(verts, faces, tol=tol, storage="f32", visibility="raycast", nearfield="dense", leaf_size=128,
                max_rank=256, max_rhs=Rb, lowp=lowp, verbose=True)
    build_s = time.perf_counter() - t0
    st = H.stats()
    log(f"built in {build_s:.1f} s: {st}")
    batches = []
    t0 = time.perf_counter()
    for b0 in range(0, len(suns), Rb):
        sb = suns[b0:b0 + Rb]
        Q = H.insolation(sb, flux=S, order="tree_rmajor")
        batches.append((albedo * Q, torch.zeros_like(Q), sb.shape[0]))
    torch.cuda.synchronize()
    log(f"insolation of {len(suns)} suns: {time.perf_counter() - t0:.2f} s")

    def sweep(refine, rt):
        tot_outer, tot_inner = 0, 0
        for E, B, R in batches:
            _, info = H.solve(E, rho=albedo, rtol=rt, out=B, order="tree_rmajor", R=R, refine=refine,
                              inner_iters=inner, max_iter=200)
            tot_outer += info["total_iters"]
            tot_inner += info["inner_iters"]
        return tot_outer, tot_inner

    tune = H.autotune(Rb, nrep=3)
    log(f"autotuned FP32 launch configuration for R={Rb}: {tune}")
    results = {}
    for name, refine in (("refined_16bit", True), ("fp32_jacobi", False)):
        E, B, R = batches[0]
        H.solve(E, rho=albedo, rtol=rtol, out=B, order="tree_rmajor", R=R, refine=refine, inner_iters=inner,
                max_iter=200)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            outer, inner_n = sweep(refine, rtol)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        results[name] = {"seconds_per_sweep": dt, "solves_per_s": len(suns) / dt, "outer_iters": outer,
                         "inner_iters": inner_n}
        log(f"{name}: {dt:.3f} s per sweep of {len(suns)} suns, {len(suns) / dt:.1f} solves/s, "
            f"outer {outer} inner {inner_n}")
    # the refined sweep last, so B holds its result for the accuracy check
    sweep(True, rtol)
    torch.cuda.synchronize()

    # single right-hand side FP32 product (GEMV path): streaming bound on the operator
    x = torch.rand(N, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        H.matvec(x, out=y, order="tree")
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(10):
        H.matvec(x, out=y, order="tree")
    ev1.record(stream)
    ev1.synchronize()
    mv1_ms = ev0.elapsed_time(ev1) / 10
    op_bytes = st["bytes_dense"] + st["bytes_csr"] + st["bytes_lowrank"]
    mv1_flops = st["flops_per_rhs"]
    roof_mv1 = roofline(mv1_flops, op_bytes + 2 * N * 4, mv1_ms, PEAK_TFLOPS["f32"],
                        "whole single-RHS FP32 H-matvec (k_proj_cols, k_proj_wide, k_tile_gemv, k_gemv_finish) "
                        "on the terrain operator")
    log(f"single-RHS FP32 matvec {mv1_ms:.3f} ms, {roof_mv1['gbs']:.0f} GB/s on a {op_bytes / 1e9:.2f} GB operator")

    ph = H.time_phases(Rb, nrep=10, lowp=True)
    ph32 = H.time_phases(Rb, nrep=5)
    flops = 2.0 * Rb * (st["lowrank_row_elems"] + st["nnz_near"])
    bytes16 = (3.0 * N * Rb * 4 + 2 * st["lowrank_row_elems"] + 2 * st["nnz_near"] + st["sum_rank"] * Rb * 4)
    roof = roofline(flops, bytes16, ph[2], 2500.0,
                    f"BF16 wide expansion (k_tile_mm16s segments on leaf pairs, k_pair_finish, k_tile_mm16w) + dense near field + fused "
                    f"Jacobi update")
    bytes32 = (3.0 * N * Rb * 4 + 4 * st["lowrank_row_elems"] + st["bytes_dense"] + st["sum_rank"] * Rb * 4)
    roof32 = roofline(flops, bytes32, ph32[2], PEAK_TFLOPS["f32"],
                      f"k_tile_mm<float, 1, {tune['tn']}> (FP32 expansion + dense near field + fused Jacobi update)")
    log(f"16-bit phases ms {ph}: {roof['tflops']:.1f} TFLOP/s {roof['gbs']:.0f} GB/s; FP32 phases ms {ph32}")
    out = {
        "workload": f"polar DEM 256x256 N={N} (fBm H=0.8 RMS 30 m + 1.5 km bowl), sun 1.5 deg x 2880 azimuths "
                    f"in batches of {Rb}, tol {tol}, {lowp} operator copy, refinement to {rtol}, albedo {albedo}",
        "N": N, "suns": len(suns), "batch": Rb, "tol": tol, "build_seconds": build_s,
        "hmat_bytes": st["bytes_total"], "hmat_blocks": block_counts(st),
        "max_panel_cols": st["max_panel_cols"], "sweeps": results, "autotune": tune,
        "hmatvec_single_rhs_ms": mv1_ms, "hmatvec_single_rhs_gbs": roof_mv1["gbs"],
        "roofline_single_rhs_hmatvec": roof_mv1,
        "roofline_expansion_16bit": roof, "roofline_expansion_fp32": roof32,
        "phase_ms_16bit": {"projections": ph[0], "split_k_sum": ph[1], "expansion_jacobi": ph[2]},
        "phase_ms_fp32": {"projections": ph32[0], "split_k_sum": ph32[1], "expansion_jacobi": ph32[2]},
    }
    if fp64:
        # the plain FP64 single-RHS form on the same compressed operator: one
        # sun at a time, the same tolerance and stopping rule
        del x, y
        G = H.convert("f64", max_rhs=1)
        E0 = batches[0][0]
        cols = [E0[:, c].double().contiguous() for c in range(16)]
        leg = single_rhs_leg(G, cols, albedo, rtol)
        G.close()
        single64 = leg["solves_per_s"]
        out["fp64_single_rhs_solves_per_s"] = single64
        out["fp64_single_rhs_iterations"] = leg["iterations"]
        out["fp64_single_rhs"] = leg
        log(f"plain FP64 single-RHS: {leg['ms_per_solve']:.2f} ms per solve = {leg['solve_vs_hbm']:.2f} x its HBM "
            f"time; product {leg['product_ms']:.3f} ms ({leg['product_frac_hbm']:.2f} of HBM)")
        out["speedup_refined_vs_fp64_single_rhs"] = results["refined_16bit"]["solves_per_s"] / single64
        out["speedup_fp32_jacobi_vs_fp64_single_rhs"] = results["fp32_jacobi"]["solves_per_s"] / single64
        log(f"plain FP64 single-RHS solves on the same operator: {single64:.1f} solves/s")
    if cpu_rows > 0:
        perm = H.perm()
        E, B, R = batches[0]
        cc = [0, 1]
        Bt = B.double().cpu().numpy()[:, cc]
        Et = E.double().cpu().numpy()[:, cc]
        Bo, Eo = np.empty_like(Bt), np.empty_like(Et)
        Bo[perm], Eo[perm] = Bt, Et
        rows = sorted(np.random.default_rng(3).choice(N, size=cpu_rows, replace=False).tolist())
        log(f"CPU reference rows {rows} ...")
        t0 = time.perf_counter()
        res = sampled_row_residual(verts, faces, Bo, Eo, albedo, rows)
        dt = time.perf_counter() - t0
        from oracle import reference as ref
        out["cpu_baseline"] = {"value": len(rows) / dt, "unit": "exact view-factor rows/s",
                               "cores": ref.num_threads(), "kind": "oracle",
                               "sample": f"{len(rows)} exact FP64 rows with brute-force ray-cast visibility, "
                                         f"{dt:.1f} s"}
        out["sampled_row_residual"] = res
        log(f"sampled-row relative residual of the refined solution vs exact rows: {res:.3e}")
    if csr:
        # Algorithm 4's own near-field form (CSR) on the same terrain: same
        # tree, so the same right-hand sides; FP32 Jacobi sweep, kernels of one
        # iteration and the single-RHS product
        perm = H.perm()
        B_ref = batches[0][1].clone()
        H.close()
        out["csr_near_field"] = terrain_csr_leg(verts, faces, perm, batches, B_ref, steps, tol, rtol, albedo, Rb)
    else:
        H.close()
    return out


def terrain_csr_leg(verts, faces, perm, batches, B_ref, steps, tol, rtol, albedo, Rb):
    """The terrain operator with CSR near field (the byte rule of Algorithm 4
    unforced) and a BF16 copy: refined 16-bit and FP32 Jacobi sweeps of the
    given batches, per-iteration kernels (16-bit and FP32), single-RHS FP32
    product, and the first batch's solution against the dense near-field
    operator's (B_ref, the refined 16-bit sweep)."""
    import torch
    from paper_2209_07632_amd import HMatrix

    N = faces.shape[0]
    log("building the terrain operator with CSR near field (FP32 + BF16 copy)")
    t0 = time.perf_counter()
    H = HMatrix(verts, faces, tol=tol, storage="f32", visibility="raycast", nearfield="csr", leaf_size=128,
                max_rank=256, max_rhs=Rb, lowp="bf16")
    build_s = time.perf_counter() - t0
    st = H.stats()
    log(f"built in {build_s:.1f} s: {st}")
    if not np.array_equal(H.perm(), perm):
        raise RuntimeError("the CSR near-field operator has another tree order")
    tune = H.autotune(Rb, nrep=3)

    def sweep(refine):
        tot = 0
        for E, B, R in batches:
            _, info = H.solve(E, rho=albedo, rtol=rtol, out=B, order="tree_rmajor", R=R, refine=refine,
                              inner_iters=3, max_iter=200)
            tot += info["total_iters"]
        return tot

    nsuns = sum(R for _, _, R in batches)
    sweeps = {}
    for name, refine in (("refined_16bit", True), ("fp32_jacobi", False)):
        sweep(refine)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            iters = sweep(refine)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        sweeps[name] = {"seconds_per_sweep": dt, "solves_per_s": nsuns / dt, "outer_iters": iters}
        log(f"CSR near field, {name}: {dt:.3f} s per sweep, {nsuns / dt:.1f} solves/s ({iters} iterations)")
    B0 = batches[0][1][:, :batches[0][2]].double()
    Br = B_ref[:, :batches[0][2]].double()
    diff = float((torch.linalg.vector_norm(B0 - Br, dim=0) / torch.linalg.vector_norm(Br, dim=0)).max())
    x = torch.rand(N, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        H.matvec(x, out=y, order="tree")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(10):
        H.matvec(x, out=y, order="tree")
    ev1.record()
    torch.cuda.synchronize()
    mv1_ms = ev0.elapsed_time(ev1) / 10
    op_bytes = st["bytes_csr"] + st["bytes_lowrank"] + st["bytes_dense"]
    ph = H.time_phases(Rb, nrep=5)
    ph16 = H.time_phases(Rb, nrep=10, lowp=True)
    flops = 2.0 * Rb * (st["lowrank_row_elems"] + st["nnz_near"])
    H.close()
    log(f"CSR near field: phases FP32 {ph}, 16-bit {ph16}; single-RHS {mv1_ms:.3f} ms; max column difference "
        f"from the dense near-field solve {diff:.2e}")
    return {"build_seconds": build_s, "hmat_blocks": block_counts(st), "bytes_csr_panels": st["bytes_csr_panels"],
            "autotune": tune, "sweeps": sweeps,
            "phase_ms_fp32": {"projections": ph[0], "split_k_sum": ph[1], "expansion_jacobi": ph[2]},
            "phase_ms_16bit": {"projections": ph16[0], "split_k_sum": ph16[1], "expansion_jacobi": ph16[2]},
            "expansion_16bit_tflops": flops / (ph16[2] * 1e-3) / 1e12,
            "expansion_fp32_tflops": flops / (ph[2] * 1e-3) / 1e12,
            "hmatvec_single_rhs_ms": mv1_ms,
            "hmatvec_single_rhs_gbs": (op_bytes + 2 * N * 4) / (mv1_ms * 1e-3) / 1e9,
            "single_rhs_gbs_with_panel_copy": (st["bytes_csr_panels"] + st["bytes_lowrank"] + 2 * N * 4)
            / (mv1_ms * 1e-3) / 1e9,
            "max_col_rel_diff_vs_dense_near_field": diff}


def run_dem(args):
    """The terrain workload as its own JSON line (value: refined sweep solves/s)."""
    m = terrain_measure(args.steps, tol=args.tol, lowp=args.lowp, rtol=args.rtol, inner=args.inner,
                        cpu_rows=0 if args.no_cpu_baseline else args.cpu_rows)
    head = m["sweeps"]["refined_16bit"]
    result = {
        "metric": "sun-RHS radiosity solves/s + H-matvec HBM GB/s at 1e-3 rel err vs plain FP64",
        "value": head["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": 1e3 * head["seconds_per_sweep"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": f"{args.lowp}+f32+f64", "data": "synthetic",
        "config": {"workload": m["workload"], "N": m["N"], "rhs": m["suns"], "batch": m["batch"], "tol": m["tol"]},
        "roofline": m["roofline_expansion_16bit"],
    }
    result.update({k: v for k, v in m.items() if k not in ("workload", "roofline_expansion_16bit")})
    print(json.dumps(result), flush=True)


def cap_leg(verts, faces, suns, albedo, S, R, tol, storage, nearfield, steps, cols, Bref):
    """One more compressed operator of the cap (another eps or precision): its
    build, blocks, solve rate over all R suns, product rate, and its error on
    the oracle's columns."""
    import torch
    from paper_2209_07632_amd import HMatrix
    t0 = time.perf_counter()
    H = HMatrix(verts, faces, tol=tol, storage=storage, nearfield=nearfield, max_rhs=R)
    build_s = time.perf_counter() - t0
    st = H.stats()
    E = albedo * H.insolation(suns, flux=S, order="tree_rmajor")
    B = torch.zeros_like(E)
    H.autotune(R, nrep=3)
    for _ in range(2):
        _, info = H.solve(E, rho=albedo, rtol=1e-3, out=B, order="tree_rmajor", R=R)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, info = H.solve(E, rho=albedo, rtol=1e-3, out=B, order="tree_rmajor", R=R)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    X = torch.rand(E.shape, dtype=E.dtype, device=E.device)
    Y = torch.zeros_like(X)
    for _ in range(3):
        H.matvec(X, out=Y, order="tree_rmajor", R=R)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    ev0.record(stream)
    for _ in range(10):
        H.matvec(X, out=Y, order="tree_rmajor", R=R)
    ev1.record(stream)
    ev1.synchronize()
    mv_ms = ev0.elapsed_time(ev1) / 10
    sb = 8 if storage == "f64" else 4
    mv = roofline(st["flops_per_rhs"] * R,
                  st["bytes_dense"] + st["bytes_csr"] + st["bytes_lowrank"] + 2 * st["n"] * R * sb, mv_ms,
                  PEAK_TFLOPS[storage], f"whole H-matmat, {R} columns")
    out = {"tol": tol, "storage": storage, "build_seconds": build_s, "hmat_blocks": block_counts(st),
           "solves_per_s": R / dt, "ms_per_step": 1e3 * dt, "iterations": info["total_iters"],
           "hmatvec_ms": mv_ms, "hmatvec_gbs": mv["gbs"], "hmatvec_tflops": mv["tflops"],
           "roofline_hmatvec": mv}
    if Bref is not None:
        perm = H.perm()
        Bt = B.double().cpu().numpy()[:, :R]
        Bo = np.empty_like(Bt)
        Bo[perm] = Bt
        out["max_rel_err_vs_fp64"] = col_err(Bo[:, cols], Bref)
    log(f"cap leg tol={tol} {storage}: {out['solves_per_s']:.0f} solves/s, {out['iterations']} iterations, "
        f"matvec {mv_ms:.3f} ms, build {build_s:.1f} s, blocks {out['hmat_blocks']}, "
        f"err {out.get('max_rel_err_vs_fp64')}")
    H.close()
    return out


def run_batch(args):
    """64 independent synthetic craters (fBm terrain + 1.5 km bowl, seeds 0-63,
    5k-60k facets, log-uniform sizes), 64 suns each, all instances behind one
    grouped operator: one step solves all 4,096 right-hand sides."""
    import torch
    from paper_2209_07632_amd import HMatrix
    from paper_2209_07632_amd.rad import ldr_of
    from synth import dem_instance, dem_mesh, instance_sizes, sun_directions

    R, albedo = 64, 0.3
    sizes = instance_sizes()[:args.instances]
    parts, Es, meshes = [], [], []
    t0 = time.perf_counter()
    for k, n in enumerate(sizes):
        v, f = dem_mesh(dem_instance(k, int(n)))
        tb = time.perf_counter()
        H = HMatrix(v, f, tol=args.tol, storage="f32", visibility="raycast", nearfield=args.nearfield,
                    max_rhs=R, max_rank=256)
        suns = sun_directions(R, (5.0, 30.0), seed=1000 + k)
        Es.append(albedo * H.insolation(suns, order="tree_rmajor"))
        parts.append(H)
        meshes.append((v, f))
        log(f"instance {k}: N={f.shape[0]} built in {time.perf_counter() - tb:.1f} s, "
            f"{H.stats()['bytes_total'] / 1e6:.0f} MB")
    build_s = time.perf_counter() - t0
    G = HMatrix.group(parts, R)
    E = torch.zeros((G.N, ldr_of(R)), dtype=torch.float32, device="cuda:0")
    for k, e in enumerate(Es):
        E[int(G.offsets[k]):int(G.offsets[k] + G.sizes[k])] = e
    B = torch.zeros_like(E)
    tune = G.autotune(R, nrep=5)
    log(f"group of {len(parts)} instances, {int(G.sizes.sum())} facets ({G.N} rows): autotuned {tune}")

    def grouped():
        _, info = G.solve(E, rho=albedo, rtol=args.rtol, out=B, order="tree_rmajor", R=R)
        return info

    Bk = [torch.zeros_like(e) for e in Es]

    def separate():
        for H, e, b in zip(parts, Es, Bk):
            H.solve(e, rho=albedo, rtol=args.rtol, out=b, order="tree_rmajor", R=R)

    for _ in range(args.warmup):
        info = grouped()
        separate()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info = grouped()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        separate()
    torch.cuda.synchronize()
    dt_sep = (time.perf_counter() - t0) / args.steps
    nrhs = R * len(parts)
    log(f"grouped: {1e3 * dt:.2f} ms per step ({nrhs / dt:.0f} solves/s, {info['total_iters']} iterations); "
        f"separate: {1e3 * dt_sep:.2f} ms ({nrhs / dt_sep:.0f} solves/s)")
    st = G.stats()
    ph = G.time_phases(R, nrep=20)
    flops = 2.0 * R * (st["lowrank_row_elems"] + st["nnz_near"])
    bytes_ = (3.0 * G.N * R * 4 + st["lowrank_row_elems"] * 4 + st["bytes_dense"] + st["bytes_csr"]
              + st["sum_rank"] * R * 4)
    tf, gbs = flops / (ph[2] * 1e-3) / 1e12, bytes_ / (ph[2] * 1e-3) / 1e9
    peak = PEAK_TFLOPS["f32"]
    intensity, ridge = flops / bytes_, peak * 1e12 / (HBM_PEAK_GBS * 1e9)
    if intensity < ridge:
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
    else:
        roof = {"bound": "mfma", "achieved": tf, "peak": peak, "unit": "TFLOP/s", "frac": tf / peak}
    roof.update({"traffic": None, "kernel": f"k_tile_mm<float, 1, {tune['tn']}> over all instances "
                                            f"({'persistent' if tune['persistent'] else 'flat'} grid)",
                 "ms_per_launch": ph[2], "flops_per_launch": flops, "bytes_per_launch": bytes_,
                 "intensity_flop_per_byte": intensity, "ridge_flop_per_byte": ridge, "tflops": tf, "gbs": gbs})
    result = {
        "metric": "sun-RHS radiosity solves/s + H-matvec HBM GB/s at 1e-3 rel err vs plain FP64",
        "value": nrhs / dt, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * dt, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{len(parts)} uneven terrains (fBm H=0.8 RMS 30 m + 1.5 km bowl, seeds 0-"
                               f"{len(parts) - 1}), {int(G.sizes.min())}-{int(G.sizes.max())} facets, {R} suns each, "
                               f"one grouped operator, tol {args.tol}, near field {args.nearfield}, "
                               f"Jacobi rtol {args.rtol}",
                   "instances": len(parts), "facets": int(G.sizes.sum()), "rhs_per_instance": R, "tol": args.tol},
        "iterations": info["total_iters"], "build_seconds": build_s, "hmat_bytes": st["bytes_total"],
        "separate_solves_per_s": nrhs / dt_sep, "autotune": tune,
        "roofline": roof,
        "phase_ms": {"projections": ph[0], "split_k_sum": ph[1], "expansion_jacobi": ph[2]},
    }
    if not args.no_cpu_baseline:
        k = int(np.argmin(sizes))
        H = parts[k]
        perm = H.perm()
        o, n = int(G.offsets[k]), int(G.sizes[k])
        cols = [0, 1]
        Bt = B[o:o + n].double().cpu().numpy()[:, cols]
        Et = Es[k].double().cpu().numpy()[:, cols]
        Bo, Eo = np.empty_like(Bt), np.empty_like(Et)
        Bo[perm], Eo[perm] = Bt, Et
        rows = sorted(np.random.default_rng(3).choice(n, size=args.cpu_rows, replace=False).tolist())
        t0 = time.perf_counter()
        res = sampled_row_residual(*meshes[k], Bo, Eo, albedo, rows)
        dtc = time.perf_counter() - t0
        from oracle import reference as ref
        result["cpu_baseline"] = {"value": len(rows) / dtc, "unit": "exact view-factor rows/s",
                                  "cores": ref.num_threads(), "kind": "oracle",
                                  "sample": f"{len(rows)} exact FP64 rows (ray-cast visibility) of instance {k} "
                                            f"(N={n}), {dtc:.1f} s"}
        result["sampled_row_residual"] = res
        log(f"sampled-row relative residual of instance {k}: {res:.3e}")
    print(json.dumps(result), flush=True)


def run_terrain_phases(args):
    """Kernel phases (projections, split-K sum, expansion with the fused
    Jacobi update) of the terrain operator at R = 256, 16-bit and FP32, and
    its single-RHS FP32 product: a DEM
    of --dem-n x --dem-n cells of 10 m (the 131k terrain's generator, leaf
    128, ray-cast visibility, dense near field, BF16 copy).  With
    --save-operator the operator is built and written to that file and the
    run ends; with --load-operator it is read from a file written so, which
    keeps the build out of a profiled run."""
    import torch
    from paper_2209_07632_amd import HMatrix
    from synth import DemSpec, dem_mesh

    if args.load_operator:
        H = HMatrix.load(args.load_operator)
        build_s = None
    else:
        verts, faces = dem_mesh(DemSpec(n=args.dem_n, extent=10.0 * args.dem_n, seed=2))
        t0 = time.perf_counter()
        H = HMatrix(verts, faces, tol=args.tol, storage="f32", visibility="raycast",
                    nearfield=args.terrain_nearfield, leaf_size=128, max_rank=256, max_rhs=256, lowp=args.lowp)
        build_s = time.perf_counter() - t0
        if args.save_operator:
            H.save(args.save_operator)
            log(f"built N={H.N} in {build_s:.1f} s, saved to {args.save_operator}")
            return
    dem_n = int(round(np.sqrt(H.N / 2)))  # two triangles per cell
    st0 = H.stats()
    nf = "CSR" if st0["n_csr"] > 0 else "dense"

    X = torch.rand((H.N, 256), dtype=torch.float32, device="cuda:0")
    for _ in range(2):
        H.matvec(X, lowp=True)
    torch.cuda.synchronize()
    ph16 = H.time_phases(256, nrep=max(args.steps, 1), lowp=True)
    ph32 = H.time_phases(256, nrep=max(args.steps // 2, 1))
    st = H.stats()
    # the single-RHS FP32 product (k_proj_cols / k_proj_wide + k_tile_gemv)
    x1 = X[:, 0].contiguous()
    y1 = torch.empty_like(x1)
    for _ in range(3):
        H.matvec(x1, out=y1, order="tree")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(max(args.steps, 1)):
        H.matvec(x1, out=y1, order="tree")
    ev1.record()
    torch.cuda.synchronize()
    mv1 = ev0.elapsed_time(ev1) / max(args.steps, 1)
    if args.calib_copy:
        calib_copy()
    print(json.dumps({"metric": "terrain product phases (ms per launch, R = 256)", "value": sum(ph16), "unit": "ms",
                      "higher_is_better": False, "n_gpus": 1, "dtype": "bf16+f32", "data": "synthetic",
                      "config": {"workload": f"DEM {dem_n}x{dem_n} cells of 10 m, N={H.N}, leaf 128, "
                                             f"tol {args.tol}, {nf} near field", "N": H.N},
                      "phases_16bit_ms": ph16, "phases_fp32_ms": ph32, "single_rhs_fp32_ms": mv1,
                      "single_rhs_fp32_gbs": (st["bytes_dense"] + st["bytes_csr"] + st["bytes_lowrank"] + 2 * H.N * 4)
                      / (mv1 * 1e-3) / 1e9,
                      "build_seconds": build_s, "bytes_csr_panels": st["bytes_csr_panels"],
                      "hmat_blocks": block_counts(st)}), flush=True)


def run_cap_phases(args):
    """Kernels of one Jacobi iteration on the 40k cap's operator at --tol and
    --dtype with --rhs columns (projections, split-K sum, expansion with the
    fused Jacobi update, each timed alone), the whole product and the
    single-RHS product, on random operands in the solver's layout.  With
    --save-operator the operator is built, written there and the run ends;
    with --load-operator it is read back, which keeps the build (many small
    rank-search launches) out of a profiled run."""
    import torch
    from paper_2209_07632_amd import HMatrix
    from paper_2209_07632_amd.rad import ldr_of
    from synth import CAP_LARGE, cap_mesh

    R = args.rhs
    if args.load_operator:
        H = HMatrix.load(args.load_operator, max_rhs=R)
        build_s = None
    else:
        verts, faces = cap_mesh(CAP_LARGE)
        t0 = time.perf_counter()
        H = HMatrix(verts, faces, tol=args.tol, storage=args.dtype, nearfield=args.nearfield, max_rhs=R)
        build_s = time.perf_counter() - t0
        if args.save_operator:
            H.save(args.save_operator)
            log(f"built N={H.N} in {build_s:.1f} s, saved to {args.save_operator}")
            return
    N = H.N
    st = H.stats()
    s_bytes = 8 if H.torch_dtype == torch.float64 else 4
    if args.tn:
        H.set_config(R, args.tn, 0, 1)
        tune = dict(H.get_config(R), ms=0.0)
    else:
        tune = H.autotune(R, nrep=5)
    X = torch.rand((N, ldr_of(R)), dtype=H.torch_dtype, device="cuda:0")
    Y = torch.zeros_like(X)
    nrep = max(args.steps, 1)

    def timed(fn):
        for _ in range(3):
            fn()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(nrep):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / nrep

    mv_ms = timed(lambda: H.matvec(X, out=Y, order="tree_rmajor", R=R))
    x1 = X[:, 0].contiguous()
    y1 = torch.empty_like(x1)
    mv1_ms = timed(lambda: H.matvec(x1, out=y1, order="tree"))
    ph = H.time_phases(R, nrep=nrep)
    op_bytes = st["bytes_dense"] + st["bytes_csr"] + st["bytes_lowrank"]
    p2_bytes = expansion_bytes(st, N, R, s_bytes)
    if args.calib_copy:
        calib_copy()
    print(json.dumps({"metric": "cap operator kernels (ms per launch)", "value": ph[2], "unit": "ms",
                      "higher_is_better": False, "n_gpus": 1, "dtype": args.dtype if not args.load_operator
                      else ("f64" if s_bytes == 8 else "f32"), "data": "synthetic",
                      "config": {"workload": f"spherical-cap crater N={N}, {R} columns, operator "
                                             f"{'read from a file' if args.load_operator else f'tol {args.tol}'}",
                                 "N": N, "rhs": R},
                      "phase_ms": {"projections": ph[0], "split_k_sum": ph[1], "expansion_jacobi": ph[2]},
                      "expansion_bytes": p2_bytes, "expansion_gbs": p2_bytes / (ph[2] * 1e-3) / 1e9,
                      "hmatvec_ms": mv_ms, "hmatvec_gbs": (op_bytes + 2 * N * R * s_bytes) / (mv_ms * 1e-3) / 1e9,
                      "single_rhs_ms": mv1_ms, "single_rhs_gbs": (op_bytes + 2 * N * s_bytes) / (mv1_ms * 1e-3) / 1e9,
                      "operator_bytes": op_bytes, "autotune": tune, "build_seconds": build_s,
                      "hmat_blocks": block_counts(st)}), flush=True)


def run_warm(args):
    """Learned warm start on the 40k-facet cap: POD (64 modes) of the scattered
    radiosity B - E of 512 training suns, a 3 x 256 tanh perceptron from sun
    direction to POD coefficients trained on the GPU, then 2,048 held-out suns
    in batches of 256, each solved cold (B^0 = E) and warm (B^0 = E + Phi c),
    by FP32 Jacobi and by BF16-refined solves, to rtol 1e-3."""
    from paper_2209_07632_amd import HMatrix
    from synth import CAP_LARGE, cap_mesh, sun_directions

    verts, faces = cap_mesh(CAP_LARGE)
    t0 = time.perf_counter()
    H = HMatrix(verts, faces, tol=args.tol, storage="f32", nearfield=args.nearfield, max_rhs=512, lowp="bf16")
    build_s = time.perf_counter() - t0
    warm_measure(H, sun_directions(512, (5.0, 30.0), seed=5), sun_directions(2048, (5.0, 30.0), seed=6),
                 f"spherical-cap crater N={faces.shape[0]}", build_s, args)


def run_warm_dem(args):
    """The learned warm start on a polar terrain: a DEM of --dem-n x --dem-n
    cells of 10 m (512: the 524k-facet terrain; fBm + bowl crater recipe of
    the 131k terrain), ray-cast visibility, CSR near field (Algorithm 4's byte
    rule) with a BF16 copy, leaf 128; suns at 1-3 deg elevation, azimuth
    uniform; otherwise as the cap's warm start."""
    from paper_2209_07632_amd import HMatrix
    from synth import DemSpec, dem_mesh, sun_directions

    n = args.dem_n
    verts, faces = dem_mesh(DemSpec(n=n, extent=10.0 * n, seed=7))
    log(f"DEM {n}x{n}, N={faces.shape[0]}: building F-hat tol={args.tol}, CSR near field, BF16 copy, leaf 128")
    t0 = time.perf_counter()
    H = HMatrix(verts, faces, tol=args.tol, storage="f32", visibility="raycast", nearfield="csr", leaf_size=128,
                max_rank=256, max_rhs=512, lowp="bf16", verbose=True)
    build_s = time.perf_counter() - t0
    log(f"built in {build_s:.1f} s: {H.stats()}")
    warm_measure(H, sun_directions(512, (1.0, 3.0), seed=5), sun_directions(2048, (1.0, 3.0), seed=6),
                 f"polar DEM {n}x{n} cells of 10 m N={faces.shape[0]}, CSR near field", build_s, args)


def warm_measure(H, train, held, label, build_s, args):
    """POD (64 modes) of B - E of the training suns' solves (FP32 Jacobi to
    1e-7), a 3 x 256 x 256 x 256 x 64 tanh perceptron trained on the GPU
    (Adam), then the held-out suns in batches of 256 solved cold and warm by
    FP32 Jacobi and by BF16 refinement to --rtol; prints the JSON line."""
    import torch
    from paper_2209_07632_amd.warmstart import MLP, pod_build, pod_expand, pod_project, sun_features
    from synth import mlp_init

    S, albedo, Rb, m = 1365.0, 0.3, 256, 64
    N = H.N
    st = H.stats()
    t0 = time.perf_counter()
    Et = albedo * H.insolation(train, flux=S, order="tree_rmajor")
    Bt, _ = H.solve(Et, rho=albedo, rtol=1e-7, order="tree_rmajor", R=len(train), max_iter=200)
    Phi, sigma = pod_build((Bt - Et).contiguous(), m, R=len(train))
    sig = torch.from_numpy(sigma).to("cuda:0", torch.float32)
    A = pod_project(Phi, Bt, E=Et, scale=1.0 / sig, R=len(train))
    del Bt, Et
    w = (sig * sig) / (sig * sig).sum()
    sizes = [3, 256, 256, 256, m]
    net = MLP(sizes, mlp_init(sizes, seed=23), compute=args.mlp, max_batch=512)
    hist = net.train(torch.from_numpy(sun_features(train)).to("cuda:0"), A, w, steps=args.train_steps, lr=1e-3)
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t0
    log(f"training data, POD and {args.train_steps} Adam steps: {prep_s:.1f} s; loss {hist[0]:.3e} -> {hist[-1]:.3e}; "
        f"sigma[0..3] {sigma[:4]}")
    batches = []
    for b0 in range(0, len(held), Rb):
        sb = held[b0:b0 + Rb]
        E = albedo * H.insolation(sb, flux=S, order="tree_rmajor")
        batches.append((E, torch.from_numpy(sun_features(sb)).to("cuda:0")))
    Bout = torch.zeros_like(batches[0][0])

    def sweep(warm, refine):
        iters = []
        for E, X in batches:
            guess = None
            if warm:
                C = net.forward(X)
                guess = pod_expand(Phi, C, scale=sig, E=E, out=Bout, R=Rb)
            _, info = H.solve(E, rho=albedo, rtol=args.rtol, out=Bout, order="tree_rmajor", R=Rb, refine=refine,
                              warm=guess, max_iter=100)
            iters.append(info["iters"])
        return np.concatenate(iters)

    res = {}
    for refine in (False, True):
        for warm in (False, True):
            sweep(warm, refine)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                it = sweep(warm, refine)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.steps
            name = ("refined_bf16" if refine else "fp32_jacobi") + ("_warm" if warm else "_cold")
            res[name] = {"solves_per_s": len(held) / dt, "mean_iterations": float(np.mean(it)),
                         "max_iterations": int(np.max(it))}
            log(f"{name}: {len(held) / dt:.0f} solves/s, iterations mean {np.mean(it):.2f} max {np.max(it)}")
    head = res["refined_bf16_warm"]
    result = {
        "metric": "sun-RHS radiosity solves/s + H-matvec HBM GB/s at 1e-3 rel err vs plain FP64",
        "value": head["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": 1e3 * len(held) / head["solves_per_s"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16+f32+f64", "data": "synthetic",
        "config": {"workload": f"{label}: POD {m} modes of {len(train)} training solves, perceptron "
                               f"3x256 ({args.mlp}), {len(held)} held-out suns in batches of {Rb}, rtol {args.rtol}",
                   "N": N, "train": len(train), "held_out": len(held), "modes": m},
        "sweeps": res, "preparation_seconds": prep_s, "build_seconds": build_s,
        "final_training_loss": float(hist[-1]), "hmat_blocks": block_counts(st),
        "bytes_csr_panels": st["bytes_csr_panels"], "roofline": None,
    }
    print(json.dumps(result), flush=True)


def run_ts(args):
    """Time stepping (Algorithm 6) on the 40k-facet cap: 64 scenarios (a sun
    at its own elevation U[5, 30] deg circling once per synodic month), one
    lunation of 0.3-day steps, 20-layer columns of lunar regolith to 1 m
    under every facet, balanced surface with three Newton repeats.  A step of
    the benchmark is the whole lunation for all scenarios; value in
    scenario time steps per second."""
    import torch
    from paper_2209_07632_amd import HMatrix
    from paper_2209_07632_amd.timestep import TimeStepper
    from synth import CAP_LARGE, cap_mesh

    S, albedo, emiss, R, M = 1365.0, 0.12, 0.95, 64, 20
    dt = 0.3 * 86400.0
    n_steps = int(round(29.53 / 0.3))
    k_cond, rhoc = 0.0015, 1.2e6
    w = 1.12 ** np.arange(M)                        # layer thickness grows 12% per layer
    z = np.concatenate([[0.0], np.cumsum(1.0 * w / w.sum())])
    verts, faces = cap_mesh(CAP_LARGE)
    N = faces.shape[0]
    H = HMatrix(verts, faces, tol=args.tol, storage=args.dtype, nearfield=args.nearfield, max_rhs=2 * R)
    st = H.stats()
    rng = np.random.default_rng(11)
    el = np.deg2rad(rng.uniform(5.0, 30.0, R))
    az0 = rng.uniform(0.0, 2.0 * np.pi, R)
    dtype = torch.float64 if args.dtype == "f64" else torch.float32
    # every level's direct insolation written by rad_insolation straight into
    # the stepper's internal layout (tree order, scenarios contiguous)
    from paper_2209_07632_amd.rad import ldr_of
    ld = ldr_of(R)
    Q = torch.zeros((n_steps + 1, N, ld), dtype=dtype, device="cuda:0")
    t0 = time.perf_counter()
    for lvl in range(n_steps + 1):
        az = az0 + 2.0 * np.pi * lvl / n_steps
        suns = np.column_stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)])
        H.insolation(suns, flux=S, order="tree_rmajor", out=Q[lvl])
    torch.cuda.synchronize()
    log(f"cap N={N}: insolation of {n_steps + 1} levels x {R} scenarios in {time.perf_counter() - t0:.1f} s")
    TS = TimeStepper(H, z, k_cond, rhoc, dt, albedo, emiss, bottom_flux=0.0, R=R, surface="balanced", newton=3)
    T0 = torch.full((M + 1, N, ld), 250.0, dtype=torch.float64, device="cuda:0")

    def lunation():
        TS.init(T0, Q[0], order="tree_rmajor")
        TS.step(Q[1:], order="tree_rmajor")

    for _ in range(args.warmup):
        lunation()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lunation()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    Ts = TS.read("T", order="tree_rmajor")[0][:, :R]
    tmin, tmax = float(Ts.min()), float(Ts.max())
    # the two parts of a time step on their own: the 2R-column product and the column kernel
    X = torch.rand((N, 2 * R), dtype=dtype, device="cuda:0")
    Y = torch.empty_like(X)
    for _ in range(3):
        H.matvec(X, out=Y)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(10):
        H.matvec(X, out=Y)
    ev1.record(stream)
    ev1.synchronize()
    mv_ms = ev0.elapsed_time(ev1) / 10
    col_ms = TS.time_column(20)
    s = 8 if args.dtype == "f64" else 4
    # per column and step: the M + 1 node temperatures read and written (FP64),
    # Q_abs and Q_rad read and written (FP64), the two product values, Q_dir
    # and the next operand's two values in the matrix precision
    col_bytes = float(N * R * (16 * (M + 1) + 32 + 5 * s))
    roof = roofline(float(N * R * (12 * M + 40)), col_bytes, col_ms, PEAK_TFLOPS["f64"],
                    f"k_ts_column<{'double' if s == 8 else 'float'}> (balanced surface, M = {M})")
    roof["bound"] = "hbm"
    roof["achieved"], roof["peak"], roof["unit"] = roof["gbs"], HBM_PEAK_GBS, "GB/s"
    roof["frac"] = roof["gbs"] / HBM_PEAK_GBS
    result = {
        "metric": "scenario time steps/s (Algorithm 6 with Crank-Nicolson columns)",
        "value": R * n_steps / wall, "unit": "scenario-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": f"{args.dtype}+f64", "data": "synthetic",
        "config": {"workload": f"spherical-cap crater N={N}: {R} scenarios x {n_steps} steps of 0.3 day (one "
                               f"lunation), {M}-layer regolith columns to 1 m, balanced surface, tol {args.tol}",
                   "N": N, "scenarios": R, "levels": n_steps, "layers": M, "dt_s": dt},
        "hmat_blocks": block_counts(st), "product_ms_2R_columns": mv_ms, "column_kernel_ms": col_ms,
        "ms_per_time_step": 1e3 * wall / n_steps, "surface_T_range_K": [tmin, tmax],
        "roofline": roof,
    }
    log(f"lunation {1e3 * wall:.1f} ms ({1e3 * wall / n_steps:.3f} ms per step: product {mv_ms:.3f} ms, "
        f"column kernel {col_ms:.3f} ms = {roof['gbs']:.0f} GB/s); surface T in [{tmin:.1f}, {tmax:.1f}] K")
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="cap40k", choices=["cap40k", "dem131k", "batch64", "warm40k", "warm_dem", "ts40k", "terrain_phases",
                             "cap_phases"])
    ap.add_argument("--mlp", default="f32", choices=["f32", "bf16"])
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--tn", type=int, default=0, help="force the column-tile width (flat grid) instead of autotuning")
    ap.add_argument("--lowp", default="bf16", choices=["f16", "bf16"])
    ap.add_argument("--inner", type=int, default=3)
    ap.add_argument("--cpu-rows", type=int, default=6)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 1,000 for cap40k, whose step is under a millisecond, so that "
                         "host jitter averages out; 50 for the other workloads)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--rhs", type=int, default=1024)
    ap.add_argument("--rtol", type=float, default=1e-3)
    ap.add_argument("--nearfield", default="csr")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cols", type=int, default=8)
    ap.add_argument("--calib-copy", action="store_true", help="add a 1 GiB copy for counter calibration")
    ap.add_argument("--no-extras", action="store_true",
                    help="the cap workload alone (no eps sweep, FP64 leg or terrain keys)")
    ap.add_argument("--dem-n", type=int, default=128, help="terrain_phases: DEM cells per side")
    ap.add_argument("--terrain-nearfield", default="dense", choices=["dense", "csr"],
                    help="terrain_phases: near-field form of the built operator")
    ap.add_argument("--save-operator", default=None, help="terrain_phases, cap_phases: build, write the operator there, stop")
    ap.add_argument("--load-operator", default=None, help="terrain_phases, cap_phases: read the operator from this file")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 1000 if args.workload == "cap40k" else 50
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU runs are not part of it"}))
        sys.exit(2)
    if args.workload == "warm40k":
        return run_warm(args)
    if args.workload == "warm_dem":
        return run_warm_dem(args)
    if args.workload == "ts40k":
        return run_ts(args)
    if args.workload == "terrain_phases":
        return run_terrain_phases(args)
    if args.workload == "cap_phases":
        return run_cap_phases(args)
    if args.workload == "batch64":
        if args.nearfield == "csr":
            args.nearfield = "dense"   # terrain near field: dense panels run far faster than CSR slices
        return run_batch(args)
    if args.workload == "dem131k":
        if args.rtol == 1e-3:
            args.rtol = 1e-4
        return run_dem(args)

    import torch
    from paper_2209_07632_amd import HMatrix
    from synth import CAP_LARGE, cap_mesh, sun_directions

    dev = "cuda:0"
    S, albedo = 1365.0, 0.3
    verts, faces = cap_mesh(CAP_LARGE)
    N = faces.shape[0]
    R = args.rhs
    suns = sun_directions(R, (5.0, 30.0), seed=1)
    log(f"mesh N={N}; building F-hat tol={args.tol} {args.dtype} nearfield={args.nearfield}")
    t0 = time.perf_counter()
    H = HMatrix(verts, faces, tol=args.tol, storage=args.dtype, nearfield=args.nearfield, max_rhs=R,
                verbose=True)
    build_s = time.perf_counter() - t0
    st = H.stats()
    log(f"built in {build_s:.2f} s: {st}")
    # right-hand sides written directly in the library's internal layout
    # (tree order, right-hand-side-minor), where the solve also leaves B
    t0 = time.perf_counter()
    Q = H.insolation(suns, flux=S, order="tree_rmajor")
    torch.cuda.synchronize()
    log(f"insolation {time.perf_counter() - t0:.2f} s")
    E = albedo * Q
    B = torch.zeros_like(E)
    perm = H.perm()
    if args.tn:
        H.set_config(R, args.tn, 0, 1)
        tune = dict(H.get_config(R), ms=0.0)
        log(f"forced launch configuration for R={R}: {tune}")
    else:
        tune = H.autotune(R, nrep=5)
        log(f"autotuned launch configuration for R={R}: {tune}")

    # iteration launches: replayed graphs or direct launches (the solve keeps one
    # iteration queued ahead of the host either way); the faster one is kept
    use_graph = True

    def step():
        _, info = H.solve(E, rho=albedo, rtol=args.rtol, out=B, order="tree_rmajor", R=R, use_graph=use_graph)
        return info

    # (both modes warmed first, then timed alternately four times; the best
    # timing of each mode counts, so clock ramp-up does not decide.  Direct
    # launches spend more host time per step, which varies more between
    # steps and boxes: they are kept only when at least 3% faster)
    mode_ms = {True: float("inf"), False: float("inf")}
    for g in (True, False):
        use_graph = g
        for _ in range(max(1, args.warmup)):
            info = step()
    for _ in range(4):
        for g in (True, False):
            use_graph = g
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(8):
                step()
            torch.cuda.synchronize()
            mode_ms[g] = min(mode_ms[g], 1e3 * (time.perf_counter() - t0) / 8)
    use_graph = not (mode_ms[False] < 0.97 * mode_ms[True])
    for _ in range(args.warmup):
        info = step()
    torch.cuda.synchronize()
    log(f"warmup done, iters {int(info['total_iters'])}; ms/step with graphs {mode_ms[True]:.3f}, "
        f"direct launches {mode_ms[False]:.3f}: use_graph={use_graph}")
    # (Python's collector is paused over the timed steps, as timeit does; two
    # untimed steps right before the clock starts keep the GPU from idling
    # between the log line and the timed region)
    gc.collect()
    gc.disable()
    for _ in range(2):
        info = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gc.enable()
    ms_per_step = 1e3 * dt / args.steps
    solves_per_s = R * args.steps / dt
    iters = int(info["total_iters"])
    log(f"{ms_per_step:.3f} ms/step, {solves_per_s:.1f} solves/s, {iters} iterations")

    # H-matvec timing (tree order, all R columns) with events on the launch stream
    X = torch.rand(E.shape, dtype=E.dtype, device=dev)
    Y = torch.zeros_like(X)
    for _ in range(3):
        H.matvec(X, out=Y, order="tree_rmajor", R=R)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nrep = 20
    ev0.record(stream)
    for _ in range(nrep):
        H.matvec(X, out=Y, order="tree_rmajor", R=R)
    ev1.record(stream)
    ev1.synchronize()
    mv_ms = ev0.elapsed_time(ev1) / nrep
    s_bytes = 8 if args.dtype == "f64" else 4
    alg_bytes = st["bytes_dense"] + st["bytes_csr"] + st["bytes_lowrank"] + 2 * N * R * s_bytes
    alg_flops = st["flops_per_rhs"] * R
    gbs = alg_bytes / (mv_ms * 1e-3) / 1e9
    tflops = alg_flops / (mv_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.dtype]
    log(f"matvec {mv_ms:.3f} ms: {gbs:.1f} GB/s, {tflops:.2f} TFLOP/s")

    # dominant kernel of a solve iteration, timed alone with HIP events on the
    # stream it is launched on: expansion + near field + fused Jacobi update
    ph = H.time_phases(R, nrep=20)
    # algorithmic work of one launch of the expansion kernel (R columns):
    # flops 2 R (sum_LR m k + nnz_near); bytes: E, B_old read and B_new written
    # (3 N R s), the U' rows and near-field values once, T read once (sum_rank x R)
    p2_flops = 2.0 * R * (st["lowrank_row_elems"] + st["nnz_near"])
    p2_bytes = expansion_bytes(st, N, R, s_bytes)
    p1_flops = 2.0 * R * st["lowrank_col_elems"]
    p2_tf = p2_flops / (ph[2] * 1e-3) / 1e12
    p2_gbs = p2_bytes / (ph[2] * 1e-3) / 1e9
    p1_tf = p1_flops / (ph[0] * 1e-3) / 1e12 if ph[0] > 0 else 0.0
    intensity = p2_flops / p2_bytes
    ridge = peak * 1e12 / (HBM_PEAK_GBS * 1e9)
    if intensity < ridge:
        roof = {"bound": "hbm", "achieved": p2_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": p2_gbs / HBM_PEAK_GBS}
    else:
        roof = {"bound": "mfma", "achieved": p2_tf, "peak": peak, "unit": "TFLOP/s", "frac": p2_tf / peak}
    roof.update({"traffic": measured_traffic(args.dtype, R, tune["tn"]),
                 "kernel": f"k_tile_mm<{'double' if args.dtype == 'f64' else 'float'}, 1, {tune['tn']}> "
                           f"(expansion + near field + fused Jacobi update, "
                           f"{'persistent' if tune['persistent'] else 'flat'} grid)",
                 "ms_per_launch": ph[2], "flops_per_launch": p2_flops, "bytes_per_launch": p2_bytes,
                 "intensity_flop_per_byte": intensity, "ridge_flop_per_byte": ridge,
                 "tflops": p2_tf, "gbs": p2_gbs})
    log(f"phases ms {ph}: expansion {p2_tf:.2f} TFLOP/s {p2_gbs:.0f} GB/s (I={intensity:.1f}), "
        f"projections {p1_tf:.2f} TFLOP/s")
    if args.calib_copy:
        calib_copy()

    result = {
        "metric": "sun-RHS radiosity solves/s + H-matvec HBM GB/s at 1e-3 rel err vs plain FP64",
        "value": solves_per_s, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"spherical-cap crater N={N}, {R} sun RHS, tol {args.tol}, "
                               f"near-field {args.nearfield}, Jacobi rtol {args.rtol}, albedo {albedo}",
                   "N": N, "rhs": R, "tol": args.tol, "nearfield": args.nearfield},
        "iterations": iters,
        "build_seconds": build_s,
        "hmat_bytes": st["bytes_total"],
        "hmatvec_ms": mv_ms, "hmatvec_gbs": gbs, "hmatvec_tflops": tflops,
        "roofline": roof,
        # the whole product Y = F-hat X (both phases, all launches) and the
        # phase-1 projections, each against the peak its intensity selects
        "roofline_hmatvec": roofline(alg_flops, alg_bytes, mv_ms, peak,
                                     f"whole H-matmat, {R} columns (projections, split-K sum, expansion)"),
        "roofline_projections": roofline(
            p1_flops, st["lowrank_col_elems"] * s_bytes + N * R * s_bytes + st["sum_rank"] * R * s_bytes, ph[0],
            peak, f"k_proj_mm<{'double' if args.dtype == 'f64' else 'float'}> (phase-1 split-K projections)"),
        "hmat_blocks": block_counts(st),
        "phase_ms": {"projections": ph[0], "split_k_sum": ph[1], "expansion_jacobi": ph[2]},
        "projections_tflops": p1_tf,
        "autotune": tune,
        "use_graph": use_graph,
    }
    # the plain form the batched solve replaces: FP64 operator, one sun at a
    # time (single-RHS products), same tolerance and stopping rule
    del X, Y
    H64 = HMatrix(verts, faces, tol=args.tol, storage="f64", nearfield=args.nearfield, max_rhs=1)
    cols64 = [E[:, c].double().contiguous() for c in range(16)]
    leg = single_rhs_leg(H64, cols64, albedo, args.rtol)
    del H64
    single64 = leg["solves_per_s"]
    log(f"plain FP64 single-RHS solves: {single64:.1f} solves/s ({len(cols64)} suns one at a time; "
        f"{leg['solve_vs_hbm']:.1f} x the HBM time of its iterations; product {leg['product_ms']:.4f} ms)")
    result["fp64_single_rhs_solves_per_s"] = single64
    result["fp64_single_rhs"] = leg
    result["speedup_vs_fp64_single_rhs"] = solves_per_s / single64
    ok = True
    if not args.no_cpu_baseline:
        cols = spread_columns(suns, args.cpu_cols)
        Bt = B.double().cpu().numpy()[:, :R]
        Bo = np.empty_like(Bt)
        Bo[perm] = Bt
        Bc = Bo[:, cols]
        log(f"CPU reference on sun columns {cols} ...")
        cb, err, Bref = cpu_baseline(verts, faces, suns, albedo, Bc, cols, S)
        result["cpu_baseline"] = cb
        result["max_rel_err_vs_fp64"] = err
        result["accuracy_columns"] = cols
        result["accuracy_tol"] = ACCURACY_TOL
        ok = err <= ACCURACY_TOL
        result["accuracy_ok"] = ok
        log(f"cpu baseline {cb}; GPU vs FP64 reference max rel err {err:.3e} over columns {cols}")
    if not args.no_extras:
        # the other configurations of the measurement, as extra keys of this
        # line: the cap at other tolerances and in FP64 (errors on the oracle's
        # columns above), then the 131k-facet terrain
        Bref_cols = Bref if not args.no_cpu_baseline else None
        cols = spread_columns(suns, args.cpu_cols)
        gc.collect()
        result["eps_sweep"] = [cap_leg(verts, faces, suns, albedo, S, R, t, args.dtype, args.nearfield, 5, cols,
                                       Bref_cols) for t in (1e-2, 1e-4, 1e-5)]
        result["fp64"] = cap_leg(verts, faces, suns, albedo, S, R, args.tol, "f64", args.nearfield, 5, cols,
                                 Bref_cols)
        H.close()
        gc.collect()
        torch.cuda.empty_cache()
        result["dem131k"] = terrain_measure(2, cpu_rows=0 if args.no_cpu_baseline else 2)
    print(json.dumps(result), flush=True)
    if not ok:
        log(f"ACCURACY GATE FAILED: max relative error {result['max_rel_err_vs_fp64']:.3e} > {ACCURACY_TOL}")
        sys.exit(3)


if __name__ == "__main__":
    main()
