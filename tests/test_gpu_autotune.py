"""Launch configurations of the multi-RHS kernels (64/128-column tiles, flat
or persistent work-queue grids) and the autotuner that picks among them:
every configuration gives the same products, solves and graph replays."""
import json

import numpy as np
import pytest

from synth import CAP_SMALL, CapSpec, cap_mesh, dem_instance, dem_mesh, sun_directions

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
CONFIGS = [(tn, 0, 1) for tn in (64, 128)] + [(tn, 1, b) for tn in (64, 128) for b in (1, 2, 4)]


def _hm(verts, faces, **kw):
    from paper_2209_07632_amd import HMatrix
    print(f"[build] N={faces.shape[0]} {kw}", flush=True)
    return HMatrix(verts, faces, **kw)


@pytest.mark.parametrize("storage", ["f32", "f64"])
@pytest.mark.parametrize("R", [37, 130])
def test_every_configuration_gives_the_same_product(storage, R):
    from paper_2209_07632_amd.rad import ldr_of
    verts, faces = cap_mesh(CAP_SMALL)
    H = _hm(verts, faces, tol=1e-4, storage=storage, nearfield="csr", max_rhs=R)
    dt = torch.float64 if storage == "f64" else torch.float32
    X = torch.from_numpy(np.random.default_rng(R).random((H.N, ldr_of(R)))).to(DEV, dt)
    assert H.get_config(R)["tn"] == (64 if R <= 64 else 128)
    Y0 = H.matvec(X, order="tree_rmajor", R=R)
    for tn, pe, bpc in CONFIGS:
        print(f"[config] tn={tn} persistent={pe} blocks_per_cu={bpc}", flush=True)
        H.set_config(R, tn, pe, bpc)
        for _ in range(2):                      # the work counter resets itself
            Y = H.matvec(X, order="tree_rmajor", R=R)
            assert torch.equal(Y[:, :R], Y0[:, :R]), (tn, pe, bpc)


def test_group_configurations_and_graph_replays():
    """Persistent grids over a group of uneven instances, replayed from cached
    graphs with eager work in between, equal the eager flat-grid solve."""
    from paper_2209_07632_amd import HMatrix
    from paper_2209_07632_amd.rad import ldr_of
    R = 64
    meshes = [cap_mesh(CapSpec(h=h, seed=s)) for h, s in ((150.0, 1), (80.0, 2))]
    meshes += [dem_mesh(dem_instance(7, 1500))]
    parts = [_hm(v, f, tol=1e-5, storage="f32", max_rhs=R, leaf_size=32,
                 visibility="raycast" if i == 2 else "backface") for i, (v, f) in enumerate(meshes)]
    G = HMatrix.group(parts, R)
    E = torch.zeros((G.N, ldr_of(R)), dtype=torch.float32, device=DEV)
    for k, p in enumerate(parts):
        o, n = int(G.offsets[k]), int(G.sizes[k])
        E[o:o + n] = 0.3 * p.insolation(sun_directions(R, seed=k), order="tree_rmajor")
    G.set_config(R, 128, 0, 1)
    B0, i0 = G.solve(E, rho=0.3, rtol=1e-6, order="tree_rmajor", R=R, use_graph=False)
    for tn, pe, bpc in [(128, 1, 2), (64, 1, 4), (64, 0, 1)]:
        G.set_config(R, tn, pe, bpc)
        for rep in range(3):
            B, info = G.solve(E, rho=0.3, rtol=1e-6, order="tree_rmajor", R=R, use_graph=True)
            if tn == 128:
                assert torch.equal(B, B0)
                np.testing.assert_array_equal(info["iters"], i0["iters"])
            else:
                assert torch.allclose(B, B0, rtol=1e-5, atol=1e-5 * float(B0.abs().max()))
            G.matvec(E, order="tree_rmajor", R=R)
            torch.cuda.synchronize()


def test_autotune_picks_a_candidate_and_caches_it(tmp_path):
    verts, faces = cap_mesh(CAP_SMALL)
    R = 96
    cache = tmp_path / "tune.json"
    H = _hm(verts, faces, tol=1e-4, storage="f32", max_rhs=R)
    res = H.autotune(R, nrep=3, cache=cache)
    print("tuned", res)
    assert (res["tn"], res["persistent"], res["blocks_per_cu"]) in [(a, b, c if b else 0) for a, b, c in CONFIGS]
    assert res["ms"] > 0
    entries = json.loads(cache.read_text())
    assert len(entries) == 1 and list(entries.values())[0]["tn"] == res["tn"]
    # a second matrix of the same shape reads the cache instead of timing
    H2 = _hm(verts, faces, tol=1e-4, storage="f32", max_rhs=R)
    res2 = H2.autotune(R, nrep=3, cache=cache)
    assert res2["ms"] == 0.0
    assert {k: res2[k] for k in ("tn", "persistent")} == {k: res[k] for k in ("tn", "persistent")}
    assert H2.get_config(R)["tn"] == res["tn"]
