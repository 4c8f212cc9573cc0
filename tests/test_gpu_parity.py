"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Neighbour lists and CSR layout must match bit for bit; weights and direct
terms within one FP32 evaluation; propagated radiance and pixels within
|err| <= max(1e-4 |ref|, 1e-5).
"""
from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle
import scenegen
import paper_2404_11894_amd as pg
from tests.gpu_util import (PIX_ABS, PIX_REL, W_ABS, W_REL, assert_within, crop, synthetic)

pytestmark = pytest.mark.gpu


def gpu_render(scene, k, D, g, g_s=None, init="pt", fg=0, schedule=0, shift=0, grid=None):
    paths = pg.DevicePaths(scene, albedo_grid=grid)
    q = pg.params(k=k, D=D, g=g, g_s=g_s, init=init, final_gather=fg, schedule=schedule, cell_shift=shift,
                  flags=pg.PG_FLAG_CHECK)
    img, gr = pg.pg_render(paths, q, graph=True)
    torch.cuda.synchronize()
    return img.cpu().numpy(), {n: t.cpu().numpy() for n, t in gr.items()}


def compare_all(scene, k, img, gr, ref_img, ref, what=""):
    N = scene.n_vertices
    K = min(k, N)
    assert np.array_equal(gr["row_ptr"], np.arange(N + 1, dtype=np.int64) * K), what
    assert np.array_equal(gr["col"].reshape(N, K), ref["col"]), what + " col"
    for name in ("w_ind", "w_ph", "w_env"):
        assert_within(gr[name].reshape(N, K), ref[name], W_REL, W_ABS, f"{what} {name}")
    assert_within(gr["b"], ref["b"], W_REL, W_ABS, f"{what} b")
    assert_within(gr["d_pt"], ref["d_pt"], W_REL, W_ABS, f"{what} d_pt")
    assert_within(gr["lplus"], ref["lplus"], PIX_REL, PIX_ABS, f"{what} lplus")
    assert_within(img, ref_img, PIX_REL, PIX_ABS, f"{what} image")


@pytest.fixture(scope="module")
def tiny():
    return scenegen.generate(scenegen.WORKLOADS["tiny"].scene)


@pytest.mark.parametrize("schedule", [pg.PG_SCHED_TWO_PASS, pg.PG_SCHED_SHIFTED, pg.PG_SCHED_SCATTER])
def test_render_tiny_matches_oracle(tiny, schedule):
    w = scenegen.WORKLOADS["tiny"]
    print(f"tiny N={tiny.n_vertices} schedule={schedule}", flush=True)
    img, gr = gpu_render(tiny, w.k, w.D, w.g, schedule=schedule)
    ref_img, ref = oracle.render(tiny, oracle.params(k=w.k, D=w.D, g=w.g), trace=True)
    compare_all(tiny, w.k, img, gr, ref_img, ref, f"tiny/sched{schedule}")


@pytest.mark.parametrize("init,fg,g_s", [("zero", 0, None), ("pt", 1, None), ("pt", 0, 0.3), ("zero", 1, 0.7)])
def test_render_variants(init, fg, g_s):
    sc = crop("tiny", 32, 32, 2)
    print(f"variant init={init} fg={fg} g_s={g_s} N={sc.n_vertices}", flush=True)
    img, gr = gpu_render(sc, 8, 6, 0.5, g_s=g_s, init=init, fg=fg)
    ref_img, ref = oracle.render(sc, oracle.params(k=8, D=6, g=0.5, g_s=g_s, init=init, final_gather=fg),
                                 trace=True)
    compare_all(sc, 8, img, gr, ref_img, ref, f"{init}/{fg}/{g_s}")


EMIT_L = (3.0, 2.0, 1.0)


@pytest.mark.parametrize("init,fg,schedule", [("pt", 0, pg.PG_SCHED_TWO_PASS), ("zero", 0, pg.PG_SCHED_SHIFTED),
                                              ("zero", 1, pg.PG_SCHED_SCATTER), ("pt", 1, pg.PG_SCHED_TWO_PASS)])
def test_render_with_volume_emission(init, fg, schedule):
    sc = crop("tiny", 32, 32, 2, emit_L=EMIT_L)
    assert (sc.l_emit > 0).any()
    print(f"emission init={init} fg={fg} schedule={schedule} N={sc.n_vertices}", flush=True)
    img, gr = gpu_render(sc, 8, 6, 0.5, init=init, fg=fg, schedule=schedule)
    ref_img, ref = oracle.render(sc, oracle.params(k=8, D=6, g=0.5, init=init, final_gather=fg), trace=True)
    compare_all(sc, 8, img, gr, ref_img, ref, f"emission {init}/{fg}/{schedule}")
    dark, _ = gpu_render(replace(sc, l_emit=None), 8, 6, 0.5, init=init, fg=fg, schedule=schedule)
    assert not np.allclose(img, dark)


@pytest.mark.parametrize("init", ["pt", "zero"])
def test_entry_points_compose_with_emission(init):
    sc = crop("tiny", 24, 24, 2, emit_L=EMIT_L)
    print(f"compose emission init={init} N={sc.n_vertices}", flush=True)
    paths = pg.DevicePaths(sc)
    q = pg.params(k=8, D=5, g=0.5, init=init, flags=pg.PG_FLAG_CHECK)
    rp, col = pg.pg_knn(paths, 8)
    e = pg.pg_edges(paths, q, rp, col)
    lplus = pg.pg_propagate(paths, q, rp, col, e["w_ind"], e["b"], e["lplus0"].clone())
    img = pg.pg_gather(paths, pg.params(k=8, D=5, g=0.5, init=init), rp, col, e["w_ind"], e["d_pt"], lplus)
    torch.cuda.synchronize()
    ref_img, ref = oracle.render(sc, oracle.params(k=8, D=5, g=0.5, init=init), trace=True)
    assert_within(e["b"].cpu().numpy(), ref["b"], W_REL, W_ABS, "b")
    assert_within(e["lplus0"].cpu().numpy(), ref["lplus0"], W_REL, W_ABS, "lplus0")
    assert_within(lplus.cpu().numpy(), ref["lplus"], PIX_REL, PIX_ABS, "lplus")
    assert_within(img.cpu().numpy(), ref_img, PIX_REL, PIX_ABS, "image")


@pytest.mark.parametrize("fg,clusters", [(0, False), (1, False), (0, True)])
def test_render_with_extra_first_vertex_samples(fg, clusters):
    cfg = replace(scenegen.crop_of(scenegen.WORKLOADS["tiny"].scene, 32, 32, 2), extra_samples=4)
    sc = scenegen.generate(cfg)
    assert sc.fb_l_env.shape == (sc.n_paths, 4, 3)
    if clusters:
        sc = replace(sc, cluster_key=scenegen.cluster_keys(sc.n_vertices, 7))
    print(f"extra samples fg={fg} clusters={clusters} N={sc.n_vertices}", flush=True)
    fl = pg.PG_FLAG_CHECK | (pg.PG_FLAG_CLUSTERS if clusters else 0)
    img = pg.pg_render(pg.DevicePaths(sc), pg.params(k=8, D=6, g=0.5, final_gather=fg, flags=fl))
    torch.cuda.synchronize()
    op = oracle.params(k=8, D=6, g=0.5, final_gather=fg, neighbours="clusters" if clusters else "knn")
    ref = oracle.render(sc, op)
    assert_within(img.cpu().numpy(), ref, PIX_REL, PIX_ABS, "extra samples")
    plain = oracle.render(replace(sc, fb_l_sun=None, fb_dir_env=None, fb_l_env=None), op)
    assert not np.allclose(ref, plain)


@pytest.mark.parametrize("fg,clusters,extra", [(0, False, 0), (1, False, 0), (0, True, 0), (0, False, 3)])
def test_render_with_point_light(fg, clusters, extra):
    cfg = replace(scenegen.crop_of(scenegen.WORKLOADS["tiny"].scene, 32, 32, 2), pl_I=(0.4, 0.3, 0.2),
                  extra_samples=extra)
    sc = scenegen.generate(cfg)
    assert sc.l_pl is not None
    if clusters:
        sc = replace(sc, cluster_key=scenegen.cluster_keys(sc.n_vertices, 7))
    print(f"point light fg={fg} clusters={clusters} extra={extra} N={sc.n_vertices}", flush=True)
    op = oracle.params(k=8, D=6, g=0.5, final_gather=fg, neighbours="clusters" if clusters else "knn")
    if clusters:
        fl = pg.PG_FLAG_CHECK | pg.PG_FLAG_CLUSTERS
        img, gr = pg.pg_render(pg.DevicePaths(sc), pg.params(k=8, D=6, g=0.5, final_gather=fg, flags=fl), graph=True)
        torch.cuda.synchronize()
        ref_img, ref = oracle.render(sc, op, trace=True)
        assert_within(gr["b"].cpu().numpy(), ref["b"], W_REL, W_ABS, "b")
        assert_within(gr["d_pt"].cpu().numpy(), ref["d_pt"], W_REL, W_ABS, "d_pt")
        assert_within(img.cpu().numpy(), ref_img, PIX_REL, PIX_ABS, "image")
    else:
        img, gr = gpu_render(sc, 8, 6, 0.5, fg=fg)
        ref_img, ref = oracle.render(sc, op, trace=True)
        compare_all(sc, 8, img, gr, ref_img, ref, f"point light {fg}/{extra}")
    dark = oracle.render(replace(sc, dir_pl=None, l_pl=None), op)
    assert not np.allclose(ref_img, dark)


def test_entry_points_compose_with_point_light():
    sc = scenegen.generate(replace(scenegen.crop_of(scenegen.WORKLOADS["tiny"].scene, 24, 24, 2),
                                   pl_I=(0.4, 0.3, 0.2)))
    paths = pg.DevicePaths(sc)
    q = pg.params(k=8, D=4, g=0.5, flags=pg.PG_FLAG_CHECK)
    rp, col = pg.pg_knn(paths, 8)
    e = pg.pg_edges(paths, q, rp, col)
    torch.cuda.synchronize()
    _, ref = oracle.render(sc, oracle.params(k=8, D=4, g=0.5), trace=True)
    assert_within(e["b"].cpu().numpy(), ref["b"], W_REL, W_ABS, "b")
    assert_within(e["d_pt"].cpu().numpy(), ref["d_pt"], W_REL, W_ABS, "d_pt")
    assert_within(e["lplus0"].cpu().numpy(), ref["lplus0"], W_REL, W_ABS, "lplus0")


@pytest.mark.parametrize("k", [1, 2, 5, 12, 16, 33, 64])
def test_neighbour_counts(k):
    sc = crop("tiny", 24, 24, 2)
    print(f"k={k} N={sc.n_vertices}", flush=True)
    img, gr = gpu_render(sc, k, 4, 0.5)
    ref_img, ref = oracle.render(sc, oracle.params(k=k, D=4, g=0.5), trace=True)
    compare_all(sc, k, img, gr, ref_img, ref, f"k={k}")


def test_neighbours_invariant_to_cell_size(tiny):
    ref = None
    for shift in (12, 14, 15, 16, 17, 18, 20):
        print(f"shift={shift}", flush=True)
        paths = pg.DevicePaths(tiny)
        rp, col = pg.pg_knn(paths, 8, shift)
        col = col.cpu().numpy()
        if ref is None:
            ref = oracle.knn(tiny.pos, 8).ravel()
        assert np.array_equal(col, ref), f"shift {shift}"


def test_entry_points_compose(tiny):
    """pg_knn -> pg_edges -> pg_propagate -> pg_gather equals pg_render and the oracle."""
    w = scenegen.WORKLOADS["tiny"]
    paths = pg.DevicePaths(tiny)
    q = pg.params(k=w.k, D=w.D, g=w.g, flags=pg.PG_FLAG_CHECK)
    rp, col = pg.pg_knn(paths, w.k)
    e = pg.pg_edges(paths, q, rp, col)
    lplus = e["lplus0"].clone()
    lplus, traj = pg.pg_propagate(paths, q, rp, col, e["w_ind"], e["b"], lplus, traj=True)
    # pg_gather takes no workspace, so it has no device flag to report through
    img = pg.pg_gather(paths, pg.params(k=w.k, D=w.D, g=w.g), rp, col, e["w_ind"], e["d_pt"], lplus)
    torch.cuda.synchronize()
    ref_img, ref = oracle.render(tiny, oracle.params(k=w.k, D=w.D, g=w.g), trace=True, traj=True)
    N, K = tiny.n_vertices, w.k
    assert np.array_equal(col.cpu().numpy().reshape(N, K), ref["col"])
    assert_within(e["w_ind"].cpu().numpy().reshape(N, K), ref["w_ind"], W_REL, W_ABS, "w_ind")
    assert_within(e["b"].cpu().numpy(), ref["b"], W_REL, W_ABS, "b")
    assert_within(e["lplus0"].cpu().numpy(), ref["lplus0"], W_REL, W_ABS, "lplus0")
    assert_within(traj.cpu().numpy(), ref["traj"][1:], PIX_REL, PIX_ABS, "trajectory")
    assert_within(img.cpu().numpy(), ref_img, PIX_REL, PIX_ABS, "image")
    img2 = pg.pg_render(paths, q)
    torch.cuda.synchronize()
    assert_within(img.cpu().numpy(), img2.cpu().numpy(), 1e-6, 1e-9, "render vs composed")


def test_render_is_deterministic(tiny):
    w = scenegen.WORKLOADS["tiny"]
    a = gpu_render(tiny, w.k, w.D, w.g)
    b = gpu_render(tiny, w.k, w.D, w.g)
    assert np.array_equal(a[0], b[0])
    for n in a[1]:
        assert np.array_equal(a[1][n], b[1][n]), n


def test_albedo_grid_render(tiny):
    rng = np.random.default_rng(2)
    grid = rng.uniform(0.6, 0.99, size=(16, 16, 16)).astype(np.float32)
    w = scenegen.WORKLOADS["tiny"]
    img, gr = gpu_render(tiny, w.k, w.D, w.g, grid=grid)
    alpha = oracle.albedo_from_grid(tiny.pos, grid)
    ref_img, ref = oracle.render(tiny, oracle.params(k=w.k, D=w.D, g=w.g), alpha=alpha, trace=True)
    compare_all(tiny, w.k, img, gr, ref_img, ref, "albedo grid")


# ------------------------------------------------------------ edge cases ---

def test_hand_derived_example():
    from tests.golden.fixtures import load
    sc, d = load("two_paths_isotropic.json")
    for case in d["cases"]:
        img, gr = gpu_render(sc, d["k"], case["D"], d["g"], init=case["init"], fg=case["final_gather"])
        assert gr["col"].reshape(3, 2).tolist() == d["expected_col"]
        assert np.allclose(img[0, :, 1], case["image"], rtol=1e-6), case


def test_no_vertices():
    rng = np.random.default_rng(0)
    P = 4 * 4 * 2
    z = np.zeros((0, 3), np.float32)
    sc = scenegen.Scene(width=4, height=4, spp=2, path_offsets=np.zeros(P + 1, np.int64), pos=z, dir_in=z,
                        dir_out=z, albedo=np.zeros(0, np.float32), l_sun=z, dir_env=z, l_env=z, l_phase=z,
                        e_cam=rng.random((P, 3), dtype=np.float32))
    paths = pg.DevicePaths(sc)
    img = pg.pg_render(paths, pg.params(k=8, D=3, flags=pg.PG_FLAG_CHECK))
    torch.cuda.synchronize()
    assert_within(img.cpu().numpy(), sc.e_cam.reshape(4, 4, 2, 3).mean(2), 1e-6, 1e-7, "empty")


def test_fewer_vertices_than_k():
    rng = np.random.default_rng(1)
    sc = synthetic(rng.random((5, 3)), rng)
    img, gr = gpu_render(sc, 8, 3, 0.4)
    ref_img, ref = oracle.render(sc, oracle.params(k=8, D=3, g=0.4), trace=True)
    compare_all(sc, 8, img, gr, ref_img, ref, "N<k")


def test_duplicate_positions():
    rng = np.random.default_rng(2)
    sc = synthetic(np.full((300, 3), 0.37), rng, lengths=np.full(30, 10))
    img, gr = gpu_render(sc, 8, 5, 0.6)
    ref_img, ref = oracle.render(sc, oracle.params(k=8, D=5, g=0.6), trace=True)
    compare_all(sc, 8, img, gr, ref_img, ref, "duplicates")


@pytest.mark.parametrize("init", ["pt", "zero"])
def test_paths_longer_than_a_wave(init):
    """The path pass takes a path 64 vertices at a time: paths of 1, 41, 64,
    65, 129 and 200 vertices and an empty one; D = 0 compares the initial
    value itself, D = 3 its propagation."""
    rng = np.random.default_rng(9)
    lengths = np.array([200, 1, 64, 65, 129, 0, 41])
    sc = synthetic(rng.random((int(lengths.sum()), 3)), rng, lengths=lengths)
    for D in (0, 3):
        img, gr = gpu_render(sc, 8, D, 0.5, init=init)
        ref_img, ref = oracle.render(sc, oracle.params(k=8, D=D, g=0.5, init=init), trace=True)
        compare_all(sc, 8, img, gr, ref_img, ref, f"long paths init={init} D={D}")


def test_lattice_ties():
    rng = np.random.default_rng(3)
    g = np.array([(x, y, z) for z in range(8) for y in range(8) for x in range(8)], np.float64)
    pos = ((g + 0.5) / 8.0).astype(np.float32)
    sc = synthetic(pos, rng, lengths=np.full(64, 8))
    for k in (7, 19, 27):
        img, gr = gpu_render(sc, k, 4, 0.3)
        ref_img, ref = oracle.render(sc, oracle.params(k=k, D=4, g=0.3), trace=True)
        compare_all(sc, k, img, gr, ref_img, ref, f"lattice k={k}")


def test_exact_search_fallback_matches_fast_path(tiny):
    """The exact (d^2, id) search the fast path hands saturated queries to,
    forced for every query: same neighbours and bit-identical images, and the
    oracle's neighbour lists, on the scene, a tie-heavy lattice and a pile of
    coincident points."""
    rng = np.random.default_rng(9)
    g = np.array([(x, y, z) for z in range(6) for y in range(6) for x in range(6)], np.float64)
    lattice = synthetic(((g + 0.5) / 6.0).astype(np.float32), rng, lengths=np.full(27, 8))
    pile = synthetic(np.concatenate([np.full((120, 3), 0.6), rng.random((40, 3))]), rng, lengths=np.full(16, 10))
    for name, sc, k in (("tiny", tiny, 8), ("lattice", lattice, 19), ("pile", pile, 12)):
        print(f"exact fallback {name} N={sc.n_vertices} k={k}", flush=True)
        paths = pg.DevicePaths(sc)
        fast, gf = pg.pg_render(paths, pg.params(k=k, D=4, g=0.5, flags=pg.PG_FLAG_CHECK), graph=True)
        exact, ge = pg.pg_render(paths, pg.params(k=k, D=4, g=0.5, flags=pg.PG_FLAG_CHECK | pg.PG_FLAG_EXACT_KNN),
                                 graph=True)
        torch.cuda.synchronize()
        assert torch.equal(gf["col"], ge["col"]), name
        assert torch.equal(fast, exact), name
        ref_img, ref = oracle.render(sc, oracle.params(k=k, D=4, g=0.5), trace=True)
        assert np.array_equal(ge["col"].cpu().numpy().reshape(sc.n_vertices, -1), ref["col"]), name


def test_phase_profiler_records_every_phase(tiny):
    """pg_profile_start / pg_profile_stop: HIP events around each phase of a
    render, on the launch stream; every phase of the two-pass schedule shows
    up with its launch count."""
    import ctypes
    L = pg.lib()
    paths = pg.DevicePaths(tiny)
    q = pg.params(k=8, D=5, g=0.5)
    pg.pg_render(paths, q)
    torch.cuda.synchronize()
    assert L.pg_profile_start() == 0
    pg.pg_render(paths, q)
    pg.pg_render(paths, q)
    torch.cuda.synchronize()
    arr = (pg.ProfileEntry * 64)()
    n = ctypes.c_int32()
    assert L.pg_profile_stop(64, arr, ctypes.byref(n)) == 0
    got = {arr[i].name.decode(): (arr[i].count, arr[i].total_ms) for i in range(n.value)}
    for name, count in (("grid", 2), ("knn", 2), ("edges", 2), ("paths", 2), ("spmv", 10), ("shift", 10),
                        ("pixels", 2)):
        assert name in got, (name, sorted(got))
        assert got[name][0] == count and got[name][1] > 0.0, (name, got[name])


def test_device_input_errors_are_reported():
    rng = np.random.default_rng(4)
    sc = synthetic(rng.random((64, 3)), rng, lengths=np.full(8, 8))
    sc.pos[5, 1] = np.nan
    paths = pg.DevicePaths(sc)
    with pytest.raises(pg.PathGraphError) as e:
        pg.pg_render(paths, pg.params(k=4, D=2, flags=pg.PG_FLAG_CHECK))
    assert e.value.code == pg.PG_ERR_INPUT
    sc = synthetic(rng.random((64, 3)), rng, lengths=np.full(8, 8))
    sc.path_offsets[3] = 40   # path 2 = [16, 40), path 3 = [40, 32): not monotone
    paths = pg.DevicePaths(sc)
    with pytest.raises(pg.PathGraphError) as e:
        pg.pg_render(paths, pg.params(k=4, D=2, flags=pg.PG_FLAG_CHECK))
    assert e.value.code == pg.PG_ERR_INPUT
    torch.cuda.synchronize()


@pytest.mark.parametrize("tile,group", [(64, 1), (128, 3), (512, 2), (1024, 1), (256, 16), (256, 5000)])
def test_launch_shape_leaves_results_unchanged(tile, group):
    # workgroup size and the tiles-per-XCD grouping only move work between
    # workgroups: images and L+ equal the default launch bit for bit, also
    # where the row count leaves a partial chunk of tiles
    sc = crop("tiny", 40, 40, 4)
    paths = pg.DevicePaths(sc)
    out = []
    for t, g in ((0, 0), (tile, group)):
        r = pg.Renderer(paths, pg.params(k=12, D=7, g=0.5, tile=t, tile_group=g, flags=pg.PG_FLAG_CHECK))
        lp = torch.empty(sc.n_vertices, 3, device="cuda")
        img = r(graph={"lplus": lp})
        torch.cuda.synchronize()
        out.append((img.cpu(), lp.cpu()))
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])


def test_compact_ids_equal_full_ids_on_a_graph_with_far_neighbours():
    # 0.5M vertices of the benchmark's ball: in the spatially sorted order some
    # neighbours lie more than 32767 rows away, so the two-pass aggregation's
    # 16-bit ids take the escape list there.  The scatter schedule reads the
    # full 32-bit ids with the same row sums: images and L+ bit for bit.
    sc = crop("mid", 160, 160, 4)
    assert sc.n_vertices > 200_000
    paths = pg.DevicePaths(sc)
    out = []
    for sched in (pg.PG_SCHED_TWO_PASS, pg.PG_SCHED_SCATTER):
        r = pg.Renderer(paths, pg.params(k=16, D=6, g=0.8, schedule=sched, flags=pg.PG_FLAG_CHECK))
        lp = torch.empty(sc.n_vertices, 3, device="cuda")
        img = r(graph={"lplus": lp})
        torch.cuda.synchronize()
        out.append((img.cpu(), lp.cpu()))
        del r
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
