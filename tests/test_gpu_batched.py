"""Batched rendering of independent scenes: equal to per-scene renders and to
the oracle; a reusable plan (eager or one hipGraph launch) replayed with other
GPU work in between gives the same images every time."""
from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle
import scenegen
import paper_2404_11894_amd as pg
from paper_2404_11894_amd import autotune
from tests.gpu_util import PIX_ABS, PIX_REL, assert_within

pytestmark = pytest.mark.gpu


def small_batch():
    base = scenegen.WORKLOADS["tiny"].scene
    specs = [
        (replace(base, width=24, height=20, spp=2, seed=11), 8, 6, 0.5),
        (replace(base, R=16, sigma_max=12.0, g=-0.2, width=16, height=16, spp=1, max_depth=5, seed=12), 5, 3, -0.2),
        (replace(base, albedo=(0.99, 0.99), g=0.8, width=30, height=18, spp=2, max_depth=12, seed=13), 16, 9, 0.8),
        (replace(base, width=8, height=8, spp=1, look_at=(0.5, 5.0, -3.0), seed=14), 8, 4, 0.5),   # no vertices
        (replace(base, sigma_max=4.0, width=20, height=20, spp=1, seed=15), 12, 0, 0.3),
        (replace(base, width=16, height=24, spp=3, seed=16), 1, 5, 0.5),
        (replace(base, width=20, height=16, spp=2, emit_L=(2.0, 1.5, 1.0), seed=17), 8, 5, 0.5),   # emissive
        (replace(base, width=16, height=16, spp=2, pl_I=(0.4, 0.3, 0.2), extra_samples=2, seed=18), 8, 4, 0.5),
    ]
    scenes, params, oparams = [], [], []
    for cfg, k, D, g in specs:
        scenes.append(scenegen.generate(cfg))
        params.append(pg.params(k=k, D=D, g=g, flags=pg.PG_FLAG_CHECK))
        oparams.append(oracle.params(k=k, D=D, g=g))
    assert scenes[3].n_vertices == 0
    return scenes, params, oparams


def test_batched_equals_per_scene_and_oracle():
    scenes, params, oparams = small_batch()
    paths = [pg.DevicePaths(s) for s in scenes]
    imgs = pg.pg_render_batched(paths, params)
    torch.cuda.synchronize()
    for s, (sc, p, op) in enumerate(zip(scenes, params, oparams)):
        single = pg.pg_render(paths[s], p)
        torch.cuda.synchronize()
        got = imgs[s].cpu().numpy()
        assert np.array_equal(got, single.cpu().numpy()), f"scene {s}"
        assert_within(got, oracle.render(sc, op), PIX_REL, PIX_ABS, f"scene {s} vs oracle")


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_mixes_cluster_and_knn_scenes(use_graph):
    scenes, params, oparams = small_batch()
    for s in (0, 2, 6):   # these use the cluster relation, the others the k nearest
        scenes[s] = replace(scenes[s], cluster_key=scenegen.cluster_keys(scenes[s].n_vertices, 30 + s))
        params[s] = pg.params(k=params[s].k, D=params[s].D, g=params[s].g,
                              flags=pg.PG_FLAG_CHECK | pg.PG_FLAG_CLUSTERS)
        oparams[s] = dict(oparams[s], neighbours="clusters")
    paths = [pg.DevicePaths(sc) for sc in scenes]
    imgs = [im.clone() for im in pg.pg_render_batched(paths, params)]
    torch.cuda.synchronize()
    for s, (sc, p, op) in enumerate(zip(scenes, params, oparams)):
        single = pg.pg_render(paths[s], p)
        torch.cuda.synchronize()
        got = imgs[s].cpu().numpy()
        assert np.array_equal(got, single.cpu().numpy()), f"scene {s}"
        assert_within(got, oracle.render(sc, op), PIX_REL, PIX_ABS, f"scene {s} vs oracle")
    plan = pg.Batch(paths, [pg.params(k=p.k, D=p.D, g=p.g, flags=p.flags & pg.PG_FLAG_CLUSTERS) for p in params],
                    use_graph=use_graph)
    for rep in range(3):
        out = plan()
        torch.cuda.synchronize()
        for s in range(len(scenes)):
            assert torch.equal(out[s], imgs[s]), (rep, s)


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_plan_replays(use_graph):
    scenes, params, _ = small_batch()
    paths = [pg.DevicePaths(s) for s in scenes]
    ref = [im.clone() for im in pg.pg_render_batched(paths, params)]
    plan = pg.Batch(paths, [pg.params(k=p.k, D=p.D, g=p.g) for p in params], use_graph=use_graph)
    other = pg.DevicePaths(scenes[0])
    for rep in range(4):
        out = plan()
        torch.cuda.synchronize()
        for s in range(len(scenes)):
            assert torch.equal(out[s], ref[s]), f"replay {rep} scene {s}"
        # the program's own eager work between replays
        pg.pg_render(other, params[0])
        (torch.rand(1000, device="cuda") * 2).sum().item()
        for im in out:
            im.zero_()
        torch.cuda.synchronize()
    plan.close()


def test_tuned_cell_size_leaves_results_unchanged():
    scenes, params, _ = small_batch()
    paths = [pg.DevicePaths(s) for s in scenes]
    ref = pg.pg_render_batched(paths, params)
    tuned = []
    for pth, p in zip(paths, params):
        q = pg.params(k=p.k, D=p.D, g=p.g, cell_shift=autotune.tune_cell_shift(pth, p.k) if pth.n_vertices else 0)
        tuned.append(q)
    alt = [pg.params(k=p.k, D=p.D, g=p.g, cell_shift=14) for p in params]
    # the batch's edge tile: workgroup size and tiles per XCD of the batched iterations
    tiles = [pg.params(k=p.k, D=p.D, g=p.g, tile=t, tile_group=grp)
             for p, (t, grp) in zip(params, [(128, 3)] * len(params))]
    tiles2 = [pg.params(k=p.k, D=p.D, g=p.g, tile=1024, tile_group=2) for p in params]
    for qs in (tuned, alt, tiles, tiles2):
        out = pg.pg_render_batched(paths, qs)
        torch.cuda.synchronize()
        for s in range(len(scenes)):
            assert torch.equal(out[s], ref[s]), f"scene {s}"


def test_autotuned_batch_plan_leaves_results_unchanged():
    scenes, params, _ = small_batch()
    paths = [pg.DevicePaths(s) for s in scenes]
    ref = [im.clone() for im in pg.pg_render_batched(paths, params)]
    plan = pg.Batch(paths, [pg.params(k=p.k, D=p.D, g=p.g) for p in params], use_graph=True, tune=True)
    assert plan.tuned is not None and plan.tuned["tile"] in autotune.TILES + (256,)
    out = plan()
    torch.cuda.synchronize()
    for s in range(len(scenes)):
        assert torch.equal(out[s], ref[s]), f"scene {s}"
    plan.close()
    # the tuner itself on a scene large enough to time its propagation
    sc = scenegen.generate(scenegen.crop_of(scenegen.WORKLOADS["mid"].scene, 64, 64, 4))
    p = pg.DevicePaths(sc)
    t = autotune.tune(p, 16, 0.8, probe_D=2)
    assert t["tile"] in autotune.TILES and t["tile_group"] in autotune.GROUPS and 11 <= t["cell_shift"] <= 20
    a = pg.pg_render(p, pg.params(k=16, D=3, g=0.8))
    b = pg.pg_render(p, pg.params(k=16, D=3, g=0.8, **t))
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_benchmark_batch_matches_oracle_on_sampled_scenes():
    # the 64-scene batching workload as the benchmark runs it (one graph
    # launch of a plan); the oracle renders its three smallest scenes and the
    # first of at least 50k vertices in full
    items = scenegen.generate_batch(64)
    paths = [pg.DevicePaths(sc) for _, sc in items]
    params = [pg.params(k=w.k, D=w.D, g=w.g) for w, _ in items]
    plan = pg.Batch(paths, params, use_graph=True)
    imgs = [im.clone() for im in plan()]
    torch.cuda.synchronize()
    plan.close()
    sizes = np.array([sc.n_vertices for _, sc in items])
    order = np.argsort(sizes, kind="stable")
    pick = list(order[:3]) + [int(order[np.searchsorted(sizes[order], 50_000)])]
    for s in pick:
        w, sc = items[s]
        print(f"batch scene {s}: N={sc.n_vertices} k={w.k} D={w.D} g={w.g:.3f}", flush=True)
        ref = oracle.render(sc, oracle.params(k=w.k, D=w.D, g=w.g))
        assert_within(imgs[s].cpu().numpy(), ref, PIX_REL, PIX_ABS, f"batch scene {s} vs oracle")


@pytest.mark.parametrize("use_graph", [False, True])
def test_persistent_schedule_equals_default(use_graph):
    # PG_FLAG_PERSISTENT: every iteration of every scene in one cooperative
    # launch with grid barriers; the same images bit for bit, eagerly and over
    # graph replays with other GPU work in between
    scenes, params, _ = small_batch()
    paths = [pg.DevicePaths(s) for s in scenes]
    ref = [im.clone() for im in pg.pg_render_batched(paths, params)]
    pers = [pg.params(k=p.k, D=p.D, g=p.g, flags=pg.PG_FLAG_PERSISTENT) for p in params]
    out = pg.pg_render_batched(paths, pers)
    torch.cuda.synchronize()
    for s in range(len(scenes)):
        assert torch.equal(out[s], ref[s]), f"eager scene {s}"
    plan = pg.Batch(paths, pers, use_graph=use_graph)
    for rep in range(3):
        got = plan()
        torch.cuda.synchronize()
        for s in range(len(scenes)):
            assert torch.equal(got[s], ref[s]), f"replay {rep} scene {s}"
        pg.pg_render(paths[0], params[0])
        for im in got:
            im.zero_()
        torch.cuda.synchronize()
    plan.close()
