"""The GPU path tracer (pg_trace_count / pg_trace_records) against the CPU
generator it shares its definition with: the same PCG32 streams, double
precision, no contraction.  The double-precision elementary functions (log,
sin, cos) of the two sides may round their last place differently, which
moves a float record by an ulp (seen: the environment direction after its
normalisation) or, in principle, flips a tracking decision.  So: path
offsets bit-exact on these scenes, camera-ray escapes bit-exact, every record
within 2 float ulps, and at most one path in 10^4 (at least 2) may differ
by more."""
import ctypes
from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle
import scenegen
import paper_2404_11894_amd as pg
from tests.gpu_util import PIX_ABS, PIX_REL, assert_within

pytestmark = pytest.mark.gpu

FIELDS = ("pos", "dir_in", "dir_out", "albedo", "l_sun", "dir_env", "l_env", "l_phase")


def traced(cfg):
    sigma, alb, maj = scenegen.medium(cfg)
    rec = pg.pg_trace(scenegen.tracer_settings(cfg), sigma, alb, maj)
    torch.cuda.synchronize()
    return rec


def compare(cfg, max_bad=1e-4):
    ref = scenegen.generate(cfg)
    rec = traced(cfg)
    off = rec.path_offsets.cpu().numpy()
    assert off.shape == ref.path_offsets.shape and off[0] == 0
    lens, rlens = np.diff(off), np.diff(ref.path_offsets)
    P = len(lens)
    same_len = lens == rlens
    assert np.array_equal(rec.e_cam.cpu().numpy()[same_len], ref.e_cam[same_len])
    got = {f: getattr(rec, f).cpu().numpy() for f in FIELDS}
    bad = int((~same_len).sum())
    # records of paths with the same length, compared path by path
    vs = np.repeat(np.arange(P), rlens)           # path of each reference vertex
    idx_ref = np.arange(len(vs))
    ok_v = same_len[vs]
    gv = off[vs[ok_v]] + (idx_ref[ok_v] - ref.path_offsets[vs[ok_v]])
    diff_path = np.zeros(P, bool)
    ulp_paths = np.zeros(P, bool)
    for f in FIELDS if len(gv) else ():
        a = got[f][gv].reshape(len(gv), -1)
        b = getattr(ref, f)[idx_ref[ok_v]].reshape(len(gv), -1)
        ulps = np.abs(a.view(np.int32).astype(np.int64) - b.view(np.int32).astype(np.int64))
        far = np.any((ulps > 2) & (a != b), axis=1)
        diff_path[vs[ok_v][far]] = True
        ulp_paths[vs[ok_v][np.any(a != b, axis=1)]] = True
    bad += int(diff_path.sum())
    print(f"{P} paths, {ref.n_vertices} vertices: {int((~same_len).sum())} lengths differ, "
          f"{int(ulp_paths.sum())} paths differ by <= 2 ulps, {bad} by more", flush=True)
    assert np.array_equal(off, ref.path_offsets) or bad > 0
    assert bad <= max(2, int(max_bad * P)), bad
    return ref, rec


def test_trace_tiny_matches_cpu_generator():
    compare(scenegen.WORKLOADS["tiny"].scene)


def test_trace_ball_crop_per_voxel_albedo():
    # the benchmark's medium (128^3 ball, per-voxel albedo, g 0.8, depth 64), centred 96x96 crop
    compare(scenegen.crop_of(scenegen.WORKLOADS["mid"].scene, 96, 96, 2))


@pytest.mark.parametrize("case", ["g_negative_short", "empty_medium", "isotropic"])
def test_trace_variants(case):
    base = scenegen.crop_of(scenegen.WORKLOADS["tiny"].scene, 40, 24, 3)
    cfg = {"g_negative_short": replace(base, g=-0.4, max_depth=3, seed=5),
           "empty_medium": replace(base, sigma_max=0.0),
           "isotropic": replace(base, g=0.0, albedo=(0.7, 0.95), seed=9)}[case]
    ref, rec = compare(cfg)
    if case == "empty_medium":
        assert ref.n_vertices == 0 and rec.n_vertices == 0


def test_trace_extra_first_vertex_samples():
    cfg = replace(scenegen.crop_of(scenegen.WORKLOADS["mid"].scene, 48, 48, 2), extra_samples=3)
    ref, rec = compare(cfg)
    for name in ("fb_l_sun", "fb_dir_env", "fb_l_env"):
        a = getattr(rec, name).cpu().numpy()
        b = getattr(ref, name)
        assert a.shape == b.shape, name
        ulps = np.abs(a.view(np.int32).astype(np.int64) - b.view(np.int32).astype(np.int64))
        far = (ulps > 2) & (a != b)
        assert far.any(axis=(1, 2)).sum() <= max(2, int(1e-4 * a.shape[0])), name
    # the paths do not depend on the extra samples
    plain = traced(replace(cfg, extra_samples=0))
    assert torch.equal(plain.path_offsets, rec.path_offsets)
    assert torch.equal(plain.pos, rec.pos)


def test_trace_point_light():
    cfg = replace(scenegen.crop_of(scenegen.WORKLOADS["mid"].scene, 48, 48, 2), pl_I=(0.5, 0.4, 0.3),
                  pl_pos=(0.2, 1.3, 0.4))
    ref, rec = compare(cfg)
    if np.array_equal(rec.path_offsets.cpu().numpy(), ref.path_offsets):
        for name in ("dir_pl", "l_pl"):
            a, b = getattr(rec, name).cpu().numpy(), getattr(ref, name)
            ulps = np.abs(a.view(np.int32).astype(np.int64) - b.view(np.int32).astype(np.int64))
            assert ((ulps > 2) & (a != b)).any(axis=1).sum() <= max(2, int(1e-4 * len(a))), name


def test_traced_records_render_like_host_records():
    cfg = scenegen.crop_of(scenegen.WORKLOADS["tiny"].scene, 48, 48, 2)
    ref = scenegen.generate(cfg)
    rec = traced(cfg)
    q = pg.params(k=8, D=6, g=0.5, flags=pg.PG_FLAG_CHECK)
    a = pg.pg_render(pg.DevicePaths(rec), q)
    b = pg.pg_render(pg.DevicePaths(ref), q)
    torch.cuda.synchronize()
    assert_within(a.cpu().numpy(), b.cpu().numpy(), PIX_REL, PIX_ABS, "device vs host records")


def host_scene(rec, cfg):
    """The device-traced records as a host Scene (numpy copies)."""
    h = lambda name: None if getattr(rec, name, None) is None else getattr(rec, name).cpu().numpy()  # noqa: E731
    return scenegen.Scene(width=rec.width, height=rec.height, spp=rec.spp, path_offsets=h("path_offsets"),
                          pos=h("pos"), dir_in=h("dir_in"), dir_out=h("dir_out"), albedo=h("albedo"),
                          l_sun=h("l_sun"), dir_env=h("dir_env"), l_env=h("l_env"), l_phase=h("l_phase"),
                          e_cam=h("e_cam"), config=cfg, sun_dir=tuple(cfg.sun_dir), fb_l_sun=h("fb_l_sun"),
                          fb_dir_env=h("fb_dir_env"), fb_l_env=h("fb_l_env"), dir_pl=h("dir_pl"), l_pl=h("l_pl"))


@pytest.mark.parametrize("extra,pl", [(0, False), (2, True)])
def test_traced_records_render_like_the_oracle(extra, pl):
    # the records the GPU tracer wrote, rendered by the oracle (FP64) and by
    # the GPU from the same device arrays
    cfg = replace(scenegen.crop_of(scenegen.WORKLOADS["tiny"].scene, 40, 40, 2), extra_samples=extra,
                  pl_I=(0.4, 0.3, 0.2) if pl else (0.0, 0.0, 0.0))
    rec = traced(cfg)
    sc = host_scene(rec, cfg)
    print(f"traced N={sc.n_vertices} extra={extra} point light={pl}", flush=True)
    q = pg.params(k=8, D=6, g=0.5, flags=pg.PG_FLAG_CHECK)
    got = pg.pg_render(pg.DevicePaths(rec), q)
    torch.cuda.synchronize()
    ref = oracle.render(sc, oracle.params(k=8, D=6, g=0.5))
    assert_within(got.cpu().numpy(), ref, PIX_REL, PIX_ABS, "device-traced records vs oracle")


def test_trace_records_rejects_foreign_offsets():
    cfg = scenegen.crop_of(scenegen.WORKLOADS["tiny"].scene, 8, 8, 1)
    sigma, alb, maj = scenegen.medium(cfg)
    rec = pg.pg_trace(scenegen.tracer_settings(cfg), sigma, alb, maj)
    st = scenegen.tracer_settings(replace(cfg, seed=cfg.seed + 1))   # other paths, same offsets
    t = pg.Tracer()
    # re-use the binding to build the struct, then call pg_trace_records with the first offsets
    sg = torch.as_tensor(sigma).cuda().contiguous()
    al = torch.as_tensor(alb).cuda().contiguous() if alb is not None else None
    t.R, t.width, t.height, t.spp, t.max_depth = st["R"], st["width"], st["height"], st["spp"], st["max_depth"]
    t.crop_x0, t.crop_y0, t.crop_w, t.crop_h = st["crop"]
    t.sigma, t.albedo = sg.data_ptr(), (al.data_ptr() if al is not None else None)
    t.albedo_const, t.majorant, t.g, t.vfov_deg = st["albedo_const"], maj, st["g"], st["vfov_deg"]
    for name in ("cam_pos", "look_at", "sun_dir", "sun_E", "env_L"):
        getattr(t, name)[:] = st[name]
    t.seed = st["seed"]
    N = rec.n_vertices
    bufs = {f: torch.full((N * (1 if f == "albedo" else 3),), -3.0, device="cuda") for f in FIELDS}
    e_cam = torch.empty(64 * 3, device="cuda")
    r = pg.Records(*(bufs[f].data_ptr() for f in FIELDS), e_cam.data_ptr(), None, None, None, None, None)
    nb = ctypes.c_size_t()
    L = pg.lib()
    pg._check(L.pg_trace_workspace_size(ctypes.byref(t), ctypes.byref(nb)))
    _, ws, n = pg._workspace(nb.value, torch.device("cuda"))
    # pass 1 of the other seed fills the workspace; pass 2 is offered the first seed's offsets
    off2 = torch.empty(rec.path_offsets.numel(), dtype=torch.int64, device="cuda")
    n2 = ctypes.c_int64()
    pg._check(L.pg_trace_count(ctypes.byref(t), pg._ptr(off2), ctypes.byref(n2), pg._ptr(ws), n,
                               pg._stream(torch.device("cuda"))))
    assert not torch.equal(off2, rec.path_offsets)
    rc = L.pg_trace_records(ctypes.byref(t), pg._ptr(rec.path_offsets),
                            ctypes.byref(r), pg._ptr(ws), n, pg._stream(torch.device("cuda")))
    torch.cuda.synchronize()
    assert rc == pg.PG_ERR_INPUT
