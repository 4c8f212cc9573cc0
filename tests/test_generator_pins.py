"""Pins of the instrumented path tracer that produces the vertex records
(paper, Sec. "Volume Path Tracing": analog delta tracking, eqs. mc and mc-pa;
Sec. "Rendering System", the instrumented path tracer).  The GPU tracer is
checked record by record against this generator, so a transport mistake the
two shared would pass there; these tests pin the generator itself against
closed forms of the transport, computed here independently of it.

The reference quantity throughout is the optical depth tau(o, d, t) =
integral of sigma_t along the ray, written out exactly for the nearest-voxel
density grid (the ray is cut at every voxel face it crosses, and each piece
contributes its voxel's sigma_t times its length):

* free flights: given the continuation ray and the distance t_e to where it
  leaves the cube, a collision distance s from analog delta tracking has
  P(s <= x | collision) = (1 - e^{-tau(x)}) / (1 - e^{-tau(t_e)}), so that
  ratio is uniform on [0, 1] (Kolmogorov-Smirnov test);
* escapes: a continuation ray escapes with probability e^{-tau(t_e)};
* shadow rays: the ratio-tracking transmittance in the sun and environment
  records has mean e^{-tau} toward the light (the environment direction is
  uniform on the sphere, p_e = 1/(4 pi), so the environment record is an
  unbiased next-event estimate of the transmitted environment radiance);
* a homogeneous slab seen head on: the camera ray misses every collision
  with probability e^{-sigma_t} and the first collision depth is exponential
  truncated to the slab.
"""
import math
from dataclasses import replace

import numpy as np
import pytest
from scipy import stats

import scenegen


def box_interval(o, d):
    """Entry and exit parameters of rays o + t d through the unit cube
    (slab test); rays that miss get an empty interval."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        ta = (0.0 - o) * inv
        tb = (1.0 - o) * inv
    lo = np.where(d == 0, np.where((o >= 0) & (o <= 1), -np.inf, np.inf), np.minimum(ta, tb))
    hi = np.where(d == 0, np.where((o >= 0) & (o <= 1), np.inf, -np.inf), np.maximum(ta, tb))
    return lo.max(1), hi.min(1)


def optical_depth(sigma, o, d, tmax):
    """tau = integral over t in [0, tmax] of sigma_t(o + t d) for the nearest-
    voxel grid sigma [R, R, R] (z, y, x) on the unit cube, zero outside."""
    R = sigma.shape[0]
    o = np.asarray(o, np.float64)
    d = np.asarray(d, np.float64)
    t0, t1 = box_interval(o, d)
    a = np.clip(t0, 0.0, None)
    b = np.minimum(t1, tmax)
    b = np.maximum(a, b)
    planes = np.arange(R + 1, dtype=np.float64) / R
    with np.errstate(divide="ignore", invalid="ignore"):
        ts = [(planes[None, :] - o[:, k:k + 1]) / d[:, k:k + 1] for k in range(3)]
    t = np.concatenate([a[:, None], b[:, None]] + ts, axis=1)
    t = np.where(np.isfinite(t), t, b[:, None])
    t = np.clip(t, a[:, None], b[:, None])
    t.sort(axis=1)
    mid = 0.5 * (t[:, 1:] + t[:, :-1])
    seg = t[:, 1:] - t[:, :-1]
    p = o[:, None, :] + mid[:, :, None] * d[:, None, :]
    idx = np.clip(np.floor(p * R).astype(np.int64), 0, R - 1)
    s = sigma[idx[..., 2], idx[..., 1], idx[..., 0]].astype(np.float64)
    return (s * seg).sum(1)


def exit_distance(o, d):
    _, t1 = box_interval(np.asarray(o, np.float64), np.asarray(d, np.float64))
    return np.clip(t1, 0.0, None)


# a heterogeneous medium: 16^3 fBm with sigma_t in [0, 6] (majorant 6 > most
# voxels, so ratio tracking is not the binary track-length estimate)
HET = scenegen.SceneConfig(R=16, sigma_max=6.0, density_contrast=1.5, mask=0, albedo=(0.9, 0.9), g=0.5,
                           width=48, height=48, spp=8, max_depth=12, vfov_deg=45.0, seed=21)


@pytest.fixture(scope="module")
def het():
    sc = scenegen.generate(HET)
    sigma, _, maj = scenegen.medium(HET)
    assert sc.n_vertices > 20000
    assert sigma.min() < 0.5 * maj                    # the majorant is loose in parts of the medium
    return sc, sigma, maj


def path_structure(sc):
    off = sc.path_offsets
    lens = np.diff(off)
    depth = np.arange(sc.n_vertices) - np.repeat(off[:-1], lens)
    last = np.zeros(sc.n_vertices, bool)
    last[off[1:][lens > 0] - 1] = True
    return depth, last


def test_records_chain_along_each_path(het):
    sc, _, _ = het
    depth, last = path_structure(sc)
    v = np.flatnonzero(~last)
    # the next vertex arrives along the continuation direction ...
    assert np.array_equal(sc.dir_in[v + 1], sc.dir_out[v])
    # ... and lies on the continuation ray
    step = sc.pos[v + 1].astype(np.float64) - sc.pos[v].astype(np.float64)
    s = np.linalg.norm(step, axis=1)
    cross = np.linalg.norm(np.cross(step, sc.dir_out[v].astype(np.float64)), axis=1)
    assert np.all(cross <= 1e-6 + 1e-6 * s)
    assert np.all(np.einsum("ij,ij->i", step, sc.dir_out[v].astype(np.float64)) > -1e-6)
    # an empty path is a camera escape and carries the environment radiance
    lens = np.diff(sc.path_offsets)
    env = np.asarray(HET.env_L, np.float32)
    assert np.all(sc.e_cam[lens == 0] == env) and not sc.e_cam[lens > 0].any()
    # a path ends by escaping (escaped radiance recorded) or at the maximum depth (none)
    esc = np.any(sc.l_phase != 0, axis=1)
    assert np.array_equal(esc, last & (depth < HET.max_depth - 1))
    assert np.all(sc.l_phase[esc] == env)
    assert depth.max() <= HET.max_depth - 1


def test_free_flights_follow_delta_tracking(het):
    sc, sigma, _ = het
    _, last = path_structure(sc)
    v = np.flatnonzero(~last)
    o = sc.pos[v].astype(np.float64)
    d = sc.dir_out[v].astype(np.float64)
    s = np.linalg.norm(sc.pos[v + 1].astype(np.float64) - o, axis=1)
    te = exit_distance(o, d)
    u = -np.expm1(-optical_depth(sigma, o, d, s)) / -np.expm1(-optical_depth(sigma, o, d, te))
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    # a flight with sigma_t <= 6 is never longer than the exit distance
    assert np.all(s <= te + 1e-5)


def test_camera_flights_follow_delta_tracking(het):
    sc, sigma, _ = het
    lens = np.diff(sc.path_offsets)
    first = sc.path_offsets[:-1][lens > 0]
    cam = np.broadcast_to(np.asarray(HET.cam_pos, np.float64), (len(first), 3))
    d = sc.dir_in[first].astype(np.float64)
    s = np.linalg.norm(sc.pos[first].astype(np.float64) - cam, axis=1)
    u = -np.expm1(-optical_depth(sigma, cam, d, s)) / -np.expm1(-optical_depth(sigma, cam, d, np.full(len(d), 1e9)))
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_continuation_escapes_with_the_transmittance(het):
    sc, sigma, _ = het
    depth, last = path_structure(sc)
    v = np.flatnonzero(depth < HET.max_depth - 1)
    esc = np.any(sc.l_phase[v] != 0, axis=1).astype(np.float64)
    o = sc.pos[v].astype(np.float64)
    d = sc.dir_out[v].astype(np.float64)
    p = np.exp(-optical_depth(sigma, o, d, exit_distance(o, d)))
    z = (esc - p).sum() / math.sqrt((p * (1 - p)).sum())
    assert abs(z) < 4.5, z
    # and the escapes are not a constant fraction: they track the transmittance
    hi, lo = p > np.quantile(p, 0.8), p < np.quantile(p, 0.2)
    assert esc[hi].mean() > esc[lo].mean() + 0.2


def check_unbiased(T, Tref, what):
    r = T - Tref
    se = r.std() / math.sqrt(r.size)
    assert abs(r.mean()) < 4.5 * se + 1e-12, f"{what}: mean error {r.mean():.3e}, standard error {se:.3e}"


def test_sun_shadow_rays_are_unbiased_transmittance(het):
    sc, sigma, _ = het
    o = sc.pos.astype(np.float64)
    d = np.broadcast_to(np.asarray(HET.sun_dir, np.float64), o.shape)
    T = sc.l_sun[:, 0].astype(np.float64) / HET.sun_E[0]
    # the three channels carry one transmittance
    assert np.allclose(sc.l_sun[:, 1] / HET.sun_E[1], T, rtol=1e-6, atol=1e-7)
    Tref = np.exp(-optical_depth(sigma, o, d, exit_distance(o, d)))
    check_unbiased(T, Tref, "sun")
    assert np.all((T >= 0) & (T <= 1 + 1e-6))
    # ratio tracking, not a 0/1 track-length estimate, where the majorant is loose
    assert np.mean((T > 1e-6) & (T < 1 - 1e-6)) > 0.3


def test_environment_shadow_rays_are_unbiased_next_event_estimates(het):
    sc, sigma, _ = het
    d = sc.dir_env.astype(np.float64)
    # directions uniform on the sphere: z and the azimuth uniform, unit length
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-6)
    assert stats.kstest(d[:, 2], "uniform", args=(-1, 2)).pvalue > 1e-3
    phi = np.arctan2(d[:, 1], d[:, 0])
    assert stats.kstest(phi, "uniform", args=(-math.pi, 2 * math.pi)).pvalue > 1e-3
    o = sc.pos.astype(np.float64)
    T = sc.l_env[:, 2].astype(np.float64) / HET.env_L[2]
    Tref = np.exp(-optical_depth(sigma, o, d, exit_distance(o, d)))
    check_unbiased(T, Tref, "environment")
    # so 4 pi * mean(record) estimates the transmitted environment radiance
    # integrated over the sphere at each vertex


def test_point_light_shadow_rays_stop_at_the_light(het):
    cfg = replace(HET, width=24, height=24, spp=4, pl_I=(0.5, 0.4, 0.3), pl_pos=(0.45, 0.7, 0.55))
    sc = scenegen.generate(cfg)
    sigma, _, _ = scenegen.medium(cfg)
    o = sc.pos.astype(np.float64)
    dl = np.asarray(cfg.pl_pos) - o
    r2 = (dl ** 2).sum(1)
    dist = np.sqrt(r2)
    d = dl / dist[:, None]
    assert np.allclose(sc.dir_pl, d, atol=1e-6)
    T = sc.l_pl[:, 0].astype(np.float64) * r2 / cfg.pl_I[0]
    Tref = np.exp(-optical_depth(sigma, o, d, np.minimum(dist, exit_distance(o, d))))
    check_unbiased(T, Tref, "point light")


def test_homogeneous_slab_camera_escape_closed_form():
    # a homogeneous cube seen head on through a very narrow field of view: every
    # camera ray crosses one unit of sigma_t = 2, so a path is empty (the ray
    # escapes) with probability e^-2, and the first collision depth z is
    # exponential with rate 2 truncated to [0, 1]
    sig = 2.0
    cfg = scenegen.SceneConfig(R=8, sigma_max=sig, density_contrast=0.0, density_bias=0.5, mask=0,
                               albedo=(0.9, 0.9), g=0.3, width=64, height=64, spp=8, max_depth=1,
                               cam_pos=(0.5, 0.5, -1.0), look_at=(0.5, 0.5, 0.5), vfov_deg=0.05, seed=33)
    sigma, _, maj = scenegen.medium(cfg)
    assert np.all(sigma == np.float32(sig)) and maj == sig
    sc = scenegen.generate(cfg)
    lens = np.diff(sc.path_offsets)
    n = lens.size
    p = math.exp(-sig)
    z = ((lens == 0).sum() - n * p) / math.sqrt(n * p * (1 - p))
    assert abs(z) < 4.5, z
    depth = sc.pos[:, 2].astype(np.float64)
    u = -np.expm1(-sig * depth) / -math.expm1(-sig)
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    # a homogeneous medium at its majorant: ratio tracking is the 0/1 estimate
    # and its mean is e^{-sigma_t d} along the sun direction
    d = exit_distance(sc.pos.astype(np.float64), np.broadcast_to(np.asarray(cfg.sun_dir), sc.pos.shape))
    T = sc.l_sun[:, 0].astype(np.float64) / cfg.sun_E[0]
    assert set(np.unique(T)) <= {0.0, 1.0}
    check_unbiased(T, np.exp(-sig * d), "homogeneous sun")


def test_optical_depth_reference_closed_forms():
    # the reference integral itself: a constant grid gives sigma times the chord
    # inside the cube; a two-valued grid splits at the voxel face
    R = 4
    const = np.full((R, R, R), 3.0, np.float32)
    o = np.array([[0.5, 0.5, -1.0], [0.2, 0.3, 0.4]])
    d = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    tau = optical_depth(const, o, d, np.array([10.0, 10.0]))
    assert np.allclose(tau, [3.0, 3.0 * 0.8])
    tau = optical_depth(const, o, d, np.array([1.5, 0.5]))
    assert np.allclose(tau, [1.5, 1.5])
    half = np.zeros((R, R, R), np.float32)
    half[:, :, R // 2:] = 5.0                                  # x >= 0.5
    tau = optical_depth(half, np.array([[0.1, 0.5, 0.5]]), np.array([[1.0, 0.0, 0.0]]), np.array([10.0]))
    assert np.allclose(tau, [2.5])
    diag = np.array([[1.0, 1.0, 1.0]]) / math.sqrt(3.0)
    assert np.allclose(optical_depth(const, np.zeros((1, 3)), diag, np.array([10.0])), [3.0 * math.sqrt(3.0)])
