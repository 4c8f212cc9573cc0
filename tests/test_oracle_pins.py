"""Pins of the FP64 oracle against things other than itself.

Each test checks the oracle against a closed form, a textbook property, a
library routine, brute force, the unbiasedness of the paper's estimators or a
dense linear-algebra restatement -- chosen so that a dropped term, a wrong
sign, index or operand fails at least one of them.
"""
import math
from dataclasses import replace

import numpy as np
import pytest
from scipy import integrate, spatial, stats

import oracle
import scenegen

FOUR_PI = 4.0 * math.pi


def hg_textbook(g, mu):
    """Henyey-Greenstein (1941) phase function in its usual form."""
    return (1.0 - g * g) / (FOUR_PI * (1.0 + g * g - 2.0 * g * mu) ** 1.5)


# ----------------------------------------------------------------- phase ---

@pytest.mark.parametrize("g", [-0.3, 0.0, 0.5, 0.8, 0.9])
def test_hg_normalised_and_mean_cosine(g):
    # integral over the sphere is 1 and the mean cosine is g (textbook HG);
    # the oracle's argument is u = 1 - cos
    norm, _ = integrate.quad(lambda u: 2 * math.pi * oracle.hg(g, u), 0.0, 2.0, epsabs=1e-13, epsrel=1e-12)
    mean, _ = integrate.quad(lambda u: 2 * math.pi * (1 - u) * oracle.hg(g, u), 0.0, 2.0,
                             epsabs=1e-13, epsrel=1e-12)
    assert abs(norm - 1.0) < 1e-10
    assert abs(mean - g) < 1e-10


def test_hg_closed_forms():
    assert abs(oracle.hg(0.0, 0.7) - 1 / FOUR_PI) < 1e-16
    for g in (-0.3, 0.5, 0.9):
        assert math.isclose(oracle.hg(g, 0.0), (1 + g) / (FOUR_PI * (1 - g) ** 2), rel_tol=1e-14)
        assert math.isclose(oracle.hg(g, 2.0), (1 - g) / (FOUR_PI * (1 + g) ** 2), rel_tol=1e-14)
        for mu in (-0.9, -0.2, 0.3, 0.99):
            assert math.isclose(oracle.hg(g, 1 - mu), hg_textbook(g, mu), rel_tol=1e-12)


@pytest.mark.parametrize("g", [-0.3, 0.4, 0.9])
def test_hg_dlog_matches_finite_difference(g):
    h = 1e-6
    for u in (0.0, 0.01, 0.5, 1.3, 2.0):
        fd = (math.log(oracle.hg(g + h, u)) - math.log(oracle.hg(g - h, u))) / (2 * h)
        assert abs(oracle.hg_dlog(g, u) - fd) < 1e-6 * max(1.0, abs(fd))


def test_generator_samples_hg_about_arriving_direction(tiny_scene):
    # the path tracer's continuation cosines follow HG_g with mu = <dir_in, dir_out>,
    # the same convention the oracle's receiver phase uses
    g = scenegen.WORKLOADS["tiny"].g
    mu = np.einsum("ij,ij->i", tiny_scene.dir_in.astype(np.float64), tiny_scene.dir_out.astype(np.float64))
    mu = np.clip(mu, -1.0, 1.0)

    def cdf(m):
        return (1 - g * g) / (2 * g) * (1 / np.sqrt(1 + g * g - 2 * g * m) - 1 / (1 + g))

    assert stats.kstest(mu, cdf).pvalue > 1e-3
    assert abs(mu.mean() - g) < 5 * mu.std() / math.sqrt(mu.size)


# ------------------------------------------------------------ quantise ---

def test_quantize_special_values():
    pos = np.array([[0.0, 0.5, 1.0], [2.0 ** -20, 1 - 2.0 ** -24, 0.25]], np.float32)
    q, ok = oracle.quantize(pos)
    assert ok
    assert q.tolist() == [[0, 2 ** 19, 2 ** 20 - 1], [1, 2 ** 20 - 1, 2 ** 18]]
    _, ok = oracle.quantize(np.array([[0.1, np.nan, 0.2]], np.float32))
    assert not ok
    _, ok = oracle.quantize(np.array([[0.1, 1.5, 0.2]], np.float32))
    assert not ok


# ----------------------------------------------------------- neighbours ---

def knn_brute(pos, k):
    q = np.floor(pos.astype(np.float64) * 2 ** 20).clip(0, 2 ** 20 - 1).astype(np.int64)
    n = len(q)
    K = min(k, n)
    out = np.empty((n, K), np.int64)
    idx = np.arange(n)
    for i in range(n):
        d2 = ((q - q[i]) ** 2).sum(1)
        d2[i] = -1                      # self first
        order = np.lexsort((idx, d2))   # by (d2, index)
        out[i] = order[:K]
    return out


@pytest.mark.parametrize("n,k", [(1, 8), (5, 8), (300, 1), (300, 8), (500, 16), (64, 64)])
def test_knn_matches_brute_force(n, k):
    rng = np.random.default_rng(n * 100 + k)
    pos = rng.random((n, 3), dtype=np.float32)
    assert np.array_equal(oracle.knn(pos, k), knn_brute(pos, k))


def test_knn_distances_match_kdtree():
    rng = np.random.default_rng(7)
    pos = rng.random((3000, 3), dtype=np.float32) ** 2   # non-uniform density
    k = 16
    col = oracle.knn(pos, k)
    q, _ = oracle.quantize(pos)
    qf = q.astype(np.float64)
    d_or = ((qf[col] - qf[:, None, :]) ** 2).sum(-1)
    d_kd, _ = spatial.cKDTree(qf).query(qf, k=k)
    # the K distances (self first at 0) are unique even where indices tie
    assert np.array_equal(d_or, np.round(d_kd ** 2))


def test_knn_lattice_ties_broken_by_index():
    # 5x5x5 lattice: the interior point's 6 face neighbours are equidistant and
    # must come in index order, then the 12 edge neighbours, in index order
    h = 1.0 / 8
    g = np.array([(x, y, z) for z in range(5) for y in range(5) for x in range(5)], np.float64)
    pos = ((g + 1) * h).astype(np.float32)
    center = 2 + 5 * 2 + 25 * 2
    col = oracle.knn(pos, 19, rows=[center])[0]
    face = sorted(center + d for d in (1, -1, 5, -5, 25, -25))
    edge = sorted(center + a + b for a, b in [(1, 5), (1, -5), (-1, 5), (-1, -5), (1, 25), (1, -25),
                                              (-1, 25), (-1, -25), (5, 25), (5, -25), (-5, 25), (-5, -25)])
    assert col.tolist() == [center] + face + edge


def test_knn_duplicates_and_degenerate():
    pos = np.full((10, 3), 0.3, np.float32)
    col = oracle.knn(pos, 4)
    for i in range(10):
        assert col[i].tolist() == [i] + [j for j in range(10) if j != i][:3]
    assert oracle.knn(np.zeros((0, 3), np.float32), 4).shape == (0, 0)


def test_knn_relabelling_invariance():
    rng = np.random.default_rng(11)
    pos = rng.random((800, 3), dtype=np.float32)
    perm = rng.permutation(800)
    a = oracle.knn(pos, 8)
    b = oracle.knn(pos[perm], 8)
    # generic positions: no distance ties, so the sets map through the relabelling
    assert np.array_equal(perm[b], a[perm])


# --------------------------------------------------------- edge weights ---

def make_scene(pos, dir_in, dir_out, dir_env, l_sun=None, l_env=None, l_phase=None, albedo=None,
               offsets=None, e_cam=None, width=None, height=1, spp=1):
    n = len(pos)
    z3 = np.zeros((n, 3), np.float32)
    if offsets is None:
        offsets = np.arange(n + 1, dtype=np.int64)   # one vertex per path
    P = len(offsets) - 1
    return scenegen.Scene(width=width or P // (height * spp), height=height, spp=spp,
                          path_offsets=np.asarray(offsets, np.int64), pos=np.asarray(pos, np.float32),
                          dir_in=np.asarray(dir_in, np.float32), dir_out=np.asarray(dir_out, np.float32),
                          albedo=np.ones(n, np.float32) if albedo is None else np.asarray(albedo, np.float32),
                          l_sun=z3 if l_sun is None else np.asarray(l_sun, np.float32),
                          dir_env=np.asarray(dir_env, np.float32),
                          l_env=z3 if l_env is None else np.asarray(l_env, np.float32),
                          l_phase=z3 if l_phase is None else np.asarray(l_phase, np.float32),
                          e_cam=np.zeros((P, 3), np.float32) if e_cam is None else np.asarray(e_cam, np.float32))


def unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def sample_hg(rng, t, g):
    """Textbook inversion sampling of HG about unit directions t."""
    n = len(t)
    u1, u2 = rng.random(n), rng.random(n)
    s = (1 - g * g) / (1 - g + 2 * g * u1)
    mu = np.clip((1 + g * g - s * s) / (2 * g), -1, 1)
    a = np.where(np.abs(t[:, 0:1]) < 0.9, [[1.0, 0, 0]], [[0, 1.0, 0]])
    e1 = np.cross(t, a)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(t, e1)
    phi = 2 * math.pi * u2
    st = np.sqrt(1 - mu * mu)[:, None]
    return mu[:, None] * t + st * (np.cos(phi)[:, None] * e1 + np.sin(phi)[:, None] * e2)


def clustered(rng, trials, K, g_s, env_fn):
    """``trials`` clusters of K coincident vertices, far apart; neighbour rows by hand."""
    n = trials * K
    centers = rng.random((trials, 3)) * 0.9 + 0.05
    pos = np.repeat(centers, K, axis=0)
    t = unit(rng, n)
    w = sample_hg(rng, t, g_s)
    we = unit(rng, n)
    sc = make_scene(pos, t, w, we, l_env=env_fn(we), l_phase=env_fn(w))
    col = np.empty((n, K), np.int32)
    for c in range(trials):
        m = np.arange(c * K, (c + 1) * K)
        for a in range(K):
            col[c * K + a] = [m[a]] + [x for x in m if x != m[a]]
    return sc, col, t


@pytest.mark.parametrize("K", [1, 4, 8])
def test_aggregation_estimators_are_unbiased(K):
    # With one HG_{g_s} sample per technique (neighbour), the balance-heuristic
    # estimators of the paper are unbiased:  E[sum_j w+_ij f(w_j)] = int rho_i f,
    # E[d_agg_i] = int rho_i L_env  (environment unoccluded, no sun), and the same
    # holds for the plain path-traced direct term.
    rng = np.random.default_rng(K)
    g, g_s = 0.7, 0.4
    trials = 20000 // K
    env = lambda d: np.repeat((d[:, 2:3] + 2.0), 3, axis=1)  # noqa: E731, positive env radiance
    sc, col, t = clustered(rng, trials, K, g_s, env)
    p = oracle.params(k=K, D=0, g=g, g_s=g_s)
    e = oracle.edges(sc, p, col)
    rows = np.arange(0, trials * K, K)            # receiver = first member of each cluster
    w_dirs = sc.dir_out.astype(np.float64)[col[rows]]
    wi = e["w_ind"][rows]
    t0 = t[rows]

    def check(samples, expected):
        m, s = samples.mean(0), samples.std(0) / math.sqrt(len(samples))
        assert np.all(np.abs(m - expected) < 5 * s + 1e-12), (m, expected, s)

    check(wi.sum(1), np.ones(1))                                          # f = 1
    check(np.einsum("ij,ijc->ic", wi, w_dirs) - g * t0, np.zeros(3))        # f = w: mean cosine g
    check(e["d_agg"][rows, 0] - (2.0 + g * t0[:, 2]), np.zeros(1))        # int rho L_env
    check(e["d_pt"][rows, 0] - (2.0 + g * t0[:, 2]), np.zeros(1))


def test_isotropic_weights_closed_form():
    # g = g_s = 0: every density is 1/(4 pi), so w+ = 1/K, w_p = w_e = 1/(2K),
    # d_agg = mean(Ls)/(4 pi) + sum(Le + Lp)/(2K), d_pt = Ls/(4 pi) + (Le + Lp)/2, r = 1
    rng = np.random.default_rng(3)
    n, k = 200, 6
    pos = rng.random((n, 3), dtype=np.float32)
    sc = make_scene(pos, unit(rng, n), unit(rng, n), unit(rng, n), l_sun=rng.random((n, 3)),
                    l_env=rng.random((n, 3)), l_phase=rng.random((n, 3)))
    p = oracle.params(k=k, D=0, g=0.0)
    col = oracle.knn(pos, k)
    e = oracle.edges(sc, p, col)
    assert np.allclose(e["w_ind"], 1 / k, rtol=1e-14)
    assert np.allclose(e["w_ph"], 1 / (2 * k), rtol=1e-14)
    assert np.allclose(e["w_env"], 1 / (2 * k), rtol=1e-14)
    ls, le, lp = (a.astype(np.float64) for a in (sc.l_sun, sc.l_env, sc.l_phase))
    dagg = ls[col].mean(1) / FOUR_PI + (le[col] + lp[col]).sum(1) / (2 * k)
    dpt = ls / FOUR_PI + (le + lp) / 2
    assert np.allclose(e["d_agg"], dagg, rtol=1e-13)
    assert np.allclose(e["d_pt"], dpt, rtol=1e-13)
    assert np.allclose(e["r"], 1.0)


def test_identical_techniques_give_uniform_weights():
    # every neighbour arrives along the same direction -> all K techniques are
    # the same pdf, and with g = g_s the indirect weight is exactly 1/K
    rng = np.random.default_rng(5)
    n, k = 64, 8
    t = np.tile(unit(rng, 1), (n, 1))
    sc = make_scene(rng.random((n, 3)), t, unit(rng, n), unit(rng, n))
    e = oracle.edges(sc, oracle.params(k=k, D=0, g=0.8), oracle.knn(sc.pos, k))
    assert np.allclose(e["w_ind"], 1 / k, rtol=1e-12)


def test_single_neighbour_reduces_to_path_tracing_weights():
    rng = np.random.default_rng(6)
    n = 50
    sc = make_scene(rng.random((n, 3)), unit(rng, n), unit(rng, n), unit(rng, n), l_sun=rng.random((n, 3)),
                    l_env=rng.random((n, 3)), l_phase=rng.random((n, 3)))
    p = oracle.params(k=1, D=0, g=0.6, g_s=0.3)
    e = oracle.edges(sc, p, oracle.knn(sc.pos, 1))
    assert np.allclose(e["w_ind"][:, 0], e["r"], rtol=1e-13)
    assert np.allclose(e["d_agg"], e["d_pt"], rtol=1e-13)


# ------------------------------------------------------ whole pipeline ---

EMIT_L = (3.0, 2.0, 1.0)


def small_scene(w=16, h=16, spp=2, name="tiny", emit=False):
    cfg = scenegen.crop_of(scenegen.WORKLOADS[name].scene, w, h, spp)
    if emit:
        cfg = replace(cfg, emit_L=EMIT_L)
    return scenegen.generate(cfg)


def path_traced_image(sc, g, g_s, sun_dir, pe=1 / FOUR_PI):
    """Plain volumetric path tracing estimate of each pixel from the records:
    I = E_cam + sum_m (prod_{u<m} alpha_u rho_u/p_u) (e_m + alpha_m d_m), with
    the textbook HG form (written independently of the oracle); e_m is the
    emission collected at the collision (collision estimator)."""
    din, dout, denv = (a.astype(np.float64) for a in (sc.dir_in, sc.dir_out, sc.dir_env))
    sd = np.asarray(sun_dir, np.float64)
    f = lambda gg, a, b: hg_textbook(gg, np.clip((a * b).sum(-1), -1, 1))  # noqa: E731
    d = (f(g, din, sd[None])[:, None] * sc.l_sun
         + (f(g, din, denv) / (f(g_s, din, denv) + pe))[:, None] * sc.l_env
         + (f(g, din, dout) / (f(g_s, din, dout) + pe))[:, None] * sc.l_phase)
    if sc.dir_pl is not None:      # point light: its own shadow-ray sample, no MIS
        d = d + f(g, din, sc.dir_pl.astype(np.float64))[:, None] * sc.l_pl
    ratio = f(g, din, dout) / f(g_s, din, dout)
    img = np.zeros((sc.height * sc.width, 3))
    off = sc.path_offsets
    for p in range(sc.n_paths):
        L, beta = np.zeros(3), 1.0
        for v in range(off[p], off[p + 1]):
            if sc.l_emit is not None:
                L += beta * sc.l_emit[v]
            beta *= sc.albedo[v]
            L += beta * d[v]
            beta *= ratio[v]
        img[p // sc.spp] += (sc.e_cam[p] + L) / sc.spp
    return img.reshape(sc.height, sc.width, 3)


@pytest.mark.parametrize("init,D", [("pt", 0), ("pt", 3), ("zero", 7), ("zero", 12)])
def test_single_neighbour_reproduces_path_tracing(init, D):
    sc = small_scene()
    g, g_s = 0.5, 0.3
    p = oracle.params(k=1, D=D, g=g, g_s=g_s, init=init)
    ref = path_traced_image(sc, g, g_s, p["sun_dir"])
    # zero init needs D >= max depth - 1 iterations to reach every vertex.  The
    # reference evaluates cos as a dot product of float32 unit vectors, the
    # oracle as 1 - |a-b|^2/2: they differ by the vectors' norm error (~1e-7).
    assert np.allclose(oracle.render(sc, p), ref, rtol=2e-6, atol=1e-12)
    # and the own-sample output (final gather) is the same estimator at K = 1
    p["final_gather"] = 1
    assert np.allclose(oracle.render(sc, p), ref, rtol=2e-6, atol=1e-12)


@pytest.mark.parametrize("init,D", [("pt", 0), ("pt", 4), ("zero", 12)])
def test_single_neighbour_with_volume_emission_reproduces_path_tracing(init, D):
    sc = small_scene(emit=True)
    assert sc.l_emit is not None and (sc.l_emit > 0).any() and (sc.l_emit == 0).any()
    g, g_s = 0.5, 0.3
    p = oracle.params(k=1, D=D, g=g, g_s=g_s, init=init)
    ref = path_traced_image(sc, g, g_s, p["sun_dir"])
    assert np.allclose(oracle.render(sc, p), ref, rtol=2e-6, atol=1e-12)
    p["final_gather"] = 1
    assert np.allclose(oracle.render(sc, p), ref, rtol=2e-6, atol=1e-12)


def test_extra_first_vertex_samples_are_unbiased():
    # one-vertex paths, nothing occluded, environment radiance (w_z + 2) and a
    # sun of irradiance E: the pixel's direct term from M extra emitter
    # samples estimates rho(sun) E + int rho (w_z + 2) = rho(sun) E + 2 + g t_z
    rng = np.random.default_rng(21)
    n, M, g = 20000, 3, 0.6
    t = unit(rng, n)
    pos = rng.random((n, 3)) * 0.9 + 0.05
    sc = make_scene(pos, t, unit(rng, n), unit(rng, n))
    dirs = unit(rng, n * M).reshape(n, M, 3)
    E = np.array([0.7, 0.5, 0.3])
    sc = replace(sc, fb_l_sun=np.broadcast_to(E, (n, M, 3)).astype(np.float32).copy(),
                 fb_dir_env=dirs.astype(np.float32), fb_l_env=np.repeat(dirs[..., 2:3] + 2.0, 3, axis=2).astype(np.float32))
    p = oracle.params(k=1, D=0, g=g, g_s=g)
    img = oracle.render(sc, p).reshape(n, 3)
    sd = np.asarray(p["sun_dir"])
    rho_sun = hg_textbook(g, np.clip(t @ sd, -1, 1))
    dev = img - rho_sun[:, None] * E[None, :] - (2.0 + g * t[:, 2])[:, None]
    m, se = dev.mean(0), dev.std(0) / math.sqrt(n)
    assert np.all(np.abs(m) < 5 * se + 1e-12), (m, se)
    # the extra samples replace the path-traced direct term: without them the
    # same pixels use d_pt, which these records (all zero) make 0
    img0 = oracle.render(replace(sc, fb_l_sun=None, fb_dir_env=None, fb_l_env=None), p)
    assert np.allclose(img0, 0.0)


@pytest.mark.parametrize("init", ["pt", "zero"])
def test_single_neighbour_with_point_light_reproduces_path_tracing(init):
    sc = scenegen.generate(replace(scenegen.crop_of(scenegen.WORKLOADS["tiny"].scene, 16, 16, 2),
                                   pl_I=(0.4, 0.3, 0.2)))
    assert sc.l_pl is not None and (sc.l_pl > 0).any()
    g, g_s = 0.5, 0.3
    p = oracle.params(k=1, D=12, g=g, g_s=g_s, init=init)
    ref = path_traced_image(sc, g, g_s, p["sun_dir"])
    assert np.allclose(oracle.render(sc, p), ref, rtol=2e-6, atol=1e-12)


def test_point_light_aggregates_as_a_delta_light():
    # groups of coincident points: one light direction per group, so the
    # aggregated point-light term is rho_i(d) times the group's mean irradiance
    rng = np.random.default_rng(8)
    K, trials, g = 5, 30, 0.7
    centres = rng.random((trials, 3)) * 0.9 + 0.05
    pos = np.repeat(centres, K, axis=0)
    n = len(pos)
    t = unit(rng, n)
    dpl = np.repeat(unit(rng, trials), K, axis=0)
    lpl = rng.random((n, 3))
    sc = replace(make_scene(pos, t, unit(rng, n), unit(rng, n)), dir_pl=dpl.astype(np.float32),
                 l_pl=lpl.astype(np.float32))
    _, tr = oracle.render(sc, oracle.params(k=K, D=0, g=g, g_s=g), trace=True)
    rho = hg_textbook(g, np.clip((t * dpl).sum(1), -1, 1))
    mean = lpl.astype(np.float32).astype(np.float64).reshape(trials, K, 3).mean(1).repeat(K, axis=0)
    assert np.allclose(tr["d_agg"], rho[:, None] * mean, rtol=2e-6, atol=1e-12)
    assert np.allclose(tr["d_pt"], rho[:, None] * lpl.astype(np.float32), rtol=2e-6, atol=1e-12)


def test_zero_albedo_sees_first_collision_emission():
    # no scattering: a pixel averages what its camera rays see directly, the
    # environment if they escape and the emission of their first collision
    sc = small_scene(emit=True)
    sc.albedo[:] = 0.0
    img = oracle.render(sc, oracle.params(k=8, D=4))
    first = np.zeros((sc.n_paths, 3))
    has = np.diff(sc.path_offsets) > 0
    first[has] = sc.l_emit[sc.path_offsets[:-1][has]]
    expect = (sc.e_cam + first).reshape(sc.height, sc.width, sc.spp, 3).mean(2)
    assert np.allclose(img, expect, rtol=1e-15, atol=0)


def test_emission_inside_direct_radiance_decomposition():
    """The paper splits L = L^o + L^+ with the volume emission inside the known
    direct part L^o: the emission e_u collected at a vertex's successor is a
    phase-sampled direct sample, aggregated with the indirect weights, and the
    unknown L^+ starts from zero.  Written with dense operators from an
    emission-free trace, this must equal the render with l_emit."""
    sc = small_scene(10, 10, 2, emit=True)
    D = 7
    for init in ("zero", "pt"):
        p = oracle.params(k=6, D=D, g=0.5, init=init)
        img, tr = oracle.render(sc, p, trace=True)
        dark = replace(sc, l_emit=None)
        _, tr0 = oracle.render(dark, p, trace=True)
        M, c0, W = dense_operator(dark, tr0)
        N = sc.n_vertices
        # E_s(v): emission collected at v's successor (0 at a path's end)
        Es = np.zeros((N, 3))
        off = sc.path_offsets
        for q in range(sc.n_paths):
            Es[off[q]:off[q + 1] - 1] = sc.l_emit[off[q] + 1:off[q + 1]]
        alpha = sc.albedo.astype(np.float64)[:, None]
        shift = np.zeros((N, N))
        for q in range(sc.n_paths):
            for v in range(off[q], off[q + 1] - 1):
                shift[v, v + 1] = 1.0
        # scattered direct L-bar^o = alpha (d_agg + W E_s); L^+_t = M L^+_{t-1} + S L-bar^o
        c = c0 + shift @ (alpha * (W @ Es))
        Lp = (tr["lplus0"] - Es) if init == "pt" else np.zeros((N, 3))
        for _ in range(D):
            Lp = M @ Lp + c
        assert np.allclose(tr["lplus"], Es + Lp, rtol=1e-11, atol=1e-13), init
        first = off[:-1]
        has = np.diff(off) > 0
        o = np.zeros((sc.n_paths, 3))
        o[has] = (sc.l_emit[first[has]]
                  + alpha[first[has]] * (tr0["d_pt"][first[has]] + (W @ (Es + Lp))[first[has]]))
        expect = (sc.e_cam + o).reshape(sc.height, sc.width, sc.spp, 3).mean(2)
        assert np.allclose(img, expect, rtol=1e-11, atol=1e-14), init


def test_affine_in_volume_emission():
    sc = small_scene(12, 12, 2, emit=True)
    p = oracle.params(k=8, D=6, g=0.5)
    dark = oracle.render(replace(sc, l_emit=None), p)
    one = oracle.render(sc, p)
    two = oracle.render(replace(sc, l_emit=sc.l_emit * np.float32(2.0)), p)
    assert not np.allclose(one, dark)
    assert np.allclose(two - one, one - dark, rtol=1e-10, atol=1e-14)


def test_zero_albedo_leaves_camera_emission_only():
    sc = small_scene()
    sc.albedo[:] = 0.0
    img = oracle.render(sc, oracle.params(k=8, D=4))
    expect = sc.e_cam.astype(np.float64).reshape(sc.height, sc.width, sc.spp, 3).mean(2)
    assert np.array_equal(img, expect)


def test_linear_in_light_radiance():
    sc = scenegen.generate(replace(scenegen.crop_of(scenegen.WORKLOADS["tiny"].scene, 16, 16, 2),
                                   pl_I=(0.4, 0.3, 0.2)))
    p = oracle.params(k=8, D=5)
    a = oracle.render(sc, p)
    for name in ("l_sun", "l_env", "l_phase", "e_cam", "l_pl"):
        setattr(sc, name, getattr(sc, name) * np.float32(2.0))
    assert np.allclose(oracle.render(sc, p), 2 * a, rtol=1e-12)


def dense_operator(sc, tr):
    """M = S diag(alpha) W and c = S b as dense matrices (S: shift to predecessor)."""
    N = sc.n_vertices
    rows = np.repeat(np.arange(N), np.diff(tr["row_ptr"]))
    W = np.zeros((N, N))
    np.add.at(W, (rows, tr["col"].ravel()), tr["w_ind"].ravel())
    A = sc.albedo.astype(np.float64)[:, None] * W
    S = np.zeros((N, N))
    off = sc.path_offsets
    for p in range(sc.n_paths):
        for v in range(off[p], off[p + 1] - 1):
            S[v, v + 1] = 1.0
    return S @ A, S @ tr["b"], W


@pytest.mark.parametrize("init", ["zero", "pt"])
def test_iteration_is_truncated_neumann_series(init):
    sc = small_scene(12, 12, 2)
    D = 9
    p = oracle.params(k=6, D=D, g=0.5, init=init)
    img, tr = oracle.render(sc, p, trace=True)
    M, c, W = dense_operator(sc, tr)
    L = tr["lplus0"] if init == "pt" else np.zeros_like(c)
    if init == "zero":
        assert not tr["lplus0"].any()
    L = np.linalg.matrix_power(M, D) @ L + sum(np.linalg.matrix_power(M, t) @ c for t in range(D))
    assert np.allclose(tr["lplus"], L, rtol=1e-12, atol=1e-14)
    # output: o_p = alpha_v0 (d_pt_v0 + (W L_D)_v0), averaged with E_cam per pixel
    first = sc.path_offsets[:-1]
    has = np.diff(sc.path_offsets) > 0
    o = np.zeros((sc.n_paths, 3))
    o[has] = sc.albedo[first[has], None] * (tr["d_pt"][first[has]] + (W @ tr["lplus"])[first[has]])
    expect = ((sc.e_cam + o).reshape(sc.height, sc.width, sc.spp, 3)).mean(2)
    assert np.allclose(img, expect, rtol=1e-12, atol=1e-15)


def test_iteration_converges_to_linear_solve():
    # D -> infinity: the fixed point solves (I - M) L = c (eq. rte-mff)
    sc = small_scene(10, 10, 2)
    p = oracle.params(k=6, D=200, g=0.5, init="zero")
    _, tr = oracle.render(sc, p, trace=True)
    M, c, _ = dense_operator(sc, tr)
    assert max(abs(np.linalg.eigvals(M))) < 0.95
    Lstar = np.linalg.solve(np.eye(len(c)) - M, c)
    assert np.allclose(tr["lplus"], Lstar, rtol=1e-9, atol=1e-12)


# ------------------------------------------------ cluster neighbours ---

def keyed(sc, seed=7):
    return replace(sc, cluster_key=scenegen.cluster_keys(sc.n_vertices, seed))


def test_cluster_centres_and_nearest_assignment():
    # K = 64 on 3000 uniform points: the ~47 initial clusters average 64
    # members, under 2K, so nothing is split and every vertex's centre is the
    # nearest centre -- checked with scipy's kd-tree on the quantised positions
    rng = np.random.default_rng(3)
    pos = rng.random((3000, 3), dtype=np.float32)
    key = scenegen.cluster_keys(3000, 5)
    K = 64
    ctr = oracle.clusters(pos, key, K)
    is_c = (key.astype(np.uint64) < (2 ** 32) // K)
    is_c[np.argmin(key)] = True
    centres = np.flatnonzero(is_c)
    assert set(np.unique(ctr)) <= set(centres)
    sizes = np.bincount(ctr, minlength=3000)[centres]
    if sizes.max() <= 2 * K:
        q, _ = oracle.quantize(pos)
        _, nn = spatial.cKDTree(q[centres].astype(np.float64)).query(q.astype(np.float64))
        assert np.array_equal(ctr, centres[nn])
    else:
        pytest.fail("seed gives a large cluster; pick another")
    assert np.array_equal(ctr[centres], centres)      # a centre is in its own cluster
    # about N/K centres: binomial(3000, 1/64) within 5 sigma
    assert abs(len(centres) - 3000 / K) < 5 * math.sqrt(3000 / K)


def test_cluster_split_refines_and_evens_out():
    # clustered input: one dense blob gets few centres' worth of points, so
    # large clusters appear and are split; the result refines the initial
    # nearest-centre partition and leaves no cluster above 2K
    rng = np.random.default_rng(9)
    pos = np.concatenate([rng.random((2000, 3)) * 0.05 + 0.5, rng.random((2000, 3))]).astype(np.float32)
    key = scenegen.cluster_keys(4000, 11)
    K = 8
    ctr = oracle.clusters(pos, key, K)
    is_c = key.astype(np.uint64) < (2 ** 32) // K
    is_c[np.argmin(key)] = True
    centres = np.flatnonzero(is_c)
    q, _ = oracle.quantize(pos)
    _, nn = spatial.cKDTree(q[centres].astype(np.float64)).query(q.astype(np.float64))
    init = centres[nn]
    big = np.bincount(init, minlength=4000).max()
    assert big > 2 * K                                   # the split is exercised
    # refinement: members of a final cluster share their initial cluster
    for c in np.unique(ctr):
        assert len(np.unique(init[ctr == c])) == 1
    assert np.bincount(ctr, minlength=4000).max() <= 2 * K
    # relabelling invariance (distinct keys, generic positions)
    perm = rng.permutation(4000)
    ctr_p = oracle.clusters(pos[perm], key[perm], K)
    assert np.array_equal(perm[ctr_p], ctr[perm])


def test_cluster_weights_equal_knn_weights_on_separated_groups():
    # groups of K coincident points, far apart, one centre each: the cluster
    # of a vertex is exactly its k nearest set, so the cluster relation must
    # give the kNN relation's (pinned) weights and direct terms, row by row
    rng = np.random.default_rng(4)
    K, trials = 6, 40
    sc, _, _ = clustered(rng, trials, K, 0.4, lambda d: np.repeat((d[:, 2:3] + 2.0), 3, axis=1))
    key = np.full(sc.n_vertices, 2 ** 32 - 1, np.uint32)
    key[::K] = np.arange(trials, dtype=np.uint32)         # the first of each group is its centre
    sc = replace(sc, cluster_key=key)
    assert np.array_equal(oracle.clusters(sc.pos, key, K), np.repeat(np.arange(0, trials * K, K), K))
    pk = oracle.params(k=K, D=3, g=0.6, g_s=0.4)
    pc = dict(pk, neighbours="clusters")
    img_k, tk = oracle.render(sc, pk, trace=True)
    img_c, tc = oracle.render(sc, pc, trace=True)
    assert np.array_equal(tc["row_ptr"], np.arange(sc.n_vertices + 1) * K)
    for i in range(sc.n_vertices):
        a, b = tc["row_ptr"][i], tc["row_ptr"][i + 1]
        order_k = np.argsort(tk["col"][i])
        assert np.array_equal(tc["col"][a:b], tk["col"][i][order_k])
        for name in ("w_ind", "w_ph", "w_env"):
            assert np.allclose(tc[name][a:b], tk[name][i][order_k], rtol=1e-13, atol=0)
    for name in ("b", "d_pt", "lplus"):
        assert np.allclose(tc[name], tk[name], rtol=1e-12, atol=1e-15)
    assert np.allclose(img_c, img_k, rtol=1e-12, atol=1e-15)


def test_cluster_rows_share_one_marginal():
    # every receiver of a cluster combines the same techniques, so for a
    # sample j the weight w+_ij times rho_i(w_j)^-1 (textbook HG) is the same
    # for all receivers i of the cluster: 1 / sum_l p_l(w_j)
    sc = keyed(small_scene(10, 10, 2))
    g, g_s = 0.5, 0.3
    p = oracle.params(k=8, D=2, g=g, g_s=g_s, neighbours="clusters")
    _, tr = oracle.render(sc, p, trace=True)
    rp, col = tr["row_ptr"], tr["col"]
    ctr = oracle.clusters(sc.pos, sc.cluster_key, 8)
    assert np.array_equal((rp, col)[1], oracle.cluster_rows(ctr)[1])
    din, dout = sc.dir_in.astype(np.float64), sc.dir_out.astype(np.float64)
    inv_m = {}
    for i in range(sc.n_vertices):
        js = col[rp[i]:rp[i + 1]]
        assert i in js and np.all(np.diff(js) > 0)
        rho = hg_textbook(g, np.clip((din[i] * dout[js]).sum(1), -1, 1))
        for j, v in zip(js, tr["w_ind"][rp[i]:rp[i + 1]] / rho):
            if j in inv_m:
                assert abs(v - inv_m[j]) <= 1e-6 * inv_m[j]
            else:
                inv_m[j] = v
    for j, v in inv_m.items():
        members = col[rp[j]:rp[j + 1]]
        m = hg_textbook(g_s, np.clip((din[members] * dout[j]).sum(1), -1, 1)).sum()
        assert abs(v * m - 1.0) <= 1e-6


def test_cluster_weights_are_column_stochastic_when_g_equals_g_s():
    # every receiver of a cluster is also one of its techniques, so with
    # rho = p (g = g_s) the weights a sample gets over the cluster's
    # receivers sum to exactly 1: sum_i rho_i(w_j) / sum_l p_l(w_j) = 1.
    # The k nearest relation lacks this (neighbour sets are not shared).
    sc = keyed(small_scene(12, 12, 2))
    N = sc.n_vertices
    for g in (0.8, 0.3, -0.2):
        for neigh in ("clusters", "knn"):
            _, tr = oracle.render(sc, oracle.params(k=8, D=1, g=g, g_s=g, neighbours=neigh), trace=True)
            colsum = np.zeros(N)
            np.add.at(colsum, tr["col"].ravel(), tr["w_ind"].ravel())
            if neigh == "clusters":
                assert np.allclose(colsum, 1.0, rtol=0, atol=1e-12), g
            else:
                assert colsum.max() > 1.2, g     # hubs: samples shared by many receivers


@pytest.mark.parametrize("init", ["pt", "zero"])
def test_cluster_single_member_reproduces_path_tracing(init):
    # k = 1: every key is below 2^32, every vertex is its own cluster
    sc = keyed(small_scene())
    g, g_s = 0.5, 0.3
    p = oracle.params(k=1, D=12, g=g, g_s=g_s, init=init, neighbours="clusters")
    ref = path_traced_image(sc, g, g_s, p["sun_dir"])
    assert np.allclose(oracle.render(sc, p), ref, rtol=2e-6, atol=1e-12)


def test_cluster_iteration_is_truncated_neumann_series():
    sc = keyed(small_scene(12, 12, 2))
    D = 8
    p = oracle.params(k=6, D=D, g=0.5, init="zero", neighbours="clusters")
    img, tr = oracle.render(sc, p, trace=True)
    M, c, W = dense_operator(sc, tr)
    # block structure: W's pattern is symmetric
    assert np.array_equal(W != 0, (W != 0).T)
    L = sum(np.linalg.matrix_power(M, t) @ c for t in range(D))
    assert np.allclose(tr["lplus"], L, rtol=1e-12, atol=1e-14)


def test_cluster_adjoint_matches_central_differences():
    sc = keyed(small_scene(8, 8, 2))
    rng = np.random.default_rng(6)
    p = oracle.params(k=6, D=4, g=0.6, g_s=0.6, neighbours="clusters")
    alpha = rng.uniform(0.6, 0.95, sc.n_vertices)
    img = oracle.render(sc, p, alpha=alpha)
    target = rng.uniform(0, 2 * img.mean(), size=img.shape)
    sc2 = replace(sc, albedo=alpha.astype(np.float32))
    alpha = sc2.albedo.astype(np.float64)
    img = oracle.render(sc2, p)
    out = oracle.backward(sc2, p, 2.0 * (img - target))
    h = 1e-5
    loss = lambda q, a: ((oracle.render(sc2, q, alpha=a) - target) ** 2).sum()  # noqa: E731
    fd_g = (loss(dict(p, g=p["g"] + h), alpha) - loss(dict(p, g=p["g"] - h), alpha)) / (2 * h)
    assert abs(out["grad_g"] - fd_g) <= 1e-6 * abs(fd_g) + 1e-9
    for i in np.argsort(-np.abs(out["grad_alpha"]))[:5]:
        e = np.zeros_like(alpha)
        e[i] = h
        fd = (loss(p, alpha + e) - loss(p, alpha - e)) / (2 * h)
        assert abs(out["grad_alpha"][i] - fd) <= 1e-6 * abs(fd) + 1e-9


# ------------------------------------------------------------- adjoint ---

def loss_and_grad(sc, p, grid, target):
    out = oracle.backward(sc, p, 2.0 * (oracle.render(sc, p, alpha=oracle.albedo_from_grid(sc.pos, grid))
                                        - target), grid=grid)
    return out


@pytest.mark.parametrize("init,fg,emit", [("pt", 0, False), ("zero", 0, False), ("pt", 1, False),
                                           ("pt", 0, True), ("zero", 0, True), ("pt", 1, "extra"),
                                           ("pt", 0, "point"), ("zero", 1, "extra+point")])
def test_adjoint_matches_central_differences(init, fg, emit):
    if emit in ("extra", "point", "extra+point"):
        cfg = scenegen.crop_of(scenegen.WORKLOADS["tiny"].scene, 8, 8, 2)
        if "extra" in emit:
            cfg = replace(cfg, extra_samples=3)
        if "point" in emit:
            cfg = replace(cfg, pl_I=(0.4, 0.3, 0.2))
        sc = scenegen.generate(cfg)
    else:
        sc = small_scene(8, 8, 2, emit=emit)
    rng = np.random.default_rng(5)
    R = 6
    grid = rng.uniform(0.6, 0.95, size=(R, R, R)).astype(np.float32)
    p = oracle.params(k=6, D=5, g=0.6, g_s=0.6, init=init, final_gather=fg)
    alpha = oracle.albedo_from_grid(sc.pos, grid)
    img = oracle.render(sc, p, alpha=alpha)
    target = rng.uniform(0, 2 * img.mean(), size=img.shape)

    def loss(gr, g):
        q = dict(p, g=g)
        return ((oracle.render(sc, q, alpha=oracle.albedo_from_grid(sc.pos, gr)) - target) ** 2).sum()

    out = oracle.backward(sc, p, 2.0 * (img - target), grid=grid)
    assert np.allclose(out["image"], img, rtol=1e-14)
    h = 1e-5
    fd_g = (loss(grid, p["g"] + h) - loss(grid, p["g"] - h)) / (2 * h)
    assert abs(out["grad_g"] - fd_g) <= 1e-6 * abs(fd_g) + 1e-9
    gg = out["grad_grid"]
    for flat in np.argsort(-np.abs(gg).ravel())[:6]:
        # the grid enters only through alpha, linearly: alpha(A + h e) = alpha + h w,
        # w = the voxel's trilinear weight per vertex (interpolate a one-hot grid)
        onehot = np.zeros(grid.size, np.float32)
        onehot[flat] = 1.0
        w = oracle.albedo_from_grid(sc.pos, onehot.reshape(grid.shape))
        lp = ((oracle.render(sc, p, alpha=alpha + h * w) - target) ** 2).sum()
        lm = ((oracle.render(sc, p, alpha=alpha - h * w) - target) ** 2).sum()
        fd = (lp - lm) / (2 * h)
        assert abs(gg.ravel()[flat] - fd) <= 1e-6 * abs(fd) + 1e-9


def test_adjoint_per_vertex_albedo_matches_central_differences():
    sc = small_scene(8, 8, 2)
    rng = np.random.default_rng(9)
    p = oracle.params(k=6, D=4, g=0.5)
    img = oracle.render(sc, p)
    target = rng.uniform(0, 2 * img.mean(), size=img.shape)
    out = oracle.backward(sc, p, 2.0 * (img - target))
    a0 = sc.albedo.astype(np.float64)
    h = 1e-6
    for v in rng.choice(sc.n_vertices, 8, replace=False):
        ap, am = a0.copy(), a0.copy()
        ap[v] += h
        am[v] -= h
        fd = (((oracle.render(sc, p, alpha=ap) - target) ** 2).sum()
              - ((oracle.render(sc, p, alpha=am) - target) ** 2).sum()) / (2 * h)
        assert abs(out["grad_alpha"][v] - fd) <= 1e-6 * abs(fd) + 1e-9


# ------------------------------------------------- hand-derived example ---

def test_two_path_worked_example():
    from tests.golden.fixtures import load
    sc, d = load("two_paths_isotropic.json")
    for case in d["cases"]:
        p = oracle.params(k=d["k"], D=case["D"], g=d["g"], init=case["init"],
                          final_gather=case["final_gather"])
        img, tr = oracle.render(sc, p, trace=True)
        assert tr["col"].tolist() == d["expected_col"]
        assert np.allclose(tr["d_pt"][:, 0], d["expected_d_pt"], rtol=1e-15)
        assert np.allclose(tr["b"][:, 0], d["expected_b"], rtol=1e-15)
        assert np.allclose(img[0, :, 1], case["image"], rtol=1e-15), case


def test_trilinear_albedo_reproduces_linear_fields():
    # cell-centred trilinear interpolation is exact for a linear field away from
    # the outer half cell, and clamps (constant extension) inside it
    R = 8
    c = (np.arange(R) + 0.5) / R
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    grid = (0.2 + 0.3 * X + 0.1 * Y + 0.25 * Z).astype(np.float32)
    rng = np.random.default_rng(2)
    pos = rng.uniform(0.5 / R, 1 - 0.5 / R, size=(500, 3)).astype(np.float32)
    ref = 0.2 + 0.3 * pos[:, 0] + 0.1 * pos[:, 1] + 0.25 * pos[:, 2]
    assert np.allclose(oracle.albedo_from_grid(pos, grid), ref, atol=1e-6)
    edge = np.array([[0.01, 0.5, 0.5]], np.float32)   # x inside the first half cell
    inner = np.array([[0.5 / R, 0.5, 0.5]], np.float32)
    assert np.allclose(oracle.albedo_from_grid(edge, grid), oracle.albedo_from_grid(inner, grid), atol=1e-7)


@pytest.mark.parametrize("n,k", [(1, 8), (7, 8), (400, 16), (300, 1)])
def test_knn_row_scan_matches_brute_force(n, k):
    # a few given rows take the direct scan over every vertex; lattice ties and
    # duplicate positions exercise the (d2, index) order there as well
    rng = np.random.default_rng(n + 17 * k)
    pos = rng.random((n, 3), dtype=np.float32)
    if n >= 400:
        pos[:64] = ((np.indices((4, 4, 4)).reshape(3, -1).T + 1) / 8.0).astype(np.float32)
        pos[64:70] = pos[3]
    rows = np.unique(rng.integers(0, n, size=min(n, 40)))
    assert np.array_equal(oracle.knn(pos, k, rows=rows), knn_brute(pos, k)[rows])
    assert np.array_equal(oracle.knn(pos, k, rows=rows), oracle.knn(pos, k)[rows])
