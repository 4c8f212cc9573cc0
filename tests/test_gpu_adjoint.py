"""GPU reverse mode against the FP64 oracle's gradient (itself pinned to FP64
central differences), the autograd wrapper, and GPU central differences.

Gradient tolerance (tests.gpu_util.grad_close): |err| <= 1e-4 |ref| per
component; the albedo gradients take a floor of 1e-5 times the same gradient
of |grad_image| (the summed magnitude of the terms, which bounds the FP32
accumulation error where terms of both signs cancel); dL/dg has no floor.
"""
import numpy as np
import pytest
import torch

import oracle
import scenegen
import paper_2404_11894_amd as pg
from tests.gpu_util import crop, grad_close, synthetic

pytestmark = pytest.mark.gpu


def case(sc, R, k, D, g, init="pt", fg=0, seed=5, lo=0.6, hi=0.95):
    rng = np.random.default_rng(seed)
    grid = rng.uniform(lo, hi, size=(R, R, R)).astype(np.float32)
    op = oracle.params(k=k, D=D, g=g, init=init, final_gather=fg)
    alpha = oracle.albedo_from_grid(sc.pos, grid)
    img = oracle.render(sc, op, alpha=alpha)
    target = scenegen.target_image(img.shape, float(img.mean()), seed=4).astype(np.float64)
    gimg = 2.0 * (img - target)                  # d/dI of sum (I - T)^2 at the oracle image
    ref = oracle.backward(sc, op, gimg, grid=grid)
    ref["mag"] = oracle.backward(sc, op, np.abs(gimg), grid=grid)
    return grid, gimg, ref


@pytest.mark.parametrize("init,fg,emit", [("pt", 0, False), ("zero", 0, False), ("pt", 1, False),
                                           ("pt", 0, True), ("zero", 1, True)])
def test_backward_matches_oracle(init, fg, emit):
    sc = crop("tiny", 32, 32, 2, emit_L=(3.0, 2.0, 1.0) if emit else None)
    print(f"adjoint init={init} fg={fg} emission={emit} N={sc.n_vertices}", flush=True)
    grid, gimg, ref = case(sc, 8, 8, 6, 0.5, init, fg)
    paths = pg.DevicePaths(sc, albedo_grid=grid)
    q = pg.params(k=8, D=6, g=0.5, init=init, final_gather=fg, flags=pg.PG_FLAG_CHECK)
    out = pg.pg_backward(paths, q, torch.from_numpy(gimg.astype(np.float32)), grad_albedo=True)
    torch.cuda.synchronize()
    grad_close(out["grad_grid"].cpu().numpy(), ref["grad_grid"], "grad grid", ref["mag"]["grad_grid"])
    grad_close(out["grad_albedo"].cpu().numpy(), ref["grad_alpha"], "grad albedo", ref["mag"]["grad_alpha"])
    grad_close([out["grad_g"].item()], [ref["grad_g"]], "grad g")


@pytest.mark.parametrize("D", [0, 3])
def test_backward_paths_longer_than_a_wave(D):
    """The adjoint of the path-traced initial value takes a path 64 vertices
    at a time: paths of 1, 41, 64, 65, 129 and 200 vertices and an empty one."""
    rng = np.random.default_rng(9)
    lengths = np.array([200, 1, 64, 65, 129, 0, 41])
    sc = synthetic(rng.random((int(lengths.sum()), 3)), rng, lengths=lengths)
    print(f"adjoint long paths D={D} N={sc.n_vertices}", flush=True)
    grid, gimg, ref = case(sc, 8, 8, D, 0.5, "pt", 0)
    paths = pg.DevicePaths(sc, albedo_grid=grid)
    q = pg.params(k=8, D=D, g=0.5, flags=pg.PG_FLAG_CHECK)
    out = pg.pg_backward(paths, q, torch.from_numpy(gimg.astype(np.float32)), grad_albedo=True)
    torch.cuda.synchronize()
    grad_close(out["grad_grid"].cpu().numpy(), ref["grad_grid"], "grad grid", ref["mag"]["grad_grid"])
    grad_close(out["grad_albedo"].cpu().numpy(), ref["grad_alpha"], "grad albedo", ref["mag"]["grad_alpha"])
    grad_close([out["grad_g"].item()], [ref["grad_g"]], "grad g")


@pytest.mark.parametrize("extra,point", [(3, False), (0, True), (2, True)])
def test_backward_with_extra_samples_and_point_light(extra, point):
    from dataclasses import replace
    cfg = replace(scenegen.crop_of(scenegen.WORKLOADS["tiny"].scene, 32, 32, 2), extra_samples=extra)
    if point:
        cfg = replace(cfg, pl_I=(0.4, 0.3, 0.2))
    sc = scenegen.generate(cfg)
    print(f"adjoint extra={extra} point={point} N={sc.n_vertices}", flush=True)
    grid, gimg, ref = case(sc, 8, 8, 6, 0.5, "pt", 0)
    paths = pg.DevicePaths(sc, albedo_grid=grid)
    q = pg.params(k=8, D=6, g=0.5, flags=pg.PG_FLAG_CHECK)
    out = pg.pg_backward(paths, q, torch.from_numpy(gimg.astype(np.float32)), grad_albedo=True)
    torch.cuda.synchronize()
    grad_close(out["grad_grid"].cpu().numpy(), ref["grad_grid"], "grad grid", ref["mag"]["grad_grid"])
    grad_close(out["grad_albedo"].cpu().numpy(), ref["grad_alpha"], "grad albedo", ref["mag"]["grad_alpha"])
    grad_close([out["grad_g"].item()], [ref["grad_g"]], "grad g")


def test_backward_with_transpose_overflow():
    """200 coincident points: the lowest ids among them are everyone's
    tie-broken neighbours, so their in-degree (about 200) exceeds the 2k
    entries a row of the transposed operator holds and the excess takes the
    overflow list."""
    rng = np.random.default_rng(7)
    pos = np.concatenate([np.full((200, 3), 0.41), rng.random((100, 3))])
    sc = synthetic(pos, rng, lengths=np.full(30, 10))
    print(f"overflow N={sc.n_vertices}", flush=True)
    grid, gimg, ref = case(sc, 4, 4, 5, 0.6)
    paths = pg.DevicePaths(sc, albedo_grid=grid)
    q = pg.params(k=4, D=5, g=0.6, flags=pg.PG_FLAG_CHECK)
    out = pg.pg_backward(paths, q, torch.from_numpy(gimg.astype(np.float32)), grad_albedo=True)
    torch.cuda.synchronize()
    grad_close(out["grad_grid"].cpu().numpy(), ref["grad_grid"], "grad grid", ref["mag"]["grad_grid"])
    grad_close(out["grad_albedo"].cpu().numpy(), ref["grad_alpha"], "grad albedo", ref["mag"]["grad_alpha"])
    grad_close([out["grad_g"].item()], [ref["grad_g"]], "grad g")


@pytest.mark.parametrize("k", [33, 40, 64])
def test_backward_rows_longer_than_32(k):
    """Rows of more than 32 neighbours: the transposed operator's counting
    pass takes one global atomic per edge there, and the reverse rows their
    generic width."""
    rng = np.random.default_rng(11)
    sc = synthetic(rng.random((600, 3)), rng, lengths=np.full(30, 20))
    print(f"adjoint k={k} N={sc.n_vertices}", flush=True)
    grid, gimg, ref = case(sc, 4, k, 4, 0.6)
    paths = pg.DevicePaths(sc, albedo_grid=grid)
    q = pg.params(k=k, D=4, g=0.6, flags=pg.PG_FLAG_CHECK)
    out = pg.pg_backward(paths, q, torch.from_numpy(gimg.astype(np.float32)), grad_albedo=True)
    torch.cuda.synchronize()
    grad_close(out["grad_grid"].cpu().numpy(), ref["grad_grid"], "grad grid", ref["mag"]["grad_grid"])
    grad_close(out["grad_albedo"].cpu().numpy(), ref["grad_alpha"], "grad albedo", ref["mag"]["grad_alpha"])
    grad_close([out["grad_g"].item()], [ref["grad_g"]], "grad g")


def test_backward_workload_crop_matches_oracle():
    """The differentiation workload: the 128^3 ball's paths held fixed, albedo
    from a 64^3 grid (U[0.95,0.999], seed 2), k 16, D 64, g 0.8, on the
    centred 64x64-pixel, 2-spp crop where the oracle gradient is affordable."""
    w = scenegen.WORKLOADS["mid"]
    sc = scenegen.generate(scenegen.crop_of(w.scene, 64, 64, 2))
    print(f"workload crop N={sc.n_vertices}", flush=True)
    grid = scenegen.albedo_grid(64, 0.95, 0.999, seed=2)
    op = oracle.params(k=w.k, D=w.D, g=w.g)
    img = oracle.render(sc, op, alpha=oracle.albedo_from_grid(sc.pos, grid))
    target = scenegen.target_image(img.shape, float(img.mean()), seed=4).astype(np.float64)
    gimg = 2.0 * (img - target)
    ref = oracle.backward(sc, op, gimg, grid=grid)
    mag = oracle.backward(sc, op, np.abs(gimg), grid=grid)
    paths = pg.DevicePaths(sc, albedo_grid=grid)
    q = pg.params(k=w.k, D=w.D, g=w.g, flags=pg.PG_FLAG_CHECK)
    out = pg.pg_backward(paths, q, torch.from_numpy(gimg.astype(np.float32)))
    torch.cuda.synchronize()
    grad_close(out["grad_grid"].cpu().numpy(), ref["grad_grid"], "grad grid", mag["grad_grid"])
    grad_close([out["grad_g"].item()], [ref["grad_g"]], "grad g")


def test_autograd_function_uses_the_tape():
    sc = crop("tiny", 32, 32, 2)
    rng = np.random.default_rng(7)
    grid0 = rng.uniform(0.6, 0.95, size=(8, 8, 8)).astype(np.float32)
    paths = pg.DevicePaths(sc)
    q = pg.params(k=8, D=5, g=0.5)
    grid = torch.tensor(grid0, device="cuda", requires_grad=True)
    g = torch.tensor(0.5, device="cuda", requires_grad=True)
    img = pg.render_differentiable(paths, q, grid, g)
    target = torch.rand_like(img) * img.mean().detach() * 2
    loss = ((img - target) ** 2).sum()
    loss.backward()
    # same gradients as a stateless pg_backward that recomputes the forward pass
    paths2 = pg.DevicePaths(sc, albedo_grid=grid0)
    out = pg.pg_backward(paths2, q, 2.0 * (img.detach() - target))
    torch.cuda.synchronize()
    assert np.allclose(grid.grad.cpu().numpy(), out["grad_grid"].cpu().numpy(), rtol=1e-5, atol=1e-7)
    assert np.isclose(g.grad.item(), out["grad_g"].item(), rtol=1e-5)
    # and the forward image is the plain render's
    img2 = pg.pg_render(paths2, q)
    torch.cuda.synchronize()
    assert torch.equal(img.detach(), img2)


def test_backward_matches_gpu_central_differences():
    """FP32 central differences (h = 1e-3) of the GPU loss on 32 voxels and g."""
    sc = crop("tiny", 32, 32, 2)
    rng = np.random.default_rng(8)
    R = 8
    grid0 = rng.uniform(0.6, 0.95, size=(R, R, R)).astype(np.float32)
    q = pg.params(k=8, D=6, g=0.5)
    paths = pg.DevicePaths(sc, albedo_grid=grid0)
    img = pg.pg_render(paths, q).double()
    target = torch.rand_like(img) * img.mean() * 2

    def loss(grid, g):
        paths.set_albedo_grid(grid)
        qq = pg.params(k=8, D=6, g=g, g_s=0.5)
        return float(((pg.pg_render(paths, qq).double() - target) ** 2).sum())

    paths.set_albedo_grid(grid0)
    out = pg.pg_backward(paths, q, (2.0 * (img - target)).float())
    gg = out["grad_grid"].cpu().numpy().ravel()
    h = 1e-3
    picks = rng.choice(np.flatnonzero(np.abs(gg) > 0), 32, replace=False)
    fd = []
    for flat in picks:
        gp, gm = grid0.copy().ravel(), grid0.copy().ravel()
        gp[flat] += h
        gm[flat] -= h
        fd.append((loss(gp.reshape(grid0.shape), 0.5) - loss(gm.reshape(grid0.shape), 0.5)) / (2 * h))
    fd = np.array(fd)
    adj = gg[picks]
    scale = np.abs(gg).max()
    assert np.all(np.abs(fd - adj) <= 0.02 * np.abs(adj) + 2e-3 * scale), np.c_[fd, adj]
    fd_g = (loss(grid0, 0.5 + h) - loss(grid0, 0.5 - h)) / (2 * h)
    assert abs(fd_g - out["grad_g"].item()) <= 0.02 * abs(fd_g) + 1e-3


@pytest.mark.parametrize("k,init", [(8, "pt"), (16, "zero"), (12, "pt"), (20, "pt")])
def test_stored_sums_match_the_oracle_and_the_recomputing_sweep(k, init):
    """PG_FLAG_STORE_Z: the taped forward keeps z_t and dz_t/dg and the
    reverse rows read them (k = 20 has no stored sums: the flag leaves the
    recomputing sweep).  Against the oracle at the usual tolerance; against
    the recomputing sweep to 1e-6 relative (the two calls build their own
    sorted layouts, whose in-cell order, and so the reverse sums' order, may
    differ in the last bits); the taped render's image equals the plain one."""
    sc = crop("mid", 40, 40, 1)
    print(f"stored sums k={k} init={init} N={sc.n_vertices}", flush=True)
    D = 6
    grid, gimg, ref = case(sc, 8, k, D, 0.7, init)
    paths = pg.DevicePaths(sc, albedo_grid=grid)
    base = dict(k=k, D=D, g=0.7, init=init)
    gi = torch.from_numpy(gimg.astype(np.float32))
    plain = pg.pg_backward(paths, pg.params(**base, flags=pg.PG_FLAG_CHECK), gi, grad_albedo=True)
    stored = pg.pg_backward(paths, pg.params(**base, flags=pg.PG_FLAG_CHECK | pg.PG_FLAG_STORE_Z), gi,
                            grad_albedo=True)
    torch.cuda.synchronize()
    for key in ("grad_grid", "grad_albedo"):
        a, b = stored[key].cpu().numpy(), plain[key].cpu().numpy()
        scale = np.abs(b).max()
        assert np.allclose(a, b, rtol=1e-6, atol=1e-6 * scale), key
    assert np.isclose(stored["grad_g"].item(), plain["grad_g"].item(), rtol=1e-6)
    grad_close(stored["grad_grid"].cpu().numpy(), ref["grad_grid"], "grad grid", ref["mag"]["grad_grid"])
    grad_close(stored["grad_albedo"].cpu().numpy(), ref["grad_alpha"], "grad albedo", ref["mag"]["grad_alpha"])
    grad_close([stored["grad_g"].item()], [ref["grad_g"]], "grad g")
    # the taped forward (aggregation with the sums stored) renders the plain
    # image, and pg_backward on its workspace (sized by the query, so the
    # stored sums must fit in it) gives the stateless call's gradients
    import ctypes
    q_tape = pg.params(**base, flags=pg.PG_FLAG_TAPE | pg.PG_FLAG_STORE_Z)
    s = paths.struct()
    nb = ctypes.c_size_t()
    pg._check(pg.lib().pg_render_workspace_size(ctypes.byref(s), ctypes.byref(q_tape), ctypes.byref(nb)))
    _, ws, n = pg._workspace(nb.value, paths.device)
    img_tape = torch.empty(sc.height, sc.width, 3, device=paths.device)
    pg._check(pg.lib().pg_render(ctypes.byref(s), ctypes.byref(q_tape), pg._ptr(img_tape), None, pg._ptr(ws), n,
                                 pg._stream(paths.device)))
    reused = pg.pg_backward(paths, q_tape, gi, grad_albedo=True, workspace=(ws, n))
    img = pg.pg_render(paths, pg.params(**base))
    torch.cuda.synchronize()
    assert torch.equal(img_tape, img)
    for key in ("grad_grid", "grad_albedo"):
        a, b = reused[key].cpu().numpy(), plain[key].cpu().numpy()
        assert np.allclose(a, b, rtol=1e-6, atol=1e-6 * np.abs(b).max()), key
    assert np.isclose(reused["grad_g"].item(), plain["grad_g"].item(), rtol=1e-6)
