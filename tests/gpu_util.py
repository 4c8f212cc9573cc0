"""Helpers shared by the GPU tests: tolerances and small synthetic scenes."""
import math
from dataclasses import replace

import numpy as np

import scenegen

# Pixel radiance and propagated radiance: |err| <= max(1e-4 |ref|, 1e-5).
PIX_REL, PIX_ABS = 1e-4, 1e-5
# Edge weights and direct terms: one FP32 evaluation of the same formula,
# accumulated over at most 2K terms.
W_REL, W_ABS = 2e-5, 1e-9


def within(got, ref, rel, abs_):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    err = np.abs(got - ref)
    tol = np.maximum(rel * np.abs(ref), abs_)
    return bool(np.all(err <= tol)), float(err.max(initial=0.0)), float((err / np.maximum(np.abs(ref), abs_)).max(initial=0.0))


def assert_within(got, ref, rel, abs_, what=""):
    ok, emax, rmax = within(got, ref, rel, abs_)
    assert ok, f"{what}: max abs err {emax:.3e}, max rel err {rmax:.3e}"


def grad_close(got, ref, what, mag=None):
    """Gradient parity: |err| <= 1e-4 |ref| per component, with a floor of
    1e-5 mag where ``mag`` is the same gradient taken with |grad_image| (the
    image is a polynomial in the albedos with non-negative coefficients, so
    that is the sum of the magnitudes of the terms the component adds up, and
    FP32 accumulation error is relative to it; it matters only where terms of
    both signs cancel).  Without ``mag`` the bound is relative only.  Prints
    how many components rely on the floor."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    err = np.abs(got - ref)
    rel = 1e-4 * np.abs(ref)
    floor = np.zeros_like(ref) if mag is None else 1e-5 * np.abs(np.asarray(mag, np.float64))
    tol = np.maximum(rel, floor)
    on_floor = int(np.count_nonzero((err > rel) & (err <= floor)))
    print(f"{what}: {ref.size} components, {on_floor} within the floor only, max err {err.max(initial=0):.3e}",
          flush=True)
    bad = err > tol
    assert not bad.any(), (f"{what}: {int(bad.sum())} components off, max err {err.max():.3e} "
                           f"(max |ref| {np.abs(ref).max():.3e})")


def crop(name, w, h, spp=None, emit_L=None):
    cfg = scenegen.crop_of(scenegen.WORKLOADS[name].scene, w, h, spp)
    if emit_L is not None:
        cfg = replace(cfg, emit_L=tuple(emit_L))
    return scenegen.generate(cfg)


def unit(rng, n):
    v = rng.normal(size=(n, 3))
    return (v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)


def synthetic(pos, rng, spp=1, width=None, lengths=None):
    """A scene over given positions with random directions and records.
    lengths: vertices per path (default: one path per vertex)."""
    pos = np.asarray(pos, np.float32)
    n = len(pos)
    if lengths is None:
        lengths = np.ones(n, np.int64)
    off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    P = len(lengths)
    width = width or P // spp
    height = P // (spp * width)
    t = unit(rng, n)
    return scenegen.Scene(width=width, height=height, spp=spp, path_offsets=off, pos=pos, dir_in=t,
                          dir_out=unit(rng, n), albedo=rng.uniform(0.5, 0.99, n).astype(np.float32),
                          l_sun=rng.random((n, 3), dtype=np.float32), dir_env=unit(rng, n),
                          l_env=rng.random((n, 3), dtype=np.float32),
                          l_phase=(rng.random((n, 3), dtype=np.float32) * (rng.random((n, 1)) < 0.3)),
                          e_cam=rng.random((P, 3), dtype=np.float32) * (rng.random((P, 1)) < 0.2))


SUN = tuple(v / math.sqrt(0.3 ** 2 + 1.0 + 0.4 ** 2) for v in (0.3, 1.0, -0.4))
