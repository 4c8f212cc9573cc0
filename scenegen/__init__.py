"""Seeded synthetic scenes for path-graph rendering of participating media.

This module is the input side shared by the FP64 oracle and the GPU library:
a deterministic generator of volume path vertices (see ``scenegen.c``) plus the
workload presets.  It contains none of the path-graph arithmetic.

A :class:`Scene` holds, in path order (paper, "Instrumented path tracer"
paragraph of Sec. "Rendering System"):

* ``path_offsets`` int64[P+1]: path p owns vertices [off[p], off[p+1]);
  path p belongs to pixel p // spp, sample p % spp;
* per vertex (float32): ``pos`` [N,3], ``dir_in`` [N,3] (travel direction of
  the path arriving at the vertex), ``dir_out`` [N,3] (phase-sampled
  continuation direction), ``albedo`` [N], ``l_sun`` [N,3] (sun irradiance times
  the shadow-ray transmittance estimate), ``dir_env`` [N,3] and ``l_env`` [N,3]
  (uniform-sphere environment shadow ray and its transmitted radiance),
  ``l_phase`` [N,3] (environment radiance if the continuation ray escaped);
* per path: ``e_cam`` [P,3] (environment radiance if the camera ray escaped);
* optionally ``dir_pl``, ``l_pl`` [N,3]: a point light's shadow-ray direction
  and irradiance (intensity x transmittance / distance^2);
* optionally ``l_emit`` [N,3]: the volume emission collected at the collision,
  L_v / sigma_t = (1 - albedo) L_e(pos) for an emissive medium whose emitted
  radiance L_e is a smooth blob (``SceneConfig.emit_L`` nonzero), else None.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field, replace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_DIR = os.path.join(_HERE, "_lib")
_SANITIZE = os.environ.get("PG_SANITIZE") == "1"
_LIB_PATH = os.path.join(_LIB_DIR, "libscenegen_san.so" if _SANITIZE else "libscenegen.so")
_SRC = os.path.join(_HERE, "scenegen.c")
_CLANG = "/opt/rocm/llvm/bin/clang"
_SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
              "-g", "-O1", "-shared-libsan"]


def build(verbose: bool = False, sanitize: bool | None = None) -> str:
    """Compile the generator into scenegen/_lib/libscenegen.so (gcc, OpenMP);
    with ``sanitize`` (default: PG_SANITIZE=1 in the environment) an
    ASan + UBSan build with clang and its OpenMP runtime, libscenegen_san.so."""
    sanitize = _SANITIZE if sanitize is None else sanitize
    os.makedirs(_LIB_DIR, exist_ok=True)
    out = os.path.join(_LIB_DIR, "libscenegen_san.so" if sanitize else "libscenegen.so")
    tmp = out + ".tmp"
    if sanitize:
        cmd = [_CLANG, *_SAN_FLAGS, "-fopenmp", "-shared", "-fPIC", "-ffp-contract=off", "-Wall", "-Wextra", _SRC,
               "-lm", "-Wl,-rpath,/opt/rocm/llvm/lib", "-o", tmp]
    else:
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-ffp-contract=off",
               "-Wall", "-Wextra", _SRC, "-lm", "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


class _Config(ctypes.Structure):
    _fields_ = [
        ("R", ctypes.c_int32), ("mask", ctypes.c_int32), ("albedo_mode", ctypes.c_int32),
        ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("spp", ctypes.c_int32),
        ("max_depth", ctypes.c_int32),
        ("crop_x0", ctypes.c_int32), ("crop_y0", ctypes.c_int32),
        ("crop_w", ctypes.c_int32), ("crop_h", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("sigma_max", ctypes.c_double),
        ("density_contrast", ctypes.c_double), ("density_bias", ctypes.c_double),
        ("mask_r0", ctypes.c_double), ("mask_r1", ctypes.c_double),
        ("albedo_lo", ctypes.c_double), ("albedo_hi", ctypes.c_double),
        ("g", ctypes.c_double),
        ("cam_pos", ctypes.c_double * 3), ("look_at", ctypes.c_double * 3), ("vfov_deg", ctypes.c_double),
        ("sun_dir", ctypes.c_double * 3), ("sun_E", ctypes.c_double * 3), ("env_L", ctypes.c_double * 3),
        ("seed", ctypes.c_uint64), ("extra_samples", ctypes.c_int32), ("point_light", ctypes.c_int32),
        ("pl_pos", ctypes.c_double * 3), ("pl_I", ctypes.c_double * 3),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.sg_trace.restype = ctypes.c_void_p
        lib.sg_trace.argtypes = [ctypes.POINTER(_Config), ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                 ctypes.c_char_p, ctypes.c_int]
        lib.sg_fetch.restype = ctypes.c_int
        lib.sg_fetch.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 10
        lib.sg_density.restype = ctypes.c_double
        lib.sg_density.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.sg_fetch_point_light.restype = ctypes.c_int
        lib.sg_fetch_point_light.argtypes = [ctypes.c_void_p] * 3
        lib.sg_fetch_extra.restype = ctypes.c_int
        lib.sg_fetch_extra.argtypes = [ctypes.c_void_p] * 4
        lib.sg_albedo.restype = ctypes.c_int
        lib.sg_albedo.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.sg_release.restype = None
        lib.sg_release.argtypes = [ctypes.c_void_p]
        _lib = lib
    return _lib


SUN_DIR = tuple(v / math.sqrt(0.3 ** 2 + 1.0 + 0.4 ** 2) for v in (0.3, 1.0, -0.4))


@dataclass(frozen=True)
class SceneConfig:
    """Medium, lights, camera and path-tracer settings of one synthetic scene."""
    R: int = 32
    sigma_max: float = 8.0
    density_contrast: float = 1.0  # sigma_t = sigma_max * clamp(0.5 + c (fbm - 0.5) + b, 0, 1)
    density_bias: float = 0.0
    mask: int = 0                 # 0 none, 1 soft sphere 1 - smoothstep(r0, r1, |x - c|)
    mask_radii: tuple = (0.3, 0.5)
    albedo: tuple = (0.9, 0.9)    # (lo, hi); lo == hi means constant
    g: float = 0.5                # HG parameter of phase sampling
    width: int = 64
    height: int = 64
    spp: int = 4
    max_depth: int = 8
    crop: tuple = (0, 0, 0, 0)    # (x0, y0, w, h); w == 0: full image
    cam_pos: tuple = (0.5, 0.5, -1.2)
    look_at: tuple = (0.5, 0.5, 0.5)
    vfov_deg: float = 40.0
    sun_dir: tuple = SUN_DIR
    sun_E: tuple = (2.0, 1.9, 1.7)
    env_L: tuple = (0.25, 0.35, 0.5)
    seed: int = 1
    # emissive blob: L_e(x) = emit_L * (1 - |x - emit_center|^2 / emit_radius^2)^2 inside the radius
    emit_L: tuple = (0.0, 0.0, 0.0)
    emit_center: tuple = (0.5, 0.55, 0.5)
    emit_radius: float = 0.25
    # extra emitter samples at each path's first vertex (sun + environment shadow rays, own stream)
    extra_samples: int = 0
    # point light: intensity pl_I (all zero: none) at pl_pos
    pl_I: tuple = (0.0, 0.0, 0.0)
    pl_pos: tuple = (0.5, 1.1, 0.5)

    def _c(self) -> _Config:
        c = _Config()
        c.R, c.mask = self.R, self.mask
        lo, hi = self.albedo
        c.albedo_mode = 0 if lo == hi else 1
        c.albedo_lo, c.albedo_hi = lo, hi
        c.width, c.height, c.spp, c.max_depth = self.width, self.height, self.spp, self.max_depth
        c.crop_x0, c.crop_y0, c.crop_w, c.crop_h = self.crop
        c.sigma_max, c.g, c.vfov_deg = self.sigma_max, self.g, self.vfov_deg
        c.density_contrast, c.density_bias = self.density_contrast, self.density_bias
        c.mask_r0, c.mask_r1 = self.mask_radii
        c.cam_pos[:] = self.cam_pos
        c.look_at[:] = self.look_at
        c.sun_dir[:] = self.sun_dir
        c.sun_E[:] = self.sun_E
        c.env_L[:] = self.env_L
        c.seed = self.seed
        c.extra_samples = self.extra_samples
        c.point_light = 1 if any(self.pl_I) else 0
        c.pl_pos[:] = self.pl_pos
        c.pl_I[:] = self.pl_I
        return c

    @property
    def image_size(self):
        """(width, height) of the traced window."""
        if self.crop[2]:
            return self.crop[2], self.crop[3]
        return self.width, self.height


@dataclass
class Scene:
    """Path-ordered vertex records of one traced image (all numpy, host)."""
    width: int
    height: int
    spp: int
    path_offsets: np.ndarray
    pos: np.ndarray
    dir_in: np.ndarray
    dir_out: np.ndarray
    albedo: np.ndarray
    l_sun: np.ndarray
    dir_env: np.ndarray
    l_env: np.ndarray
    l_phase: np.ndarray
    e_cam: np.ndarray
    config: SceneConfig | None = None
    l_emit: np.ndarray | None = None
    cluster_key: np.ndarray | None = None   # uint32 [N], see cluster_keys
    # extra first-vertex emitter samples [P, M, 3] each (None: M = 0)
    fb_l_sun: np.ndarray | None = None
    fb_dir_env: np.ndarray | None = None
    fb_l_env: np.ndarray | None = None
    # point light [N, 3] each (None: no point light)
    dir_pl: np.ndarray | None = None
    l_pl: np.ndarray | None = None
    sun_dir: tuple = SUN_DIR
    env_pdf: float = 1.0 / (4.0 * math.pi)

    @property
    def n_vertices(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_paths(self) -> int:
        return int(self.path_offsets.shape[0] - 1)

    ARRAYS = ("path_offsets", "pos", "dir_in", "dir_out", "albedo", "l_sun",
              "dir_env", "l_env", "l_phase", "e_cam")


def generate(cfg: SceneConfig, threads: int = 0) -> Scene:
    """Trace every path of ``cfg`` and return the path-ordered records."""
    lib = _load()
    c = cfg._c()
    nv = ctypes.c_int64()
    npath = ctypes.c_int64()
    err = ctypes.create_string_buffer(256)
    h = lib.sg_trace(ctypes.byref(c), int(threads), ctypes.byref(nv), ctypes.byref(npath), err, 256)
    if not h:
        raise RuntimeError("scenegen: " + err.value.decode())
    try:
        N, P = nv.value, npath.value
        off = np.empty(P + 1, np.int64)
        a3 = lambda n: np.empty((n, 3), np.float32)  # noqa: E731
        pos, din, dout, ls, denv, le, lp = (a3(N) for _ in range(7))
        alb = np.empty(N, np.float32)
        ecam = a3(P)
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        rc = lib.sg_fetch(h, ptr(off), ptr(pos), ptr(din), ptr(dout), ptr(alb), ptr(ls),
                          ptr(denv), ptr(le), ptr(lp), ptr(ecam))
        if rc != 0:
            raise RuntimeError("scenegen: fetch failed")
        pl = None
        if any(cfg.pl_I):
            pl = (a3(N), a3(N))
            lib.sg_fetch_point_light(h, ptr(pl[0]), ptr(pl[1]))
        fb = None
        if cfg.extra_samples > 0:
            fb = tuple(np.zeros((P, cfg.extra_samples, 3), np.float32) for _ in range(3))
            lib.sg_fetch_extra(h, *(ptr(a) for a in fb))
    finally:
        lib.sg_release(h)
    w, hgt = cfg.image_size
    return Scene(width=w, height=hgt, spp=cfg.spp, path_offsets=off, pos=pos, dir_in=din,
                 dir_out=dout, albedo=alb, l_sun=ls, dir_env=denv, l_env=le, l_phase=lp,
                 e_cam=ecam, config=cfg, sun_dir=tuple(cfg.sun_dir), l_emit=emission(cfg, pos, alb),
                 fb_l_sun=fb[0] if fb else None, fb_dir_env=fb[1] if fb else None,
                 fb_l_env=fb[2] if fb else None, dir_pl=pl[0] if pl else None, l_pl=pl[1] if pl else None)


def emission(cfg: SceneConfig, pos: np.ndarray, albedo: np.ndarray) -> np.ndarray | None:
    """Per-vertex collected volume emission (1 - albedo) L_e(pos) [N,3], or None
    when the medium does not emit.  With delta tracking a real collision
    estimates the emission integral by L_v / sigma_t, and L_v = sigma_a L_e."""
    if not any(cfg.emit_L):
        return None
    d2 = ((pos.astype(np.float64) - np.asarray(cfg.emit_center)) ** 2).sum(1)
    prof = np.clip(1.0 - d2 / cfg.emit_radius ** 2, 0.0, None) ** 2
    le = prof[:, None] * np.asarray(cfg.emit_L, np.float64)[None, :]
    return ((1.0 - albedo.astype(np.float64))[:, None] * le).astype(np.float32)


def density(cfg: SceneConfig) -> tuple[np.ndarray, float]:
    """The density grid sigma_t [R,R,R] (z, y, x) and its maximum."""
    lib = _load()
    c = replace(cfg, width=1, height=1, spp=1, crop=(0, 0, 0, 0))._c()
    nv = ctypes.c_int64()
    npath = ctypes.c_int64()
    err = ctypes.create_string_buffer(256)
    h = lib.sg_trace(ctypes.byref(c), 0, ctypes.byref(nv), ctypes.byref(npath), err, 256)
    if not h:
        raise RuntimeError("scenegen: " + err.value.decode())
    try:
        out = np.empty((cfg.R, cfg.R, cfg.R), np.float32)
        maj = lib.sg_density(h, out.ctypes.data_as(ctypes.c_void_p))
    finally:
        lib.sg_release(h)
    return out, maj


def medium(cfg: SceneConfig) -> tuple[np.ndarray, np.ndarray | None, float]:
    """The medium of ``cfg``: sigma_t [R,R,R] (z, y, x), the per-voxel albedo
    grid (None when constant) and the majorant the tracer uses."""
    lib = _load()
    c = replace(cfg, width=1, height=1, spp=1, crop=(0, 0, 0, 0))._c()
    nv = ctypes.c_int64()
    npath = ctypes.c_int64()
    err = ctypes.create_string_buffer(256)
    h = lib.sg_trace(ctypes.byref(c), 0, ctypes.byref(nv), ctypes.byref(npath), err, 256)
    if not h:
        raise RuntimeError("scenegen: " + err.value.decode())
    try:
        sigma = np.empty((cfg.R, cfg.R, cfg.R), np.float32)
        maj = lib.sg_density(h, sigma.ctypes.data_as(ctypes.c_void_p))
        alb = np.empty((cfg.R, cfg.R, cfg.R), np.float32)
        if lib.sg_albedo(h, alb.ctypes.data_as(ctypes.c_void_p)) != 0:
            alb = None
    finally:
        lib.sg_release(h)
    return sigma, alb, float(maj)


def tracer_settings(cfg: SceneConfig) -> dict:
    """Camera, lights, sampling and image settings of ``cfg`` as plain values
    (the medium comes from ``medium``)."""
    return {"R": cfg.R, "width": cfg.width, "height": cfg.height, "spp": cfg.spp, "max_depth": cfg.max_depth,
            "crop": tuple(cfg.crop), "albedo_const": float(cfg.albedo[0]), "g": cfg.g,
            "cam_pos": tuple(cfg.cam_pos), "look_at": tuple(cfg.look_at), "vfov_deg": cfg.vfov_deg,
            "sun_dir": tuple(cfg.sun_dir), "sun_E": tuple(cfg.sun_E), "env_L": tuple(cfg.env_L), "seed": cfg.seed,
            "extra_samples": cfg.extra_samples, "pl_I": tuple(cfg.pl_I), "pl_pos": tuple(cfg.pl_pos)}


def cluster_keys(n: int, seed: int = 7) -> np.ndarray:
    """Seeded uniform 32-bit keys [n]: the random draw that picks the cluster
    centres of the cluster neighbour relation."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2 ** 32, size=n, dtype=np.uint32)


def albedo_grid(res: int = 64, lo: float = 0.95, hi: float = 0.999, seed: int = 2) -> np.ndarray:
    """Seeded per-voxel albedo grid [res,res,res] (z, y, x), uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(res, res, res)).astype(np.float32)


def target_image(shape, scale: float, seed: int = 4) -> np.ndarray:
    """Seeded target image for the L2 loss: uniform in [0, 2*scale)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 2.0 * scale, size=shape).astype(np.float32)


# Method settings that accompany each workload: k neighbours (self included),
# D propagation iterations, HG g evaluated at the receiver and g_s of the pdfs.
@dataclass(frozen=True)
class Workload:
    name: str
    scene: SceneConfig
    k: int
    D: int

    @property
    def g(self) -> float:
        return self.scene.g


WORKLOADS = {
    # 32^3 fBm, sigma_t in [0,8], albedo 0.9, g 0.5, 64x64x4, depth 8, k 8, D 8
    # (about 30k vertices).
    "tiny": Workload("tiny", SceneConfig(R=32, sigma_max=8.0, mask=0, albedo=(0.9, 0.9), g=0.5,
                                         width=64, height=64, spp=4, max_depth=8, vfov_deg=50.0,
                                         seed=1), k=8, D=8),
    # 128^3 fBm x soft sphere, sigma_t in [0,32], albedo U[0.95,0.999] per voxel,
    # g 0.8, 512x512x4, depth 64, k 16, D 64.  The fBm is contrast-stretched so
    # the ball is dense; with sigma_t <= 32 and g = 0.8 delta-tracking paths
    # average about 20 vertices, i.e. about 21M vertices in all.
    "mid": Workload("mid", SceneConfig(R=128, sigma_max=32.0, density_contrast=2.0, density_bias=0.75,
                                       mask=1, mask_radii=(0.42, 0.5), albedo=(0.95, 0.999), g=0.8,
                                       width=512, height=512, spp=4, max_depth=64, vfov_deg=20.0,
                                       seed=2), k=16, D=64),
    # 512^3 fBm, sigma_t up to 64, albedo 0.999, g 0.9, 1024x1024x1, depth 128, k 16, D 128.
    # A dense cloud seen close up: the fBm is contrast-stretched so most of the
    # cube sits at sigma_t = 64 with thinner fBm pockets, and the 10 degree view
    # fills the image with the cloud's front face.  Paths average about 66
    # vertices (about 69M in all): with the camera outside the unit cube, a
    # medium of sigma_t <= 64 and g = 0.9 cannot hold the paths much longer (a
    # homogeneous sigma_t = 64 half-space, the densest and widest medium a
    # camera outside it can face, averages 81 vertices per path at depth 128).
    "large": Workload("large", SceneConfig(R=512, sigma_max=64.0, density_contrast=2.0, density_bias=0.75,
                                           mask=0, albedo=(0.999, 0.999), g=0.9,
                                           width=1024, height=1024, spp=1, max_depth=128,
                                           vfov_deg=10.0, seed=3), k=16, D=128),
}


def crop_of(cfg: SceneConfig, w: int, h: int, spp: int | None = None) -> SceneConfig:
    """Centred w x h window of ``cfg`` (same paths as the full image there)."""
    x0 = (cfg.width - w) // 2
    y0 = (cfg.height - h) // 2
    return replace(cfg, crop=(x0, y0, w, h), spp=cfg.spp if spp is None else spp)


def _batch_specs(n, seed, n_min, n_max):
    """Seeded draws of the batching workload: per scene the medium, method
    settings and a log-uniform vertex-count target."""
    rng = np.random.default_rng(seed)
    specs = []
    for s in range(n):
        R = int(rng.choice([32, 64, 128, 256]))
        alb = float(rng.uniform(0.8, 0.999))
        g = float(rng.uniform(-0.3, 0.9))
        k = int(rng.integers(8, 17))
        D = int(rng.integers(16, 65))
        target = float(np.exp(rng.uniform(np.log(n_min), np.log(n_max))))
        sigma = float(rng.uniform(6.0, 24.0))
        cfg = SceneConfig(R=R, sigma_max=sigma, albedo=(alb, alb), g=g, width=32, height=32, spp=1,
                          max_depth=D, vfov_deg=40.0, seed=seed + s)
        specs.append((f"batch{s}", cfg, k, D, target))
    return specs


def _sized(spec, per_pixel):
    name, cfg, k, D, target = spec
    pixels = target / max(per_pixel, 0.05)
    spp = 1 if pixels < 512 * 512 else 4
    side = int(max(8, round(np.sqrt(pixels / spp))))
    return Workload(name, replace(cfg, width=side, height=side, spp=spp), k=k, D=D)


def batch_workload(n: int = 64, seed: int = 1000, n_min: float = 1e4, n_max: float = 2e6):
    """Independent scenes of the batching workload: scene s is seeded 1000+s
    (grid 32^3..256^3 fBm, albedo U[0.8, 0.999], HG g U[-0.3, 0.9], k 8..16,
    D 16..64), its vertex count drawn log-uniform in [n_min, n_max] and reached
    by choosing the image size from a 32x32-pixel probe render.
    Returns a list of Workload."""
    return [_sized(sp, generate(sp[1]).n_vertices / (32 * 32)) for sp in _batch_specs(n, seed, n_min, n_max)]


def generate_batch(n: int = 64, seed: int = 1000, n_min: float = 1e4, n_max: float = 2e6):
    """The batching workload's scenes, traced: a list of (Workload, Scene).
    Each scene is traced right after its probe, so its medium is built once."""
    out = []
    for sp in _batch_specs(n, seed, n_min, n_max):
        w = _sized(sp, generate(sp[1]).n_vertices / (32 * 32))
        out.append((w, generate(w.scene)))
    return out
