"""MI355X (gfx950) path-graph rendering of participating media.

Thin Python binding of the C ABI in ``include/pathgraph.h``: the functions
below carry the same names as the C entry points and only marshal arguments
(torch device tensors -> pointers, the current HIP stream, a workspace
tensor).  Every step runs in the HIP kernels of ``libpathgraph.so``; there is
no fallback.  Build the library with :func:`build` (``__graft_entry__.build``).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from ._build import LIB_PATH, build  # noqa: F401

PG_OK, PG_ERR_ARG, PG_ERR_WORKSPACE, PG_ERR_HIP, PG_ERR_INPUT, PG_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
PG_INIT_PT, PG_INIT_ZERO = 0, 1
PG_FLAG_CHECK, PG_FLAG_TAPE, PG_FLAG_EXACT_KNN, PG_FLAG_CLUSTERS, PG_FLAG_PERSISTENT = 1, 2, 4, 8, 16
PG_FLAG_STORE_Z = 32
PG_SCHED_TWO_PASS, PG_SCHED_SHIFTED, PG_SCHED_SCATTER = 1, 2, 3
PG_MAX_K = 64

EXPORTS = ("pg_version", "pg_last_error", "pg_default_cell_shift", "pg_profile_start", "pg_profile_stop",
           "pg_trace_workspace_size", "pg_trace_count", "pg_trace_records",
           "pg_knn_workspace_size", "pg_knn", "pg_clusters_workspace_size", "pg_clusters",
           "pg_edges_workspace_size", "pg_edges",
           "pg_propagate_workspace_size", "pg_propagate", "pg_propagate_static", "pg_gather",
           "pg_render_workspace_size", "pg_render", "pg_backward_workspace_size", "pg_backward",
           "pg_render_batched_workspace_size", "pg_render_batched", "pg_batch_create", "pg_batch_launch",
           "pg_batch_destroy")


class PathGraphError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pathgraph error {code}: {msg}")
        self.code = code


class Paths(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("n_paths", ctypes.c_int64),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("spp", ctypes.c_int32),
                ("albedo_grid_res", ctypes.c_int32)] + [
        (n, ctypes.c_void_p) for n in ("path_offsets", "pos", "dir_in", "dir_out", "albedo", "l_sun",
                                       "dir_env", "l_env", "l_phase", "e_cam", "albedo_grid", "l_emit",
                                       "cluster_key", "fb_l_sun", "fb_dir_env", "fb_l_env")] + [
        ("n_extra", ctypes.c_int32), ("pad_", ctypes.c_int32), ("dir_pl", ctypes.c_void_p), ("l_pl", ctypes.c_void_p)]


class Tracer(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int32), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("spp", ctypes.c_int32), ("max_depth", ctypes.c_int32), ("crop_x0", ctypes.c_int32),
                ("crop_y0", ctypes.c_int32), ("crop_w", ctypes.c_int32), ("crop_h", ctypes.c_int32),
                ("extra_samples", ctypes.c_int32), ("sigma", ctypes.c_void_p), ("albedo", ctypes.c_void_p),
                ("albedo_const", ctypes.c_double), ("majorant", ctypes.c_double), ("g", ctypes.c_double),
                ("cam_pos", ctypes.c_double * 3), ("look_at", ctypes.c_double * 3), ("vfov_deg", ctypes.c_double),
                ("sun_dir", ctypes.c_double * 3), ("sun_E", ctypes.c_double * 3), ("env_L", ctypes.c_double * 3),
                ("seed", ctypes.c_uint64), ("pl_pos", ctypes.c_double * 3), ("pl_I", ctypes.c_double * 3)]


class Records(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("pos", "dir_in", "dir_out", "albedo", "l_sun", "dir_env", "l_env",
                                               "l_phase", "e_cam", "fb_l_sun", "fb_dir_env", "fb_l_env", "dir_pl",
                                               "l_pl")]


class Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("D", ctypes.c_int32), ("g", ctypes.c_float), ("g_s", ctypes.c_float),
                ("sun_dir", ctypes.c_float * 3), ("env_pdf", ctypes.c_float), ("init", ctypes.c_int32),
                ("final_gather", ctypes.c_int32), ("cell_shift", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("tile", ctypes.c_int32), ("tile_group", ctypes.c_int32)]


class ProfileEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("count", ctypes.c_int32), ("total_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double)]


class GraphOut(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("row_ptr", "col", "w_ind", "w_ph", "w_env", "b", "d_pt", "lplus")] + [
        ("edge_capacity", ctypes.c_int64), ("n_far", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: the HIP library has not been built "
                               "(run __graft_entry__.build() or paper_2404_11894_amd.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)
        P, Q = ctypes.POINTER(Paths), ctypes.POINTER(Params)
        sig = {
            "pg_version": (ctypes.c_char_p, []),
            "pg_last_error": (ctypes.c_char_p, []),
            "pg_default_cell_shift": (i32, [i64]),
            "pg_profile_start": (i32, []),
            "pg_profile_stop": (i32, [i32, ctypes.POINTER(ProfileEntry), ctypes.POINTER(ctypes.c_int32)]),
            "pg_knn_workspace_size": (i32, [P, i32, i32, sz]),
            "pg_knn": (i32, [P, i32, i32, vp, vp, vp, ctypes.c_size_t, vp]),
            "pg_trace_workspace_size": (i32, [ctypes.POINTER(Tracer), sz]),
            "pg_trace_count": (i32, [ctypes.POINTER(Tracer), vp, ctypes.POINTER(ctypes.c_int64), vp,
                                     ctypes.c_size_t, vp]),
            "pg_trace_records": (i32, [ctypes.POINTER(Tracer), vp, ctypes.POINTER(Records), vp, ctypes.c_size_t,
                                       vp]),
            "pg_clusters_workspace_size": (i32, [P, i32, i32, sz]),
            "pg_clusters": (i32, [P, i32, i32, vp, vp, ctypes.c_size_t, vp]),
            "pg_edges_workspace_size": (i32, [P, Q, sz]),
            "pg_edges": (i32, [P, Q, vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]),
            "pg_propagate_workspace_size": (i32, [P, Q, sz]),
            "pg_propagate": (i32, [P, Q, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]),
            "pg_propagate_static": (i32, [P, Q, vp, vp, vp, vp, vp, vp, vp]),
            "pg_gather": (i32, [P, Q, vp, vp, vp, vp, vp, vp, vp]),
            "pg_render_workspace_size": (i32, [P, Q, sz]),
            "pg_render": (i32, [P, Q, vp, ctypes.POINTER(GraphOut), vp, ctypes.c_size_t, vp]),
            "pg_backward_workspace_size": (i32, [P, Q, sz]),
            "pg_backward": (i32, [P, Q, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]),
            "pg_render_batched_workspace_size": (i32, [i32, P, Q, sz]),
            "pg_render_batched": (i32, [i32, P, Q, vp, vp, ctypes.c_size_t, vp]),
            "pg_batch_create": (i32, [i32, P, Q, vp, vp, ctypes.c_size_t, i32, vp, ctypes.POINTER(vp)]),
            "pg_batch_launch": (i32, [vp, vp]),
            "pg_batch_destroy": (i32, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != PG_OK:
        raise PathGraphError(rc, lib().pg_last_error().decode())


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _workspace(nbytes: int, device):
    torch = _torch()
    # 256-byte aligned view into a byte tensor
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf[off:off + int(nbytes)], int(nbytes)


class DevicePaths:
    """The path records of one image as device tensors, plus the C struct
    pointing at them.  ``scene`` is any object with the record arrays (numpy or
    torch) and width / height / spp attributes; an optional ``l_emit`` [N,3]
    attribute (None: no emission) carries the per-vertex volume emission and
    an optional ``cluster_key`` [N] (uint32) the keys of the cluster relation."""

    ARRAYS = ("path_offsets", "pos", "dir_in", "dir_out", "albedo", "l_sun", "dir_env", "l_env", "l_phase",
              "e_cam")

    def __init__(self, scene, device="cuda", albedo_grid=None):
        torch = _torch()
        self.device = torch.device(device)
        self.tensors = {}
        for name in self.ARRAYS:
            a = getattr(scene, name)
            t = torch.as_tensor(a)
            dt = torch.int64 if name == "path_offsets" else torch.float32
            self.tensors[name] = t.to(device=self.device, dtype=dt).contiguous()
        self.width, self.height, self.spp = int(scene.width), int(scene.height), int(scene.spp)
        self.n_vertices = int(self.tensors["pos"].shape[0])
        self.n_paths = int(self.tensors["path_offsets"].shape[0]) - 1
        em = getattr(scene, "l_emit", None)
        self.l_emit = None if em is None else torch.as_tensor(em).to(
            device=self.device, dtype=torch.float32).contiguous()
        self.cluster_key = None
        self.set_cluster_key(getattr(scene, "cluster_key", None))
        self.pl = None   # point light records [N, 3] x 2
        if getattr(scene, "dir_pl", None) is not None:
            self.pl = {n: torch.as_tensor(getattr(scene, n)).to(device=self.device, dtype=torch.float32).contiguous()
                       for n in ("dir_pl", "l_pl")}
        self.fb = None   # extra first-vertex samples [P, M, 3] x 3
        if getattr(scene, "fb_l_sun", None) is not None:
            self.fb = {n: torch.as_tensor(getattr(scene, n)).to(device=self.device, dtype=torch.float32).contiguous()
                       for n in ("fb_l_sun", "fb_dir_env", "fb_l_env")}
        self.albedo_grid = None
        self.set_albedo_grid(albedo_grid)

    def set_cluster_key(self, key):
        """uint32 keys [N] (numpy) or an int32 tensor holding their bits."""
        torch = _torch()
        if key is None:
            self.cluster_key = None
            return
        if not isinstance(key, torch.Tensor):
            key = torch.from_numpy(np.ascontiguousarray(key, dtype=np.uint32).view(np.int32))
        self.cluster_key = key.to(device=self.device, dtype=torch.int32).contiguous()

    def set_albedo_grid(self, grid):
        torch = _torch()
        self.albedo_grid = None if grid is None else torch.as_tensor(grid).to(
            device=self.device, dtype=torch.float32).contiguous()

    def struct(self) -> Paths:
        s = Paths()
        s.n_vertices, s.n_paths = self.n_vertices, self.n_paths
        s.width, s.height, s.spp = self.width, self.height, self.spp
        for name, t in self.tensors.items():
            setattr(s, name, t.data_ptr() if t.numel() else None)
        if self.albedo_grid is not None:
            s.albedo_grid = self.albedo_grid.data_ptr()
            s.albedo_grid_res = int(self.albedo_grid.shape[0])
        if self.l_emit is not None and self.l_emit.numel():
            s.l_emit = self.l_emit.data_ptr()
        if self.cluster_key is not None and self.cluster_key.numel():
            s.cluster_key = self.cluster_key.data_ptr()
        if self.pl is not None and self.pl["dir_pl"].numel():
            for n, t in self.pl.items():
                setattr(s, n, t.data_ptr())
        if self.fb is not None and self.fb["fb_l_sun"].numel():
            for n, t in self.fb.items():
                setattr(s, n, t.data_ptr())
            s.n_extra = int(self.fb["fb_l_sun"].shape[1])
        return s


def params(k=8, D=8, g=0.5, g_s=None, sun_dir=None, env_pdf=None, init="pt", final_gather=0, cell_shift=0,
           schedule=0, flags=0, tile=0, tile_group=0) -> Params:
    """Method parameters (defaults of the small workload)."""
    q = Params()
    q.k, q.D = int(k), int(D)
    q.g = float(g)
    q.g_s = float(g if g_s is None else g_s)
    if sun_dir is None:
        n = math.sqrt(0.3 ** 2 + 1.0 + 0.4 ** 2)
        sun_dir = (0.3 / n, 1.0 / n, -0.4 / n)
    q.sun_dir[:] = [float(v) for v in sun_dir]
    q.env_pdf = float(1.0 / (4.0 * math.pi) if env_pdf is None else env_pdf)
    q.init = {"pt": PG_INIT_PT, "zero": PG_INIT_ZERO}[init] if isinstance(init, str) else int(init)
    q.final_gather = int(final_gather)
    q.cell_shift = int(cell_shift)
    q.schedule = int(schedule)
    q.flags = int(flags)
    q.tile = int(tile)
    q.tile_group = int(tile_group)
    return q


def resolved_schedule(q: Params) -> str:
    """Name of the propagation schedule a call with these params uses."""
    return {PG_SCHED_SHIFTED: "shifted", PG_SCHED_SCATTER: "scatter"}.get(q.schedule, "two-pass")


def _K(paths: DevicePaths, k: int) -> int:
    return min(int(k), paths.n_vertices)


def pg_version() -> str:
    return lib().pg_version().decode()


def pg_default_cell_shift(n_vertices: int) -> int:
    return int(lib().pg_default_cell_shift(int(n_vertices)))


def pg_knn(paths: DevicePaths, k: int, cell_shift: int = 0):
    """Neighbour lists: (row_ptr int64[N+1], col int32[N*K])."""
    torch = _torch()
    L, s = lib(), paths.struct()
    nb = ctypes.c_size_t()
    _check(L.pg_knn_workspace_size(ctypes.byref(s), int(k), int(cell_shift), ctypes.byref(nb)))
    _, ws, n = _workspace(nb.value, paths.device)
    N, K = paths.n_vertices, _K(paths, k)
    row_ptr = torch.empty(N + 1, dtype=torch.int64, device=paths.device)
    col = torch.empty(N * K, dtype=torch.int32, device=paths.device)
    _check(L.pg_knn(ctypes.byref(s), int(k), int(cell_shift), _ptr(row_ptr), _ptr(col), _ptr(ws), n,
                    _stream(paths.device)))
    return row_ptr, col


class DeviceRecords:
    """Path records traced on the GPU (pg_trace): device tensors with the
    names DevicePaths reads, plus width / height / spp."""

    def __init__(self, width, height, spp, tensors):
        self.width, self.height, self.spp = width, height, spp
        for name, t in tensors.items():
            setattr(self, name, t)

    @property
    def n_vertices(self) -> int:
        return int(self.pos.shape[0])


def pg_trace(settings: dict, sigma, albedo=None, majorant=None, device="cuda") -> DeviceRecords:
    """Trace every path of an image on the GPU (pg_trace_count, then
    pg_trace_records).  ``settings``: R, width, height, spp, max_depth, crop
    (x0, y0, w, h; w = 0 for the full image), albedo_const, g, cam_pos,
    look_at, vfov_deg, sun_dir, sun_E, env_L, seed.  ``sigma`` / ``albedo``:
    [R,R,R] (z, y, x) grids, numpy or torch; majorant defaults to sigma's max."""
    torch = _torch()
    dev = torch.device(device)
    sg = torch.as_tensor(sigma).to(device=dev, dtype=torch.float32).contiguous()
    al = None if albedo is None else torch.as_tensor(albedo).to(device=dev, dtype=torch.float32).contiguous()
    t = Tracer()
    t.R, t.width, t.height = int(settings["R"]), int(settings["width"]), int(settings["height"])
    t.spp, t.max_depth = int(settings["spp"]), int(settings["max_depth"])
    t.crop_x0, t.crop_y0, t.crop_w, t.crop_h = (int(v) for v in settings.get("crop", (0, 0, 0, 0)))
    t.sigma = sg.data_ptr()
    t.albedo = al.data_ptr() if al is not None else None
    t.albedo_const = float(settings["albedo_const"])
    t.majorant = float(sg.max().item()) if majorant is None else float(majorant)
    t.g, t.vfov_deg = float(settings["g"]), float(settings["vfov_deg"])
    for name in ("cam_pos", "look_at", "sun_dir", "sun_E", "env_L"):
        getattr(t, name)[:] = [float(v) for v in settings[name]]
    t.seed = int(settings["seed"])
    t.extra_samples = int(settings.get("extra_samples", 0))
    t.pl_pos[:] = [float(v) for v in settings.get("pl_pos", (0.0, 0.0, 0.0))]
    t.pl_I[:] = [float(v) for v in settings.get("pl_I", (0.0, 0.0, 0.0))]
    point_light = any(v != 0.0 for v in t.pl_I)
    w = t.crop_w if t.crop_w else t.width
    h = t.crop_h if t.crop_w else t.height
    P = w * h * t.spp
    L = lib()
    nb = ctypes.c_size_t()
    _check(L.pg_trace_workspace_size(ctypes.byref(t), ctypes.byref(nb)))
    _, ws, n = _workspace(nb.value, dev)
    off = torch.empty(P + 1, dtype=torch.int64, device=dev)
    N = ctypes.c_int64()
    _check(L.pg_trace_count(ctypes.byref(t), _ptr(off), ctypes.byref(N), _ptr(ws), n, _stream(dev)))
    N = int(N.value)
    # at least one row each, so every pointer is valid (an empty tensor has none); the views keep n rows
    f = lambda n, *sh: torch.empty(max(n, 1), *sh, dtype=torch.float32, device=dev)  # noqa: E731
    base = {"pos": f(N, 3), "dir_in": f(N, 3), "dir_out": f(N, 3), "albedo": f(N), "l_sun": f(N, 3),
            "dir_env": f(N, 3), "l_env": f(N, 3), "l_phase": f(N, 3), "e_cam": f(P, 3)}
    if point_light:
        base["dir_pl"], base["l_pl"] = f(N, 3), f(N, 3)
    M = t.extra_samples
    if M > 0:
        for name in ("fb_l_sun", "fb_dir_env", "fb_l_env"):
            base[name] = torch.empty(max(P, 1), M, 3, dtype=torch.float32, device=dev)
    r = Records()
    for name, t_ in base.items():
        setattr(r, name, t_.data_ptr())
    ten = {"path_offsets": off,
           **{name: t_[:(P if name == "e_cam" or name.startswith("fb_") else N)] for name, t_ in base.items()}}
    _check(L.pg_trace_records(ctypes.byref(t), _ptr(off), ctypes.byref(r), _ptr(ws), n, _stream(dev)))
    return DeviceRecords(w, h, t.spp, ten)


def pg_clusters(paths: DevicePaths, k: int, cell_shift: int = 0):
    """Centre id (path order) of every vertex's cluster, int32 [N]."""
    torch = _torch()
    L, s = lib(), paths.struct()
    nb = ctypes.c_size_t()
    _check(L.pg_clusters_workspace_size(ctypes.byref(s), int(k), int(cell_shift), ctypes.byref(nb)))
    _, ws, n = _workspace(nb.value, paths.device)
    centre = torch.empty(paths.n_vertices, dtype=torch.int32, device=paths.device)
    _check(L.pg_clusters(ctypes.byref(s), int(k), int(cell_shift), _ptr(centre), _ptr(ws), n,
                         _stream(paths.device)))
    return centre


def cluster_edge_count(centre) -> int:
    """Edges of the cluster relation: the sum over clusters of size^2."""
    torch = _torch()
    c = torch.as_tensor(centre).to(torch.int64)
    if c.numel() == 0:
        return 0
    size = torch.bincount(c, minlength=c.numel())
    return int((size * size).sum().item())


def pg_edges(paths: DevicePaths, q: Params, row_ptr, col):
    """Aggregation weights and direct terms: dict of w_ind, w_ph, w_env [N*K],
    b, d_pt, lplus0 [N,3]."""
    torch = _torch()
    L, s = lib(), paths.struct()
    nb = ctypes.c_size_t()
    _check(L.pg_edges_workspace_size(ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb)))
    _, ws, n = _workspace(nb.value, paths.device)
    N, K = paths.n_vertices, _K(paths, q.k)
    f = lambda *sh: torch.empty(*sh, dtype=torch.float32, device=paths.device)  # noqa: E731
    out = {"w_ind": f(N * K), "w_ph": f(N * K), "w_env": f(N * K), "b": f(N, 3), "d_pt": f(N, 3),
           "lplus0": f(N, 3)}
    _check(L.pg_edges(ctypes.byref(s), ctypes.byref(q), _ptr(row_ptr), _ptr(col), _ptr(out["w_ind"]),
                      _ptr(out["w_ph"]), _ptr(out["w_env"]), _ptr(out["b"]), _ptr(out["d_pt"]),
                      _ptr(out["lplus0"]), _ptr(ws), n, _stream(paths.device)))
    return out


def pg_propagate(paths: DevicePaths, q: Params, row_ptr, col, w_ind, b, lplus, traj: bool = False):
    """D iterations of aggregation + propagation.  lplus (L_0, [N,3]) is
    updated in place to L_D; with traj also returns L_1..L_D [D,N,3]."""
    torch = _torch()
    L, s = lib(), paths.struct()
    nb = ctypes.c_size_t()
    _check(L.pg_propagate_workspace_size(ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb)))
    _, ws, n = _workspace(nb.value, paths.device)
    tr = torch.empty(q.D, paths.n_vertices, 3, dtype=torch.float32, device=paths.device) if traj else None
    _check(L.pg_propagate(ctypes.byref(s), ctypes.byref(q), _ptr(row_ptr), _ptr(col), _ptr(w_ind), _ptr(b),
                          _ptr(lplus), _ptr(tr), _ptr(ws), n, _stream(paths.device)))
    return (lplus, tr) if traj else lplus


def pg_propagate_static(paths: DevicePaths, q: Params, row_ptr, col, w_ind, b, lplus, traj=None):
    """pg_propagate without a workspace (the library's static device scratch):
    lplus (L_0, [N,3]) is updated in place to L_D; ``traj``, if given, is a
    caller tensor [D,N,3] that receives L_1..L_D.  Allocates nothing."""
    _check(lib().pg_propagate_static(ctypes.byref(paths.struct()), ctypes.byref(q), _ptr(row_ptr), _ptr(col),
                                     _ptr(w_ind), _ptr(b), _ptr(lplus), _ptr(traj), _stream(paths.device)))
    return lplus


def pg_gather(paths: DevicePaths, q: Params, row_ptr, col, w_ind, d_pt, lplus):
    """Pixel radiance [H, W, 3]."""
    torch = _torch()
    s = paths.struct()
    image = torch.empty(paths.height, paths.width, 3, dtype=torch.float32, device=paths.device)
    _check(lib().pg_gather(ctypes.byref(s), ctypes.byref(q), _ptr(row_ptr), _ptr(col), _ptr(w_ind), _ptr(d_pt),
                           _ptr(lplus), _ptr(image), _stream(paths.device)))
    return image


class Renderer:
    """Holds the workspace of repeated pg_render calls on one set of paths."""

    def __init__(self, paths: DevicePaths, q: Params):
        L = lib()
        self.paths, self.q = paths, q
        self.s = paths.struct()
        nb = ctypes.c_size_t()
        _check(L.pg_render_workspace_size(ctypes.byref(self.s), ctypes.byref(q), ctypes.byref(nb)))
        self._buf, self.ws, self.ws_bytes = _workspace(nb.value, paths.device)

    def __call__(self, image=None, graph: dict | None = None):
        torch = _torch()
        if image is None:
            image = torch.empty(self.paths.height, self.paths.width, 3, dtype=torch.float32,
                                device=self.paths.device)
        out = None
        if graph is not None:
            out = GraphOut()
            for name, t in graph.items():
                setattr(out, name, t.data_ptr())
            out.edge_capacity = int(graph["col"].numel()) if "col" in graph else 0
        _check(lib().pg_render(ctypes.byref(self.s), ctypes.byref(self.q), _ptr(image),
                               ctypes.byref(out) if out is not None else None, _ptr(self.ws), self.ws_bytes,
                               _stream(self.paths.device)))
        return image


def pg_render(paths: DevicePaths, q: Params, graph: bool = False):
    """Image [H, W, 3]; with graph=True also the path-order graph
    (row_ptr, col, w_ind, w_ph, w_env, b, d_pt, lplus)."""
    torch = _torch()
    g = None
    if graph:
        N = paths.n_vertices
        if q.flags & PG_FLAG_CLUSTERS:
            E = cluster_edge_count(pg_clusters(paths, q.k, q.cell_shift)) if N else 0
        else:
            E = N * _K(paths, q.k)
        f = lambda *sh: torch.empty(*sh, dtype=torch.float32, device=paths.device)  # noqa: E731
        g = {"row_ptr": torch.empty(N + 1, dtype=torch.int64, device=paths.device),
             "col": torch.empty(E, dtype=torch.int32, device=paths.device),
             "w_ind": f(E), "w_ph": f(E), "w_env": f(E), "b": f(N, 3), "d_pt": f(N, 3),
             "lplus": f(N, 3)}
    image = Renderer(paths, q)(graph=g)
    return (image, g) if graph else image


def pg_backward(paths: DevicePaths, q: Params, grad_image, grad_grid=True, grad_albedo=False, grad_g=True,
                workspace=None):
    """Reverse mode: gradient of sum(grad_image * image) w.r.t. the albedo
    grid (paths.albedo_grid), the per-vertex albedo and g.  ``workspace`` is a
    (tensor, bytes) pair holding a PG_FLAG_TAPE render's tape, or None to
    recompute the forward pass."""
    torch = _torch()
    L, s = lib(), paths.struct()
    if workspace is None:
        nb = ctypes.c_size_t()
        _check(L.pg_backward_workspace_size(ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb)))
        _, ws, n = _workspace(nb.value, paths.device)
    else:
        ws, n = workspace
    gi = grad_image.to(device=paths.device, dtype=torch.float32).contiguous()
    out = {}
    gg = gr = ga = None
    if grad_grid and paths.albedo_grid is not None:
        gr = torch.empty_like(paths.albedo_grid)
        out["grad_grid"] = gr
    if grad_albedo:
        ga = torch.empty(paths.n_vertices, dtype=torch.float32, device=paths.device)
        out["grad_albedo"] = ga
    if grad_g:
        gg = torch.empty(1, dtype=torch.float32, device=paths.device)
        out["grad_g"] = gg
    _check(L.pg_backward(ctypes.byref(s), ctypes.byref(q), _ptr(gi), _ptr(gr), _ptr(ga), _ptr(gg), _ptr(ws), n,
                         _stream(paths.device)))
    return out


def _render_function():
    torch = _torch()

    class RenderFunction(torch.autograd.Function):
        """image = render(albedo grid, g) with the paths and sampling pdfs fixed.
        forward: pg_render with PG_FLAG_TAPE; backward: pg_backward on the tape."""

        @staticmethod
        def forward(ctx, grid, g, paths, q):
            qq = Params.from_buffer_copy(q)
            qq.g = float(g)
            qq.flags = qq.flags | PG_FLAG_TAPE
            paths.set_albedo_grid(grid.detach())
            s = paths.struct()
            nb = ctypes.c_size_t()
            _check(lib().pg_render_workspace_size(ctypes.byref(s), ctypes.byref(qq), ctypes.byref(nb)))
            buf, ws, n = _workspace(nb.value, paths.device)
            image = torch.empty(paths.height, paths.width, 3, dtype=torch.float32, device=paths.device)
            _check(lib().pg_render(ctypes.byref(s), ctypes.byref(qq), _ptr(image), None, _ptr(ws), n,
                                   _stream(paths.device)))
            ctx.paths, ctx.q, ctx.ws = paths, qq, (buf, ws, n)
            return image

        @staticmethod
        def backward(ctx, grad_image):
            _, ws, n = ctx.ws
            out = pg_backward(ctx.paths, ctx.q, grad_image, workspace=(ws, n))
            ctx.ws = None
            return out["grad_grid"], out["grad_g"].reshape(()), None, None

    return RenderFunction


_RF = None


def render_differentiable(paths: DevicePaths, q: Params, albedo_grid, g):
    """Image as a differentiable function of the albedo grid [R,R,R] and the
    scalar HG parameter g (torch tensors); paths and the sampling pdfs
    (q.g_s) stay fixed."""
    global _RF
    if _RF is None:
        _RF = _render_function()
    return _RF.apply(albedo_grid, g, paths, q)


def _batch_structs(paths_list, params_list):
    n = len(paths_list)
    P = (Paths * n)(*[p.struct() for p in paths_list])
    Q = (Params * n)(*[Params.from_buffer_copy(q) for q in params_list])
    return n, P, Q


def pg_render_batched(paths_list, params_list):
    """Render independent scenes in one batched pass; returns their images."""
    torch = _torch()
    L = lib()
    n, P, Q = _batch_structs(paths_list, params_list)
    nb = ctypes.c_size_t()
    _check(L.pg_render_batched_workspace_size(n, P, Q, ctypes.byref(nb)))
    dev = paths_list[0].device
    _, ws, nbytes = _workspace(nb.value, dev)
    images = [torch.empty(p.height, p.width, 3, dtype=torch.float32, device=dev) for p in paths_list]
    ptrs = (ctypes.c_void_p * n)(*[im.data_ptr() for im in images])
    _check(L.pg_render_batched(n, P, Q, ptrs, _ptr(ws), nbytes, _stream(dev)))
    return images


class Batch:
    """A reusable batch plan (optionally one hipGraph launch per render).
    Work runs on a stream of its own, ordered after the current stream's work
    and before anything enqueued on the current stream afterwards."""

    def __init__(self, paths_list, params_list, use_graph=True, tune=False):
        """tune: pick every scene's cell shift and the batch's edge tile with
        the autotuner (results unchanged; recorded in ``self.tuned``)."""
        torch = _torch()
        L = lib()
        self.paths_list = list(paths_list)
        self.tuned = None
        if tune:
            from . import autotune
            params_list = [Params.from_buffer_copy(q) for q in params_list]
            shifts = []
            for p, q in zip(self.paths_list, params_list):
                if p.n_vertices and not (q.flags & PG_FLAG_CLUSTERS):
                    q.cell_shift = autotune.tune_cell_shift(p, q.k)
                shifts.append(q.cell_shift)
            # the batched iterations are one launch shape for all scenes: tuned on the largest
            big = max(range(len(params_list)), key=lambda s: self.paths_list[s].n_vertices)
            qb = params_list[big]
            tile, group = autotune.tune_tile(self.paths_list[big], qb.k, qb.g, cell_shift=qb.cell_shift,
                                             default=autotune.BATCH_DEFAULT)
            for q in params_list:
                q.tile, q.tile_group = tile, group
            self.tuned = {"cell_shift": shifts, "tile": tile, "tile_group": group}
        n, self._P, self._Q = _batch_structs(paths_list, params_list)
        nb = ctypes.c_size_t()
        _check(L.pg_render_batched_workspace_size(n, self._P, self._Q, ctypes.byref(nb)))
        self.device = paths_list[0].device
        self.stream = torch.cuda.Stream(self.device)
        self._buf, self.ws, self.ws_bytes = _workspace(nb.value, self.device)
        self.images = [torch.empty(p.height, p.width, 3, dtype=torch.float32, device=self.device)
                       for p in paths_list]
        self._ptrs = (ctypes.c_void_p * n)(*[im.data_ptr() for im in self.images])
        self.handle = ctypes.c_void_p()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        _check(L.pg_batch_create(n, self._P, self._Q, self._ptrs, _ptr(self.ws), self.ws_bytes, int(use_graph),
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self.handle)))

    def __call__(self):
        torch = _torch()
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        _check(lib().pg_batch_launch(self.handle, ctypes.c_void_p(self.stream.cuda_stream)))
        cur.wait_stream(self.stream)
        return self.images

    def close(self):
        if self.handle:
            _torch().cuda.synchronize(self.device)
            lib().pg_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
