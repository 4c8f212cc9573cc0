"""FP64 CPU oracle for path-graph rendering of participating media.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2404_11894_amd``) never does, and the two share no code.

The arithmetic lives in ``pg_oracle.c`` (plain single-threaded C, double
precision).  This module only builds it, marshals numpy arrays and returns
numpy arrays.  Method parameters are a plain mapping:

* ``k``  neighbours per vertex, the vertex itself included (K = min(k, N));
* ``D``  number of aggregation + propagation iterations;
* ``g``  HG parameter of the receiver's phase function; ``g_s`` that of the
  sampling pdfs (defaults to ``g``; the gradient holds ``g_s`` fixed);
* ``init``  ``"pt"`` (path-traced initial estimate, paper's default) or ``"zero"``;
* ``final_gather``  0: aggregate at the first vertex; 1: own continuation only;
* ``sun_dir``  unit vector toward the sun; ``env_pdf`` (1/(4 pi)).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_DIR = os.path.join(_HERE, "_lib")
_SANITIZE = os.environ.get("PG_SANITIZE") == "1"
_LIB_PATH = os.path.join(_LIB_DIR, "liboracle_san.so" if _SANITIZE else "liboracle.so")
_SRC = os.path.join(_HERE, "pg_oracle.c")
# AddressSanitizer + UndefinedBehaviorSanitizer build (PG_SANITIZE=1): clang,
# so that one sanitizer runtime serves the oracle, the generator and the host
# side of the HIP library in one process.
CLANG = "/opt/rocm/llvm/bin/clang"
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
             "-g", "-O1", "-shared-libsan"]


def build(verbose: bool = False, sanitize: bool | None = None) -> str:
    """Compile pg_oracle.c into oracle/_lib/liboracle.so (gcc, no fast-math);
    with ``sanitize`` (default: PG_SANITIZE=1 in the environment) an
    ASan + UBSan build with clang, liboracle_san.so."""
    sanitize = _SANITIZE if sanitize is None else sanitize
    os.makedirs(_LIB_DIR, exist_ok=True)
    out = os.path.join(_LIB_DIR, "liboracle_san.so" if sanitize else "liboracle.so")
    tmp = out + ".tmp"
    if sanitize:
        cmd = [CLANG, *SAN_FLAGS, "-shared", "-fPIC", "-ffp-contract=off", "-Wall", "-Wextra", _SRC, "-lm",
               "-o", tmp]
    else:
        cmd = ["gcc", "-O2", "-shared", "-fPIC", "-ffp-contract=off", "-Wall", "-Wextra", _SRC, "-lm", "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


class _Scene(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("n_paths", ctypes.c_int64),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("spp", ctypes.c_int32),
                ("pad_", ctypes.c_int32)] + [
        (name, ctypes.c_void_p) for name in ("path_offsets", "pos", "dir_in", "dir_out", "albedo",
                                             "l_sun", "dir_env", "l_env", "l_phase", "e_cam",
                                             "l_emit", "cluster_key", "fb_l_sun", "fb_dir_env",
                                             "fb_l_env")] + [("n_extra", ctypes.c_int32), ("pad2_", ctypes.c_int32),
                                                             ("dir_pl", ctypes.c_void_p), ("l_pl", ctypes.c_void_p)]


class _Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("D", ctypes.c_int32), ("init", ctypes.c_int32),
                ("final_gather", ctypes.c_int32), ("neighbours", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("g", ctypes.c_double), ("g_s", ctypes.c_double),
                ("env_pdf", ctypes.c_double), ("sun_dir", ctypes.c_double * 3)]


class _Trace(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in
                ("row_ptr", "col", "w_ind", "w_ph", "w_env", "d_agg", "b", "d_pt", "r", "lplus0", "lplus",
                 "traj", "out_path")]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        lib.or_hg.restype = ctypes.c_double
        lib.or_hg.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.or_hg_dlog.restype = ctypes.c_double
        lib.or_hg_dlog.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.or_quantize.argtypes = [i64, vp, vp]
        lib.or_knn.argtypes = [i64, vp, i32, i64, vp, vp]
        lib.or_clusters.argtypes = [i64, vp, vp, i32, vp]
        lib.or_edges.argtypes = [ctypes.POINTER(_Scene), ctypes.POINTER(_Params), i32, i64, vp, vp,
                                 vp, vp, vp, vp, vp, vp]
        lib.or_albedo_from_grid.argtypes = [i64, vp, i32, vp, vp]
        lib.or_render.argtypes = [ctypes.POINTER(_Scene), ctypes.POINTER(_Params), vp, vp,
                                  ctypes.POINTER(_Trace)]
        lib.or_backward.argtypes = [ctypes.POINTER(_Scene), ctypes.POINTER(_Params), i32, vp, vp, vp,
                                    vp, vp, vp]
        for f in ("or_quantize", "or_knn", "or_clusters", "or_edges", "or_albedo_from_grid", "or_render", "or_backward"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


ERRORS = {-1: "invalid argument", -4: "invalid input data", -6: "out of memory"}


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise OracleError(rc, f"{what}: {ERRORS.get(rc, rc)}")


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None:
        a = a.reshape(shape)
    return a


class _Bound:
    """Keeps contiguous copies of the scene arrays alive while C reads them."""

    def __init__(self, scene):
        N = int(np.asarray(scene.pos).shape[0])
        P = int(np.asarray(scene.path_offsets).shape[0]) - 1
        self.arrays = {
            "path_offsets": np.ascontiguousarray(scene.path_offsets, dtype=np.int64),
            "pos": _f32(scene.pos, (N, 3)), "dir_in": _f32(scene.dir_in, (N, 3)),
            "dir_out": _f32(scene.dir_out, (N, 3)), "albedo": _f32(scene.albedo, (N,)),
            "l_sun": _f32(scene.l_sun, (N, 3)), "dir_env": _f32(scene.dir_env, (N, 3)),
            "l_env": _f32(scene.l_env, (N, 3)), "l_phase": _f32(scene.l_phase, (N, 3)),
            "e_cam": _f32(scene.e_cam, (P, 3)),
        }
        if getattr(scene, "l_emit", None) is not None:   # volume emission, optional
            self.arrays["l_emit"] = _f32(scene.l_emit, (N, 3))
        if getattr(scene, "cluster_key", None) is not None:   # cluster neighbour relation
            self.arrays["cluster_key"] = np.ascontiguousarray(scene.cluster_key, dtype=np.uint32).reshape(N)
        if getattr(scene, "dir_pl", None) is not None:         # point light
            self.arrays["dir_pl"] = _f32(scene.dir_pl, (N, 3))
            self.arrays["l_pl"] = _f32(scene.l_pl, (N, 3))
        M = 0
        if getattr(scene, "fb_l_sun", None) is not None:       # extra first-vertex samples
            M = int(np.asarray(scene.fb_l_sun).shape[1])
            for name in ("fb_l_sun", "fb_dir_env", "fb_l_env"):
                self.arrays[name] = _f32(getattr(scene, name), (P, M, 3))
        s = _Scene()
        s.n_vertices, s.n_paths = N, P
        s.width, s.height, s.spp = int(scene.width), int(scene.height), int(scene.spp)
        for name, arr in self.arrays.items():
            setattr(s, name, _p(arr))
        s.n_extra = M
        self.c = s
        self.N, self.P = N, P


def params(k=8, D=8, g=0.5, g_s=None, init="pt", final_gather=0, sun_dir=None, env_pdf=None,
           neighbours="knn") -> dict:
    """Method parameters as a plain dict (defaults of the small workload).
    neighbours: "knn" (k nearest) or "clusters" (the scene's cluster_key
    chooses the centres, k is the expected cluster size)."""
    if sun_dir is None:
        n = math.sqrt(0.3 ** 2 + 1.0 + 0.4 ** 2)
        sun_dir = (0.3 / n, 1.0 / n, -0.4 / n)
    return {"k": k, "D": D, "g": g, "g_s": g if g_s is None else g_s, "init": init,
            "final_gather": final_gather, "sun_dir": tuple(sun_dir),
            "env_pdf": 1.0 / (4.0 * math.pi) if env_pdf is None else env_pdf, "neighbours": neighbours}


def _params(p: dict) -> _Params:
    c = _Params()
    c.k, c.D = int(p["k"]), int(p["D"])
    c.init = {"pt": 0, "zero": 1}[p.get("init", "pt")]
    c.final_gather = int(p.get("final_gather", 0))
    c.neighbours = {"knn": 0, "clusters": 1}[p.get("neighbours", "knn")]
    c.g = float(p["g"])
    c.g_s = float(p.get("g_s", p["g"]) if p.get("g_s") is not None else p["g"])
    c.env_pdf = float(p.get("env_pdf", 1.0 / (4.0 * math.pi)))
    c.sun_dir[:] = [float(x) for x in p["sun_dir"]]
    return c


def hg(g: float, u) -> np.ndarray:
    """Henyey-Greenstein density at u = 1 - cos(theta)."""
    lib = _load()
    return np.vectorize(lambda x: lib.or_hg(float(g), float(x)))(np.asarray(u, dtype=np.float64))


def hg_dlog(g: float, u) -> np.ndarray:
    """d ln HG / d g at u = 1 - cos(theta)."""
    lib = _load()
    return np.vectorize(lambda x: lib.or_hg_dlog(float(g), float(x)))(np.asarray(u, dtype=np.float64))


def quantize(pos) -> tuple[np.ndarray, bool]:
    """20-bit integer coordinates [N,3] and whether every input was in [0,1]."""
    lib = _load()
    pos = _f32(pos).reshape(-1, 3)
    q = np.empty(pos.shape, np.int64)
    rc = lib.or_quantize(pos.shape[0], _p(pos), _p(q))
    return q, rc == 0


def knn(pos, k: int, rows=None) -> np.ndarray:
    """Neighbour lists [nq, K]: the vertex itself, then the K-1 nearest others
    by (squared quantised distance, index); K = min(k, N)."""
    lib = _load()
    pos = _f32(pos).reshape(-1, 3)
    n = pos.shape[0]
    K = min(int(k), n)
    if rows is None:
        r = None
        nq = n
    else:
        r = np.ascontiguousarray(rows, dtype=np.int64)
        nq = r.shape[0]
    col = np.empty((nq, max(K, 0)), np.int32)
    rc = lib.or_knn(n, _p(pos), int(k), nq, _p(r), _p(col))
    if rc not in (0, -4):
        _check(rc, "knn")
    return col


def clusters(pos, key, k: int) -> np.ndarray:
    """Centre id [N] of every vertex's cluster (or_clusters): centres where
    key < 2^32 // k (and the smallest key), nearest centre by (squared
    quantised distance, id), clusters above 2k members split again."""
    lib = _load()
    pos = _f32(pos).reshape(-1, 3)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1)
    n = pos.shape[0]
    assert key.shape[0] == n
    out = np.empty(n, np.int32)
    rc = lib.or_clusters(n, _p(pos), _p(key), int(k), _p(out))
    if rc not in (0, -4):
        _check(rc, "clusters")
    return out


def cluster_rows(centre) -> tuple[np.ndarray, np.ndarray]:
    """CSR of the cluster neighbour relation: row i lists the members of i's
    cluster in ascending id.  Returns (row_ptr [N+1], col [E])."""
    centre = np.asarray(centre)
    n = centre.shape[0]
    order = np.lexsort((np.arange(n), centre))
    size = np.bincount(centre, minlength=n) if n else np.zeros(0, np.int64)
    start = np.zeros(n + 1, np.int64)
    start[1:] = np.cumsum(size)
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum(size[centre]) if n else []
    col = np.empty(int(rp[-1]), np.int32)
    for i in range(n):
        c = centre[i]
        col[rp[i]:rp[i + 1]] = order[start[c]:start[c + 1]]
    return rp, col


def albedo_from_grid(pos, grid) -> np.ndarray:
    """Per-vertex albedo: cell-centred trilinear interpolation of grid [R,R,R] (z,y,x)."""
    lib = _load()
    pos = _f32(pos).reshape(-1, 3)
    grid = _f32(grid)
    R = grid.shape[0]
    out = np.empty(pos.shape[0], np.float64)
    _check(lib.or_albedo_from_grid(pos.shape[0], _p(pos), R, _p(grid), _p(out)), "albedo_from_grid")
    return out


def edges(scene, p: dict, col: np.ndarray, rows=None) -> dict:
    """Edge weights and direct terms of the receivers ``rows`` (default: all),
    given their neighbour lists ``col`` [nq, K]."""
    lib = _load()
    b = _Bound(scene)
    col = np.ascontiguousarray(col, dtype=np.int32)
    nq, K = col.shape
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    out = {"w_ind": np.empty((nq, K)), "w_ph": np.empty((nq, K)), "w_env": np.empty((nq, K)),
           "d_agg": np.empty((nq, 3)), "d_pt": np.empty((nq, 3)), "r": np.empty(nq)}
    cp = _params(p)
    _check(lib.or_edges(ctypes.byref(b.c), ctypes.byref(cp), K, nq, _p(r), _p(col), _p(out["w_ind"]),
                        _p(out["w_ph"]), _p(out["w_env"]), _p(out["d_agg"]), _p(out["d_pt"]), _p(out["r"])),
           "edges")
    return out


def render(scene, p: dict, alpha=None, trace: bool = False, traj: bool = False):
    """FP64 image [H, W, 3]; with ``trace`` also every intermediate result."""
    lib = _load()
    b = _Bound(scene)
    N, P = b.N, b.P
    K = min(int(p["k"]), N) if N else 0
    image = np.empty((int(scene.height), int(scene.width), 3), np.float64)
    a = None if alpha is None else np.ascontiguousarray(alpha, dtype=np.float64)
    out = None
    tr = None
    if trace:
        if p.get("neighbours", "knn") == "clusters":
            E = int(cluster_rows(clusters(scene.pos, scene.cluster_key, p["k"]))[0][-1]) if N else 0
            shape = (E,)
        else:
            shape = (N, K)
        out = {"row_ptr": np.empty(N + 1, np.int64), "col": np.empty(shape, np.int32), "w_ind": np.empty(shape),
               "w_ph": np.empty(shape), "w_env": np.empty(shape), "d_agg": np.empty((N, 3)), "b": np.empty((N, 3)),
               "d_pt": np.empty((N, 3)), "r": np.empty(N), "lplus0": np.empty((N, 3)),
               "lplus": np.empty((N, 3)), "out_path": np.empty((P, 3))}
        if traj:
            out["traj"] = np.empty((int(p["D"]) + 1, N, 3))
        tr = _Trace()
        for name, arr in out.items():
            setattr(tr, name, _p(arr))
    cp = _params(p)
    _check(lib.or_render(ctypes.byref(b.c), ctypes.byref(cp), _p(a), _p(image),
                         ctypes.byref(tr) if tr is not None else None), "render")
    return (image, out) if trace else image


def backward(scene, p: dict, grad_image, grid=None) -> dict:
    """Reverse-mode gradient of <grad_image, I> w.r.t. per-vertex albedo, the
    albedo grid (if given; the albedo is then its trilinear interpolation) and g."""
    lib = _load()
    b = _Bound(scene)
    N = b.N
    gi = np.ascontiguousarray(grad_image, dtype=np.float64).reshape(int(scene.height), int(scene.width), 3)
    ga = np.empty(N, np.float64)
    gg = np.zeros(1, np.float64)
    image = np.empty((int(scene.height), int(scene.width), 3), np.float64)
    R = 0
    gr = None
    gp = None
    if grid is not None:
        gp = _f32(grid)
        R = gp.shape[0]
        gr = np.empty(gp.shape, np.float64)
    cp = _params(p)
    _check(lib.or_backward(ctypes.byref(b.c), ctypes.byref(cp), R, _p(gp), _p(gi), _p(ga), _p(gr), _p(gg),
                           _p(image)), "backward")
    out = {"grad_alpha": ga, "grad_g": float(gg[0]), "image": image}
    if grid is not None:
        out["grad_grid"] = gr
    return out
