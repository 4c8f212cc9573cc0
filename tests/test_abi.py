"""The C ABI library on the CPU: it loads, exports every symbol the header
declares, and rejects invalid arguments on the host before touching a GPU."""
import ctypes
import math
import os
import re
import subprocess

import pytest

import paper_2404_11894_amd as pg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pathgraph.h")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]*?\b(pg_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    names = declared()
    assert "pg_render" in names and "pg_backward" in names and "pg_render_batched" in names
    lib = pg.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(pg.EXPORTS)


STRUCTS = {"pg_paths": "Paths", "pg_params": "Params", "pg_graph_out": "GraphOut",
           "pg_profile_entry": "ProfileEntry", "pg_tracer": "Tracer", "pg_records": "Records"}


def test_ctypes_structs_match_the_header(tmp_path):
    """Every struct the binding mirrors has the header's size and field offsets
    (a C program built against the header prints them); equal sizes also mean
    no header field is missing from the binding."""
    lines = ['#include <stdio.h>', '#include "pathgraph.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for field, _ in getattr(pg, pyname)._fields_:
            lines.append(f'printf("{cname}.{field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.splitlines())
    for cname, pyname in STRUCTS.items():
        cls = getattr(pg, pyname)
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert int(got[f"{cname}.{field}"]) == getattr(cls, field).offset, f"{cname}.{field}"


def test_version_and_default_shift():
    assert pg.pg_version().startswith("pathgraph-gfx950")
    assert pg.pg_default_cell_shift(0) == 20
    assert pg.pg_default_cell_shift(30000) == 16      # 16^3 <= 30000 < 32^3
    assert pg.pg_default_cell_shift(22_000_000) == 12
    assert pg.pg_default_cell_shift(1000) == 17       # 8^3 <= 1000 < 16^3
    assert pg.pg_default_cell_shift(10 ** 12) == 11   # capped at 512 cells per axis


def fake_paths(N=100, P=16, w=4, h=4, spp=1):
    """A paths struct with non-NULL dummy pointers; never dereferenced on the host."""
    s = pg.Paths()
    s.n_vertices, s.n_paths, s.width, s.height, s.spp = N, P, w, h, spp
    for name in ("path_offsets", "pos", "dir_in", "dir_out", "albedo", "l_sun", "dir_env", "l_env",
                 "l_phase", "e_cam"):
        setattr(s, name, 0x1000)
    return s


def status(fn, *args):
    rc = fn(*args)
    return rc, pg.lib().pg_last_error().decode()


def test_workspace_queries_validate_arguments():
    L = pg.lib()
    s, q = fake_paths(), pg.params(k=8, D=4)
    nb = ctypes.c_size_t()
    assert L.pg_render_workspace_size(ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb)) == 0
    assert nb.value > 0 and nb.value % 256 == 0
    small = nb.value
    q.flags = pg.PG_FLAG_TAPE
    assert L.pg_render_workspace_size(ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb)) == 0
    assert nb.value > small                 # the tape keeps every iterate
    q.flags = pg.PG_FLAG_CHECK | pg.PG_FLAG_EXACT_KNN
    assert L.pg_render_workspace_size(ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb)) == 0
    assert nb.value == small
    for bad in (dict(k=0), dict(k=65), dict(D=-1), dict(g=1.0), dict(g=0.3, g_s=-1.0), dict(env_pdf=0.0),
                dict(init=2), dict(final_gather=3), dict(cell_shift=5), dict(schedule=9), dict(flags=64)):
        kw = dict(k=8, D=4)
        kw.update(bad)
        qq = pg.params(**{k: v for k, v in kw.items() if k in ("k", "D", "g", "g_s", "env_pdf", "init",
                                                                "final_gather", "cell_shift", "schedule",
                                                                "flags")})
        rc, msg = status(L.pg_render_workspace_size, ctypes.byref(s), ctypes.byref(qq), ctypes.byref(nb))
        assert rc == pg.PG_ERR_ARG, (bad, rc)
        assert msg
    qq = pg.params(k=8, D=4)
    qq.sun_dir[1] = math.nan
    assert L.pg_render_workspace_size(ctypes.byref(s), ctypes.byref(qq), ctypes.byref(nb)) == pg.PG_ERR_ARG


def test_paths_validation():
    L = pg.lib()
    q = pg.params()
    nb = ctypes.c_size_t()
    s = fake_paths(P=15)          # P != w*h*spp
    assert L.pg_render_workspace_size(ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb)) == pg.PG_ERR_ARG
    s = fake_paths(N=-1)
    assert L.pg_render_workspace_size(ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb)) == pg.PG_ERR_ARG
    s = fake_paths(N=2 ** 31)
    assert L.pg_render_workspace_size(ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb)) == pg.PG_ERR_ARG
    s = fake_paths()
    s.dir_env = None
    assert L.pg_render_workspace_size(ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb)) == pg.PG_ERR_ARG
    s = fake_paths()
    s.albedo = None               # neither per-vertex albedo nor a grid
    assert L.pg_render_workspace_size(ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb)) == pg.PG_ERR_ARG
    s.albedo_grid, s.albedo_grid_res = 0x2000, 64
    assert L.pg_render_workspace_size(ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb)) == 0
    s = fake_paths(N=0)
    s.pos = s.dir_in = None       # nothing to read when there are no vertices
    assert L.pg_render_workspace_size(ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb)) == 0
    assert L.pg_render_workspace_size(None, ctypes.byref(q), ctypes.byref(nb)) == pg.PG_ERR_ARG
    assert L.pg_render_workspace_size(ctypes.byref(s), None, ctypes.byref(nb)) == pg.PG_ERR_ARG


def test_cluster_flag_validation():
    L = pg.lib()
    nb = ctypes.c_size_t()
    s = fake_paths()
    q = pg.params(k=8, D=4, flags=pg.PG_FLAG_CLUSTERS)
    rc, msg = status(L.pg_render_workspace_size, ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb))
    assert rc == pg.PG_ERR_ARG and "cluster_key" in msg
    s.cluster_key = 0x1000
    assert L.pg_render_workspace_size(ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb)) == 0
    qq = pg.params(k=8, D=4, flags=pg.PG_FLAG_CLUSTERS, schedule=pg.PG_SCHED_SHIFTED)
    rc, _ = status(L.pg_render_workspace_size, ctypes.byref(s), ctypes.byref(qq), ctypes.byref(nb))
    assert rc == pg.PG_ERR_UNSUPPORTED
    qt = pg.params(k=8, D=4, flags=pg.PG_FLAG_CLUSTERS | pg.PG_FLAG_TAPE)
    assert L.pg_render_workspace_size(ctypes.byref(s), ctypes.byref(qt), ctypes.byref(nb)) == 0
    assert L.pg_backward_workspace_size(ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb)) == 0
    assert L.pg_clusters_workspace_size(ctypes.byref(s), 8, 0, ctypes.byref(nb)) == 0 and nb.value > 0
    s.cluster_key = None
    rc, _ = status(L.pg_clusters, ctypes.byref(s), 8, 0, ctypes.c_void_p(0x4000), ctypes.c_void_p(0x10000),
                   nb.value, None)
    assert rc == pg.PG_ERR_ARG


def test_tracer_validation():
    L = pg.lib()
    nb = ctypes.c_size_t()
    t = pg.Tracer()
    t.R, t.width, t.height, t.spp, t.max_depth = 8, 4, 4, 1, 3
    t.sigma, t.majorant, t.g = 0x1000, 1.0, 0.5
    assert L.pg_trace_workspace_size(ctypes.byref(t), ctypes.byref(nb)) == 0 and nb.value > 0
    for field, bad in (("R", 0), ("spp", 0), ("max_depth", 0), ("g", 1.0), ("majorant", -1.0), ("sigma", None),
                       ("crop_w", 5)):
        tt = pg.Tracer.from_buffer_copy(t)
        setattr(tt, field, bad)
        if field == "crop_w":
            tt.crop_h = 1
        rc, msg = status(L.pg_trace_workspace_size, ctypes.byref(tt), ctypes.byref(nb))
        assert rc == pg.PG_ERR_ARG and msg, field
    rc, _ = status(L.pg_trace_count, ctypes.byref(t), None, None, None, 0, None)
    assert rc == pg.PG_ERR_ARG


def test_tracer_workspace_holds_max_depth_records_per_path():
    # the counting pass keeps every path's records in the workspace: 88 bytes
    # per slot (seven 3-vectors and the albedo), max_depth slots per path, and
    # 24 more per slot with a point light
    L = pg.lib()
    t = pg.Tracer()
    t.R, t.width, t.height, t.spp = 8, 64, 32, 2
    t.sigma, t.majorant, t.g = 0x1000, 1.0, 0.5
    P = 64 * 32 * 2

    def ws(depth, pl=0.0):
        tt = pg.Tracer.from_buffer_copy(t)
        tt.max_depth = depth
        tt.pl_I[0] = pl
        nb = ctypes.c_size_t()
        assert L.pg_trace_workspace_size(ctypes.byref(tt), ctypes.byref(nb)) == 0
        return nb.value

    grow = ws(96) - ws(32)
    assert 88 * P * 64 <= grow <= 88 * P * 64 + 4096   # alignment padding of the carved arrays
    grow_pl = ws(96, 1.0) - ws(32, 1.0)
    assert 112 * P * 64 <= grow_pl <= 112 * P * 64 + 4096


def test_stored_sums_are_part_of_the_tape_workspace():
    # PG_FLAG_STORE_Z keeps 6 floats per vertex per iteration; the sizing
    # pass (null base) must carve them like the real one, for every entry
    # point that takes a tape: 24 D N more bytes, for K rounded up to 8, 12 or
    # 16 only
    L = pg.lib()
    s = pg.Paths()
    s.n_vertices, s.width, s.height, s.spp = 100000, 64, 64, 2
    s.n_paths = 64 * 64 * 2
    for name in ("path_offsets", "pos", "dir_in", "dir_out", "albedo", "l_sun", "dir_env", "l_env", "l_phase",
                 "e_cam", "albedo_grid"):
        setattr(s, name, 1 << 40)   # never dereferenced by the size queries
    s.albedo_grid_res = 8
    N, D = 100000, 7

    def sizes(k, flags):
        q = pg.params(k=k, D=D, flags=flags)
        out = []
        for fn in (L.pg_render_workspace_size, L.pg_backward_workspace_size):
            nb = ctypes.c_size_t()
            assert fn(ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb)) == 0
            out.append(nb.value)
        return out

    for k in (8, 12, 16):
        a, b = sizes(k, pg.PG_FLAG_TAPE), sizes(k, pg.PG_FLAG_TAPE | pg.PG_FLAG_STORE_Z)
        for x, y in zip(a, b):
            assert 24 * D * N <= y - x <= 24 * D * N + 512, (k, x, y)
    for k in (4, 20):   # no stored sums: the flag has no effect
        assert sizes(k, pg.PG_FLAG_TAPE) == sizes(k, pg.PG_FLAG_TAPE | pg.PG_FLAG_STORE_Z)
    # without the tape the flag has no effect either
    assert sizes(16, 0)[0] == sizes(16, pg.PG_FLAG_STORE_Z)[0]


def test_calls_reject_bad_workspace_before_launching():
    L = pg.lib()
    s, q = fake_paths(), pg.params(k=8, D=4)
    nb = ctypes.c_size_t()
    assert L.pg_render_workspace_size(ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb)) == 0
    img = ctypes.c_void_p(0x3000)
    rc, msg = status(L.pg_render, ctypes.byref(s), ctypes.byref(q), img, None, None, nb.value, None)
    assert rc == pg.PG_ERR_WORKSPACE and "NULL" in msg
    rc, msg = status(L.pg_render, ctypes.byref(s), ctypes.byref(q), img, None, ctypes.c_void_p(0x10100),
                     nb.value - 1, None)
    assert rc == pg.PG_ERR_WORKSPACE and "too small" in msg
    rc, msg = status(L.pg_render, ctypes.byref(s), ctypes.byref(q), img, None, ctypes.c_void_p(0x10010),
                     nb.value, None)
    assert rc == pg.PG_ERR_WORKSPACE and "aligned" in msg
    rc, _ = status(L.pg_render, ctypes.byref(s), ctypes.byref(q), None, None, ctypes.c_void_p(0x10100),
                   nb.value, None)
    assert rc == pg.PG_ERR_ARG
    rc, _ = status(L.pg_knn, ctypes.byref(s), 0, 0, ctypes.c_void_p(0x4000), ctypes.c_void_p(0x5000), None, 0,
                   None)
    assert rc == pg.PG_ERR_ARG
    rc, _ = status(L.pg_gather, ctypes.byref(s), ctypes.byref(q), None, None, None, None, None,
                   ctypes.c_void_p(0x3000), None)
    assert rc == pg.PG_ERR_ARG


def test_product_path_refuses_to_run_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(pg, "_lib", None)
    monkeypatch.setattr(pg, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="has not been built"):
        pg.lib()


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asked for more it says so and exits."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_static_propagate_rejects_graphs_beyond_its_scratch_on_the_host():
    # 4M vertices need 80 MB of propagation workspace, more than the 64 MiB
    # static scratch: refused before any device call
    L = pg.lib()
    s, q = fake_paths(N=4_000_000, P=16), pg.params(k=8, D=4)
    nb = ctypes.c_size_t()
    assert L.pg_propagate_workspace_size(ctypes.byref(s), ctypes.byref(q), ctypes.byref(nb)) == 0
    assert nb.value > 64 << 20
    p = ctypes.c_void_p(0x1000)
    rc, msg = status(L.pg_propagate_static, ctypes.byref(s), ctypes.byref(q), p, p, p, p, p, None, None)
    assert rc == pg.PG_ERR_WORKSPACE and "static scratch" in msg
    rc, msg = status(L.pg_propagate_static, ctypes.byref(s), None, p, p, p, p, p, None, None)
    assert rc == pg.PG_ERR_ARG


def test_csr_entry_points_refuse_the_cluster_flag_on_the_host():
    # pg_edges / pg_propagate / pg_gather read the k-nearest layout i*K + l;
    # the cluster relation's rows have other lengths
    L = pg.lib()
    s, q = fake_paths(), pg.params(k=8, D=4, flags=pg.PG_FLAG_CLUSTERS)
    p = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x10000)
    for fn, args in ((L.pg_edges, (p, p, p, p, p, p, p, p, ws, 1 << 30, None)),
                     (L.pg_propagate, (p, p, p, p, p, None, ws, 1 << 30, None)),
                     (L.pg_gather, (p, p, p, p, p, p, None)),
                     (L.pg_propagate_static, (p, p, p, p, p, None, None))):
        rc, msg = status(fn, ctypes.byref(s), ctypes.byref(q), *args)
        assert rc == pg.PG_ERR_UNSUPPORTED and "k-nearest" in msg, fn


def test_persistent_batch_flag_needs_the_default_tile():
    L = pg.lib()
    s = (pg.Paths * 1)(fake_paths())
    q = (pg.Params * 1)(pg.params(k=8, D=4, flags=pg.PG_FLAG_PERSISTENT, tile=512))
    nb = ctypes.c_size_t()
    rc, msg = status(L.pg_render_batched_workspace_size, 1, s, q, ctypes.byref(nb))
    assert rc == pg.PG_ERR_UNSUPPORTED and "PERSISTENT" in msg
    q[0].tile = 256
    assert L.pg_render_batched_workspace_size(1, s, q, ctypes.byref(nb)) == 0
