#!/usr/bin/env python3
"""Benchmark of the path-graph hot path on one MI355X.

Headline workload (the forward line): the large dense forward-scattering
cloud -- 512^3 fBm medium (sigma_t <= 64), albedo 0.999, HG g = 0.9, sun +
environment, 1024x1024 px at 1 spp, delta-tracking paths to depth 128
(about 69M vertices); k = 16 neighbours, D = 128 iterations.  Inputs are
generated on the host, copied to HBM, and are resident before the timed
region starts.

One step = one pg_render call: grid build + exact kNN, aggregation operators,
path pass, D iterations of aggregation + propagation, output to pixels.
value = E * D / step time  (E = N * K edges), in Gedge-updates/s.

The other legs run on the mid workload (128^3 fBm ball, 512x512 px at 4 spp,
depth 64, k = 16, D = 64), on which the differentiation workload is defined:
its forward line, the GPU path tracer, the cluster relation, forward +
adjoint; then the 64-scene batch.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import dataclasses
import ctypes
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gedge-updates/s fwd, fwd+adjoint, batched vs per-scene on 1 GPU; % HBM peak"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(step, N, K, starts, n_far=None):
    """Compulsory HBM bytes of one launch of a propagation step (every input
    read once, every output written once):
      spmv with the compact ids (n_far given): per row the 16-bit ids and the
      weights (2K + 4K), one x gather, b, albedo, one y write (12 + 12 + 4 +
      12), plus 4 bytes per far id read from the side list and one 4-byte
      list start per 64-row slice: N (6K + 40) + 4 n_far + 4 (N/64 + 1)
      spmv / spmv_shifted with 32-bit ids: col + weight per edge (8 B), one x
      gather, b (or c) and albedo or row mask per row, one y write:
      N (8K + 12 + 12 + 4 + 12)
      spmv_scatter: the same plus the predecessor id, for the N - starts rows
      that have a predecessor; a path's first vertex reads only that id
      shift: successor id, one y gather, one x write: N (4 + 12 + 12)."""
    if step == "spmv" and n_far is not None:
        return N * (6 * K + 40) + 4 * n_far + 4 * (-(-N // 64) + 1)
    if step in ("spmv", "spmv_shifted"):
        return N * (8 * K + 40)
    if step == "spmv_scatter":
        return (N - starts) * (8 * K + 44) + starts * 4
    if step == "shift":
        return N * 28
    return None


SOURCES = {"spmv": ("pg_prop.hip", "pg_internal.h"), "shift": ("pg_prop.hip", "pg_internal.h"),
           "cagg": ("pg_clusters.hip", "pg_internal.h"), "rev_rows": ("pg_backward.hip", "pg_internal.h"),
           "rev_cols": ("pg_backward.hip", "pg_internal.h"), "spmv_tape": ("pg_backward.hip", "pg_internal.h")}


def kernel_source_hash(kernel="spmv"):
    """sha256 over the kernel's source file and the header it includes."""
    hsh = hashlib.sha256()
    for f in SOURCES[kernel]:
        hsh.update(open(os.path.join(ROOT, "paper_2404_11894_amd", "csrc", f), "rb").read())
    return hsh.hexdigest()


def read_traffic(kernel, workload, variant=None):
    """HBM bytes per launch measured with rocprofv3 counters, if the summary
    under profiles/ was taken from the current kernel source (and, with
    `variant`, names that kernel in its title)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if variant is not None and variant not in text.splitlines()[0]:
        return None
    m = re.search(r"bytes_per_launch:\s*([0-9.eE+]+)", text)
    h = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    if not m or not h:
        return None
    if kernel_source_hash(kernel if kernel in SOURCES else "spmv") != h.group(1):
        return None
    return float(m.group(1))


def profile_entries(pg):
    L = pg.lib()
    arr = (pg.ProfileEntry * 64)()
    n = ctypes.c_int32()
    pg._check(L.pg_profile_stop(64, arr, ctypes.byref(n)))
    return {arr[i].name.decode(): (arr[i].count, arr[i].total_ms, arr[i].max_ms) for i in range(min(n.value, 64))}


def cpu_baseline(workload, sc_full, seconds=10.0):
    """The FP64 oracle, single-threaded, on a centred square crop of the same
    workload (all its samples per pixel): the whole pipeline.  The crop starts
    at about 1e8 edge-updates (E D) and its work doubles until one run takes
    at least `seconds` (the oracle slows per edge as its arrays outgrow the
    host caches, so the size is found by measuring, not extrapolated); the
    last run is reported."""
    import oracle
    import scenegen
    k, D, g = workload.k, workload.D, workload.g
    per_px = sc_full.n_vertices / (sc_full.width * sc_full.height)

    def side_for(work):
        return int(max(8, min(sc_full.width, round((work / (k * D * per_px)) ** 0.5 / 8) * 8)))

    work = 1e8
    while True:
        side = side_for(work)
        sc = scenegen.generate(scenegen.crop_of(workload.scene, side, side))
        t0 = time.perf_counter()
        oracle.render(sc, oracle.params(k=k, D=D, g=g))
        dt = time.perf_counter() - t0
        log(f"cpu baseline: {side}x{side} crop, N={sc.n_vertices}, {dt:.1f} s")
        if dt >= seconds or side >= sc_full.width:
            break
        work *= 2
    K = min(k, sc.n_vertices)
    E = sc.n_vertices * K
    return {"value": E * D / dt / 1e9, "unit": "Gedge-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"centred {side}x{side}-pixel crop of the same image, {sc.spp} spp: N={sc.n_vertices}, E={E}, "
                      f"D={D}; whole pipeline (kNN, weights, {D} iterations, pixels) in {dt:.2f} s",
            "host": host_cpu()}


def host_cpu():
    """The host's CPU model and logical CPU count (the oracle uses one core)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def time_fwd_adjoint(pg, torch, sc, w, steps, warmup, store_z=True):
    """The differentiation workload: the same paths, albedo from a 64^3 grid
    (U[0.95, 0.999], seed 2), loss = sum (I - T)^2 against a seeded target.
    One step = pg_render with the tape (and, with store_z, every iteration's
    neighbour sums) + pg_backward on it.  Counts 2 E D."""
    import ctypes as C
    import scenegen
    dev = torch.device("cuda:0")
    grid = scenegen.albedo_grid(64, 0.95, 0.999, seed=2)
    paths = pg.DevicePaths(sc, device=dev, albedo_grid=grid)
    q = pg.params(k=w.k, D=w.D, g=w.g, flags=pg.PG_FLAG_TAPE | (pg.PG_FLAG_STORE_Z if store_z else 0))
    s = paths.struct()
    nb = C.c_size_t()
    pg._check(pg.lib().pg_render_workspace_size(C.byref(s), C.byref(q), C.byref(nb)))
    _, ws, n = pg._workspace(nb.value, dev)
    image = torch.empty(sc.height, sc.width, 3, device=dev)
    target = torch.from_numpy(scenegen.target_image((sc.height, sc.width, 3), 0.3, seed=4)).to(dev)

    def step():
        pg._check(pg.lib().pg_render(C.byref(s), C.byref(q), pg._ptr(image), None, pg._ptr(ws), n,
                                     pg._stream(dev)))
        gi = 2.0 * (image - target)
        return pg.pg_backward(paths, q, gi, workspace=(ws, n))

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    pg._check(pg.lib().pg_profile_start())
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    prof = profile_entries(pg)
    phases = {k: round(v[1] / steps, 3) for k, v in prof.items()}
    N = sc.n_vertices
    K = min(w.k, N)
    E = N * K
    # the reverse sweep's kernels against the HBM peak, by algorithmic bytes:
    # rev_rows per row, recomputing the sums: compact ids + weights + dw/dg
    # (2K + 4K + 4K), x_{t-1} gather 12, lambda gather at the predecessor 12 +
    # its position 4, albedo 4, dL/dalpha and dL/db each read and written
    # (2 x 4 + 2 x 12), zbar write 12: 10K + 76, plus the far ids' side list;
    # reading the stored sums instead: z and dz/dg 24 + the same 64 = 88;
    # rev_cols per T-row: source id + weight per entry (8K over the real
    # entries), zbar gather 12, lambda write 12.  With the stored sums the
    # forward's aggregation also reads dw/dg (4K) and writes the sums (24).
    nf = torch.zeros(1, dtype=torch.int64, device=dev)
    qn = pg.params(k=w.k, D=0, g=w.g)
    pg.Renderer(paths, qn)(graph={"n_far": nf})
    n_far = int(nf.item())
    rev = {}
    taped = store_z and K >= 5 and K <= 16
    rows_bytes = 88 * N if taped else N * (10 * K + 76) + 4 * n_far
    for name, ab in (("rev_rows", rows_bytes), ("rev_cols", N * (8 * K + 24))):
        if name in prof:
            cnt, tot, _ = prof[name]
            avg = tot / cnt / 1e3
            variant = None if name != "rev_rows" else ("k_rev_rows_taped" if taped else "k_rev_rows<")
            tr = read_traffic(name, w.name, variant)
            rev[name] = {"avg_launch_ms": round(avg * 1e3, 4), "algorithmic_bytes_per_launch": ab,
                         "achieved_GBs": round(ab / avg / 1e9, 1), "hbm_frac": round(ab / avg / 1e9 / HBM_PEAK_GBS, 4),
                         "traffic": tr, "traffic_GBs": round(tr / avg / 1e9, 1) if tr else None}
    if len(rev) == 2:
        t_it = rev["rev_rows"]["avg_launch_ms"] + rev["rev_cols"]["avg_launch_ms"]
        b_it = rev["rev_rows"]["algorithmic_bytes_per_launch"] + rev["rev_cols"]["algorithmic_bytes_per_launch"]
        rev["iteration"] = {"ms": round(t_it, 4), "hbm_frac": round(b_it / (t_it / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    if taped and "spmv" in prof:
        cnt, tot, _ = prof["spmv"]
        avg = tot / cnt / 1e3
        ab = N * (12 * K + 64)
        tr = read_traffic("spmv_tape", w.name)
        rev["taped_aggregation"] = {"avg_launch_ms": round(avg * 1e3, 4), "algorithmic_bytes_per_launch": ab,
                                    "hbm_frac": round(ab / avg / 1e9 / HBM_PEAK_GBS, 4),
                                    "bytes": "(8K + 40) N of the aggregation + 4K N (dw/dg) + 24 N (z, dz/dg)",
                                    "traffic": tr, "traffic_GBs": round(tr / avg / 1e9, 1) if tr else None}
    rev["stored_sums"] = bool(taped)
    ok = bool(torch.isfinite(out["grad_grid"]).all().item()) and bool(torch.isfinite(out["grad_g"]).all().item())
    del ws, paths
    torch.cuda.empty_cache()
    return {"value": round(2 * E * w.D / (ms / 1e3) / 1e9, 2), "unit": "Gedge-updates/s", "ms_per_step": round(ms, 3),
            "counts": "2*E*D per step (forward + reverse sweep)", "finite": ok, "phases_ms": phases,
            "reverse": rev,
            "workload": "same paths, albedo = trilinear 64^3 grid, L2 loss, grad wrt grid and g"}


def time_clusters(pg, torch, sc, w, steps, warmup, knn_ms):
    """The paper's own neighbour relation on the same paths: clusters of
    expected size k around centres drawn by seeded uniform keys (seed 7).
    One step = pg_render with PG_FLAG_CLUSTERS.  Counts E_c D, E_c = the sum
    over clusters of size^2 (every member aggregates every member); also one
    forward + reverse step with the albedo from the 64^3 grid (2 E_c D)."""
    import scenegen
    dev = torch.device("cuda:0")
    sck = dataclasses.replace(sc, cluster_key=scenegen.cluster_keys(sc.n_vertices, 7))
    paths = pg.DevicePaths(sck, device=dev)
    centre = pg.pg_clusters(paths, w.k)
    torch.cuda.synchronize()
    size = torch.bincount(centre.to(torch.int64), minlength=sc.n_vertices)
    nz = size[size > 0]
    E = int((nz * nz).sum().item())
    q = pg.params(k=w.k, D=w.D, g=w.g, flags=pg.PG_FLAG_CLUSTERS)
    render = pg.Renderer(paths, q)
    image = torch.empty(sc.height, sc.width, 3, device=dev)
    for _ in range(warmup):
        render(image)
    torch.cuda.synchronize()
    pg._check(pg.lib().pg_profile_start())
    t0 = time.perf_counter()
    for _ in range(steps):
        render(image)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    prof = profile_entries(pg)
    phases = {k: round(v[1] / steps, 4) for k, v in prof.items()}
    cnt, tot, _ = prof["spmv"]
    avg_s = tot / cnt / 1e3
    N = sc.n_vertices
    # forward + reverse mode with the cluster relation (albedo from the 64^3 grid, as fwd_adjoint)
    del render
    torch.cuda.empty_cache()
    paths.set_albedo_grid(scenegen.albedo_grid(64, 0.95, 0.999, seed=2))
    qt = pg.params(k=w.k, D=w.D, g=w.g, flags=pg.PG_FLAG_CLUSTERS | pg.PG_FLAG_TAPE)
    rt = pg.Renderer(paths, qt)
    target = torch.from_numpy(scenegen.target_image((sc.height, sc.width, 3), 0.3, seed=4)).to(dev)

    def adj_step():
        rt(image)
        return pg.pg_backward(paths, qt, 2.0 * (image - target), workspace=(rt.ws, rt.ws_bytes))

    adj_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_adj = max(2, steps // 2)
    for _ in range(n_adj):
        g_out = adj_step()
    torch.cuda.synchronize()
    adj_ms = (time.perf_counter() - t0) * 1e3 / n_adj
    adj_ok = bool(torch.isfinite(g_out["grad_grid"]).all().item())
    del rt
    # per row: (t, albedo) 16, range 8, b 12, y 12; each member's (w, 1/M+) 16 once, and its x: 12 read
    # (first iteration) or successor id 4 + gathered y 12 (the others, propagation folded in)
    ab = N * (76 + 80 * (w.D - 1)) / w.D
    flops = 22 * E  # per edge: 1 - cos 9, HG 7 (one rsqrt), 1/M+ 1, accumulate 6 (FMA = 2)
    del paths
    torch.cuda.empty_cache()
    return {"value": round(E * w.D / (ms / 1e3) / 1e9, 2), "unit": "Gedge-updates/s", "ms_per_step": round(ms, 3),
            "fwd_adjoint": {"value": round(2 * E * w.D / (adj_ms / 1e3) / 1e9, 2), "ms_per_step": round(adj_ms, 3),
                            "finite": adj_ok},
            "vs_knn_render": round(knn_ms / ms, 3) if knn_ms == knn_ms else None, "E": E, "clusters": int(nz.numel()),
            "mean_size": round(N / max(1, int(nz.numel())), 2), "max_size": int(nz.max().item()),
            "phases_ms": phases,
            "aggregation": {"kernel": "k_cagg", "avg_launch_ms": round(avg_s * 1e3, 4),
                            "algorithmic_bytes_per_launch": int(ab),
                            "traffic": read_traffic("cagg", "mid") if w.name == "mid" else None,
                            "algorithmic_GBs": round(ab / avg_s / 1e9, 1), "hbm_frac": round(ab / avg_s / 1e9 / HBM_PEAK_GBS, 4),
                            "TFLOPs": round(flops / avg_s / 1e12, 2), "fp32_frac": round(flops / avg_s / 1e12 / 157.3, 4),
                            "gedge_per_s_per_launch": round(E / avg_s / 1e9, 1)},
            "workload": "same paths, cluster relation (k = expected cluster size), keys seed 7"}


def time_tracer(pg, torch, w, host_gen_s, host_copy_s):
    """Generating the workload's records on the GPU (pg_trace: the count pass
    traces into the workspace, a scan, the record pass compacts) against the
    host generator plus the copy to HBM."""
    import scenegen
    dev = torch.device("cuda:0")
    sigma, alb, maj = scenegen.medium(w.scene)
    st = scenegen.tracer_settings(w.scene)
    rec = pg.pg_trace(st, sigma, alb, maj, device=dev)        # warm-up (and the grid upload)
    torch.cuda.synchronize()
    sg = torch.as_tensor(sigma).to(dev)
    ag = None if alb is None else torch.as_tensor(alb).to(dev)
    times = []
    for _ in range(3):
        del rec
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec = pg.pg_trace(st, sg, ag, maj, device=dev)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    ms = min(times) * 1e3
    n = rec.n_vertices
    del rec, sg, ag
    torch.cuda.empty_cache()
    return {"ms_device": round(ms, 2), "n_vertices": n, "paths": w.scene.width * w.scene.height * w.scene.spp,
            "ms_host_generate": round(host_gen_s * 1e3, 1), "ms_host_to_device_copy": round(host_copy_s * 1e3, 1),
            "speedup_vs_host_plus_copy": round((host_gen_s + host_copy_s) * 1e3 / ms, 2),
            "note": "records traced once into the workspace (pg_trace_count), then compacted (pg_trace_records); host: all cores of the box"}


def study(pg, torch, w):
    """Convergence and quality of the path graph on the workload's medium.

    Convergence: with the paths of the workload fixed, the relative change of
    the image and of L+ between iteration counts, for both initialisations.
    Quality: at 1 spp over the full image, the mean squared error over the
    centred 64x64 crop of plain path tracing (k = 1, D = 0), the path graph
    (k nearest and clusters) and its iteration count, against a 1024-spp
    path-traced reference of that crop (independent seed); mean of 4 seeds."""
    import numpy as np
    import scenegen
    dev = torch.device("cuda:0")
    res = {}

    def render(paths, k, D, init="pt", clusters=False, lplus=False):
        fl = pg.PG_FLAG_CLUSTERS if clusters else 0
        q = pg.params(k=k, D=D, g=w.g, init=init, flags=fl)
        if lplus:
            r = pg.Renderer(paths, q)
            img = torch.empty(paths.height, paths.width, 3, device=dev)
            lp = torch.empty(paths.n_vertices, 3, device=dev)
            r(img, graph={"lplus": lp})
            return img.cpu().numpy().astype(np.float64), lp.cpu().numpy()
        return pg.pg_render(paths, q).cpu().numpy().astype(np.float64)

    def rel(a, b):
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))

    log("study: convergence")
    sc = scenegen.generate(w.scene)
    sck = pg.DevicePaths(dataclasses.replace(sc, cluster_key=scenegen.cluster_keys(sc.n_vertices, 7)), device=dev)
    del sc
    ts = [0, 1, 2, 3, 4, 6, 8, 10, 12, 16, 24, 32, 48, 64]
    conv = {}
    for init in ("pt", "zero"):
        for clusters in (False, True):
            imgs, lps = {}, {}
            for t in ts:
                imgs[t], lps[t] = render(sck, w.k, t, init, clusters, lplus=True)
            last = ts[-1]
            conv[f"{init}/{'clusters' if clusters else 'knn'}"] = {
                "image_change_vs_D64": {t: round(rel(imgs[t], imgs[last]), 6) for t in ts[:-1]},
                "lplus_step_change": {t: round(rel(lps[t], lps[ts[i - 1]]), 6) for i, t in enumerate(ts) if i > 0}}
    res["convergence"] = conv
    del sck, imgs, lps
    torch.cuda.empty_cache()

    log("study: 1-spp error against a 1024-spp reference")
    x0, y0 = (w.scene.width - 64) // 2, (w.scene.height - 64) // 2
    ref_cfg = dataclasses.replace(w.scene, spp=1024, crop=(x0, y0, 64, 64), seed=w.scene.seed + 1000)
    ref_paths = pg.DevicePaths(scenegen.generate(ref_cfg), device=dev)
    ref = render(ref_paths, 1, 0)
    del ref_paths
    torch.cuda.empty_cache()
    Ds = [0, 1, 2, 4, 8, 16, 64]
    mse = {"pt": []}
    for D in Ds:
        mse[f"knn_D{D}"] = []
        mse[f"clusters_D{D}"] = []
    for seed in range(4):
        cfg = dataclasses.replace(w.scene, spp=1, seed=w.scene.seed + 2000 + seed)
        s1 = scenegen.generate(cfg)
        s1 = pg.DevicePaths(dataclasses.replace(s1, cluster_key=scenegen.cluster_keys(s1.n_vertices, 100 + seed)),
                            device=dev)
        crop = lambda im: im[y0:y0 + 64, x0:x0 + 64]  # noqa: E731
        err = lambda im: float(((crop(im) - ref) ** 2).mean())  # noqa: E731
        mse["pt"].append(err(render(s1, 1, 0)))
        for D in Ds:
            mse[f"knn_D{D}"].append(err(render(s1, w.k, D)))
            mse[f"clusters_D{D}"].append(err(render(s1, w.k, D, clusters=True)))
        del s1
        torch.cuda.empty_cache()
    m = {k: float(np.mean(v)) for k, v in mse.items()}
    res["quality"] = {"mse": {k: round(v, 8) for k, v in m.items()},
                      "mse_over_pt": {k: round(v / m["pt"], 4) for k, v in m.items()},
                      "reference_mean": round(float(ref.mean()), 6), "seeds": 4,
                      "setup": f"1 spp {w.scene.width}x{w.scene.height}, error on the centred 64x64 crop, "
                               f"reference 1024 spp path tracing, k {w.k}"}
    return res


def time_batched(pg, torch, steps, tune=True):
    """64 independent scenes: one hipGraph launch of a batch plan (each
    scene's cell size and the batch's edge tile from the autotuner) vs 64
    sequential pg_render calls (library defaults).  Counts sum_s E_s D_s."""
    import scenegen
    dev = torch.device("cuda:0")
    log("generating the 64-scene batch")
    t0 = time.perf_counter()
    items = scenegen.generate_batch(64)
    log(f"batch generated in {time.perf_counter() - t0:.1f} s")
    paths = [pg.DevicePaths(sc, device=dev) for _, sc in items]
    params = [pg.params(k=w.k, D=w.D, g=w.g) for w, _ in items]
    work = sum(p.n_vertices * min(w.k, p.n_vertices) * w.D for (w, _), p in zip(items, paths))
    nverts = sum(p.n_vertices for p in paths)
    # per scene: one Renderer (workspace allocated once), launched one after another
    rends = [pg.Renderer(p, q) for p, q in zip(paths, params)]
    imgs = [torch.empty(p.height, p.width, 3, device=dev) for p in paths]

    def per_scene():
        for r, im in zip(rends, imgs):
            r(im)

    t0 = time.perf_counter()
    plan = pg.Batch(paths, params, use_graph=True, tune=tune)
    tune_s = time.perf_counter() - t0
    for f in (per_scene, plan):
        f()
    torch.cuda.synchronize()
    res = {}
    for name, f in (("per_scene", per_scene), ("batched", plan)):
        t0 = time.perf_counter()
        for _ in range(steps):
            f()
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) * 1e3 / steps
    same = all(torch.equal(a, b) for a, b in zip(imgs, plan.images))
    tuned = plan.tuned
    plan.close()
    # the opt-in persistent schedule: every iteration in one cooperative launch
    pers = pg.Batch(paths, [pg.params(k=q.k, D=q.D, g=q.g, flags=pg.PG_FLAG_PERSISTENT) for q in params],
                    use_graph=True)
    pers()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pers()
    torch.cuda.synchronize()
    pers_ms = (time.perf_counter() - t0) * 1e3 / steps
    pers_same = all(torch.equal(a, b) for a, b in zip(imgs, pers.images))
    pers.close()
    del rends, plan
    torch.cuda.empty_cache()
    return {"value": round(work / (res["batched"] / 1e3) / 1e9, 2), "unit": "Gedge-updates/s",
            "ms_batched": round(res["batched"], 3), "ms_per_scene_sequential": round(res["per_scene"], 3),
            "speedup": round(res["per_scene"] / res["batched"], 3),
            "per_scene_value": round(work / (res["per_scene"] / 1e3) / 1e9, 2), "images_equal": same,
            "persistent": {"ms_batched": round(pers_ms, 3), "images_equal": pers_same,
                           "note": "PG_FLAG_PERSISTENT: all iterations in one cooperative launch with grid barriers"},
            "autotuned": None if tuned is None else {"tile": tuned["tile"], "tile_group": tuned["tile_group"],
                                                     "cell_shift_vs_default": sum(
                                                         1 for sh, p in zip(tuned["cell_shift"], paths)
                                                         if p.n_vertices and sh != pg.pg_default_cell_shift(
                                                             p.n_vertices)),
                                                     "plan_build_s_with_tuning": round(tune_s, 2)},
            "workload": f"64 scenes, sum N = {nverts}, sum E*D = {work}, k 8-16, D 16-64 (one hipGraph launch)"}


def time_forward(pg, torch, sc, w, name, steps, warmup, schedule=0, cell_shift=0, growth=True, tile=0, tile_group=0,
                 tune=False):
    """Times `steps` pg_render calls on the workload's paths (already in HBM)
    after `warmup` untimed ones.  Returns the headline fields and the roofline
    of the dominant propagation kernel, timed with HIP events on the stream the
    library launches it on (the caller's current stream)."""
    dev = torch.device("cuda:0")
    paths = pg.DevicePaths(sc, device=dev)
    tuned = None
    if tune:   # the autotuner's cell size and edge tile (results unchanged); explicit flags win
        from paper_2404_11894_amd import autotune
        t0 = time.perf_counter()
        tuned = autotune.tune(paths, w.k, w.g)
        torch.cuda.synchronize()
        tuned["tune_s"] = round(time.perf_counter() - t0, 2)
        log(f"{name}: autotuned {tuned}")
        cell_shift = cell_shift or tuned["cell_shift"]
        tile = tile or tuned["tile"]
        tile_group = tile_group or tuned["tile_group"]
    q = pg.params(k=w.k, D=w.D, g=w.g, schedule=schedule, cell_shift=cell_shift, tile=tile, tile_group=tile_group)
    N = sc.n_vertices
    K = min(w.k, N)
    E = N * K
    render = pg.Renderer(paths, q)
    image = torch.empty(sc.height, sc.width, 3, device=dev)
    for _ in range(warmup):
        render(image)
    torch.cuda.synchronize()
    log(f"{name}: warm-up done ({warmup} steps); timing {steps} steps")
    pg._check(pg.lib().pg_profile_start())
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    marks[0].record(stream)
    for k in range(steps):
        render(image)
        marks[k + 1].record(stream)   # HIP events between steps (the render runs on this stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    step_ms = sorted(marks[k].elapsed_time(marks[k + 1]) for k in range(steps))
    median_ms = step_ms[len(step_ms) // 2] if len(step_ms) % 2 else 0.5 * (step_ms[len(step_ms) // 2 - 1] +
                                                                           step_ms[len(step_ms) // 2])
    prof = profile_entries(pg)
    ms = dt * 1e3 / steps
    value = E * w.D / (ms / 1e3) / 1e9
    log(f"{name}: {ms:.2f} ms/step, {value:.1f} Gedge-updates/s")
    phases = {k: round(v[1] / steps, 4) for k, v in prof.items()}
    prop_steps = [s for s in ("spmv", "shift", "spmv_shifted", "spmv_scatter") if s in prof]
    prop_ms = sum(prof[s][1] for s in prop_steps) / steps
    dom = max(prop_steps, key=lambda s: prof[s][1])
    cnt, tot, _ = prof[dom]
    avg_s = tot / cnt / 1e3
    starts = int((sc.path_offsets[1:] > sc.path_offsets[:-1]).sum())
    nf = torch.zeros(1, dtype=torch.int64, device=dev)
    render(image, graph={"n_far": nf})
    n_far = int(nf.item()) if dom == "spmv" and pg.resolved_schedule(q) == "two-pass" else None
    # achieved: the per-row bytes of the problem's definition (int32 id + fp32
    # weight per edge, x gather, b, albedo, y write: N (8K + 40)); the compact
    # ids move fewer, reported under own_format, and the counters under traffic
    ab = algorithmic_bytes(dom, N, K, starts)
    achieved = ab / avg_s / 1e9
    traffic = read_traffic(dom, w.name)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
            "algorithmic_bytes_per_launch": ab, "avg_launch_ms": round(avg_s * 1e3, 4),
            "traffic_GBs": round(traffic / avg_s / 1e9, 1) if traffic else None}
    if n_far is not None:
        fb = algorithmic_bytes(dom, N, K, starts, n_far)
        roof["own_format"] = {"ids": "16-bit offsets from the row, far ids from a side list", "n_far": n_far,
                              "far_fraction": round(n_far / max(1, N * (K - 1)), 4), "bytes_per_launch": fb,
                              "achieved": round(fb / avg_s / 1e9, 1),
                              "frac": round(fb / avg_s / 1e9 / HBM_PEAK_GBS, 4),
                              "note": "the bytes this kernel's layout must move: N (6K + 40) + 4 n_far + "
                                      "4 (N/64 + 1)"}
    prop_bytes = (8 * K + 68) * N * w.D
    fmt_bytes = None if n_far is None else (algorithmic_bytes("spmv", N, K, starts, n_far) + 28 * N) * w.D
    out = {
        "value": round(value, 2), "ms_per_step": round(ms, 3), "ms_per_step_median": round(median_ms, 3),
        "config": {"workload": f"{name}: {w.scene.R}^3 fBm medium, {w.scene.width}x{w.scene.height} px, "
                               f"{w.scene.spp} spp, depth {w.scene.max_depth}, k {w.k}, D {w.D}",
                   "N": N, "E": E, "P": sc.n_paths, "K": K, "D": w.D,
                   "schedule": pg.resolved_schedule(q), "cell_shift": cell_shift or pg.pg_default_cell_shift(N),
                   "tile": tile or 512, "tile_group": tile_group or 1, "autotuned": tuned},
        "propagation": {"ms_per_step": round(prop_ms, 3), "gedge_updates_per_s": round(E * w.D / prop_ms / 1e6, 2),
                        "algorithmic_GBs": round(prop_bytes / (prop_ms / 1e3) / 1e9, 1),
                        "hbm_frac": round(prop_bytes / (prop_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                        "bytes_per_iteration": "(8K + 68) N: col + weight per edge, x gather, b, albedo, y "
                                               "write; successor, y gather, x write",
                        "hbm_frac_own_format": None if fmt_bytes is None else
                        round(fmt_bytes / (prop_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
        "phases_ms": phases,
        "roofline": roof,
    }
    if growth:
        out["iteration"] = iteration_growth(pg, torch, paths, w, render.ws, render.ws_bytes)
    del render, paths
    torch.cuda.empty_cache()
    return out


def iteration_growth(pg, torch, paths, w, ws, ws_bytes):
    """Whether the timed iteration settles on this workload.  From zero,
    L+_t - L+_{t-1} = M^(t-1) c with M = S diag(albedo) W, so the ratio of
    successive-difference norms D/2 iterations apart, to the power 2/D,
    estimates the spectral radius of M: above 1 the iterates grow without
    bound (the k-nearest relation with per-receiver marginals at this g)."""
    import ctypes as C
    dev = paths.device
    N = paths.n_vertices
    s = paths.struct()

    def lplus(D):
        q = pg.params(k=w.k, D=D, g=w.g, init="zero")
        out = pg.GraphOut()
        lp = torch.empty(N, 3, device=dev)
        out.lplus = lp.data_ptr()
        img = torch.empty(paths.height, paths.width, 3, device=dev)
        pg._check(pg.lib().pg_render(C.byref(s), C.byref(q), pg._ptr(img), C.byref(out), pg._ptr(ws), ws_bytes,
                                     pg._stream(dev)))
        return lp.double()

    a, b = w.D // 2, w.D
    d0 = torch.linalg.vector_norm(lplus(a) - lplus(a - 1)).item()
    d1 = torch.linalg.vector_norm(lplus(b) - lplus(b - 1)).item()
    rate = (d1 / d0) ** (1.0 / (b - a)) if d0 > 0 else float("nan")
    return {"growth_per_iteration": round(rate, 4), "converges": bool(rate < 1.0),
            "estimate": f"(|L+_{b} - L+_{b - 1}| / |L+_{a} - L+_{a - 1}|)^(1/{b - a}) from zero: the spectral "
                        f"radius of S diag(albedo) W",
            "note": "the timed iteration count and work do not depend on it; "
                    "tests/test_convergence.py pins the radius on a crop of the mid medium"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=["tiny", "mid", "large"],
                    help="workload of the headline forward line (the other legs run on mid)")
    ap.add_argument("--schedule", type=int, default=0, help="0 default, 1 two-pass, 2 shifted, 3 scatter")
    ap.add_argument("--cell-shift", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0, help="workgroup size of the propagation kernels (0 = 512)")
    ap.add_argument("--tile-group", type=int, default=0, help="consecutive row tiles per XCD in the aggregation")
    ap.add_argument("--no-autotune", action="store_true",
                    help="library defaults instead of the autotuner's cell size and edge tile")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-clusters", action="store_true")
    ap.add_argument("--no-tracer", action="store_true")
    ap.add_argument("--no-mid", action="store_true", help="skip the mid forward line")
    ap.add_argument("--no-growth", action="store_true", help="skip the iteration-growth estimate (for profiling)")
    ap.add_argument("--only", choices=["clusters", "tracer", "adjoint", "batched"],
                    help="run only this leg (on mid) and print its JSON")
    ap.add_argument("--study", action="store_true",
                    help="convergence and 1-spp error study instead of the timing (one JSON line)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="run a 1 GiB device copy then the render steps (for rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import scenegen
    import paper_2404_11894_amd as pg

    w = scenegen.WORKLOADS[args.workload]
    if args.study:
        print(json.dumps({"study": args.workload, **study(pg, torch, w)}), flush=True)
        return
    dev = torch.device("cuda:0")
    wm = scenegen.WORKLOADS["mid"]

    def generate(wl):
        log(f"generating workload {wl.name}")
        t0 = time.perf_counter()
        sc = scenegen.generate(wl.scene)
        gen_s = time.perf_counter() - t0
        log(f"{wl.name}: N={sc.n_vertices} P={sc.n_paths} generated in {gen_s:.1f} s")
        return sc, gen_s

    if args.pmc_probe:
        a = torch.ones(256 * 1024 * 1024, device=dev)          # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("pmc probe: copied 1 GiB (1 GiB read + 1 GiB written)")
    if args.only:
        sc, gen_s = generate(wm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        paths = pg.DevicePaths(sc, device=dev)
        torch.cuda.synchronize()
        copy_s = time.perf_counter() - t0
        del paths
        if args.only == "clusters":
            leg = time_clusters(pg, torch, sc, wm, args.steps, max(1, args.warmup), float("nan"))
        elif args.only == "tracer":
            leg = time_tracer(pg, torch, wm, gen_s, copy_s)
        elif args.only == "adjoint":
            leg = time_fwd_adjoint(pg, torch, sc, wm, args.steps, max(1, args.warmup))
        else:
            torch.cuda.empty_cache()
            leg = time_batched(pg, torch, args.steps, tune=not args.no_autotune)
        print(json.dumps({"leg": args.only, **leg}), flush=True)
        return

    sc, gen_s = generate(w)
    head = time_forward(pg, torch, sc, w, args.workload, args.steps, args.warmup, args.schedule, args.cell_shift,
                        growth=not (args.pmc_probe or args.no_growth), tile=args.tile, tile_group=args.tile_group,
                        tune=not args.no_autotune)
    if args.pmc_probe:
        print(json.dumps({"pmc_probe": True, "ms_per_step": head["ms_per_step"]}))
        return
    out = {"metric": METRIC, "value": head["value"], "unit": "Gedge-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
           "ms_per_step_median": head["ms_per_step_median"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": head["config"],
           "propagation": head["propagation"], "phases_ms": head["phases_ms"], "roofline": head["roofline"],
           "iteration": head.get("iteration")}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, sc)
    del sc
    legs = not (args.no_mid and args.no_tracer and args.no_clusters and args.no_adjoint)
    if legs:
        scm, gen_m = generate(wm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pm = pg.DevicePaths(scm, device=dev)
        torch.cuda.synchronize()
        copy_m = time.perf_counter() - t0
        del pm
        torch.cuda.empty_cache()
        mid_ms = float("nan")
        if not args.no_mid and args.workload != "mid":
            m = time_forward(pg, torch, scm, wm, "mid", args.steps, args.warmup, tune=not args.no_autotune)
            mid_ms = m["ms_per_step"]
            out["mid_forward"] = {k: m[k] for k in ("value", "ms_per_step", "config", "propagation", "phases_ms",
                                                    "roofline", "iteration")}
        elif args.workload == "mid":
            mid_ms = head["ms_per_step"]
        if not args.no_tracer:
            log("timing the GPU path tracer")
            out["tracer"] = time_tracer(pg, torch, wm, gen_m, copy_m)
            log(f"tracer {out['tracer']['ms_device']} ms on the device, N = {out['tracer']['n_vertices']}")
        if not args.no_clusters:
            log("timing the cluster relation")
            out["clusters"] = time_clusters(pg, torch, scm, wm, args.steps, max(1, args.warmup), mid_ms)
            log(f"clusters {out['clusters']['ms_per_step']} ms/step, E = {out['clusters']['E']}")
        if not args.no_adjoint:
            log("timing forward + adjoint")
            out["fwd_adjoint"] = time_fwd_adjoint(pg, torch, scm, wm, max(2, args.steps // 2), 1)
            log(f"fwd+adjoint {out['fwd_adjoint']['ms_per_step']} ms/step")
            torch.cuda.empty_cache()
            alt = time_fwd_adjoint(pg, torch, scm, wm, max(2, args.steps // 4), 1, store_z=False)
            out["fwd_adjoint"]["recomputing_sums"] = {
                "ms_per_step": alt["ms_per_step"], "value": alt["value"], "reverse": alt["reverse"],
                "note": "without PG_FLAG_STORE_Z: the reverse rows gather x_(t-1) again instead of reading the "
                        "forward's stored sums (24 D N bytes less workspace)"}
            log(f"fwd+adjoint recomputing the sums {alt['ms_per_step']} ms/step")
        del scm
    if not args.no_batched:
        torch.cuda.empty_cache()
        out["batched"] = time_batched(pg, torch, max(2, args.steps // 2), tune=not args.no_autotune)
        log(f"batched {out['batched']['ms_batched']} ms vs per-scene {out['batched']['ms_per_scene_sequential']} ms")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
