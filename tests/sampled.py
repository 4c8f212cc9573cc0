"""Propagated radiance at a few sampled vertices, computed one vertex at a time
by the oracle, for graphs too large for the oracle's whole render.

With PG_INIT_PT the starting value L+_0(v) is the path tracer's own estimate
of the indirect radiance arriving at v along its continuation (paper, Sec.
"Rendering System", path graph solver): walking v's path suffix backward from
its last vertex (where it is 0), L+_0(v) = e_u + albedo_u (d_pt_u + r_u L+_0(u))
with u the successor of v, d_pt_u the vertex's own direct estimate and r_u its
phase-to-pdf ratio.  One iteration (eqs. ag-mf, rte-pg, rte-mff) sets
y_t(u) = b_u + albedo_u sum_j w_uj L+_{t-1}(j) and L+_t(v) = y_t(succ v), 0 at
a path's last vertex.  Every d_pt, r, b and w here comes from the oracle's
per-receiver routines (oracle.knn and oracle.edges on the rows needed), so the
values test the GPU's weighted gather with non-zero input at any graph size.
"""
import numpy as np

import oracle


def last_vertices(scene) -> np.ndarray:
    """Boolean [N]: v is the last vertex of its path."""
    off = scene.path_offsets
    last = np.zeros(scene.n_vertices, bool)
    last[off[1:][np.diff(off) > 0] - 1] = True
    return last


def _path_end(scene, v):
    """One past the last vertex of v's path, for each v."""
    off = scene.path_offsets
    p = np.searchsorted(off, v, side="right") - 1
    return off[p + 1]


def own_terms(scene, p, rows):
    """(d_pt [n,3], r [n]) of the vertices ``rows``: neither depends on the
    neighbour list, so the oracle is asked with the vertex as its only neighbour."""
    rows = np.asarray(rows, np.int64)
    if rows.size == 0:
        return np.zeros((0, 3)), np.zeros(0)
    e = oracle.edges(scene, p, rows[:, None].astype(np.int32), rows=rows)
    return e["d_pt"], e["r"]


def pt_init(scene, p, verts) -> np.ndarray:
    """L+_0 [n,3] at ``verts`` with the path-traced start."""
    verts = np.asarray(verts, np.int64)
    end = _path_end(scene, verts)
    suffix = np.unique(np.concatenate([np.arange(v + 1, e) for v, e in zip(verts, end)] + [np.zeros(0, np.int64)]))
    d_pt, r = own_terms(scene, p, suffix)
    at = {int(u): i for i, u in enumerate(suffix)}
    alb = scene.albedo.astype(np.float64)
    emit = None if scene.l_emit is None else scene.l_emit.astype(np.float64)
    out = np.zeros((len(verts), 3))
    for n, (v, e) in enumerate(zip(verts, end)):
        x = np.zeros(3)
        for u in range(int(e) - 1, int(v), -1):     # u = e-1 .. v+1, so x ends as L+_0(u-1)
            i = at[u]
            x = alb[u] * (d_pt[i] + r[i] * x)
            if emit is not None:
                x = x + emit[u]
        out[n] = x
    return out


def lplus(scene, p, verts, D: int) -> np.ndarray:
    """L+_D [n,3] at ``verts`` after D iterations from the path-traced start
    (the k nearest neighbours of p["k"], weights of p's g and g_s)."""
    verts = np.asarray(verts, np.int64)
    if D == 0:
        return pt_init(scene, p, verts)
    last = last_vertices(scene)
    out = np.zeros((len(verts), 3))
    inner = np.flatnonzero(~last[verts])
    if inner.size == 0:
        return out
    u = verts[inner] + 1
    K = min(int(p["k"]), scene.n_vertices)
    col = oracle.knn(scene.pos, K, rows=u)
    e = oracle.edges(scene, p, col, rows=u)
    js = np.unique(col)
    prev = lplus(scene, p, js, D - 1)
    at = np.searchsorted(js, col)
    z = np.einsum("nk,nkc->nc", e["w_ind"], prev[at])
    alb = scene.albedo[u].astype(np.float64)[:, None]
    out[inner] = alb * e["d_agg"] + alb * z
    if scene.l_emit is not None:
        out[inner] += scene.l_emit[u].astype(np.float64)
    return out
