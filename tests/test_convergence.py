"""Convergence of the propagation on the benchmark's medium (paper, Sec.
"Rendering System": the iteration settles in fewer than ten rounds; Fig.
PG-iterations).

One iteration maps L+ to M L+ + c with M = S diag(albedo) W (eqs. ag-mf,
rte-pg, rte-mff), so it converges for every start exactly when the spectral
radius of M is below 1.  On a crop of the 128^3 fBm ball (g = g_s = 0.8,
k = 16) the k-nearest relation with per-receiver marginals gives a radius
above 1: samples shared by many receivers collect a total weight above 1, and
the iteration grows.  The paper's cluster relation, in which every receiver
of a cluster is also one of its techniques, keeps every sample's total weight
at 1 and the radius below 1.  The radius comes from ARPACK on the oracle's
sparse operator and is confirmed by the growth of the oracle's own iterates.
"""
from dataclasses import replace

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as sla

import oracle
import scenegen

MID = scenegen.WORKLOADS["mid"]


@pytest.fixture(scope="module")
def crop():
    sc = scenegen.generate(scenegen.crop_of(MID.scene, 16, 16, 4))
    return replace(sc, cluster_key=scenegen.cluster_keys(sc.n_vertices, 7))


def operator(sc, tr):
    N = sc.n_vertices
    off = sc.path_offsets
    last = np.zeros(N, bool)
    last[off[1:][np.diff(off) > 0] - 1] = True
    v = np.flatnonzero(~last)
    S = sp.csr_matrix((np.ones(len(v)), (v, v + 1)), shape=(N, N))
    W = sp.csr_matrix((tr["w_ind"].ravel(), tr["col"].ravel(), tr["row_ptr"]), shape=(N, N))
    return S @ sp.diags(sc.albedo.astype(np.float64)) @ W


def radius(M):
    ev = sla.eigs(M, k=4, which="LM", return_eigenvectors=False, tol=1e-10, maxiter=20000)
    return float(np.abs(ev).max())


@pytest.mark.parametrize("neigh", ["knn", "clusters"])
def test_spectral_radius_on_the_ball(crop, neigh):
    p = oracle.params(k=MID.k, D=1, g=MID.g, neighbours=neigh)
    _, tr = oracle.render(crop, p, trace=True)
    rho = radius(operator(crop, tr))
    print(f"{neigh}: N = {crop.n_vertices}, spectral radius {rho:.4f}")
    if neigh == "knn":
        assert rho > 1.1
    else:
        assert 0.9 < rho < 1.0
    # the oracle's iterates from zero grow (or settle) at that rate: with D
    # iterations L+_D = sum_{t<D} M^t c, so successive differences scale by rho
    Ds = (40, 60)
    diffs = []
    for D in Ds:
        a = oracle.render(crop, oracle.params(k=MID.k, D=D, g=MID.g, init="zero", neighbours=neigh), trace=True)[1]
        b = oracle.render(crop, oracle.params(k=MID.k, D=D + 1, g=MID.g, init="zero", neighbours=neigh),
                          trace=True)[1]
        diffs.append(np.linalg.norm(b["lplus"] - a["lplus"]))
    rate = (diffs[1] / diffs[0]) ** (1.0 / (Ds[1] - Ds[0]))
    assert abs(rate - rho) < 0.02 * rho, (rate, rho)


def test_knn_radius_falls_below_one_for_weaker_forward_scattering(crop):
    # the same paths at g = g_s = 0.5: the hubs' excess weight shrinks with the
    # phase function's peak and the k-nearest iteration converges again
    p = oracle.params(k=MID.k, D=1, g=0.5, g_s=0.5)
    _, tr = oracle.render(crop, p, trace=True)
    assert radius(operator(crop, tr)) < 1.0
