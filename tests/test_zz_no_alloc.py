"""pg_propagate_static, the variant of pg_propagate that allocates nothing
(its workspace is the library's static device scratch), against
pg_propagate on the same graphs: L+_D and the whole trajectory bit for bit,
on two calls in a row, the second on a smaller graph, so the scratch holds
the first call's contents when the second starts."""
import numpy as np
import pytest
import torch

import paper_2404_11894_amd as pg
from tests.gpu_util import crop

pytestmark = pytest.mark.gpu


def graph(sc, k, D, g):
    paths = pg.DevicePaths(sc)
    q = pg.params(k=k, D=D, g=g, flags=pg.PG_FLAG_CHECK)
    row_ptr, col = pg.pg_knn(paths, k)
    e = pg.pg_edges(paths, q, row_ptr, col)
    return paths, q, row_ptr, col, e


def test_static_propagate_matches_propagate_on_two_calls():
    cases = [(crop("tiny", 64, 64, 4), 8, 8, 0.5), (crop("tiny", 24, 16, 2), 5, 6, 0.3)]
    assert cases[1][0].n_vertices < cases[0][0].n_vertices
    for sc, k, D, g in cases:
        print(f"static propagate: N={sc.n_vertices} k={k} D={D}", flush=True)
        paths, q, rp, col, e = graph(sc, k, D, g)
        ref = e["lplus0"].clone()
        ref, ref_traj = pg.pg_propagate(paths, q, rp, col, e["w_ind"], e["b"], ref, traj=True)
        got = e["lplus0"].clone()
        traj = torch.full((D, sc.n_vertices, 3), float("nan"), device=got.device)
        pg.pg_propagate_static(paths, q, rp, col, e["w_ind"], e["b"], got, traj)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        assert torch.equal(traj, ref_traj)
        assert np.abs(got.cpu().numpy()).max() > 0
