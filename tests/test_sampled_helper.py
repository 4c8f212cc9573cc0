"""The sampled-vertex propagation used by the full-size GPU tests agrees with
the oracle's whole render on the small workload: the path-traced start, and
one, two and three iterations, with and without volume emission."""
import numpy as np
import pytest

import oracle
from tests import sampled
from tests.gpu_util import crop


@pytest.fixture(scope="module", params=[None, (2.0, 1.5, 1.0)], ids=["plain", "emissive"])
def scene(request):
    return crop("tiny", 24, 24, 2, emit_L=request.param)


@pytest.mark.parametrize("D", [0, 1, 2, 3])
def test_sampled_lplus_matches_whole_render(scene, D):
    p = oracle.params(k=8, D=D, g=0.5)
    _, tr = oracle.render(scene, p, trace=True)
    rng = np.random.default_rng(40 + D)
    v = np.sort(rng.choice(scene.n_vertices, 40, replace=False))
    v = np.union1d(v, np.flatnonzero(sampled.last_vertices(scene))[:3])   # some path ends too
    want = tr["lplus0"][v] if D == 0 else tr["lplus"][v]
    got = sampled.lplus(scene, p, v, D)
    assert np.abs(want).max() > 0
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-14)
