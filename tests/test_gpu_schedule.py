"""Results do not depend on the launch schedule of the FP32 rounds.

The persistent refinement kernel takes tiles from an atomic counter, lets
waves claim a tile's A blocks one at a time and, once the tile list is used
up, lets every wave join the tiles still in progress.  Which wave evaluates
which facet pairs, and in which order the per-item minima arrive, therefore
changes from run to run and with the launch shape; the per-item minima
(exact minima of the FP32 estimates) and everything decided from them must
not.  Shapes range from one wave per CU with 64-facet B ranges (every tile
has many claimable blocks and most of the work is done by joining waves) to
sixteen waves per CU with 65536-facet ranges."""
import numpy as np
import pytest

import meshgen as mg

pytestmark = pytest.mark.gpu

SHAPES = [(64, 1), (256, 2), (1024, 8), (65536, 16)]


@pytest.fixture(scope="module")
def pj():
    import paper_2604_19982_amd as pj
    return pj


@pytest.fixture(scope="module")
def mid():
    return mg.config_multilod(seed=1, n_r=400, n_s=80, box=150.0, n_seg=1280)


@pytest.mark.parametrize("tau", [0.0, 5.0, 20.0])
def test_within_same_for_every_shape(orc, pj, mid, tau):
    R, S = mid
    outs = []
    for ts, wpc in SHAPES:
        c = pj.Context(tile_s=ts, waves_per_cu=wpc, want_dist=True)
        got = c.join_within(c.meshes(R), c.meshes(S), tau)
        st = c.stats()
        assert (st["tile_s_used"], st["waves_per_cu_used"]) == (ts, wpc)
        outs.append(got)
    for got in outs[1:]:
        assert np.array_equal(got["r"], outs[0]["r"]) and np.array_equal(got["s"], outs[0]["s"])
        # FP64 distances of the result pairs come from the exact recheck
        assert np.array_equal(got["dist"], outs[0]["dist"])
    if tau == 5.0:
        ref = orc.join_within(orc.OSet(R), orc.OSet(S), tau)
        assert np.array_equal(outs[0]["r"], ref["r"]) and np.array_equal(outs[0]["s"], ref["s"])


def test_knn_same_for_every_shape(pj):
    R, S = mg.config_knn(seed=3, n_r=60, n_s=60, n_clusters=3, box=200.0, sigma=12.0, f_median=2000)
    outs = []
    for ts, wpc in SHAPES:
        c = pj.Context(tile_s=ts, waves_per_cu=wpc)
        outs.append(c.join_knn(c.meshes(R), c.meshes(S), 3))
    for got in outs[1:]:
        assert np.array_equal(got["count"], outs[0]["count"]) and np.array_equal(got["s"], outs[0]["s"])
        assert np.array_equal(got["dist"], outs[0]["dist"])


def test_repeated_runs_same_results(pj, mid):
    """The same context and shape, several times: the dynamic order differs,
    the results do not."""
    R, S = mid
    c = pj.Context(tile_s=256, waves_per_cu=2)
    gR, gS = c.meshes(R), c.meshes(S)
    first = c.join_within(gR, gS, 20.0)
    for _ in range(3):
        again = c.join_within(gR, gS, 20.0)
        assert np.array_equal(again["r"], first["r"]) and np.array_equal(again["s"], first["s"])
