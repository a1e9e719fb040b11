"""GPU: voxel-pair filtering (Section 3.2, Algorithms 1-3) in front of the
LoD rounds.  Voxels (k-means over the coarsest facets, consistent across
LoDs) only remove facet pairs that cannot decide a pair, so every join with
voxels on must return exactly what the oracle and the join without voxels
return: the same pairs, k-NN lists and FP64 distances."""
import numpy as np
import pytest

import meshgen as mg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pj():
    import paper_2604_19982_amd as pj
    return pj


@pytest.fixture(scope="module")
def mid():
    return mg.config_multilod(seed=31, n_r=400, n_s=80, box=150.0, n_seg=1280)


@pytest.fixture(scope="module")
def plain_ref(pj, mid):
    R, S = mid
    c = pj.Context(want_dist=True)
    gR, gS = c.meshes(R), c.meshes(S)
    return {tau: c.join_within(gR, gS, tau) for tau in (0.0, 5.0, 20.0)}


def _same(a, b):
    assert np.array_equal(a["r"], b["r"]) and np.array_equal(a["s"], b["s"])
    if a.get("dist") is not None and b.get("dist") is not None:
        assert np.array_equal(a["dist"], b["dist"])


@pytest.mark.parametrize("tau", [0.0, 5.0, 20.0])
def test_voxel_within_matches_plain_and_prunes(pj, mid, plain_ref, tau):
    R, S = mid
    c = pj.Context(voxels=True, want_dist=True)
    gR, gS = c.meshes(R), c.meshes(S)
    got = c.join_within(gR, gS, tau)
    st = c.stats()
    _same(got, plain_ref[tau])
    assert st["vp_pairs"] > 0 and 0 < st["vp_kept"] < st["vp_pairs"]
    assert st["vp_chunks"] >= 1


def test_voxel_within_vs_oracle_small(orc, pj):
    R, S = mg.config_multilod(seed=32, n_r=60, n_s=12, box=60.0, n_seg=256)
    c = pj.Context(voxels=True)
    gR, gS = c.meshes(R), c.meshes(S)
    O_R, O_S = orc.OSet(R), orc.OSet(S)
    for tau in (0.0, 3.0, 10.0):
        ref = orc.join_within(O_R, O_S, tau)
        assert ref["near_ties"] == 0
        got = c.join_within(gR, gS, tau)
        assert np.array_equal(got["r"], ref["r"]) and np.array_equal(got["s"], ref["s"]), tau


def test_voxel_filter_chunks_under_a_cap(pj, mid, plain_ref):
    """A small cap cuts the voxel filter into many chunks (Algorithm 3's
    double-buffered pipeline); results do not change."""
    R, S = mid
    c = pj.Context(voxels=True, mem_cap_bytes=12 << 20, want_dist=True)
    gR, gS = c.meshes(R), c.meshes(S)
    got = c.join_within(gR, gS, 20.0)
    st = c.stats()
    _same(got, plain_ref[20.0])
    assert st["vp_chunks"] > 2


@pytest.mark.parametrize("cap", [0, 6 << 20])
def test_voxel_host_resident(pj, mid, plain_ref, cap):
    R, S = mid
    c = pj.Context(voxels=True, host_resident=True, mem_cap_bytes=cap, stage_sets=3)
    gR, gS = c.meshes(R), c.meshes(S)
    for tau in (0.0, 20.0):
        got = c.join_within(gR, gS, tau)
        assert np.array_equal(got["r"], plain_ref[tau]["r"]) and np.array_equal(got["s"], plain_ref[tau]["s"])
        assert c.stats()["staged_bytes"] > 0


def test_voxel_knn_matches_plain(orc, pj):
    R, S = mg.config_knn(seed=33, n_r=80, n_s=80, n_clusters=3, box=300.0, sigma=15.0, f_median=2000)
    a = pj.Context()
    b = pj.Context(voxels=True)
    x = a.join_knn(a.meshes(R), a.meshes(S), 3)
    y = b.join_knn(b.meshes(R), b.meshes(S), 3)
    st = b.stats()
    assert np.array_equal(x["s"], y["s"]) and np.array_equal(x["dist"], y["dist"])
    assert st["vp_pairs"] > 0 and st["vp_kept"] < st["vp_pairs"]
    rs = np.arange(0, 80, 8)
    ref = orc.join_knn(orc.OSet(R), orc.OSet(S), 3, r_subset=rs)
    assert ref["near_ties"] == 0
    for r in rs:
        assert y["s"][r].tolist() == ref["s"][int(r)].tolist()


def test_voxel_orphan_facets_and_single_lod(orc, pj):
    """A coarse facet with no finest descendant (the hd case of Eq. (1)),
    device- and host-resident, and single-LoD sets (k-means on the only
    LoD)."""
    from test_gpu_parity import _orphan_sets
    R, S = _orphan_sets()
    O_R, O_S = orc.OSet(R), orc.OSet(S)
    for host in (False, True):
        c = pj.Context(voxels=True, host_resident=host)
        gR, gS = c.meshes(R), c.meshes(S)
        for tau in (0.0, 1.0, 4.6, 4.8):
            got = c.join_within(gR, gS, tau)
            ref = orc.join_within(O_R, O_S, tau)
            assert np.array_equal(got["r"], ref["r"]) and np.array_equal(got["s"], ref["s"]), (host, tau)
    R1, S1 = mg.config_small(seed=34, n_r=40, n_s=40, box=8.0)
    c = pj.Context(voxels=True)
    got = c.join_within(c.meshes(R1), c.meshes(S1), 0.5)
    ref = orc.join_within(orc.OSet(R1), orc.OSet(S1), 0.5)
    assert np.array_equal(got["r"], ref["r"]) and np.array_equal(got["s"], ref["s"])
