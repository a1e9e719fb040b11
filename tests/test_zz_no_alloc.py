"""The allocation-free LoD-bounds entry point against the allocating one:
two calls in a row on the same device (the second with fewer pairs, so its
scratch still holds the first call's contents), each compared bit for bit
with pj_pair_bounds on the same inputs.  Both reduce exact minima over the
same facet pairs, so their FP32 bounds are identical."""
import numpy as np
import pytest

import meshgen as mg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sets():
    import paper_2604_19982_amd as pj
    R, S = mg.config_multilod(seed=21, n_r=300, n_s=60, box=120.0)
    ctx = pj.Context()
    gR, gS = ctx.meshes(R), ctx.meshes(S)
    box_r, _ = gR.boxes()
    box_s, _ = gS.boxes()
    g = np.maximum(0.0, np.maximum(box_s[None, :, :3] - box_r[:, None, 3:], box_r[:, None, :3] - box_s[None, :, 3:]))
    r, s = np.nonzero(np.sqrt((g * g).sum(-1)) <= 8.0)
    return ctx, gR, gS, r.astype(np.int32), s.astype(np.int32)


@pytest.mark.parametrize("lod", [0, 2, 3])
def test_noalloc_matches_pair_bounds_twice(sets, lod):
    ctx, gR, gS, r, s = sets
    assert len(r) > 200
    first = slice(0, min(len(r), 600))
    second = slice(7, 7 + min(len(r) - 7, 150))
    for sl in (first, second):
        ref = ctx.pair_bounds(gR, gS, r[sl], s[sl], lod)
        got = ctx.pair_bounds(gR, gS, r[sl], s[sl], lod, noalloc=True)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
        assert np.all(np.isfinite(got[0])) and np.all(got[0] <= got[1])


def test_noalloc_limits(sets):
    import paper_2604_19982_amd as pj
    ctx, gR, gS, r, s = sets
    big = np.zeros(4097, np.int32)
    with pytest.raises(pj.PJError) as e:
        ctx.pair_bounds(gR, gS, big, big, 0, noalloc=True)
    assert e.value.status == 1
    c64 = pj.Context(precision="fp64")
    with pytest.raises(pj.PJError) as e:
        c64.pair_bounds(gR, gS, r[:4], s[:4], 0, noalloc=True)
    assert e.value.status == 4
    # an empty call is valid and touches nothing
    assert len(ctx.pair_bounds(gR, gS, r[:0], s[:0], 0, noalloc=True)[0]) == 0
