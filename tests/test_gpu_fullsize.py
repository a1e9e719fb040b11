"""Parity at the full size of the bench workload (10k blobs x 2k tubes,
500^3 box, tau in {0, 5, 20}) in the configuration bench.py times (learned
LoD skip, batched FP32 tiles, guard band, chunk culling, graphs).  The
oracle checks sampled outputs one by one: random reported pairs must be
within tau, random unreported MBB candidates must not be; properties that
hold at any size (nesting in tau) are checked on the whole result."""
import os
import sys

import numpy as np
import pytest

import meshgen as mg

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def full(tmp_path_factory):
    sys.path.insert(0, ROOT)
    import torch
    import bench
    import paper_2604_19982_amd as pj
    stream = torch.cuda.current_stream()
    model, _, _ = bench.train_model(pj, mg, stream, str(tmp_path_factory.mktemp("lod")))
    R, S = mg.config_multilod(seed=1)
    ctx = pj.Context(stream=stream.cuda_stream, learned_skip=True, model_path=model)
    gR, gS = ctx.meshes(R), ctx.meshes(S)
    res = {tau: ctx.join_within(gR, gS, tau) for tau in bench.TAUS}
    return R, S, res


def test_results_nest_in_tau(full):
    _, _, res = full
    sets = {t: set(zip(v["r"].tolist(), v["s"].tolist())) for t, v in res.items()}
    assert sets[0.0] <= sets[5.0] <= sets[20.0]
    assert len(sets[0.0]) > 50 and len(sets[20.0]) > 10000


@pytest.mark.parametrize("tau", [0.0, 5.0, 20.0])
def test_sampled_pairs_match_oracle(orc, full, tau):
    R, S, res = full
    O_R, O_S = orc.OSet(R), orc.OSet(S)
    rng = np.random.default_rng(int(tau) + 7)
    got = set(zip(res[tau]["r"].tolist(), res[tau]["s"].tolist()))
    # candidate pairs by box gap (exact), to sample negatives from
    bR, _ = orc.mbbs(O_R)
    bS, _ = orc.mbbs(O_S)
    cand = []
    for c0 in range(0, R.n_objects, 2000):
        md = orc.mindist(bR[c0:c0 + 2000], bS)
        i, j = np.nonzero(md <= tau)
        cand += list(zip((i + c0).tolist(), j.tolist()))
    neg = [p for p in cand if p not in got]
    pos = sorted(got)
    sp = [pos[i] for i in rng.choice(len(pos), min(40, len(pos)), replace=False)]
    sn = [neg[i] for i in rng.choice(len(neg), min(40, len(neg)), replace=False)]
    pairs = sp + sn
    d, hit = orc.pair_distances(O_R, O_S, [p[0] for p in pairs], [p[1] for p in pairs])
    inside = hit if tau == 0.0 else d <= tau
    M = np.maximum(np.abs(bR[[p[0] for p in pairs]]).max(1), np.abs(bS[[p[1] for p in pairs]]).max(1))
    # no near ties in the sample (a pair that meets is decided by the exact test, not by d)
    assert not np.any(~hit.astype(bool) & (np.abs(d - tau) <= 1e-12 * np.maximum(M, tau)))
    assert np.all(inside[:len(sp)]), [pairs[k] for k in np.nonzero(~inside[:len(sp)])[0]]
    assert not np.any(inside[len(sp):]), [pairs[len(sp) + k] for k in np.nonzero(inside[len(sp):])[0]]


# ---------------------------------------------------------------------------
# The learned-skip workload (100k blobs x 20k tubes, 5000^3, tau = 10) in the
# bench configuration: the oracle decides every MBB candidate, so the whole
# result set is compared.
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def learned_full(tmp_path_factory):
    sys.path.insert(0, ROOT)
    import torch
    import bench
    import paper_2604_19982_amd as pj
    stream = torch.cuda.current_stream()
    work = str(tmp_path_factory.mktemp("lod_learned"))
    model, _, _ = bench.train_model(pj, mg, stream, work)
    R, S = mg.config_learned()
    ctx = pj.Context(stream=stream.cuda_stream, learned_skip=True, model_path=model, autotune=True,
                     autotune_path=os.path.join(work, "shapes.txt"))
    gR, gS = ctx.meshes(R), ctx.meshes(S)
    res = ctx.join_within(gR, gS, 10.0)
    return R, S, res


def test_learned_workload_full_parity(orc, learned_full):
    """Every MBB candidate (box gap <= 10, found by an x sweep over the
    oracle's boxes) is decided by the oracle's exact distance."""
    import bench
    R, S, res = learned_full
    tau = 10.0
    O_R, O_S = orc.OSet(R), orc.OSet(S)
    cr, cs = bench.sample_candidates(orc, O_R, O_S, tau, max_r=R.n_objects)
    assert len(cr) > 1000
    d, hit = orc.pair_distances(O_R, O_S, cr, cs)
    bR, _ = orc.mbbs(O_R)
    bS, _ = orc.mbbs(O_S)
    M = orc.pair_scale(bR[cr], bS[cs])
    assert not np.any(~hit & (np.abs(d - tau) <= 1e-12 * np.maximum(M, tau)))  # no near ties
    keep = d <= tau
    want = sorted(zip(cr[keep].tolist(), cs[keep].tolist()))
    got = list(zip(res["r"].tolist(), res["s"].tolist()))
    assert got == want


# ---------------------------------------------------------------------------
# The k-NN workload (k = 3, 20k x 20k clustered blob/tube mix): sampled
# queries against the oracle's exact k-NN of the same r.
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def knn_full(tmp_path_factory):
    import torch
    import paper_2604_19982_amd as pj
    stream = torch.cuda.current_stream()
    work = str(tmp_path_factory.mktemp("knn_full"))
    R, S = mg.config_knn()
    ctx = pj.Context(stream=stream.cuda_stream, autotune=True, autotune_path=os.path.join(work, "shapes.txt"))
    res = ctx.join_knn(ctx.meshes(R), ctx.meshes(S), 3)
    return R, S, res


def test_knn_workload_sampled_parity(orc, knn_full):
    R, S, res = knn_full
    rs = np.sort(np.random.default_rng(11).choice(R.n_objects, 24, replace=False))
    O_R, O_S = orc.OSet(R), orc.OSet(S)
    ref = orc.join_knn(O_R, O_S, 3, r_subset=rs)
    assert ref["near_ties"] == 0
    bR, _ = orc.mbbs(O_R)
    bS, _ = orc.mbbs(O_S)
    M = float(max(np.abs(bR).max(), np.abs(bS).max()))
    assert np.all(res["count"] == 3)
    for r in rs:
        assert res["s"][r].tolist() == ref["s"][int(r)].tolist(), r
        d, e = res["dist"][r], ref["d"][int(r)]
        assert np.all(np.abs(d - e) <= np.maximum(1e-5 * e, 1e-12 * M)), (r, d, e)
