"""GPU tests of the LoD-skip network: forward/backward kernels against the
FP64 CPU reference (BF16 weights, FP32 accumulation), and training on the
join's own resolution logs with a held-out comparison against the plain
progressive schedule (same result set, fewer items and less work)."""
import os

import numpy as np
import pytest

import meshgen as mg

pytestmark = pytest.mark.gpu

SHAPES = [(16, 64), (64,), (64, 64), (64,), (64, 4), (4,)]


@pytest.fixture(scope="module")
def pj():
    import paper_2604_19982_amd as pj
    return pj


def bf16(a):
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def test_mlp_forward_backward_vs_oracle(orc, pj):
    rng = np.random.default_rng(0)
    flat = np.concatenate([rng.normal(scale=0.3, size=s).ravel() for s in SHAPES]).astype(np.float32)
    x = rng.normal(size=(300, 16)).astype(np.float32)
    y = rng.integers(0, 4, size=300).astype(np.int32)
    c = pj.Context()
    logits, loss, grads = c.mlp_eval(flat, x, y)
    # reference: FP64 with the BF16-rounded weights the kernels use
    wq = bf16(flat).astype(np.float64)
    P, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        P.append(wq[o:o + n].reshape(s))
        o += n
    ref_logits, _ = orc.mlp_forward(P, x.astype(np.float64))
    ref_loss, ref_grads = orc.mlp_loss_grad(P, x.astype(np.float64), y)
    assert np.allclose(logits, ref_logits, rtol=1e-4, atol=1e-4)
    assert abs(loss - ref_loss) <= 1e-5 * max(1.0, ref_loss)
    g = np.concatenate([r.ravel() for r in ref_grads])
    assert np.all(np.abs(grads - g) <= 1e-4 * np.abs(g).max() + 1e-6), np.max(np.abs(grads - g))


def test_mlp_forward_hand_values_gpu(pj):
    """The forward kernel on the hand-built network of the oracle's pin: every
    weight and input is a small dyadic number, so the BF16 weights and FP32
    sums are exact and the logits must equal the hand values."""
    import test_oracle_mlp as hand
    flat = np.concatenate([p.ravel() for p in hand.hand_net()]).astype(np.float32)
    assert np.array_equal(bf16(flat), flat)
    logits, _, _ = pj.Context().mlp_eval(flat, hand.HAND_X.astype(np.float32))
    assert np.array_equal(logits.astype(np.float64), hand.hand_logits(hand.HAND_X)), logits


@pytest.fixture(scope="module")
def trained(tmp_path_factory, pj):
    """The LoD model trained on resolution logs of a held-out multi-LoD
    workload (seed 101, 10k x 2k in 500^3, tau in {0, 2, 5, 10, 20}) written
    by joins with voxel-pair filtering, as the bench trains it; plus k-NN
    logs of a held-out clustered set."""
    d = tmp_path_factory.mktemp("lod")
    log = str(d / "res.log")
    R, S = mg.config_multilod(seed=101, n_r=10000, n_s=2000, box=500.0)
    c = pj.Context(log_path=log, voxels=True)
    gR, gS = c.meshes(R), c.meshes(S)
    for tau in (0.0, 2.0, 5.0, 10.0, 20.0):
        c.join_within(gR, gS, tau)
    KR, KS = mg.config_knn(seed=102, n_r=300, n_s=300, n_clusters=4, box=600.0, sigma=25.0, f_median=1500)
    c.join_knn(c.meshes(KR), c.meshes(KS), 3)
    n_rec = os.path.getsize(log) // 72
    model = str(d / "lod.model")
    loss = c.train_lod_model(log, model, epochs=40, batch=512, lr=3e-3, seed=1)
    return dict(model=model, loss=loss, n_rec=n_rec)


def test_training_reduces_loss(trained):
    assert trained["n_rec"] > 3000
    assert trained["loss"] < 0.9 * np.log(4.0)


@pytest.fixture(scope="module")
def held_out(pj):
    return mg.config_multilod(seed=13, n_r=2000, n_s=400, box=300.0)


@pytest.mark.parametrize("tau", [0.0, 10.0, 20.0])
def test_learned_skip_same_results_less_work(pj, trained, held_out, tau):
    """What the trained network gains over the plain progressive order, on
    held-out inputs, with a measure that depends only on the schedule's
    decisions (not on tile order or timing): the (pair, LoD) items visited
    fall by at least 10%, and the sum over them of sqrt(n_r * n_s) (the
    work the network's choice minimises; with box culling the evaluated
    facet pairs grow like it) falls strictly.  The result sets are equal."""
    R, S = held_out
    base = pj.Context(voxels=True)
    gR, gS = base.meshes(R), base.meshes(S)
    ref = base.join_within(gR, gS, tau)
    st0 = base.stats()
    lc = pj.Context(voxels=True, learned_skip=True, model_path=trained["model"])
    got = lc.join_within(gR, gS, tau)
    st1 = lc.stats()
    assert np.array_equal(got["r"], ref["r"]) and np.array_equal(got["s"], ref["s"])
    i0, i1 = sum(st0["lod_items"]), sum(st1["lod_items"])
    print(f"tau={tau}: plain progressive items {st0['lod_items'][:4]} sqrt-work {st0['planned_sqrt']:.4e} "
          f"evaluated {st0['facet_pairs']:.3e}; learned items {st1['lod_items'][:4]} sqrt-work "
          f"{st1['planned_sqrt']:.4e} evaluated {st1['facet_pairs']:.3e}")
    assert i0 > 0
    assert i1 <= 0.9 * i0
    assert st1["planned_sqrt"] < st0["planned_sqrt"]


def test_learned_skip_knn_same_results(pj, trained):
    """The learned first LoD in the k-NN join (threshold feature: the
    query's theta_r) never changes the lists or distances."""
    R, S = mg.config_knn(seed=103, n_r=300, n_s=300, n_clusters=4, box=600.0, sigma=25.0, f_median=1500)
    base = pj.Context(voxels=True)
    gR, gS = base.meshes(R), base.meshes(S)
    ref = base.join_knn(gR, gS, 3)
    st0 = base.stats()
    lc = pj.Context(voxels=True, learned_skip=True, model_path=trained["model"])
    got = lc.join_knn(gR, gS, 3)
    st1 = lc.stats()
    assert np.array_equal(got["s"], ref["s"]) and np.array_equal(got["dist"], ref["dist"])
    print(f"k-NN: plain items {st0['lod_items'][:4]} sqrt-work {st0['planned_sqrt']:.4e}; learned items "
          f"{st1['lod_items'][:4]} sqrt-work {st1['planned_sqrt']:.4e}")


def test_missing_model_falls_back(pj):
    c = pj.Context(learned_skip=True, model_path="/nonexistent/lod.model")
    R, S = mg.config_small(seed=0, n_r=10, n_s=10, box=4.0)
    assert isinstance(c.join_within(c.meshes(R), c.meshes(S), 0.5)["r"], np.ndarray)
