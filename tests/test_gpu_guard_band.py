"""The FP32 guard band at scale: over 1e8 facet pairs (random, adversarial
and facet pairs of the workload meshes) the FP32 lower and upper facet
distance estimates bracket the FP64 distance to within eps/8, eps = 2^-16 x
the pair's half-extent about its float centre, an FP32 "sure" crossing is
always a real meet, and few pairs are left open (lower < upper) for the FP64
recheck.

The FP64 reference here is the library's FP64 facet-pair path, which
tests/test_gpu_parity.py pins to the CPU oracle (exact predicates) on random,
adversarial and integer-grid pairs; a 200k subset is also checked against the
oracle directly."""
import numpy as np
import pytest

import meshgen as mg

pytestmark = pytest.mark.gpu

BLOCK = 1 << 22
BLOCKS = 24


@pytest.fixture(scope="module")
def ctx():
    import paper_2604_19982_amd as pj
    return pj.Context(device=0)


def _eps(T1, T2):
    P = np.concatenate([T1, T2], 1)
    lo, hi = P.min(1), P.max(1)
    o = (0.5 * (lo + hi)).astype(np.float32)
    M = np.maximum(hi - o, o - lo).max(1)
    return np.ldexp(M.astype(np.float64), -16)


def _unit(x):
    return x / np.linalg.norm(x, axis=-1, keepdims=True)


def _block(rng, n):
    """Random and adversarial triangle pairs, vectorised (float32 [n, 3, 3])."""
    k = rng.integers(0, 7, size=n)
    g = lambda *shape: rng.standard_normal(size=shape, dtype=np.float32)  # noqa: E731
    T1 = g(n, 3, 3)
    T2 = g(n, 3, 3)
    c = T1.mean(1)
    nrm = _unit(np.cross(T1[:, 1] - T1[:, 0], T1[:, 2] - T1[:, 0]))
    # 0: independent random pairs at a random offset
    m = k == 0
    T2[m] += g(m.sum(), 1, 3) * 2.0
    # 1: nearly parallel copies with a tiny offset
    m = k == 1
    T2[m] = T1[m] + g(m.sum(), 1, 3) * 1e-3 + \
        nrm[m][:, None, :] * rng.uniform(-1e-2, 1e-2, size=(m.sum(), 1, 1)).astype(np.float32)
    # 2: thin (tube-like) facets close to each other
    m = k == 2
    a = g(m.sum(), 3)
    u = g(m.sum(), 3)
    T1[m] = np.stack([a, a + u, a + 0.02 * g(m.sum(), 3)], 1)
    T2[m] = T1[m] + g(m.sum(), 1, 3) * 0.05
    # 3: a segment through the interior (crossing)
    m = k == 3
    T2[m] = np.stack([c[m] - 0.5 * nrm[m], c[m] + 0.5 * nrm[m], c[m] + g(m.sum(), 3)], 1)
    # 4: a vertex pushed onto the face
    m = k == 4
    T2[m] = np.stack([c[m], c[m] + g(m.sum(), 3), c[m] + g(m.sum(), 3)], 1)
    # 5: edge-edge near misses
    m = k == 5
    T2[m] = g(m.sum(), 3, 3) * 0.5 + c[m][:, None, :]
    # 6: small pairs far from the origin (coordinates carry large offsets)
    m = k == 6
    off = rng.uniform(-2e4, 2e4, size=(m.sum(), 1, 3)).astype(np.float32)
    T1[m] = T1[m] * 0.3 + off
    T2[m] = T2[m] * 0.3 + off + g(m.sum(), 1, 3) * 0.5
    # scale spread
    s = (10.0 ** rng.uniform(-2, 2, size=(n, 1, 1))).astype(np.float32)
    s[k == 6] = 1.0
    return T1 * s, T2 * s


def _mesh_pairs(rng, n_want):
    """Facet pairs of nearby blob/tube objects (finest LoD): for sampled
    facets of a blob, the tube facets with the nearest centroids."""
    R, S = mg.config_multilod(seed=7, n_r=150, n_s=30, box=40.0, n_seg=1280)
    L = R.n_lods
    out1, out2 = [], []
    have = 0
    for r in range(R.n_objects):
        if have >= n_want:
            break
        vr = R.verts[R.vert_begin[r]:R.vert_begin[r] + R.vert_count[r]]
        tr = R.tris[R.tri_begin[r * L + L - 1]:R.tri_begin[r * L + L - 1] + R.tri_count[r * L + L - 1]]
        Fr = vr[tr]
        cr = Fr.mean(1)
        for s in range(S.n_objects):
            vs = S.verts[S.vert_begin[s]:S.vert_begin[s] + S.vert_count[s]]
            if np.min(np.linalg.norm(vs - cr.mean(0), axis=1)) > 4.0:
                continue
            ts = S.tris[S.tri_begin[s * L + L - 1]:S.tri_begin[s * L + L - 1] + S.tri_count[s * L + L - 1]]
            Fs = vs[ts]
            cs = Fs.mean(1)
            pick = rng.choice(len(Fr), 256, replace=False)
            d2 = ((cr[pick][:, None, :] - cs[None, :, :]) ** 2).sum(-1)
            near = np.argsort(d2, axis=1)[:, :16]
            out1.append(np.repeat(Fr[pick], 16, axis=0))
            out2.append(Fs[near.reshape(-1)])
            have += 256 * 16
    return np.concatenate(out1).astype(np.float32), np.concatenate(out2).astype(np.float32)


def _check(ctx, T1, T2, max_open=0.05):
    lo, hi, sure = ctx.facet_pairs(T1, T2, "fp32", bounds=True)
    d64, h64 = ctx.facet_pairs(T1, T2, "fp64")
    eps = _eps(T1, T2)
    # the lower estimate never exceeds the distance, nor the upper one falls
    # below it, by more than eps/8 ...
    under, over = (lo - d64) / eps, (d64 - hi) / eps
    assert np.all(under <= 0.125), (int((under > 0.125).sum()), float(under.max()), int(np.argmax(under)))
    assert np.all(over <= 0.125), (int((over > 0.125).sum()), float(over.max()), int(np.argmax(over)))
    # ... a certain crossing is a real meet with upper estimate 0 ...
    assert not np.any(sure & ~h64)
    assert np.all(hi[sure] == 0.0)
    assert np.all(lo <= hi)
    # ... and only a few pairs stay open for the FP64 recheck
    n_open = int((lo < hi).sum())
    assert n_open <= max_open * len(lo), n_open
    err = np.abs(np.where(lo < hi, 0.0, lo - d64)) / eps
    return float(err.max()), int(h64.sum()), n_open


def test_guard_band_subset_against_oracle(orc, ctx):
    rng = np.random.default_rng(20)
    T1, T2 = _block(rng, 200000)
    d_ref, h_ref = orc.tri_tri_batch(T1, T2)
    d64, h64 = ctx.facet_pairs(T1, T2, "fp64")
    assert np.array_equal(h64, h_ref)
    scale = 1.0 + np.abs(np.concatenate([T1, T2], 1)).reshape(len(T1), -1).max(1)
    assert np.all(np.abs(d64 - d_ref) <= 1e-12 * scale)
    lo, hi, sure = ctx.facet_pairs(T1, T2, "fp32", bounds=True)
    # a certain crossing is a real meet by the oracle's exact predicates
    assert not np.any(sure & ~h_ref)
    _check(ctx, T1, T2)


def test_guard_band_near_coplanar_thin_pair(ctx):
    """Two thin facets, one an in-plane shifted copy of the other, 7.2e-3
    apart: their plane distances are FP32 rounding noise, and the plain-sign
    crossing test fires on them.  The pair must stay open (lower 0, upper the
    true distance), never a certain crossing."""
    T1 = np.array([[1.6040207, -1.1628633, -2.2375202], [0.04622463, -2.524434, -1.5271888],
                   [1.5848998, -1.2076437, -2.1975858]], np.float32)
    T2 = np.array([[1.4963719, -1.2225302, -2.226716], [-0.06142426, -2.584101, -1.5163845],
                   [1.4772509, -1.2673107, -2.1867816]], np.float32)
    lo, hi, sure = ctx.facet_pairs(T1[None], T2[None], "fp32", bounds=True)
    d64, h64 = ctx.facet_pairs(T1[None], T2[None], "fp64")
    assert not h64[0] and d64[0] > 7e-3
    assert not sure[0]
    eps = _eps(T1[None], T2[None])[0]
    assert lo[0] <= d64[0] + eps / 8 and hi[0] >= d64[0] - eps / 8


def test_guard_band_degenerate_facets(orc, ctx):
    """Zero-area facets (a segment, a point) against regular triangles: a
    segment piercing a face meets it although none of the 15 candidates is
    0, so the lower estimate must drop to 0; the upper one stays an attained
    distance."""
    rng = np.random.default_rng(22)
    n = 20000
    T2 = rng.standard_normal((n, 3, 3)).astype(np.float32)
    c = T2.mean(1)
    nrm = _unit(np.cross(T2[:, 1] - T2[:, 0], T2[:, 2] - T2[:, 0]))
    k = rng.integers(0, 3, n)
    T1 = np.empty_like(T2)
    h = rng.uniform(0.1, 1.0, (n, 1)).astype(np.float32)
    # 0: a segment (a repeated corner) through the face's interior
    seg = np.stack([c - h * nrm, c + h * nrm, c + h * nrm], 1)
    # 1: a point on or next to the face
    pt = np.repeat((c + rng.uniform(-1e-3, 1e-3, (n, 1)).astype(np.float32) * nrm)[:, None, :], 3, 1)
    # 2: three collinear corners beside the face
    d = rng.standard_normal((n, 3)).astype(np.float32)
    col = np.stack([c + 2 * nrm, c + 2 * nrm + d, c + 2 * nrm + 2 * d], 1)
    T1[k == 0], T1[k == 1], T1[k == 2] = seg[k == 0], pt[k == 1], col[k == 2]
    lo, hi, sure = ctx.facet_pairs(T1, T2, "fp32", bounds=True)
    d64, h64 = ctx.facet_pairs(T1, T2, "fp64")
    # the FP64 path against the oracle's exact predicates on these inputs
    d_ref, h_ref = orc.tri_tri_batch(T1, T2)
    assert np.array_equal(h64, h_ref)
    assert np.all(np.abs(d64 - d_ref) <= 1e-12 * (1.0 + np.abs(np.concatenate([T1, T2], 1)).reshape(n, -1).max(1)))
    eps = _eps(T1, T2)
    assert np.all(lo - d64 <= eps / 8), float(np.max((lo - d64) / eps))
    assert np.all(d64 - hi <= eps / 8), float(np.max((d64 - hi) / eps))
    assert not np.any(sure & ~h64)
    assert h64[k == 0].all()   # every piercing segment meets its face


def test_guard_band_1e8_pairs(ctx):
    rng = np.random.default_rng(21)
    worst, meets, total, n_open = 0.0, 0, 0, 0
    M1, M2 = _mesh_pairs(rng, 1 << 20)
    w, h, o = _check(ctx, M1, M2, max_open=0.01)
    worst, meets, total, n_open = max(worst, w), meets + h, total + len(M1), n_open + o
    for b in range(BLOCKS):
        T1, T2 = _block(rng, BLOCK)
        w, h, o = _check(ctx, T1, T2)
        worst, meets, total, n_open = max(worst, w), meets + h, total + len(T1), n_open + o
        print(f"block {b}: {total} pairs, worst err/eps {worst:.4f}, meets {meets}, open {n_open}", flush=True)
    assert total >= 100_000_000
    assert meets > 1000
