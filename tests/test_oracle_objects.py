"""Object-level pins for the oracle: meshes, hand-built object distances, the
anchor upper bound, brute vs culled scans, the LoD bounds of Eq. (1)/(2) and
properties of the three joins."""
import numpy as np
import pytest

import meshgen as mg


def _edges(tris):
    e = np.sort(np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]]), 1)
    u, c = np.unique(e, axis=0, return_counts=True)
    return u, c


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_icosphere_counts(level):
    v, faces, parents = mg.icosphere_template(level)
    f = faces[level]
    assert len(v) == 10 * 4 ** level + 2 and len(f) == 20 * 4 ** level
    u, c = _edges(f)
    assert np.all(c == 2)                       # closed 2-manifold
    assert len(v) - len(u) + len(f) == 2        # Euler characteristic
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0)
    if level:
        p = parents[level]
        assert np.array_equal(np.bincount(p), np.full(len(faces[level - 1]), 4))


@pytest.mark.parametrize("n_seg,n_lods", [(64, 3), (1280, 4)])
def test_tube_counts_and_parents(n_seg, n_lods):
    tl, pl = mg.tube_template(n_seg, n_lods)
    for lod in range(n_lods):
        ns = n_seg // 4 ** (n_lods - 1 - lod)
        assert len(tl[lod]) == 16 * ns + 16
        u, c = _edges(tl[lod])
        assert np.all(c == 2)
        nv = len(np.unique(tl[lod]))
        assert nv - len(u) + len(tl[lod]) == 2
        if lod:
            assert pl[lod].min() >= 0 and pl[lod].max() < len(tl[lod - 1])
            assert np.array_equal(np.bincount(pl[lod], minlength=len(tl[lod - 1]))[:16 * (ns // 4)],
                                  np.full(16 * (ns // 4), 4))


def _single(orc, ms):
    return orc.OSet(ms)


def test_cubes_face_gap_and_diagonal(orc):
    A = orc.OSet(mg.cube_mesh([0, 0, 0], [1, 1, 1]))
    for g in (0.0, 0.25, 1.5):
        B = orc.OSet(mg.cube_mesh([1 + g, 0, 0], [2 + g, 1, 1]))
        d, hit = orc.object_distance(A, 0, B, 0)
        assert d == pytest.approx(g, abs=1e-15) and hit == (g == 0.0)
    for gx, gy, gz in [(0.5, 0.25, 1.0), (3.0, 0.0, 4.0), (0.0, 0.0, 0.0)]:
        B = orc.OSet(mg.cube_mesh([1 + gx, 1 + gy, 1 + gz], [2 + gx, 2 + gy, 2 + gz]))
        d, _ = orc.object_distance(A, 0, B, 0)
        assert d == pytest.approx(np.sqrt(gx * gx + gy * gy + gz * gz), abs=1e-14)


def test_nested_cubes_surface_semantics(orc):
    # a solid inside another does not meet it: distance between surfaces
    A = orc.OSet(mg.cube_mesh([1, 1, 1], [2, 2, 2]))
    B = orc.OSet(mg.cube_mesh([0, 0, 0], [3, 3, 3]))
    d, hit = orc.object_distance(A, 0, B, 0)
    assert d == pytest.approx(1.0, abs=1e-15) and not hit


def _two_boxes(c1, c2, h=0.5):
    a = mg.cube_mesh(np.asarray(c1) - h, np.asarray(c1) + h)
    b = mg.cube_mesh(np.asarray(c2) - h, np.asarray(c2) + h)
    v = np.concatenate([a.verts, b.verts])
    t = np.concatenate([a.tris, b.tris + 8])
    return mg.single_object(v, [t])


def test_anchor_bound_fig3_case(orc):
    """Two separated objects whose MBB centres coincide (the failure case of
    upper-bounding by MBB centres, Section 2.1): the vertex-anchor bound stays
    positive and above d."""
    A = orc.OSet(_two_boxes([0, 0, 0], [9, 9, 0]))
    B = orc.OSet(_two_boxes([9, 0, 0], [0, 9, 0]))
    bA, aA = orc.mbbs(A)
    bB, aB = orc.mbbs(B)
    assert np.allclose(0.5 * (bA[0, :3] + bA[0, 3:]), 0.5 * (bB[0, :3] + bB[0, 3:]))
    d, _ = orc.object_distance(A, 0, B, 0)
    ub = np.linalg.norm(aA[0] - aB[0])
    assert d == pytest.approx(8.0)
    assert ub > 0 and ub >= d


@pytest.fixture(scope="module")
def small_multilod():
    R = mg.blob_set(mg.rng_for(100, 0), 4, (0.0, 5.0), 1, 3, radius_sigma=0.3)
    S = mg.tube_set(mg.rng_for(100, 1), 3, (0.0, 5.0), 64, 3, length_range=(6.0, 10.0))
    return R, S


def test_brute_equals_culled(orc, small_multilod):
    R, S = (orc.OSet(x) for x in small_multilod)
    rr, ss = np.meshgrid(np.arange(4), np.arange(3), indexing="ij")
    for lod in range(3):
        d0, h0 = orc.pair_distances(R, S, rr.ravel(), ss.ravel(), lod=lod, mode=0)
        d1, h1 = orc.pair_distances(R, S, rr.ravel(), ss.ravel(), lod=lod, mode=1)
        assert np.array_equal(d0, d1) and np.array_equal(h0, h1)


def test_hd_ph_bounds_are_valid(orc, small_multilod):
    """LB_l <= d <= UB_l at every LoD, LB = UB = d on the finest one
    (Eq. (1), Eq. (2))."""
    R, S = (orc.OSet(x) for x in small_multilod)
    L = 3
    hp_r = {(i, l): orc.hd_ph(R, i, l) for i in range(4) for l in range(L)}
    hp_s = {(j, l): orc.hd_ph(S, j, l) for j in range(3) for l in range(L)}
    for (i, l), (hd, ph) in hp_r.items():
        assert np.all(hd >= 0) and np.all(ph >= 0)
        if l == L - 1:
            assert not hd.any() and not ph.any()
    widths = []
    for i in range(4):
        for j in range(3):
            d, _ = orc.object_distance(R, i, S, j)
            for l in range(L):
                lb, ub = orc.lod_bounds(R, i, S, j, l, hp_r[i, l][0], hp_r[i, l][1], hp_s[j, l][0], hp_s[j, l][1])
                assert lb <= d + 1e-12 and d <= ub + 1e-12, (i, j, l, lb, d, ub)
                widths.append((l, ub - lb))
                if l == L - 1:
                    assert lb == pytest.approx(d, abs=1e-15) and ub == pytest.approx(d, abs=1e-15)
    w = {l: np.mean([x for ll, x in widths if ll == l]) for l in range(L)}
    assert w[0] > w[1] > w[2]   # bounds tighten as the LoD rises


def test_hd_covers_dense_points(orc, small_multilod):
    """hd(f', P) >= dist(x, P) for many random points x of each coarse facet
    (distance to *all* finest facets, brute force)."""
    Rm, _ = small_multilod
    R = orc.OSet(Rm)
    rng = np.random.default_rng(4)
    fine = Rm.facets(0, 2).astype(np.float64)
    for lod in (0, 1):
        hd, ph = orc.hd_ph(R, 0, lod)
        F = Rm.facets(0, lod).astype(np.float64)
        for f in rng.choice(len(F), 12, replace=False):
            w = rng.dirichlet(np.ones(3), size=20)
            X = w @ F[f]
            for x in X:
                dx = min(orc.pt_tri(x, *g) for g in fine)
                assert dx <= hd[f] + 1e-12
        # ph: every finest corner mapped to f' is within ph of f'
        assert np.all(ph <= hd + 1.0)


@pytest.fixture(scope="module")
def small_join():
    R, S = mg.config_small(seed=0, n_r=30, n_s=30, box=7.0)
    return R, S


def test_join_properties(orc, small_join):
    R, S = (orc.OSet(x) for x in small_join)
    res = {t: orc.join_within(R, S, t) for t in (0.0, 0.1, 0.5, 1.0)}
    sets = {t: set(zip(v["r"].tolist(), v["s"].tolist())) for t, v in res.items()}
    assert sets[0.0] <= sets[0.1] <= sets[0.5] <= sets[1.0]
    assert len(sets[0.0]) > 0 and len(sets[1.0]) > len(sets[0.0])
    inter = orc.join_intersect(R, S)
    assert set(zip(inter["r"].tolist(), inter["s"].tolist())) == sets[0.0]
    for v in res.values():
        assert v["near_ties"] == 0
    # the MBB skip is exact: compare with the full all-pairs scan
    rr, ss = np.meshgrid(np.arange(30), np.arange(30), indexing="ij")
    d, hit = orc.pair_distances(R, S, rr.ravel(), ss.ravel())
    full = set(zip(rr.ravel()[d <= 0.5].tolist(), ss.ravel()[d <= 0.5].tolist()))
    assert full == sets[0.5]
    assert set(zip(rr.ravel()[hit].tolist(), ss.ravel()[hit].tolist())) == sets[0.0]


def test_knn_full_order(orc, small_join):
    R, S = (orc.OSet(x) for x in small_join)
    rr, ss = np.meshgrid(np.arange(5), np.arange(30), indexing="ij")
    d, _ = orc.pair_distances(R, S, rr.ravel(), ss.ravel())
    d = d.reshape(5, 30)
    for k in (1, 3, 30, 40):
        res = orc.join_knn(R, S, k, r_subset=np.arange(5))
        for r in range(5):
            order = np.lexsort((np.arange(30), d[r]))[:min(k, 30)]
            assert np.array_equal(res["s"][r], order)
            assert np.array_equal(res["d"][r], d[r][order])


def _dist_to_unit_square(x):
    """Closed-form distance of points x [n, 3] to the square [0,1]^2 x {0}."""
    dx = np.maximum(0.0, np.maximum(-x[:, 0], x[:, 0] - 1.0))
    dy = np.maximum(0.0, np.maximum(-x[:, 1], x[:, 1] - 1.0))
    return np.sqrt(dx * dx + dy * dy + x[:, 2] * x[:, 2])


def test_hd_of_facet_without_descendants(orc):
    """A coarse facet that no finest facet descends from (a triangle at z = 5
    over the unit square) still gets an hd that bounds its distance to the
    finest mesh (Eq. (1) needs hd(f', P) >= max_x dist(x, P)); ph only has
    to cover descendants, so it is 0 there."""
    ms = mg.orphan_facet_object(5.0)
    O = orc.OSet(ms)
    hd, ph = orc.hd_ph(O, 0, 0)
    F = ms.facets(0, 0).astype(np.float64)
    rng = np.random.default_rng(3)
    for f in range(3):
        X = np.concatenate([F[f], rng.dirichlet(np.ones(3), size=200) @ F[f]])
        assert hd[f] >= _dist_to_unit_square(X).max() - 1e-12, (f, hd[f])
    assert hd[2] >= 5.0 and ph[2] == 0.0
    # the two square facets are their own descendants: hd is the grid edge
    assert hd[0] == pytest.approx(np.sqrt(2.0) / 8.0, abs=1e-12)
    assert hd[1] == pytest.approx(np.sqrt(2.0) / 8.0, abs=1e-12)
    # Eq. (1)/(2) at the coarse LoD against a small facet 0.2 above the
    # orphan: LB <= d <= UB (with hd = the grid edge alone, UB would be ~0.38)
    q = np.array([[0.1, 0.1, 5.2], [0.3, 0.1, 5.2], [0.1, 0.3, 5.2]], np.float32)
    T = orc.OSet(mg.single_object(q, [np.array([[0, 1, 2]]), np.array([[0, 1, 2]])],
                                  [np.full(1, -1, np.int32), np.zeros(1, np.int32)]))
    hq, pq = orc.hd_ph(T, 0, 0)
    d, _ = orc.object_distance(O, 0, T, 0)
    assert d == pytest.approx(5.2, abs=1e-6)
    lb, ub = orc.lod_bounds(O, 0, T, 0, 0, hd, ph, hq, pq)
    assert lb <= d <= ub
    assert ub >= 5.0
