"""Pins for the oracle's triangle distances (Section 2.2, 15 candidates plus
the exact meet test).

Independent references: closed forms on hand-built cases, an exhaustive
face-pair (KKT) enumeration of the convex distance problem, dense sampling,
and exact invariances (symmetry, integer translation, power-of-two scaling).
"""
import itertools

import numpy as np
import pytest


def tri_dist_enum(T1, T2):
    """min |sum l_i A_i - sum m_j B_j| over the two simplices by enumerating
    every pair of faces (vertex / edge / whole triangle) of the two
    triangles and keeping feasible stationary points of each face pair."""
    A = np.asarray(T1, np.float64)
    B = np.asarray(T2, np.float64)
    faces = [f for k in (1, 2, 3) for f in itertools.combinations(range(3), k)]
    best = np.inf
    for F in faces:
        for G in faces:
            P0, Q0 = A[F[0]], B[G[0]]
            cols = [A[i] - P0 for i in F[1:]] + [-(B[j] - Q0) for j in G[1:]]
            w = P0 - Q0
            if cols:
                M = np.stack(cols, 1)
                z, *_ = np.linalg.lstsq(M, -w, rcond=None)
                alpha, beta = z[:len(F) - 1], z[len(F) - 1:]
                lam = np.concatenate([[1 - alpha.sum()], alpha])
                mu = np.concatenate([[1 - beta.sum()], beta])
                if lam.min() < -1e-12 or mu.min() < -1e-12:
                    continue
                v = np.linalg.norm(w + M @ z)
            else:
                v = np.linalg.norm(w)
            best = min(best, v)
    return best


def test_point_triangle_closed_forms(orc):
    a, b, c = [0, 0, 0], [4, 0, 0], [0, 4, 0]
    assert orc.pt_tri([1, 1, 2.5], a, b, c) == pytest.approx(2.5, abs=1e-15)
    assert orc.pt_tri([-3, -4, 0], a, b, c) == pytest.approx(5.0, abs=1e-15)   # vertex region
    assert orc.pt_tri([2, -3, 4], a, b, c) == pytest.approx(5.0, abs=1e-15)    # edge region
    assert orc.pt_tri([3, 3, 0], a, b, c) == pytest.approx(np.sqrt(2.0), abs=1e-15)  # hypotenuse region
    # degenerate (collinear) triangle -> distance to the segment
    assert orc.pt_tri([1, 2, 0], [0, 0, 0], [2, 0, 0], [4, 0, 0]) == pytest.approx(2.0, abs=1e-15)


def test_segment_closed_forms(orc):
    for h in (0.5, 3.0, 1e-4):
        assert orc.seg_seg([-1, 0, 0], [1, 0, 0], [0, -1, h], [0, 1, h]) == pytest.approx(h, rel=1e-14)
    assert orc.seg_seg([0, 0, 0], [4, 0, 0], [1, 3, 4], [6, 3, 4]) == pytest.approx(5.0, rel=1e-15)  # parallel
    assert orc.seg_seg([0, 0, 0], [1, 0, 0], [3, 0, 0], [5, 0, 0]) == pytest.approx(2.0, rel=1e-15)  # collinear
    assert orc.seg_seg([0, 0, 0], [0, 0, 0], [0, 3, 4], [0, 3, 4]) == pytest.approx(5.0, rel=1e-15)  # points


def test_triangle_closed_forms(orc):
    T = np.array([[0, 0, 0], [4, 0, 0], [0, 4, 0]], np.float32)
    for h in (0.25, 2.0, 7.5):
        assert orc.tri_tri_dist(T, T + np.float32([0, 0, h])) == pytest.approx(h, rel=1e-15)
    # crossing triangles: every one of the 15 candidates is positive, d = 0
    X = np.array([[1, 1, -1], [1, 1, 1], [6, 6, 0]], np.float32)
    assert orc.tri_tri_dist(T, X) == 0.0
    # edge over edge, skew, at height 3
    E = np.array([[1, -1, 3], [1, 5, 3], [1, 2, 9]], np.float32)
    assert orc.tri_tri_dist(T, E) == pytest.approx(3.0, rel=1e-15)


def _random_pair(rng, kind):
    T1 = rng.normal(size=(3, 3))
    T2 = rng.normal(size=(3, 3)) + rng.normal(size=3) * (0.0 if kind == "close" else 2.0)
    if kind == "sliver":
        T2[2] = T2[0] + 1e-3 * (T2[1] - T2[0]) + 1e-6
    if kind == "parallel":
        T2 = T1 + np.array([0.3, -0.2, 0.7])
    return T1.astype(np.float32), T2.astype(np.float32)


@pytest.mark.parametrize("kind", ["far", "close", "sliver", "parallel"])
def test_triangle_distance_vs_face_pair_enumeration(orc, kind):
    rng = np.random.default_rng({"far": 1, "close": 2, "sliver": 3, "parallel": 4}[kind])
    for _ in range(300):
        T1, T2 = _random_pair(rng, kind)
        ref = tri_dist_enum(T1, T2)
        got = orc.tri_tri_dist(T1, T2)
        scale = 1.0 + np.abs(np.concatenate([T1, T2])).max()
        assert abs(got - ref) <= 1e-9 * scale, (kind, got, ref)
        assert (got == 0.0) == orc.tri_tri_intersect(T1, T2)


def test_triangle_distance_dense_sampling(orc):
    rng = np.random.default_rng(9)
    N = 24
    ij = np.array([(i, j) for i in range(N + 1) for j in range(N + 1 - i)], np.float64) / N
    bary = np.stack([1 - ij.sum(1), ij[:, 0], ij[:, 1]], 1)
    for _ in range(20):
        T1, T2 = _random_pair(rng, "far")
        P = bary @ T1.astype(np.float64)
        Q = bary @ T2.astype(np.float64)
        smin = np.sqrt(((P[:, None, :] - Q[None, :, :]) ** 2).sum(-1)).min()
        h = max(np.linalg.norm(np.roll(T, 1, 0) - T, axis=1).max() for T in (T1, T2)) / N
        d = orc.tri_tri_dist(T1, T2)
        assert d <= smin + 1e-12
        assert smin <= d + 2 * h + 1e-12


def test_triangle_distance_invariances(orc):
    rng = np.random.default_rng(12)
    for _ in range(200):
        T1, T2 = _random_pair(rng, "far")
        d = orc.tri_tri_dist(T1, T2)
        # symmetry (candidate order differs, so allow rounding)
        assert orc.tri_tri_dist(T2, T1) == pytest.approx(d, rel=1e-13, abs=1e-15)
        # power-of-two scaling is exact in binary floating point
        assert orc.tri_tri_dist(T1 * np.float32(4), T2 * np.float32(4)) == 4 * d
        assert orc.tri_tri_dist(T1 * np.float32(0.125), T2 * np.float32(0.125)) == 0.125 * d
        # axis permutation
        p = rng.permutation(3)
        assert orc.tri_tri_dist(T1[:, p], T2[:, p]) == pytest.approx(d, rel=1e-12, abs=1e-14)
    # translation by integers on a grid where the shifted coordinates stay exact
    for _ in range(200):
        T1 = (rng.integers(-64, 64, size=(3, 3)) / 8.0).astype(np.float32)
        T2 = (rng.integers(-64, 64, size=(3, 3)) / 8.0).astype(np.float32)
        s = rng.integers(-1000, 1000, size=3).astype(np.float32)
        d = orc.tri_tri_dist(T1, T2)
        assert orc.tri_tri_dist(T1 + s, T2 + s) == pytest.approx(d, rel=1e-12, abs=1e-12 * 1000)
        assert orc.tri_tri_intersect(T1 + s, T2 + s) == orc.tri_tri_intersect(T1, T2)


def test_distance_zero_iff_meet_near_contact(orc):
    """Triangles pushed onto each other along a random direction: the sign
    of the gap decides the meet, and d == 0 exactly when they meet."""
    rng = np.random.default_rng(21)
    seen = {True: 0, False: 0}
    for _ in range(300):
        T1 = rng.normal(size=(3, 3)).astype(np.float32)
        T2 = rng.normal(size=(3, 3)).astype(np.float32)
        n = np.cross(T1[1] - T1[0], T1[2] - T1[0])
        T2 = (T2 + (rng.uniform(-0.3, 0.3) * n / np.linalg.norm(n))).astype(np.float32)
        hit = orc.tri_tri_intersect(T1, T2)
        seen[hit] += 1
        d = orc.tri_tri_dist(T1, T2)
        assert (d == 0.0) == hit
        if not hit:
            assert d == pytest.approx(tri_dist_enum(T1, T2), abs=1e-9)
    assert seen[True] > 20 and seen[False] > 20
