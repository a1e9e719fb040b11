"""Pins for the oracle's exact orientation predicates and triangle meet test.

The references here are independent of the oracle's arithmetic: exact
rational determinants (``fractions.Fraction``) and an exact feasibility search
over barycentric coordinates, both run on small inputs.
"""
from fractions import Fraction as Fr
import itertools

import numpy as np
import pytest


def f32(x):
    return np.float32(x)


def det_rational(rows):
    """Exact determinant of a square matrix of Fractions (Laplace)."""
    n = len(rows)
    if n == 1:
        return rows[0][0]
    tot = Fr(0)
    for j in range(n):
        minor = [r[:j] + r[j + 1:] for r in rows[1:]]
        tot += (-1) ** j * rows[0][j] * det_rational(minor)
    return tot


def sgn(x):
    return (x > 0) - (x < 0)


def orient3d_exact(a, b, c, d):
    rows = [[Fr(float(v)) for v in p] + [Fr(1)] for p in (a, b, c, d)]
    return sgn(det_rational(rows))


def orient2d_exact(a, b, c):
    rows = [[Fr(float(p[0])), Fr(float(p[1])), Fr(1)] for p in (a, b, c)]
    return sgn(det_rational(rows))


def _rand_pts(rng, n, scale):
    return (rng.uniform(-1, 1, size=(n, 3)) * scale).astype(np.float32)


def test_orient3d_unit_cases(orc):
    o = [0, 0, 0]
    assert orc.orient3d(o, [1, 0, 0], [0, 1, 0], [0, 0, 1]) == orient3d_exact(o, [1, 0, 0], [0, 1, 0], [0, 0, 1]) != 0
    assert orc.orient3d(o, [1, 0, 0], [0, 1, 0], [0, 0, 1]) == -orc.orient3d(o, [1, 0, 0], [0, 1, 0], [0, 0, -1])
    assert orc.orient3d(o, [1, 0, 0], [0, 1, 0], [7, -3, 0]) == 0
    assert orc.orient3d(o, [1, 1, 1], [2, 2, 2], [5, -1, 3]) == 0  # collinear triple


@pytest.mark.parametrize("scale", [1.0, 1e3, 1e-3, 3e7])
def test_orient3d_random_and_near_coplanar(orc, scale):
    rng = np.random.default_rng(7)
    for _ in range(150):
        a, b, c, d = _rand_pts(rng, 4, scale)
        assert orc.orient3d(a, b, c, d) == orient3d_exact(a, b, c, d)
    # points on a plane through a, b, c rounded to float32: signs decided by
    # the rounding, i.e. tiny determinants the fast FP64 formula gets wrong
    for _ in range(150):
        a, b, c = _rand_pts(rng, 3, scale)
        u, v = rng.uniform(-2, 2, size=2)
        d = (a.astype(np.float64) + u * (b - a.astype(np.float64)) + v * (c - a.astype(np.float64))).astype(np.float32)
        assert orc.orient3d(a, b, c, d) == orient3d_exact(a, b, c, d)


def test_orient3d_ulp_flip(orc):
    # d exactly on the plane z = 0, then one ulp above and below
    a, b, c = [0.1, 0.2, 0.0], [3.7, -1.1, 0.0], [-2.3, 5.9, 0.0]
    a, b, c = (np.float32(x) for x in (a, b, c))
    d0 = np.array([1.3, 0.7, 0.0], np.float32)
    up = d0.copy()
    up[2] = np.nextafter(np.float32(0), np.float32(1))
    dn = d0.copy()
    dn[2] = -up[2]
    s0, su, sd = orc.orient3d(a, b, c, d0), orc.orient3d(a, b, c, up), orc.orient3d(a, b, c, dn)
    assert s0 == 0 and su == -sd != 0
    assert su == orient3d_exact(a, b, c, up)


def test_orient2d_random_and_collinear(orc):
    rng = np.random.default_rng(11)
    for _ in range(300):
        a, b, c = _rand_pts(rng, 3, 10.0)
        assert orc.orient2d(a, b, c, 0, 1) == orient2d_exact(a[:2], b[:2], c[:2])
        assert orc.orient2d(a, b, c, 1, 2) == orient2d_exact(a[1:], b[1:], c[1:])
    for _ in range(300):
        a, b = _rand_pts(rng, 2, 10.0)
        t = rng.uniform(-2, 2)
        c = (a.astype(np.float64) + t * (b.astype(np.float64) - a)).astype(np.float32)
        assert orc.orient2d(a, b, c, 0, 1) == orient2d_exact(a[:2], b[:2], c[:2])


# ---------------------------------------------------------------------------
# triangle meet test vs an exact barycentric feasibility search
# ---------------------------------------------------------------------------
def _solve_exact(A, b):
    """Unique exact solution of A x = b (A: m x n Fractions with independent
    columns), or None if inconsistent."""
    m, n = len(A), len(A[0])
    M = [row[:] + [bb] for row, bb in zip(A, b)]
    r = 0
    piv = []
    for c in range(n):
        p = next((i for i in range(r, m) if M[i][c] != 0), None)
        if p is None:
            return None  # dependent columns
        M[r], M[p] = M[p], M[r]
        inv = 1 / M[r][c]
        M[r] = [x * inv for x in M[r]]
        for i in range(m):
            if i != r and M[i][c] != 0:
                f = M[i][c]
                M[i] = [x - f * y for x, y in zip(M[i], M[r])]
        piv.append(c)
        r += 1
    for i in range(r, m):
        if M[i][n] != 0:
            return None
    return [M[i][n] for i in range(n)]


def meet_exact(T1, T2):
    """Closed triangles meet iff sum l_i T1_i = sum m_j T2_j has a solution
    with l, m >= 0, sum l = sum m = 1.  A feasible system has a basic
    feasible solution, whose support columns are independent: enumerate
    supports and solve exactly."""
    cols = []
    for p in T1:
        cols.append([Fr(float(x)) for x in p] + [Fr(1), Fr(0)])
    for p in T2:
        cols.append([-Fr(float(x)) for x in p] + [Fr(0), Fr(1)])
    rhs = [Fr(0)] * 3 + [Fr(1), Fr(1)]
    for k in range(1, 6):
        for sup in itertools.combinations(range(6), k):
            A = [[cols[c][i] for c in sup] for i in range(5)]
            x = _solve_exact(A, rhs)
            if x is not None and all(v >= 0 for v in x):
                return True
    return False


def test_meet_hand_cases(orc):
    T = np.array([[0, 0, 0], [4, 0, 0], [0, 4, 0]], np.float32)
    cases = {
        "crossing": ([[1, 1, -1], [1, 1, 1], [6, 6, 0]], True),
        "above": ([[1, 1, 1], [2, 1, 1], [1, 2, 1]], False),
        "vertex_on_face": ([[1, 1, 0], [1, 1, 2], [2, 1, 2]], True),
        "edge_on_edge": ([[2, 2, 0], [5, 5, 0], [3, 3, 3]], True),
        "vertex_touch_vertex": ([[4, 0, 0], [5, 0, 1], [5, 1, 0]], True),
        "coplanar_overlap": ([[1, 1, 0], [5, 1, 0], [1, 5, 0]], True),
        "coplanar_contained": ([[0.5, 0.5, 0], [1, 0.5, 0], [0.5, 1, 0]], True),
        "coplanar_apart": ([[3, 3, 0], [6, 3, 0], [3, 6, 0]], False),
        "coplanar_touch_edge": ([[2, 2, 0], [4, 4, 0], [1, 5, 0]], True),
        "degenerate_segment_piercing": ([[1, 1, -1], [1, 1, 1], [1, 1, 3]], True),
        "degenerate_point_inside": ([[1, 1, 0], [1, 1, 0], [1, 1, 0]], True),
        "degenerate_point_outside": ([[1, 1, 0.5], [1, 1, 0.5], [1, 1, 0.5]], False),
    }
    for name, (t2, want) in cases.items():
        t2 = np.asarray(t2, np.float32)
        assert orc.tri_tri_intersect(T, t2) == want, name
        assert orc.tri_tri_intersect(t2, T) == want, name
        assert meet_exact(T, t2) == want, name
        assert (orc.tri_tri_dist(T, t2) == 0.0) == want, name


def test_meet_small_grid_brute_force(orc):
    """Random triangles on a 4x4x4 integer grid: plenty of touching,
    coplanar, collinear and degenerate configurations."""
    rng = np.random.default_rng(3)
    n_meet = 0
    for _ in range(400):
        T1 = rng.integers(0, 4, size=(3, 3)).astype(np.float32)
        T2 = rng.integers(0, 4, size=(3, 3)).astype(np.float32)
        want = meet_exact(T1, T2)
        n_meet += want
        assert orc.tri_tri_intersect(T1, T2) == want, (T1.tolist(), T2.tolist())
    assert 50 < n_meet < 350


def test_meet_half_integer_coplanar(orc):
    rng = np.random.default_rng(5)
    for _ in range(300):
        T1 = np.zeros((3, 3), np.float32)
        T2 = np.zeros((3, 3), np.float32)
        T1[:, :2] = rng.integers(0, 8, size=(3, 2)) / 2.0
        T2[:, :2] = rng.integers(0, 8, size=(3, 2)) / 2.0
        # tilt both copies into the same oblique plane z = x + 2y (exact)
        T1[:, 2] = T1[:, 0] + 2 * T1[:, 1]
        T2[:, 2] = T2[:, 0] + 2 * T2[:, 1]
        assert orc.tri_tri_intersect(T1, T2) == meet_exact(T1, T2), (T1.tolist(), T2.tolist())
