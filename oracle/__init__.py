"""CPU FP64 oracle for the progressive polyhedral spatial join.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; never by the product path.  It
shares no code with the GPU library (``paper_2604_19982_amd``), neither
imports the other, and the only common module is ``meshgen`` (inputs only).

The heavy geometry lives in ``oracle.c`` (plain C, FP64, OpenMP over object
pairs); this module drives it and adds the pieces that are easier to read in
numpy:

* ``join_within`` / ``join_intersect`` / ``join_knn`` -- the three queries of
  Section 3 (intersection, within-tau, k-NN), computed from the plain
  definition d(r, s) = min over facet pairs (Section 2.1) on the finest LoD;
* ``knn_prune`` -- the k-NN object-pair pruning rule of Algorithm 6, in a
  corrected reading (see its docstring);
* ``mlp_*`` -- FP64 forward/backward of the 16-64-64-4 LoD-skip network.

"Parity unpinned" parts: none of the functions here lacks a pin; see the
tests under ``tests/test_oracle_*.py`` for what pins each one.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Set(ctypes.Structure):
    _fields_ = [("n_objects", ctypes.c_int32), ("n_lods", ctypes.c_int32),
                ("verts", ctypes.c_void_p), ("vert_begin", ctypes.c_void_p), ("vert_count", ctypes.c_void_p),
                ("tris", ctypes.c_void_p), ("tri_begin", ctypes.c_void_p), ("tri_count", ctypes.c_void_p),
                ("parent", ctypes.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        sp = ctypes.POINTER(_Set)
        L.oracle_orient3d.argtypes = [dp, dp, dp, dp]
        L.oracle_orient2d.argtypes = [dp, dp, dp, ctypes.c_int, ctypes.c_int]
        L.oracle_tri_tri_intersect.argtypes = [fp, fp]
        L.oracle_tri_tri_dist.argtypes = [fp, fp, ctypes.POINTER(ctypes.c_int)]
        L.oracle_tri_tri_dist.restype = ctypes.c_double
        L.oracle_pt_tri.argtypes = [dp, dp, dp, dp]
        L.oracle_pt_tri.restype = ctypes.c_double
        L.oracle_seg_seg.argtypes = [dp, dp, dp, dp]
        L.oracle_seg_seg.restype = ctypes.c_double
        L.oracle_object_distance.argtypes = [sp, ctypes.c_int, ctypes.c_int, sp, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.oracle_object_distance.restype = ctypes.c_double
        L.oracle_pair_distances.argtypes = [sp, sp, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_pair_distances_counted.argtypes = [sp, sp, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                                    ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_mbb_all.argtypes = [sp, ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_hd_ph.argtypes = [sp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_lod_bounds.argtypes = [sp, ctypes.c_int, sp, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, dp, dp]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_tri_tri_batch.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_int]
        L.oracle_tri_tri_batch.restype = None
        _lib = L
    return _lib


class OSet:
    """A mesh set pinned for the C oracle (keeps the numpy arrays alive)."""

    def __init__(self, ms):
        self.ms = ms
        self._keep = [np.ascontiguousarray(ms.verts, np.float32), np.ascontiguousarray(ms.vert_begin, np.int64),
                      np.ascontiguousarray(ms.vert_count, np.int32), np.ascontiguousarray(ms.tris, np.int32),
                      np.ascontiguousarray(ms.tri_begin, np.int64), np.ascontiguousarray(ms.tri_count, np.int32),
                      np.ascontiguousarray(ms.parent, np.int32)]
        k = self._keep
        self.c = _Set(ms.n_objects, ms.n_lods, *[a.ctypes.data for a in k])

    @property
    def ref(self):
        return ctypes.byref(self.c)


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---------------------------------------------------------------------------
# geometry primitives (thin wrappers, used by the pins)
# ---------------------------------------------------------------------------
def orient3d(a, b, c, d) -> int:
    a, b, c, d = (np.asarray(x, np.float64) for x in (a, b, c, d))
    return lib().oracle_orient3d(_p(a), _p(b), _p(c), _p(d))


def orient2d(a, b, c, i=0, j=1) -> int:
    a, b, c = (np.asarray(x, np.float64) for x in (a, b, c))
    return lib().oracle_orient2d(_p(a), _p(b), _p(c), i, j)


def tri_tri_intersect(t1, t2) -> bool:
    t1 = np.ascontiguousarray(t1, np.float32).reshape(9)
    t2 = np.ascontiguousarray(t2, np.float32).reshape(9)
    fp = ctypes.POINTER(ctypes.c_float)
    return bool(lib().oracle_tri_tri_intersect(t1.ctypes.data_as(fp), t2.ctypes.data_as(fp)))


def tri_tri_dist(t1, t2) -> float:
    t1 = np.ascontiguousarray(t1, np.float32).reshape(9)
    t2 = np.ascontiguousarray(t2, np.float32).reshape(9)
    fp = ctypes.POINTER(ctypes.c_float)
    return float(lib().oracle_tri_tri_dist(t1.ctypes.data_as(fp), t2.ctypes.data_as(fp), None))


def tri_tri_batch(t1, t2, threads: int = 0):
    """(d, hit) for many triangle pairs ([n, 9] or [n, 3, 3] float32 each)."""
    t1 = np.ascontiguousarray(t1, np.float32).reshape(-1, 9)
    t2 = np.ascontiguousarray(t2, np.float32).reshape(-1, 9)
    n = len(t1)
    d = np.empty(n, np.float64)
    h = np.zeros(n, np.int8)
    if n:
        lib().oracle_tri_tri_batch(n, t1.ctypes.data, t2.ctypes.data, d.ctypes.data, h.ctypes.data, int(threads))
    return d, h.astype(bool)


def pt_tri(p, a, b, c) -> float:
    p, a, b, c = (np.asarray(x, np.float64) for x in (p, a, b, c))
    return float(lib().oracle_pt_tri(_p(p), _p(a), _p(b), _p(c)))


def seg_seg(p0, p1, q0, q1) -> float:
    p0, p1, q0, q1 = (np.asarray(x, np.float64) for x in (p0, p1, q0, q1))
    return float(lib().oracle_seg_seg(_p(p0), _p(p1), _p(q0), _p(q1)))


# ---------------------------------------------------------------------------
# object level
# ---------------------------------------------------------------------------
def object_distance(R: OSet, r: int, S: OSet, s: int, lod: int | None = None, mode: int = 1):
    """(d, hit) of objects r and s at a LoD (default: finest)."""
    lr = R.ms.n_lods - 1 if lod is None else lod
    ls = S.ms.n_lods - 1 if lod is None else lod
    h = ctypes.c_int(0)
    d = lib().oracle_object_distance(R.ref, int(r), lr, S.ref, int(s), ls, int(mode), ctypes.byref(h))
    return float(d), bool(h.value)


def pair_distances(R: OSet, S: OSet, rr, ss, lod: int = -1, mode: int = 1, threads: int = 0):
    """Finest-LoD distances and exact meet flags for the pairs (rr[k], ss[k])."""
    rr = np.ascontiguousarray(rr, np.int32)
    ss = np.ascontiguousarray(ss, np.int32)
    d = np.empty(len(rr), np.float64)
    h = np.zeros(len(rr), np.int8)
    if len(rr):
        lib().oracle_pair_distances(R.ref, S.ref, len(rr), rr.ctypes.data, ss.ctypes.data, int(lod), int(mode),
                                    int(threads), d.ctypes.data, h.ctypes.data)
    return d, h.astype(bool)


def pair_distances_counted(R: OSet, S: OSet, rr, ss, threads: int = 0):
    """pair_distances (finest LoD, culled scan) plus the number of facet pairs
    the scan evaluated for each object pair."""
    rr = np.ascontiguousarray(rr, np.int32)
    ss = np.ascontiguousarray(ss, np.int32)
    d = np.empty(len(rr), np.float64)
    h = np.zeros(len(rr), np.int8)
    ev = np.zeros(len(rr), np.int64)
    if len(rr):
        lib().oracle_pair_distances_counted(R.ref, S.ref, len(rr), rr.ctypes.data, ss.ctypes.data, -1, 1,
                                            int(threads), d.ctypes.data, h.ctypes.data, ev.ctypes.data)
    return d, h.astype(bool), ev


def mbbs(S: OSet, anchors: bool = True):
    """(mbb [n, 6] lo|hi, anchor [n, 3]) in FP64 (anchor None when
    anchors=False)."""
    n = S.ms.n_objects
    box = np.empty((n, 6), np.float64)
    anc = np.empty((n, 3), np.float64) if anchors else None
    if n:
        lib().oracle_mbb_all(S.ref, box.ctypes.data, anc.ctypes.data if anchors else None)
    return box, anc


def mindist(boxA, boxB):
    """MINDIST between every box of A and every box of B (FP64, [nA, nB])."""
    g = np.maximum(0.0, np.maximum(boxB[None, :, :3] - boxA[:, None, 3:], boxA[:, None, :3] - boxB[None, :, 3:]))
    return np.sqrt(np.sum(g * g, -1))


def hd_ph(S: OSet, obj: int, lod: int, m: int = 8):
    """Reference per-facet (hd, ph) of one object at one LoD (FP64)."""
    n = int(S.ms.tri_count[obj * S.ms.n_lods + lod])
    hd = np.zeros(n, np.float64)
    ph = np.zeros(n, np.float64)
    rc = lib().oracle_hd_ph(S.ref, int(obj), int(lod), int(m), hd.ctypes.data, ph.ctypes.data)
    if rc != 0:
        raise ValueError("broken parent chain")
    return hd, ph


def lod_bounds(R: OSet, r, S: OSet, s, lod, hdr, phr, hds, phs):
    """(lb, ub) of Eq. (2) and Eq. (1) at one LoD, every facet pair."""
    hdr, phr, hds, phs = (np.ascontiguousarray(x, np.float64) for x in (hdr, phr, hds, phs))
    lb = ctypes.c_double()
    ub = ctypes.c_double()
    lib().oracle_lod_bounds(R.ref, int(r), S.ref, int(s), int(lod), hdr.ctypes.data, phr.ctypes.data,
                            hds.ctypes.data, phs.ctypes.data, ctypes.byref(lb), ctypes.byref(ub))
    return lb.value, ub.value


def pair_scale(boxR, boxS):
    """Coordinate magnitude M of a pair (largest absolute MBB coordinate)."""
    return np.maximum(np.abs(boxR).max(-1), np.abs(boxS).max(-1))


# ---------------------------------------------------------------------------
# the three joins (Section 3: intersection, within-tau, k-NN)
# ---------------------------------------------------------------------------
NEAR_TIE_REL = 1e-12


def join_within(R: OSet, S: OSet, tau: float, mode: int = 1, threads: int = 0, r_subset=None):
    """{(r, s): d(r, s) <= tau}; tau == 0 means "the surfaces meet" (exact).

    Object pairs whose MBBs are farther apart than tau are skipped (exact:
    a surface lies inside its MBB).  Returns a dict with the sorted pairs,
    their distances, the number of near ties |d - tau| <= 1e-12 max(M, tau)
    and the candidate count.
    """
    bR, _ = mbbs(R)
    bS, _ = mbbs(S)
    rs = np.arange(R.ms.n_objects) if r_subset is None else np.asarray(r_subset)
    cr, cs = [], []
    for c0 in range(0, len(rs), 4096):
        blk = rs[c0:c0 + 4096]
        md = mindist(bR[blk], bS)
        i, j = np.nonzero(md <= tau)
        cr.append(blk[i])
        cs.append(j)
    cr = np.concatenate(cr).astype(np.int32) if cr else np.zeros(0, np.int32)
    cs = np.concatenate(cs).astype(np.int32) if cs else np.zeros(0, np.int32)
    d, hit = pair_distances(R, S, cr, cs, -1, mode, threads)
    keep = hit if tau == 0.0 else (d <= tau)
    M = pair_scale(bR[cr], bS[cs])
    near = np.abs(d - tau) <= NEAR_TIE_REL * np.maximum(M, tau)
    near_ties = int(np.sum(near & ~(hit & (tau == 0.0))))
    if tau == 0.0:
        near_ties = int(np.sum((d == 0.0) != hit)) + int(np.sum(~hit & (d <= NEAR_TIE_REL * M)))
    order = np.lexsort((cs[keep], cr[keep]))
    return dict(r=cr[keep][order], s=cs[keep][order], d=d[keep][order], near_ties=near_ties,
                n_candidates=len(cr), cand_r=cr, cand_s=cs, cand_d=d, cand_hit=hit)


def join_intersect(R: OSet, S: OSet, mode: int = 1, threads: int = 0, r_subset=None):
    return join_within(R, S, 0.0, mode, threads, r_subset)


def join_knn(R: OSet, S: OSet, k: int, threads: int = 0, r_subset=None, batch: int = 8):
    """For each r: the first min(k, |S|) objects of S ordered by (d(r,s), s).

    s is visited in ascending MINDIST order (ties by id); the scan stops once
    MINDIST exceeds the current k-th distance, which cannot change the answer
    because d >= MINDIST.  Returns per-r lists and a near-tie count (adjacent
    result distances, or the k-th and the next, within 1e-12 M).
    """
    bR, _ = mbbs(R)
    bS, _ = mbbs(S)
    nS = S.ms.n_objects
    rs = np.arange(R.ms.n_objects) if r_subset is None else np.asarray(r_subset)
    out_s, out_d = {}, {}
    near = 0
    M_all = float(max(np.abs(bR).max(initial=0.0), np.abs(bS).max(initial=0.0)))
    for r in rs:
        md = mindist(bR[r:r + 1], bS)[0]
        order = np.lexsort((np.arange(nS), md))
        found = []  # (d, s)
        pos = 0
        while pos < nS:
            blk = order[pos:pos + batch]
            if len(found) >= k:
                kth = sorted(found)[k - 1][0]
                blk = blk[md[blk] <= kth]  # ascending MINDIST: a prefix
                if len(blk) == 0:
                    break
            d, hit = pair_distances(R, S, np.full(len(blk), r), blk, -1, 1, threads)
            found += [(float(x), int(s)) for x, s in zip(d, blk)]
            pos += batch
        found.sort()
        res = found[:min(k, nS)]
        out_s[int(r)] = np.array([s for _, s in res], np.int32)
        out_d[int(r)] = np.array([x for x, _ in res], np.float64)
        ds = [x for x, _ in found[:min(k, nS) + 1]]
        for a, b in zip(ds, ds[1:]):
            if 0.0 < abs(b - a) <= NEAR_TIE_REL * max(M_all, abs(a)):
                near += 1
    return dict(s=out_s, d=out_d, near_ties=near)


# ---------------------------------------------------------------------------
# Algorithm 6 (k-NN object-pair pruning), corrected reading
# ---------------------------------------------------------------------------
UNDECIDED, CONFIRMED, REMOVED = 0, 1, 2


def surely_precedes(lb, ub, ids, n, m) -> bool:
    """Candidate n comes before m in the (d, id) order for every d in the
    intervals: ub_n < lb_m, or ub_n == lb_m and id_n < id_m."""
    return ub[n] < lb[m] or (ub[n] == lb[m] and ids[n] < ids[m])


def knn_prune(lb, ub, ids, status, k_left):
    """One pruning round over one query's candidates (Algorithm 6).

    Reading taken (the printed rule cannot confirm a clear nearest neighbour,
    counts ties both ways and reads statuses that other threads are writing):
    among the undecided set U (decided from a snapshot), with
    kLeft = k - #confirmed,
      CONFIRM m if #{n in U\\m : not (m surely precedes n)} < kLeft,
      REMOVE  m if #{n in U\\m : n surely precedes m} >= kLeft.
    Returns the new status array (the input is not modified).
    """
    status = np.asarray(status)
    new = status.copy()
    U = [i for i in range(len(status)) if status[i] == UNDECIDED]
    if k_left <= 0:
        for m in U:
            new[m] = REMOVED
        return new
    for m in U:
        maybe_before = sum(1 for n in U if n != m and not surely_precedes(lb, ub, ids, m, n))
        surely_before = sum(1 for n in U if n != m and surely_precedes(lb, ub, ids, n, m))
        if maybe_before < k_left:
            new[m] = CONFIRMED
        elif surely_before >= k_left:
            new[m] = REMOVED
    return new


# ---------------------------------------------------------------------------
# LoD-skip MLP 16-64-64-4 (ReLU), FP64 reference
# ---------------------------------------------------------------------------
def mlp_forward(params, x):
    W1, b1, W2, b2, W3, b3 = params
    z1 = x @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    logits = h2 @ W3 + b3
    return logits, (x, z1, h1, z2, h2)


def mlp_loss_grad(params, x, y):
    """Mean softmax cross-entropy over the batch and its gradients."""
    W1, b1, W2, b2, W3, b3 = params
    logits, (x, z1, h1, z2, h2) = mlp_forward(params, x)
    m = logits.max(1, keepdims=True)
    e = np.exp(logits - m)
    p = e / e.sum(1, keepdims=True)
    B = len(x)
    loss = float(np.mean(-np.log(p[np.arange(B), y])))
    g = p.copy()
    g[np.arange(B), y] -= 1.0
    g /= B
    gW3 = h2.T @ g
    gb3 = g.sum(0)
    gh2 = g @ W3.T
    gz2 = gh2 * (z2 > 0)
    gW2 = h1.T @ gz2
    gb2 = gz2.sum(0)
    gh1 = gz2 @ W2.T
    gz1 = gh1 * (z1 > 0)
    gW1 = x.T @ gz1
    gb1 = gz1.sum(0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]
