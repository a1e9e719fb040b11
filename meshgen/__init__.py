"""Seeded synthetic triangle-mesh generators shared by the tests, the bench and
the oracle checks.

This module only *creates inputs*: vertex positions, triangle connectivity and
the parent maps that relate the triangles of consecutive levels of detail
(LoDs).  It holds none of the join's arithmetic (no distances, bounds or
predicates), so both the CPU oracle and the GPU library can consume what it
produces without sharing any method code.

Shapes follow the workloads of the paper (Section 4, "Datasets"): small
nucleus-like blobs and long vessel-like tubes, each with a coarse-to-fine
sequence of LoDs whose finest level is the original mesh (Section 2.1,
"Level of Detail").  Coarse vertices are always a subset of the fine ones, so
every object stores one vertex array and one triangle list per LoD.

Mesh-set layout (all numpy arrays, object-major):
  verts      float32 [V, 3]     all objects' vertices, concatenated
  vert_begin int64   [n]        first vertex of each object
  vert_count int32   [n]
  tris       int32   [T, 3]     vertex indices local to the object's range;
                                blocks may be shared by many objects
  tri_begin  int64   [n * L]    (object, LoD) -> first triangle in ``tris``
  tri_count  int32   [n * L]
  parent     int32   [T]        for a triangle of LoD l > 0: index (within
                                the same object's LoD l-1 list) of the coarse
                                triangle it refines; -1 at LoD 0
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math
import mmap
import multiprocessing
import time
import os

import numpy as np

__all__ = [
    "MeshSet", "rng_for", "icosphere_template", "tube_template",
    "make_blobs", "make_tubes", "concat", "config_small", "config_multilod",
    "cube_mesh", "single_object", "CONFIGS",
]


# Large sets are built in blocks (noise values per blob block, tubes per
# tube block); the arrays do not depend on these sizes.
BLOB_BLOCK_VALUES = 1 << 22
TUBE_BLOCK = 4096


def default_workers() -> int:
    """Worker processes for large sets: the host's CPU share (at most 16)."""
    env = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return max(1, min(16, env if env > 0 else (os.cpu_count() or 1)))


def _shared_array(shape, dtype):
    """A zeroed array in anonymous shared memory: processes forked after its
    creation write into the same pages."""
    nbytes = int(np.prod(shape)) * np.dtype(dtype).itemsize
    mm = mmap.mmap(-1, max(nbytes, 1))
    return np.frombuffer(mm, dtype=dtype, count=int(np.prod(shape))).reshape(shape)


_FORK_JOB = None


def _fork_entry(item):
    fn, args = _FORK_JOB
    fn(*args, *item)
    return 0


def _gpu_opened() -> bool:
    """Whether this process holds a GPU device file open (a process that has
    touched the GPU is never forked)."""
    try:
        for fd in os.listdir("/proc/self/fd"):
            try:
                target = os.readlink(os.path.join("/proc/self/fd", fd))
            except OSError:
                continue
            if target == "/dev/kfd" or target.startswith("/dev/dri/"):
                return True
    except OSError:
        return True
    return False


def _run_blocks(fn, args, blocks, workers, progress=None, label=""):
    """fn(*args, *block) for every block, in forked worker processes (which
    write their results into shared arrays among ``args``), or in threads of
    this process when it has opened the GPU (a profiler can open it before
    the program starts), or serially for one worker.  The blocks write
    disjoint slices, so the arrays do not depend on the schedule.  Without
    forked workers, progress(label done/total) is reported every few
    seconds."""
    global _FORK_JOB
    if workers <= 1 or len(blocks) <= 1 or _gpu_opened():
        from multiprocessing.pool import ThreadPool
        total = blocks[-1][1] if blocks else 0
        last = time.time()
        done = 0
        if workers <= 1 or len(blocks) <= 1:
            it = (fn(*args, *b) or b for b in blocks)
            pool = None
        else:
            pool = ThreadPool(min(workers, len(blocks)))
            it = pool.imap_unordered(lambda b: (fn(*args, *b), b)[1], blocks)
        try:
            for b in it:
                done += b[1] - b[0]
                if progress is not None and time.time() - last > 5.0:
                    progress(f"{label} {done}/{total}")
                    last = time.time()
        finally:
            if pool is not None:
                pool.close()
                pool.join()
        return
    _FORK_JOB = (fn, args)
    try:
        with multiprocessing.get_context("fork").Pool(min(workers, len(blocks))) as pool:
            pool.map(_fork_entry, blocks, chunksize=1)
    finally:
        _FORK_JOB = None


def rng_for(seed: int, stream: int) -> np.random.Generator:
    """PCG64 stream ``stream`` of experiment seed ``seed``."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


@dataclass
class MeshSet:
    n_objects: int
    n_lods: int
    verts: np.ndarray
    vert_begin: np.ndarray
    vert_count: np.ndarray
    tris: np.ndarray
    tri_begin: np.ndarray
    tri_count: np.ndarray
    parent: np.ndarray
    kind: np.ndarray = field(default=None)  # 0 = blob, 1 = tube, 2 = other

    def object_verts(self, i: int) -> np.ndarray:
        b = int(self.vert_begin[i])
        return self.verts[b:b + int(self.vert_count[i])]

    def object_tris(self, i: int, lod: int) -> np.ndarray:
        k = i * self.n_lods + lod
        b = int(self.tri_begin[k])
        return self.tris[b:b + int(self.tri_count[k])]

    def object_parent(self, i: int, lod: int) -> np.ndarray:
        k = i * self.n_lods + lod
        b = int(self.tri_begin[k])
        return self.parent[b:b + int(self.tri_count[k])]

    def facets(self, i: int, lod: int) -> np.ndarray:
        """[F, 3, 3] float32 triangle corners of object i at a LoD."""
        return self.object_verts(i)[self.object_tris(i, lod)]

    def total_facets(self, lod: int | None = None) -> int:
        c = self.tri_count.reshape(self.n_objects, self.n_lods)
        return int(c.sum() if lod is None else c[:, lod].sum())

    def subset(self, idx) -> "MeshSet":
        """Objects ``idx`` (in that order) as a new set; shares nothing."""
        idx = np.asarray(idx, dtype=np.int64)
        L = self.n_lods
        vb = self.vert_begin[idx]
        vc = self.vert_count[idx].astype(np.int64)
        new_vb = np.zeros(len(idx), np.int64)
        if len(idx):
            new_vb[1:] = np.cumsum(vc)[:-1]
        verts = np.concatenate([self.verts[b:b + c] for b, c in zip(vb, vc)]) if len(idx) else np.zeros((0, 3), np.float32)
        keys = (idx[:, None] * L + np.arange(L)[None, :]).reshape(-1)
        tb = self.tri_begin[keys]
        tc = self.tri_count[keys].astype(np.int64)
        # keep sharing of identical blocks
        uniq, inv = np.unique(np.stack([tb, tc], 1), axis=0, return_inverse=True) if len(keys) else (np.zeros((0, 2), np.int64), np.zeros(0, np.int64))
        inv = np.asarray(inv).reshape(-1)
        blocks_t, blocks_p, starts = [], [], []
        pos = 0
        for b, c in uniq:
            blocks_t.append(self.tris[b:b + c])
            blocks_p.append(self.parent[b:b + c])
            starts.append(pos)
            pos += c
        starts = np.asarray(starts, np.int64)
        tris = np.concatenate(blocks_t) if blocks_t else np.zeros((0, 3), np.int32)
        parent = np.concatenate(blocks_p) if blocks_p else np.zeros(0, np.int32)
        return MeshSet(len(idx), L, np.ascontiguousarray(verts, np.float32), new_vb,
                       self.vert_count[idx].astype(np.int32), np.ascontiguousarray(tris, np.int32),
                       starts[inv] if len(keys) else np.zeros(0, np.int64), tc.astype(np.int32),
                       np.ascontiguousarray(parent, np.int32),
                       None if self.kind is None else self.kind[idx].copy())

    def nbytes(self) -> int:
        return sum(a.nbytes for a in (self.verts, self.vert_begin, self.vert_count, self.tris,
                                      self.tri_begin, self.tri_count, self.parent))


# ---------------------------------------------------------------------------
# Icosphere: recursive 1->4 midpoint subdivision of an icosahedron, new
# vertices appended so that level l's vertices are the first 10*4^l+2 entries.
# ---------------------------------------------------------------------------
_ICO_CACHE: dict = {}


def _icosahedron():
    from scipy.spatial import ConvexHull
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = []
    for a in (-1.0, 1.0):
        for b in (-p, p):
            v += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    v = np.asarray(v, np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    hull = ConvexHull(v)
    faces = []
    for f in hull.simplices:
        a, b, c = v[f]
        if np.dot(np.cross(b - a, c - a), a + b + c) < 0:
            f = f[[0, 2, 1]]
        faces.append(f)
    faces = np.asarray(sorted(map(tuple, faces)), np.int64)
    return v, faces


def icosphere_template(level: int):
    """Unit icosphere levels 0..level.

    Returns (verts[float64, V_level x 3], [faces_0, ..., faces_level],
    [parents_0 (all -1), ..., parents_level]).
    """
    if level in _ICO_CACHE:
        return _ICO_CACHE[level]
    v, f = _icosahedron()
    verts = [tuple(x) for x in v]
    faces = [f.astype(np.int32)]
    parents = [np.full(len(f), -1, np.int32)]
    for _ in range(level):
        mid = {}
        cur = faces[-1]
        nf = np.empty((len(cur) * 4, 3), np.int32)
        par = np.repeat(np.arange(len(cur), dtype=np.int32), 4)

        def m(i, j):
            key = (i, j) if i < j else (j, i)
            if key not in mid:
                x = (np.asarray(verts[i]) + np.asarray(verts[j])) * 0.5
                x = x / np.linalg.norm(x)
                mid[key] = len(verts)
                verts.append(tuple(x))
            return mid[key]

        for t, (a, b, c) in enumerate(cur):
            ab, bc, ca = m(a, b), m(b, c), m(c, a)
            nf[4 * t + 0] = (a, ab, ca)
            nf[4 * t + 1] = (ab, b, bc)
            nf[4 * t + 2] = (ca, bc, c)
            nf[4 * t + 3] = (ab, bc, ca)
        faces.append(nf)
        parents.append(par)
    out = (np.asarray(verts, np.float64), faces, parents)
    _ICO_CACHE[level] = out
    return out


# ---------------------------------------------------------------------------
# Tube: regular octagon swept along a cubic Bezier in a rotation-minimising
# frame.  Rings 0..n_seg (8 vertices each) then two cap centres.  LoD l keeps
# every step_l-th ring, step_l = 4^(L-1-l); ends are closed by 8-triangle fans.
# ---------------------------------------------------------------------------
_TUBE_CACHE: dict = {}


def tube_template(n_seg: int, n_lods: int):
    """Connectivity of a capped 8-sided tube with ``n_seg`` finest segments.

    Returns ([tris_0..tris_{L-1}] int32, [parent_0..parent_{L-1}] int32).
    """
    key = (n_seg, n_lods)
    if key in _TUBE_CACHE:
        return _TUBE_CACHE[key]
    step0 = 4 ** (n_lods - 1)
    if n_seg % step0:
        raise ValueError("n_seg must be a multiple of 4^(n_lods-1)")
    c0 = 8 * (n_seg + 1)
    c1 = c0 + 1
    tris_l, par_l = [], []
    q = np.arange(8)
    qn = (q + 1) % 8
    for lod in range(n_lods):
        step = 4 ** (n_lods - 1 - lod)
        nsl = n_seg // step
        m = np.arange(nsl)
        i = (m * step)[:, None]
        j = ((m + 1) * step)[:, None]
        v00 = 8 * i + q[None, :]
        v01 = 8 * i + qn[None, :]
        v10 = 8 * j + q[None, :]
        v11 = 8 * j + qn[None, :]
        t0 = np.stack([v00, v01, v11], -1)
        t1 = np.stack([v00, v11, v10], -1)
        quads = np.stack([t0, t1], 2).reshape(-1, 3)          # (m, q, t) order
        start = np.stack([np.full(8, c0), qn, q], -1)            # ring 0
        last = 8 * n_seg
        end = np.stack([np.full(8, c1), last + q, last + qn], -1)
        tris = np.concatenate([quads, start, end]).astype(np.int32)
        if lod == 0:
            par = np.full(len(tris), -1, np.int32)
        else:
            mm = np.repeat(np.arange(nsl), 16)
            qq = np.tile(np.repeat(np.arange(8), 2), nsl)
            tt = np.tile(np.array([0, 1]), nsl * 8)
            coarse_m = mm // 4
            sub = mm % 4
            # centroid of the fine triangle in the coarse quad's (u, v) square:
            # tri 0 -> (u0 + h/3, 2/3), tri 1 -> (u0 + 2h/3, 1/3), h = 1/4.
            uc = sub / 4.0 + np.where(tt == 0, 1.0 / 12.0, 2.0 / 12.0)
            vc = np.where(tt == 0, 2.0 / 3.0, 1.0 / 3.0)
            coarse_t = np.where(vc >= uc, 0, 1)
            pq = ((coarse_m * 8 + qq) * 2 + coarse_t).astype(np.int32)
            nsc = nsl // 4
            caps = np.concatenate([16 * nsc + np.arange(8), 16 * nsc + 8 + np.arange(8)]).astype(np.int32)
            par = np.concatenate([pq, caps]).astype(np.int32)
        tris_l.append(tris)
        par_l.append(par)
    _TUBE_CACHE[key] = (tris_l, par_l)
    return tris_l, par_l


def _bezier(P, u):
    """P: [n, 4, 3], u: [n, k] -> points [n, k, 3] and derivatives."""
    u = u[..., None]
    w = 1.0 - u
    pts = (w ** 3) * P[:, None, 0] + 3 * w * w * u * P[:, None, 1] + 3 * w * u * u * P[:, None, 2] + (u ** 3) * P[:, None, 3]
    der = 3 * w * w * (P[:, None, 1] - P[:, None, 0]) + 6 * w * u * (P[:, None, 2] - P[:, None, 1]) + 3 * u * u * (P[:, None, 3] - P[:, None, 2])
    return pts, der


def _unit(x):
    return x / np.linalg.norm(x, axis=-1, keepdims=True)


def make_tubes(rng, centres, n_seg: int, n_lods: int, length_range=(20.0, 80.0), radius: float = 1.0,
               n_seg_per_object=None, progress=None, workers=1):
    """Tubes with MBB centres at ``centres`` (float64 [n, 3]).

    Draw order per call: directions (n x 3 normals x 3), lengths (n).
    ``n_seg_per_object`` (optional int array) overrides ``n_seg`` per tube.
    """
    centres = np.asarray(centres, np.float64)
    n = len(centres)
    d0 = _unit(rng.normal(size=(n, 3)))
    d1 = _unit(d0 + rng.normal(scale=0.5, size=(n, 3)))
    d2 = _unit(d1 + rng.normal(scale=0.5, size=(n, 3)))
    lengths = rng.uniform(length_range[0], length_range[1], size=n)
    segs = np.full(n, n_seg, np.int64) if n_seg_per_object is None else np.asarray(n_seg_per_object, np.int64)
    step = TUBE_BLOCK
    if workers > 1 and n > step and n_seg_per_object is None:
        # equal tubes: blocks in worker processes, into one shared [n, V, 3]
        out = _shared_array((n, 8 * (n_seg + 1) + 2, 3), np.float32)
        _run_blocks(_tube_block_into, (out, centres, d0, d1, d2, lengths, segs, radius),
                    [(c0, min(n, c0 + step)) for c0 in range(0, n, step)], workers, progress, "tubes")
        if progress is not None:
            progress(f"tubes {n}/{n}")
        return out, segs
    per_obj = [None] * n
    # the shapes are fixed by the draws above; build them in blocks of tubes
    for c0 in range(0, n, step):
        c1 = min(n, c0 + step)
        _tube_block(per_obj, c0, centres[c0:c1], d0[c0:c1], d1[c0:c1], d2[c0:c1], lengths[c0:c1], segs[c0:c1],
                    radius)
        if progress is not None:
            progress(f"tubes {c1}/{n}")
    return per_obj, segs


def _tube_block_into(out, centres, d0, d1, d2, lengths, segs, radius, c0, c1):
    _tube_block(out, c0, centres[c0:c1], d0[c0:c1], d1[c0:c1], d2[c0:c1], lengths[c0:c1], segs[c0:c1], radius)


def _tube_block(per_obj, c0, centres, d0, d1, d2, lengths, segs, radius):
    n = len(centres)
    P = np.zeros((n, 4, 3))
    P[:, 1] = d0
    P[:, 2] = d0 + d1
    P[:, 3] = d0 + d1 + d2
    K = 2048
    uu = np.broadcast_to(np.linspace(0.0, 1.0, K), (n, K))
    pts, _ = _bezier(P, uu)
    seglen = np.linalg.norm(np.diff(pts, axis=1), axis=-1)
    cum = np.concatenate([np.zeros((n, 1)), np.cumsum(seglen, 1)], 1)
    scale = lengths / cum[:, -1]
    P *= scale[:, None, None]
    cum *= scale[:, None]
    groups = {}
    for t in range(n):
        groups.setdefault(int(segs[t]), []).append(t)
    theta = 2.0 * np.pi * np.arange(8) / 8.0
    for ns, ids in groups.items():
        ids = np.asarray(ids)
        m = len(ids)
        s_targets = np.linspace(0.0, 1.0, ns + 1)[None, :] * lengths[ids][:, None]
        # invert arc length per tube
        u = np.empty((m, ns + 1))
        for k, t in enumerate(ids):
            u[k] = np.interp(s_targets[k], cum[t], np.linspace(0.0, 1.0, K))
        x, der = _bezier(P[ids], u)
        tan = _unit(der)
        # rotation-minimising frame by double reflection
        r = np.empty_like(tan)
        ref = np.where(np.abs(tan[:, 0, 0:1]) < 0.9, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))
        r0 = ref - np.sum(ref * tan[:, 0], -1, keepdims=True) * tan[:, 0]
        r[:, 0] = _unit(r0)
        for i in range(ns):
            v1 = x[:, i + 1] - x[:, i]
            c1 = np.sum(v1 * v1, -1, keepdims=True)
            rl = r[:, i] - (2.0 / c1) * np.sum(v1 * r[:, i], -1, keepdims=True) * v1
            tl = tan[:, i] - (2.0 / c1) * np.sum(v1 * tan[:, i], -1, keepdims=True) * v1
            v2 = tan[:, i + 1] - tl
            c2 = np.sum(v2 * v2, -1, keepdims=True)
            c2 = np.where(c2 > 0, c2, 1.0)
            r[:, i + 1] = _unit(rl - (2.0 / c2) * np.sum(v2 * rl, -1, keepdims=True) * v2)
        s = np.cross(tan, r)
        ring = x[:, :, None, :] + radius * (np.cos(theta)[None, None, :, None] * r[:, :, None, :]
                                           + np.sin(theta)[None, None, :, None] * s[:, :, None, :])
        ring = ring.reshape(m, (ns + 1) * 8, 3)
        v = np.concatenate([ring, x[:, 0:1], x[:, ns:ns + 1]], 1)
        lo, hi = v.min(1), v.max(1)
        v += (centres[ids] - 0.5 * (lo + hi))[:, None, :]
        for k, t in enumerate(ids):
            per_obj[c0 + t] = v[k].astype(np.float32)


def _blob_block(v, state, tv, centres, radii, noise, nv, i0, i1):
    g = np.random.PCG64()
    g.state = state
    g.advance(i0 * nv)
    noise_v = np.random.Generator(g).uniform(noise[0], noise[1], size=(i1 - i0, nv))
    v[i0:i1] = tv[None, :, :] * (noise_v * radii[i0:i1, None])[:, :, None] + centres[i0:i1, None, :]


def make_blobs(rng, centres, radii, level_min: int, level_max: int, noise=(0.9, 1.1), progress=None, workers=1):
    """Perturbed icospheres; LoD l is subdivision level level_min + l.

    Each finest vertex is scaled radially by U(noise) (coarse vertices are a
    subset of the finest ones and share that noise), then by the radius, then
    moved to the centre.  Draw order: noise (n x V).
    """
    centres = np.asarray(centres, np.float64)
    radii = np.asarray(radii, np.float64)
    n = len(centres)
    tv, faces, parents = icosphere_template(level_max)
    nv = 10 * 4 ** level_max + 2
    # generated in row blocks (the noise stream is the same as one n x V draw)
    step = max(1, BLOB_BLOCK_VALUES // nv)
    if workers > 1 and n > step and isinstance(rng.bit_generator, np.random.PCG64):
        # Each block draws its noise from a copy of the generator advanced by
        # the draws of the blocks before it (one 64-bit output per uniform
        # value), so the arrays are those of one pass.
        v = _shared_array((n, nv, 3), np.float32)
        state = rng.bit_generator.state
        _run_blocks(_blob_block, (v, state, tv[:nv], centres, radii, noise, nv),
                    [(i0, min(n, i0 + step)) for i0 in range(0, n, step)], workers, progress, "blobs")
        rng.bit_generator.advance(n * nv)
        if progress is not None:
            progress(f"blobs {n}/{n}")
    else:
        v = np.empty((n, nv, 3), np.float32)
        for i0 in range(0, n, step):
            i1 = min(n, i0 + step)
            noise_v = rng.uniform(noise[0], noise[1], size=(i1 - i0, nv))
            v[i0:i1] = tv[None, :nv, :] * (noise_v * radii[i0:i1, None])[:, :, None] + centres[i0:i1, None, :]
            if progress is not None and (i1 == n or (i0 // step) % 64 == 63):
                progress(f"blobs {i1}/{n}")
    lods = list(range(level_min, level_max + 1))
    tris = [faces[l] for l in lods]
    par = [parents[l] if i > 0 else np.full(len(faces[l]), -1, np.int32) for i, l in enumerate(lods)]
    return v, tris, par


def _assemble(per_obj_verts, per_obj_template, templates, n_lods, kind):
    """Build a MeshSet from per-object vertex arrays and shared templates.

    templates: dict key -> (list of tris per LoD, list of parents per LoD)
    """
    n = len(per_obj_verts)
    if isinstance(per_obj_verts, np.ndarray) and per_obj_verts.ndim == 3:
        # every object has the same vertex count: one reshape, no copy
        vc = np.full(n, per_obj_verts.shape[1], np.int64)
        verts = per_obj_verts.reshape(-1, 3)
    else:
        vc = np.array([len(v) for v in per_obj_verts], np.int64)
        verts = np.concatenate(per_obj_verts).astype(np.float32) if n else np.zeros((0, 3), np.float32)
    vb = np.zeros(n, np.int64)
    if n:
        vb[1:] = np.cumsum(vc)[:-1]
    blocks_t, blocks_p = [], []
    start = {}
    pos = 0
    for key, (tl, pl) in templates.items():
        for l in range(n_lods):
            start[(key, l)] = pos
            blocks_t.append(tl[l])
            blocks_p.append(pl[l])
            pos += len(tl[l])
    tris = np.concatenate(blocks_t).astype(np.int32)
    parent = np.concatenate(blocks_p).astype(np.int32)
    keys = list(templates.keys())
    kid = {k: j for j, k in enumerate(keys)}
    tb_k = np.array([[start[(k, l)] for l in range(n_lods)] for k in keys], np.int64).reshape(len(keys), n_lods)
    tc_k = np.array([[len(templates[k][0][l]) for l in range(n_lods)] for k in keys], np.int32).reshape(len(keys), n_lods)
    if len(keys) == 1:
        obj_k = np.zeros(n, np.int64)
    else:
        obj_k = np.array([kid[k] for k in per_obj_template], np.int64)
    tb = tb_k[obj_k].reshape(-1)
    tc = tc_k[obj_k].reshape(-1)
    return MeshSet(n, n_lods, np.ascontiguousarray(verts), vb, vc.astype(np.int32), np.ascontiguousarray(tris),
                   tb, tc, parent, np.asarray(kind, np.int8))


def blob_set(rng, n, box, level_min, level_max, radius_sigma=None, radius=1.0, progress=None, workers=1):
    """n blobs, centres U(box) then radii then noise (in that draw order)."""
    lo, hi = box
    centres = rng.uniform(lo, hi, size=(n, 3))
    if radius_sigma is None:
        radii = np.full(n, radius)
    else:
        radii = np.exp(rng.normal(0.0, radius_sigma, size=n))
    v, tris, par = make_blobs(rng, centres, radii, level_min, level_max, progress=progress, workers=workers)
    L = level_max - level_min + 1
    templ = {("ico", level_min, level_max): (tris, par)}
    return _assemble(v, [("ico", level_min, level_max)] * n, templ, L, np.zeros(n))


def tube_set(rng, n, box, n_seg, n_lods, length_range=(20.0, 80.0), radius=1.0, progress=None, workers=1):
    """n tubes, centres U(box) then tube shape draws."""
    lo, hi = box
    centres = rng.uniform(lo, hi, size=(n, 3))
    v, segs = make_tubes(rng, centres, n_seg, n_lods, length_range, radius, progress=progress, workers=workers)
    tl, pl = tube_template(n_seg, n_lods)
    templ = {("tube", n_seg, n_lods): (tl, pl)}
    return _assemble(v, [("tube", n_seg, n_lods)] * n, templ, n_lods, np.ones(n))


def concat(a: MeshSet, b: MeshSet) -> MeshSet:
    if a.n_lods != b.n_lods:
        raise ValueError("LoD counts differ")
    return MeshSet(a.n_objects + b.n_objects, a.n_lods, np.concatenate([a.verts, b.verts]),
                   np.concatenate([a.vert_begin, b.vert_begin + len(a.verts)]),
                   np.concatenate([a.vert_count, b.vert_count]), np.concatenate([a.tris, b.tris]),
                   np.concatenate([a.tri_begin, b.tri_begin + len(a.tris)]),
                   np.concatenate([a.tri_count, b.tri_count]), np.concatenate([a.parent, b.parent]),
                   np.concatenate([a.kind, b.kind]))


def single_object(verts, tris_per_lod, parents_per_lod=None) -> MeshSet:
    """A one-object set from explicit arrays (hand-built test cases)."""
    L = len(tris_per_lod)
    if parents_per_lod is None:
        parents_per_lod = [np.full(len(t), -1, np.int32) for t in tris_per_lod]
    tris = np.concatenate([np.asarray(t, np.int32).reshape(-1, 3) for t in tris_per_lod])
    par = np.concatenate([np.asarray(p, np.int32) for p in parents_per_lod])
    tc = np.array([len(np.asarray(t).reshape(-1, 3)) for t in tris_per_lod], np.int32)
    tb = np.zeros(L, np.int64)
    tb[1:] = np.cumsum(tc)[:-1]
    v = np.asarray(verts, np.float32).reshape(-1, 3)
    return MeshSet(1, L, v, np.zeros(1, np.int64), np.array([len(v)], np.int32), tris, tb, tc, par, np.array([2], np.int8))


def objects(list_of_sets) -> MeshSet:
    """Concatenate several MeshSets (same LoD count)."""
    out = list_of_sets[0]
    for s in list_of_sets[1:]:
        out = concat(out, s)
    return out


def orphan_facet_object(height: float = 5.0) -> MeshSet:
    """Two-LoD object whose coarse LoD has a facet no finest facet descends
    from: the finest LoD is the unit square [0,1]^2 at z = 0 (2 triangles);
    the coarse LoD repeats those two (each the parent of its copy) and adds
    a triangle at z = ``height`` with no children."""
    v = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                  [0, 0, height], [1, 0, height], [0, 1, height]], np.float32)
    square = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    coarse = np.concatenate([square, np.array([[4, 5, 6]], np.int32)])
    return single_object(v, [coarse, square], [np.full(3, -1, np.int32), np.array([0, 1], np.int32)])


def orphan_facet_cube(side: float = 10.0) -> MeshSet:
    """Two-LoD object: the finest LoD is the surface of the cube [0, side]^3
    (12 triangles); the coarse LoD repeats them (each the parent of its copy)
    and adds a unit triangle at the cube's centre with no children, far from
    the finest surface yet inside its bounding box."""
    cube = cube_mesh([0, 0, 0], [side, side, side])
    h = 0.5 * side
    extra = np.array([[h, h, h], [h + 1, h, h], [h, h + 1, h]], np.float32)
    v = np.concatenate([cube.verts, extra])
    coarse = np.concatenate([cube.tris, np.array([[8, 9, 10]], np.int32)])
    return single_object(v, [coarse, cube.tris], [np.full(13, -1, np.int32), np.arange(12, dtype=np.int32)])


def cube_mesh(lo, hi) -> MeshSet:
    """Axis-aligned box surface, 8 vertices, 12 triangles, one LoD."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    v = np.array([[lo[0] if (k & 1) == 0 else hi[0], lo[1] if (k & 2) == 0 else hi[1], lo[2] if (k & 4) == 0 else hi[2]]
                  for k in range(8)], np.float32)
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    t = []
    for a, b, c, d in quads:
        t += [(a, b, c), (a, c, d)]
    return single_object(v, [np.asarray(t, np.int32)])


# ---------------------------------------------------------------------------
# Workload configurations (synthetic stand-ins for the paper's datasets).
# ---------------------------------------------------------------------------
def config_small(seed: int = 0, n_r: int = 100, n_s: int = 100, box=15.0):
    """Single-LoD join: icospheres at level 2 (320 triangles), radius 1, noise
    U(0.9, 1.1), centres U([0, box]^3).  R from stream 0, S from stream 1."""
    R = blob_set(rng_for(seed, 0), n_r, (0.0, box), 2, 2)
    S = blob_set(rng_for(seed, 1), n_s, (0.0, box), 2, 2)
    return R, S


def config_multilod(seed: int = 1, n_r: int = 10000, n_s: int = 2000, box=500.0, n_seg=1280, progress=None,
                    workers=1):
    """Multi-LoD join: R = blobs with LoDs at icosphere levels 1..4
    (80/320/1280/5120 triangles), radius lognormal(0, 0.3); S = tubes of
    length U(20, 80), radius 1, 4 LoDs decimated 4x per level (finest n_seg
    segments, 16*n_seg+16 triangles).  Centres U([0, box]^3)."""
    R = blob_set(rng_for(seed, 0), n_r, (0.0, box), 1, 4, radius_sigma=0.3, progress=progress, workers=workers)
    S = tube_set(rng_for(seed, 1), n_s, (0.0, box), n_seg, 4, progress=progress, workers=workers)
    return R, S


def mixed_set(rng, centres, n_lods: int = 4, f_median: float = 7071.0, f_sigma: float = math.log(50.0) / 4,
              f_clip=(1000, 50000), radius_sigma: float = 0.3):
    """Blob/tube mix with lognormal finest facet counts.

    Per object (draw order): kind (blob/tube, 50/50), target finest facet
    count F ~ lognormal(ln f_median, f_sigma) clipped to f_clip.  A blob is
    the icosphere whose finest level (3, 4 or 5: 1280/5120/20480 triangles)
    is nearest to F in log scale, with LoDs at the n_lods levels ending there;
    a tube gets n_seg = F/16 rounded to a multiple of 4^(n_lods-1) segments.
    Then blob radii, blob noise, tube shapes (in that order).
    """
    centres = np.asarray(centres, np.float64)
    n = len(centres)
    kind = rng.integers(0, 2, size=n)
    F = np.clip(np.exp(rng.normal(math.log(f_median), f_sigma, size=n)), f_clip[0], f_clip[1])
    step = 4 ** (n_lods - 1)
    blob_lv = np.clip(np.round(np.log(F / 20.0) / math.log(4.0)), n_lods - 1, 5).astype(int)
    segs = np.clip(np.round(F / 16.0 / step) * step, step, None).astype(int)
    radii = np.exp(rng.normal(0.0, radius_sigma, size=n))
    per_v = [None] * n
    per_key = [None] * n
    templ = {}
    for lv in sorted(set(blob_lv[kind == 0].tolist())):
        ids = np.nonzero((kind == 0) & (blob_lv == lv))[0]
        v, tris, par = make_blobs(rng, centres[ids], radii[ids], lv - n_lods + 1, lv)
        templ[("ico", lv - n_lods + 1, lv)] = (tris, par)
        for k_, i in enumerate(ids):
            per_v[i] = v[k_]
            per_key[i] = ("ico", lv - n_lods + 1, lv)
    tube_ids = np.nonzero(kind == 1)[0]
    if len(tube_ids):
        v, sg = make_tubes(rng, centres[tube_ids], 0, n_lods, n_seg_per_object=segs[tube_ids])
        for k_, i in enumerate(tube_ids):
            ns = int(segs[i])
            key = ("tube", ns, n_lods)
            if key not in templ:
                templ[key] = tube_template(ns, n_lods)
            per_v[i] = v[k_]
            per_key[i] = key
    return _assemble(per_v, per_key, templ, n_lods, kind)


def config_knn(seed: int = 2, n_r: int = 20000, n_s: int = 20000, n_clusters: int = 50, box: float = 2000.0,
               sigma: float = 30.0, progress=None, **kw):
    """Clustered k-NN workload: object centres = one of n_clusters centres
    U([0, box]^3) + N(0, sigma^2); objects from ``mixed_set``.  The cluster
    centres come from stream 2, R from stream 0, S from stream 1."""
    cl = rng_for(seed, 2).uniform(0.0, box, size=(n_clusters, 3))
    out = []
    for stream, n in ((0, n_r), (1, n_s)):
        rng = rng_for(seed, stream)
        c = cl[rng.integers(0, n_clusters, size=n)] + rng.normal(0.0, sigma, size=(n, 3))
        out.append(mixed_set(rng, c, **kw))
        if progress is not None:
            progress(f"{'RS'[stream]}: {n} objects")
    return out[0], out[1]


def config_learned(seed: int = 4, n_r: int = 100000, n_s: int = 20000, box: float = 5000.0, n_seg: int = 1280,
                   progress=None, workers=None):
    """Learned-skip workload: the multi-LoD object shapes at 10x the counts in
    a 5000^3 box, joined within tau = 10."""
    return config_multilod(seed=seed, n_r=n_r, n_s=n_s, box=box, n_seg=n_seg, progress=progress,
                           workers=default_workers() if workers is None else workers)


def config_large(seed: int = 5, n_r: int = 1000000, n_s: int = 200000, box: float = 20000.0, n_seg: int = 1280,
                 progress=None, workers=None):
    """Large intersection workload: 1M blobs (80..5120 triangles) and 200k
    tubes (336..20,496 triangles) in a 20000^3 box, joined at tau = 0.  The
    vertex arrays (55 GB at full size) are built by worker processes into
    shared memory; the arrays do not depend on the worker count."""
    return config_multilod(seed=seed, n_r=n_r, n_s=n_s, box=box, n_seg=n_seg, progress=progress,
                           workers=default_workers() if workers is None else workers)


CONFIGS = {
    "small": dict(builder=config_small, tau=[0.5]),
    "multilod": dict(builder=config_multilod, tau=[0.0, 5.0, 20.0]),
    "knn": dict(builder=config_knn, k=3),
    "learned": dict(builder=config_learned, tau=[10.0]),
    "large": dict(builder=config_large, tau=[0.0]),
}
