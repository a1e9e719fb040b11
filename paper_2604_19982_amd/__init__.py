"""Python binding of the MI355X progressive polyhedral spatial join library.

Argument marshalling only: every step of the join runs in the HIP library
``_lib/libpj.so`` behind the C ABI of ``include/pj.h``.  There is no CPU
fallback; if the library is missing, importing a context raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libpj.so")

PJ_OK = 0
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "DEVICE", 4: "UNSUPPORTED", 5: "INTERNAL"}
PREC = {"fp32": 0, "fp32_band": 0, "fp64": 1}
SCHED = {"batched": 0, "plain": 1}


class PJError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("precision", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("learned_skip", ctypes.c_int32), ("want_dist", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("tile_cull", ctypes.c_int32), ("tile_s", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("host_threads", ctypes.c_int32), ("chunk_tiles", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("mesh_residency", ctypes.c_int32), ("stage_sets", ctypes.c_int32),
                ("filter_mode", ctypes.c_int32), ("knn_prune_host", ctypes.c_int32),
                ("mem_cap_bytes", ctypes.c_int64),
                ("model_path", ctypes.c_char_p), ("log_path", ctypes.c_char_p), ("autotune_path", ctypes.c_char_p),
                ("stream", ctypes.c_void_p), ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN),
                ("alloc_user", ctypes.c_void_p), ("storage_dir", ctypes.c_char_p),
                ("voxels", ctypes.c_int32), ("reserved1", ctypes.c_int32)]


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_objects", ctypes.c_int32), ("n_lods", ctypes.c_int32), ("n_verts", ctypes.c_int64),
                ("n_tris", ctypes.c_int64), ("verts", ctypes.c_void_p), ("vert_begin", ctypes.c_void_p),
                ("vert_count", ctypes.c_void_p), ("tris", ctypes.c_void_p), ("tri_begin", ctypes.c_void_p),
                ("tri_count", ctypes.c_void_p), ("parent", ctypes.c_void_p), ("hd", ctypes.c_void_p),
                ("ph", ctypes.c_void_p), ("hdph_begin", ctypes.c_void_p)]


class Pairs(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("r", ctypes.POINTER(ctypes.c_int32)), ("s", ctypes.POINTER(ctypes.c_int32)),
                ("dist", ctypes.POINTER(ctypes.c_double))]


class Knn(ctypes.Structure):
    _fields_ = [("n_r", ctypes.c_int32), ("k", ctypes.c_int32), ("count", ctypes.POINTER(ctypes.c_int32)),
                ("s", ctypes.POINTER(ctypes.c_int32)), ("dist", ctypes.POINTER(ctypes.c_double))]


class Stats(ctypes.Structure):
    _fields_ = [("t_total_ms", ctypes.c_double), ("t_filter_ms", ctypes.c_double), ("t_refine_ms", ctypes.c_double),
                ("t_band_ms", ctypes.c_double), ("t_ingest_ms", ctypes.c_double),
                ("refine_kernel_ms", ctypes.c_double), ("band_kernel_ms", ctypes.c_double),
                ("refine_launches", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("confirmed_filter", ctypes.c_int64), ("facet_pairs", ctypes.c_int64),
                ("facet_pairs_fp64", ctypes.c_int64), ("tiles", ctypes.c_int64), ("tiles_culled", ctypes.c_int64),
                ("band_pairs", ctypes.c_int64), ("resolved_at_lod", ctypes.c_int64 * 8), ("rounds", ctypes.c_int64),
                ("peak_device_bytes", ctypes.c_int64), ("chunks", ctypes.c_int64),
                ("graph_replays", ctypes.c_int64), ("tile_s_used", ctypes.c_int64),
                ("waves_per_cu_used", ctypes.c_int64), ("t_tune_ms", ctypes.c_double),
                ("staged_bytes", ctypes.c_int64), ("lod_items", ctypes.c_int64 * 8), ("lod_tiles", ctypes.c_int64 * 8),
                ("lod_pairs", ctypes.c_int64 * 8), ("lod_kernel_ms", ctypes.c_double * 8),
                ("collect_launches", ctypes.c_int64), ("collect_pairs", ctypes.c_int64),
                ("collect_kernel_ms", ctypes.c_double), ("collected_pairs", ctypes.c_int64),
                ("collect_overflow", ctypes.c_int64), ("lod_planned_pairs", ctypes.c_int64 * 8),
                ("knn_grid_cells", ctypes.c_int64), ("t_prune_ms", ctypes.c_double), ("t_prep_ms", ctypes.c_double),
                ("vp_pairs", ctypes.c_int64), ("vp_kept", ctypes.c_int64), ("vp_chunks", ctypes.c_int64),
                ("voxel_decided", ctypes.c_int64), ("t_voxel_ms", ctypes.c_double),
                ("planned_sqrt", ctypes.c_double), ("collect_regrow", ctypes.c_int64)]

    def to_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if isinstance(v, ctypes.Array) else v
        return d


class TrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


EXPORTS = ["pj_config_default", "pj_context_create", "pj_context_destroy", "pj_meshes_create", "pj_meshes_destroy",
           "pj_join_within", "pj_join_intersect", "pj_join_knn", "pj_pairs_free", "pj_knn_free", "pj_get_stats",
           "pj_last_error", "pj_train_lod_model", "pj_meshes_boxes", "pj_meshes_hdph", "pj_facet_pairs",
           "pj_pair_bounds", "pj_pair_bounds_noalloc", "pj_mlp_eval", "pj_probe_fma", "pj_probe_copy"]

_lib = None


def lib():
    """Load ``libpj.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2604_19982_amd.build.build()")
        # One HIP runtime per process: torch ships its own libamdhip64 under
        # the same soname.  Loaded first, torch's copy is the one the library
        # binds to; loaded after the library, it would be a second runtime
        # whose streams and device memory the library cannot use.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.pj_config_default.argtypes = [ctypes.POINTER(Config)]
        L.pj_config_default.restype = None
        L.pj_context_create.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(vp)]
        L.pj_context_destroy.argtypes = [vp]
        L.pj_meshes_create.argtypes = [vp, ctypes.POINTER(MeshDesc), ctypes.POINTER(vp)]
        L.pj_meshes_destroy.argtypes = [vp]
        L.pj_join_within.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.POINTER(Pairs)]
        L.pj_join_intersect.argtypes = [vp, vp, vp, ctypes.POINTER(Pairs)]
        L.pj_join_knn.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.POINTER(Knn)]
        L.pj_pairs_free.argtypes = [ctypes.POINTER(Pairs)]
        L.pj_pairs_free.restype = None
        L.pj_knn_free.argtypes = [ctypes.POINTER(Knn)]
        L.pj_knn_free.restype = None
        L.pj_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
        L.pj_last_error.argtypes = [vp]
        L.pj_last_error.restype = ctypes.c_char_p
        L.pj_train_lod_model.argtypes = [vp, ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(TrainOpts),
                                         ctypes.POINTER(ctypes.c_float)]
        L.pj_meshes_boxes.argtypes = [vp, vp, vp]
        L.pj_meshes_hdph.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp]
        L.pj_facet_pairs.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_int32, vp, vp, vp]
        L.pj_pair_bounds.argtypes = [vp, vp, vp, ctypes.c_int64, vp, vp, ctypes.c_int32, vp, vp, vp]
        L.pj_pair_bounds_noalloc.argtypes = [vp, vp, vp, ctypes.c_int64, vp, vp, ctypes.c_int32, vp, vp, vp]
        L.pj_mlp_eval.argtypes = [vp, vp, vp, vp, ctypes.c_int64, vp, vp, vp]
        L.pj_probe_fma.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
        L.pj_probe_copy.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
        _lib = L
    return _lib


def _arr(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class Meshes:
    """An ingested object set (device resident)."""

    def __init__(self, ctx: "Context", ms, hd=None, ph=None, hdph_begin=None):
        self.ctx = ctx
        self.n = int(ms.n_objects)
        self.L = int(ms.n_lods)
        keep = [_arr(ms.verts, np.float32), _arr(ms.vert_begin, np.int64), _arr(ms.vert_count, np.int32),
                _arr(ms.tris, np.int32), _arr(ms.tri_begin, np.int64), _arr(ms.tri_count, np.int32),
                _arr(ms.parent, np.int32)]
        extra = [None, None, None] if hd is None else [_arr(hd, np.float32), _arr(ph, np.float32),
                                                      _arr(hdph_begin, np.int64)]
        d = MeshDesc(self.n, self.L, len(keep[0]), len(keep[3]), *[a.ctypes.data for a in keep],
                     *[None if a is None else a.ctypes.data for a in extra])
        h = ctypes.c_void_p()
        ctx._check(lib().pj_meshes_create(ctx.h, ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        self.tri_count = keep[5].reshape(self.n, self.L) if self.n else keep[5].reshape(0, self.L)

    def boxes(self):
        box = np.zeros((self.n, 6), np.float32)
        anc = np.zeros((self.n, 3), np.float32)
        self.ctx._check(lib().pj_meshes_boxes(self.h, box.ctypes.data, anc.ctypes.data))
        return box, anc

    def hdph(self, obj, lod):
        nf = int(self.tri_count[obj, lod])
        hd = np.zeros(nf, np.float32)
        ph = np.zeros(nf, np.float32)
        self.ctx._check(lib().pj_meshes_hdph(self.h, int(obj), int(lod), hd.ctypes.data, ph.ctypes.data))
        return hd, ph

    def close(self):
        if self.h:
            lib().pj_meshes_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """A join context on one device (see ``pj_config``)."""

    def __init__(self, device=0, precision="fp32", schedule="batched", learned_skip=False, want_dist=False,
                 use_graph=True, tile_cull=True, tile_s=0, waves_per_cu=0, mem_cap_bytes=0, model_path=None,
                 log_path=None, stream=None, chunk_tiles=0, autotune=False, autotune_path=None,
                 host_resident=False, stage_sets=0, filter_mode="auto", allocator=None, storage_dir=None,
                 knn_prune_host=False, voxels=False):
        """``allocator``: optional (alloc, free) Python callables for the
        library's device memory: alloc(nbytes) -> device address (int) or
        None, free(address).  They back pj_config.dev_alloc / dev_free.
        ``storage_dir``: mesh sets keep their facet data in a file there
        (out-of-core residency; implies host_resident)."""
        L = lib()
        c = Config()
        L.pj_config_default(ctypes.byref(c))
        c.device = device
        c.precision = PREC[precision]
        c.schedule = SCHED[schedule]
        c.learned_skip = int(bool(learned_skip))
        c.want_dist = int(bool(want_dist))
        c.use_graph = int(bool(use_graph))
        c.tile_cull = int(bool(tile_cull))
        c.tile_s = int(tile_s)
        c.waves_per_cu = int(waves_per_cu)
        c.mem_cap_bytes = int(mem_cap_bytes)
        c.chunk_tiles = int(chunk_tiles)
        c.autotune = int(bool(autotune))
        c.mesh_residency = 2 if storage_dir is not None else (1 if host_resident else 0)
        c.stage_sets = int(stage_sets)
        c.filter_mode = {"auto": 0, "pairs": 1, "sweep": 2, "grid": 3}[filter_mode]
        c.knn_prune_host = int(bool(knn_prune_host))
        c.voxels = int(bool(voxels))
        self._paths = [None if p is None else os.fsencode(p) for p in (model_path, log_path, autotune_path)]
        c.model_path, c.log_path, c.autotune_path = self._paths
        self._storage = None if storage_dir is None else os.fsencode(storage_dir)
        c.storage_dir = self._storage
        c.stream = stream
        self._hooks = None
        if allocator is not None:
            fa, ff = allocator

            def _alloc(nbytes, _user):
                try:
                    p = fa(int(nbytes))
                    return int(p) if p else None
                except Exception:  # an exception may not cross into the library
                    return None

            def _free(ptr, _user):
                try:
                    ff(int(ptr))
                except Exception:
                    pass

            self._hooks = (ALLOC_FN(_alloc), FREE_FN(_free))
            c.dev_alloc, c.dev_free = self._hooks
        h = ctypes.c_void_p()
        st = L.pj_context_create(ctypes.byref(c), ctypes.byref(h))
        if st != PJ_OK:
            raise PJError(st, "pj_context_create failed")
        self.h = h
        self.cfg = c

    def _check(self, st):
        if st != PJ_OK:
            raise PJError(st, lib().pj_last_error(self.h).decode(errors="replace"))

    def meshes(self, ms, **kw) -> Meshes:
        return Meshes(self, ms, **kw)

    def join_within(self, R: Meshes, S: Meshes, tau: float):
        p = Pairs()
        self._check(lib().pj_join_within(self.h, R.h, S.h, float(tau), ctypes.byref(p)))
        return self._pairs(p)

    def join_intersect(self, R: Meshes, S: Meshes):
        p = Pairs()
        self._check(lib().pj_join_intersect(self.h, R.h, S.h, ctypes.byref(p)))
        return self._pairs(p)

    def _pairs(self, p):
        n = int(p.n)
        out = dict(r=np.ctypeslib.as_array(p.r, (n,)).copy() if n else np.zeros(0, np.int32),
                   s=np.ctypeslib.as_array(p.s, (n,)).copy() if n else np.zeros(0, np.int32),
                   dist=np.ctypeslib.as_array(p.dist, (n,)).copy() if (n and p.dist) else None)
        lib().pj_pairs_free(ctypes.byref(p))
        return out

    def join_knn(self, R: Meshes, S: Meshes, k: int):
        q = Knn()
        self._check(lib().pj_join_knn(self.h, R.h, S.h, int(k), ctypes.byref(q)))
        n, kk = int(q.n_r), int(q.k)
        count = np.ctypeslib.as_array(q.count, (n,)).copy() if n else np.zeros(0, np.int32)
        s = np.ctypeslib.as_array(q.s, (n * kk,)).copy().reshape(n, kk) if n * kk else np.zeros((n, kk), np.int32)
        d = np.ctypeslib.as_array(q.dist, (n * kk,)).copy().reshape(n, kk) if n * kk else np.zeros((n, kk))
        lib().pj_knn_free(ctypes.byref(q))
        return dict(count=count, s=s, dist=d)

    def stats(self, raw=False):
        """The last join's statistics as a dict, or (raw=True) as the ctypes
        ``Stats`` structure itself (attribute access, no conversion)."""
        st = Stats()
        self._check(lib().pj_get_stats(self.h, ctypes.byref(st)))
        return st if raw else st.to_dict()

    def facet_pairs(self, t1, t2, precision="fp32", bounds=False):
        """Facet-pair distances: (d, hit), or (d_lo, d_hi, hit) with bounds=True."""
        t1 = _arr(t1, np.float32).reshape(-1, 9)
        t2 = _arr(t2, np.float32).reshape(-1, 9)
        n = len(t1)
        d = np.zeros(n, np.float64)
        d_hi = np.zeros(n, np.float64)
        hit = np.zeros(n, np.int8)
        self._check(lib().pj_facet_pairs(self.h, t1.ctypes.data, t2.ctypes.data, n, PREC[precision], d.ctypes.data,
                                         d_hi.ctypes.data, hit.ctypes.data))
        if bounds:
            return d, d_hi, hit.astype(bool)
        return d, hit.astype(bool)

    def pair_bounds(self, R: Meshes, S: Meshes, r, s, lod, noalloc=False):
        """LoD bounds of pairs (r[i], s[i]); noalloc=True calls the
        allocation-free entry point."""
        r = _arr(r, np.int32)
        s = _arr(s, np.int32)
        n = len(r)
        lb = np.zeros(n)
        ub = np.zeros(n)
        hit = np.zeros(n, np.int8)
        fn = lib().pj_pair_bounds_noalloc if noalloc else lib().pj_pair_bounds
        self._check(fn(self.h, R.h, S.h, n, r.ctypes.data, s.ctypes.data, int(lod), lb.ctypes.data, ub.ctypes.data,
                       hit.ctypes.data))
        return lb, ub, hit.astype(bool)

    def mlp_eval(self, params, x, y=None):
        params = _arr(params, np.float32)
        x = _arr(x, np.float32).reshape(-1, 16)
        n = len(x)
        logits = np.zeros((n, 4), np.float32)
        loss = np.zeros(1, np.float32)
        grads = np.zeros_like(params)
        yy = None if y is None else _arr(y, np.int32)
        self._check(lib().pj_mlp_eval(self.h, params.ctypes.data, x.ctypes.data,
                                      None if yy is None else yy.ctypes.data, n, logits.ctypes.data,
                                      loss.ctypes.data, grads.ctypes.data))
        return logits, (float(loss[0]) if y is not None else None), (grads if y is not None else None)

    def train_lod_model(self, log_path, model_out, epochs=30, batch=1024, lr=3e-3, seed=0):
        o = TrainOpts(int(epochs), int(batch), float(lr), int(seed))
        loss = ctypes.c_float()
        self._check(lib().pj_train_lod_model(self.h, os.fsencode(log_path), os.fsencode(model_out),
                                             ctypes.byref(o), ctypes.byref(loss)))
        return float(loss.value)

    def probe_fma(self, fp64=False):
        """Measured FMA throughput (GFLOP/s) of register-only FP32 or FP64 code."""
        g = ctypes.c_double()
        self._check(lib().pj_probe_fma(self.h, int(bool(fp64)), ctypes.byref(g)))
        return g.value

    def probe_copy(self, nbytes):
        """Achieved bandwidth (GB/s, read + write) of one plain copy of nbytes."""
        g = ctypes.c_double()
        self._check(lib().pj_probe_copy(self.h, int(nbytes), ctypes.byref(g)))
        return g.value

    def close(self):
        if getattr(self, "h", None):
            lib().pj_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
