#!/usr/bin/env python
"""Benchmark of the progressive polyhedral spatial join on one MI355X.

The default workload is the large intersection join: 1M blob objects (LoDs
of 80/320/1280/5120 triangles) against 200k tube objects (336..20,496
triangles) in a 20000^3 box, tau = 0.  A step is one pass of the whole hot
path (MBB filter, progressive LoD refinement with the learned first LoD,
guard-band recheck, result assembly).  The timed steps run on mesh sets
ingested into HBM before the timed region; the same join with the sets kept
in host memory under a 32 GB device cap (chunked streaming over PCIe) is
timed after it and reported beside the headline, with the plain GPU schedule
under the same cap.  The multi-LoD and learned-skip workloads are measured
in the same run and reported in ``config.other_workloads``.

Prints ONE JSON line with the metric, a roofline entry for the FP32 tile
refinement kernel (timed with HIP events by the library on its stream), the
plain GPU schedule on the same inputs, and the CPU oracle's join over the
workload's MBB candidates.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 operations per facet pair of the bulk kernel (adds, subs,
# muls, FMA counted as 2, rcp and sqrt as 1; min/max/compare/select not
# counted): 6 vertex-plane candidates x 25 + 9 segment pairs x 49 + sqrt 1 +
# bounds 6.
FLOP_PER_PAIR = 6 * 25 + 9 * 49 + 1 + 6
# MI355X published FP32 vector peak (256 CUs, 2.4 GHz).  The build disables
# packed FP32 instructions; scalar FP32 FMA issue alone reaches half of it
# (256 CUs x 64 lanes x 2 x 2.4 GHz = 78.6 TFLOP/s, measured by the FMA probe
# reported beside it), while gfx950 can co-issue two VALU instructions per
# SIMD quad-cycle, which mixed code like the refinement kernel uses.
PEAK_FP32_TFLOPS = 157.3
SINGLE_ISSUE_FP32_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
TAUS = (0.0, 5.0, 20.0)
def counters_file(workload):
    return os.path.join(ROOT, "profiles", f"k_refine_f32_{workload}_counters.json")


def measured_traffic(workload):
    """HBM bytes per launch from the committed counter runs of this workload,
    or None when there are none or the kernel sources changed since."""
    import hashlib
    try:
        rec = json.load(open(counters_file(workload)))
        sha = hashlib.sha256(b"".join(open(os.path.join(ROOT, s), "rb").read() for s in rec["sources"])).hexdigest()
        return rec["traffic_bytes_per_launch"] if sha == rec["source_sha256"] else None
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_step(ctx, gR, gS, taus, verbose=False, k=None):
    """One pass of the hot path: a within-tau join per tau, or one k-NN join.
    ``digest`` identifies the result sets (sorted (r, s) pairs per tau, or
    the k-NN id lists), so that variants can be checked for equal results."""
    import hashlib
    import numpy as np
    h = hashlib.sha1()
    tot = dict(pairs=0, pairs64=0, pairsc=0, kms=0.0, launches=0, results=0, band=0, ms=0.0, kms64=0.0,
               planned=0, items=0, staged=0, chunks=0, prep_ms=0.0, refine_ms=0.0, peak=0)
    for tau in (taus if k is None else [None]):
        if k is None:
            res = ctx.join_within(gR, gS, tau)
            h.update(np.float64(tau).tobytes())
            h.update(np.ascontiguousarray(res["r"], np.int32).tobytes())
            h.update(np.ascontiguousarray(res["s"], np.int32).tobytes())
        else:
            kn = ctx.join_knn(gR, gS, k)
            h.update(np.ascontiguousarray(kn["s"], np.int32).tobytes())
            res = {"r": kn["s"][kn["s"] >= 0]}
        # the structure itself inside the timed steps (no dict conversion)
        st = ctx.stats() if verbose else ctx.stats(raw=True)
        if verbose:
            log(f"  {'tau=' + str(tau) if k is None else 'k=' + str(k)}: {st['t_total_ms']:.1f} ms (filter {st['t_filter_ms']:.1f}, refine {st['t_refine_ms']:.1f}, "
                f"band {st['t_band_ms']:.1f}), kernel {st['refine_kernel_ms']:.1f} ms, cand {st['candidates']}, "
                f"pairs {st['facet_pairs']:.3e}+{st['facet_pairs_fp64']:.3e}, band {st['band_pairs']}, "
                f"resolved/lod {st['resolved_at_lod'][:4]}, results {len(res['r'])}")
            log(f"    per LoD: items {st['lod_items'][:4]}, tiles {st['lod_tiles'][:4]}, "
                f"pairs {[f'{x:.2e}' for x in st['lod_pairs'][:4]]}, "
                f"kernel ms {[round(x, 2) for x in st['lod_kernel_ms'][:4]]}, chunks culled {st['tiles_culled']}")
        g = st.__getitem__ if isinstance(st, dict) else st.__getattribute__
        tot["pairs"] += g("facet_pairs")
        tot["pairs64"] += g("facet_pairs_fp64")
        tot["pairsc"] += g("collect_pairs")
        tot["kms"] += g("refine_kernel_ms")
        tot["kms64"] += g("band_kernel_ms")
        tot["launches"] += g("refine_launches")
        tot["results"] += len(res["r"])
        tot["band"] += g("band_pairs")
        tot["planned"] += sum(g("lod_planned_pairs"))
        tot["items"] += sum(g("lod_items"))
        tot["staged"] += g("staged_bytes")
        tot["chunks"] += g("chunks")
        tot["prep_ms"] += g("t_prep_ms")
        tot["refine_ms"] += g("t_refine_ms")
        tot["peak"] = max(tot["peak"], g("peak_device_bytes"))
    tot["digest"] = h.hexdigest()
    return tot


def train_model(pj, mg, stream, workdir, **cfg):
    """LoD model for the learned skip, trained on resolution logs of a
    held-out workload of the multi-LoD shape (seed 101, 10k x 2k in 500^3,
    tau in {0, 2, 5, 10, 20}), written by joins with the given context
    options (the timed joins')."""
    log = os.path.join(workdir, "resolution.log")
    model = os.path.join(workdir, "lod.model")
    if os.path.exists(log):
        os.remove(log)
    R, S = mg.config_multilod(seed=101, n_r=10000, n_s=2000, box=500.0)
    c = pj.Context(log_path=log, stream=stream.cuda_stream, **cfg)
    gR, gS = c.meshes(R), c.meshes(S)
    for tau in (0.0, 2.0, 5.0, 10.0, 20.0):
        c.join_within(gR, gS, tau)
    loss = c.train_lod_model(log, model, epochs=40, batch=1024, lr=3e-3, seed=1)
    return model, loss, os.path.getsize(log) // 72


_ROCTX = []


def roctx():
    """The roctx marker library (ranges seen by rocprofv3 --marker-trace), or
    None where it is not installed."""
    if not _ROCTX:
        import ctypes
        lib = None
        for name in ("librocprofiler-sdk-roctx.so.1", "libroctx64.so.4"):
            try:
                lib = ctypes.CDLL(name)
                lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
                break
            except (OSError, AttributeError):
                lib = None
        _ROCTX.append(lib)
    return _ROCTX[0]


def one_step(pj, stream, gR, gS, taus, k=None, warmup=1, mark=None, **cfg):
    """One timed step on another context over the already ingested mesh sets
    (a mesh set may be shared by contexts on its device), after `warmup`
    untimed ones (first-use costs: buffer growth, graph capture, tuning).
    `mark` names a roctx range around the timed step."""
    import torch
    c = pj.Context(stream=stream.cuda_stream, **cfg)
    for _ in range(warmup):
        run_step(c, gR, gS, taus, k=k)
    torch.cuda.synchronize()
    rt = roctx() if mark else None
    if rt:
        rt.roctxRangePushA(mark.encode())
    ts = time.time()
    tot = run_step(c, gR, gS, taus, k=k)
    torch.cuda.synchronize()
    tot["ms"] = (time.time() - ts) * 1e3
    if rt:
        rt.roctxRangePop()
    return tot


def sample_candidates(oracle, O_R, O_S, gap, max_r=20000, seed=0, block=8192):
    """MBB candidate pairs (box gap <= gap) of up to max_r random R objects
    (all of R when max_r >= |R|), in (r, s) order, with the oracle's FP64
    boxes: S is binned by box centre in a uniform grid, each r visits the
    cells its box (widened by gap and S's widest half extent) reaches, and
    the exact box gap decides."""
    import numpy as np
    bR, _ = oracle.mbbs(O_R, anchors=False)
    bS, _ = oracle.mbbs(O_S, anchors=False)
    if max_r >= len(bR):
        rs = np.arange(len(bR))
    else:
        rs = np.sort(np.random.default_rng(seed).permutation(len(bR))[:max_r])
    if len(bS) == 0 or len(rs) == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    cen = 0.5 * (bS[:, :3] + bS[:, 3:])
    half = (0.5 * (bS[:, 3:] - bS[:, :3])).max(0)
    lo = cen.min(0)
    ext = np.maximum(cen.max(0) - lo, 1e-9)
    # cells of about 2 (gap + widest half extent), at most 2^21 of them
    csz = max(float(2.0 * (gap + half.max())), float(ext.max()) / 128.0, 1e-6)
    while np.prod(np.floor(ext / csz) + 1) > (1 << 21):
        csz *= 1.25
    g = (np.floor(ext / csz) + 1).astype(np.int64)
    cs = np.minimum(np.floor((cen - lo) / csz).astype(np.int64), g - 1)
    cid = (cs[:, 2] * g[1] + cs[:, 1]) * g[0] + cs[:, 0]
    order = np.argsort(cid, kind="stable")
    beg = np.searchsorted(cid[order], np.arange(np.prod(g) + 1))
    cr, cso = [], []
    for b0 in range(0, len(rs), block):
        blk = rs[b0:b0 + block]
        a = np.floor((bR[blk, :3] - gap - half - lo) / csz).astype(np.int64) - 1
        z = np.floor((bR[blk, 3:] + gap + half - lo) / csz).astype(np.int64) + 1
        a = np.clip(a, 0, g - 1)
        z = np.clip(z, 0, g - 1)
        span = z - a + 1
        rr, ss = [], []
        for dz in range(int(span[:, 2].max())):
            for dy in range(int(span[:, 1].max())):
                m = (dz < span[:, 2]) & (dy < span[:, 1])
                if not m.any():
                    continue
                row = ((a[m, 2] + dz) * g[1] + (a[m, 1] + dy)) * g[0]
                c0 = beg[row + a[m, 0]]
                c1 = beg[row + z[m, 0] + 1]
                cnt = c1 - c0
                if cnt.sum() == 0:
                    continue
                r_rep = np.repeat(blk[m], cnt)
                first = np.repeat(c0 - np.concatenate([[0], np.cumsum(cnt)[:-1]]), cnt)
                rr.append(r_rep)
                ss.append(order[first + np.arange(cnt.sum())])
        if not rr:
            continue
        r_rep = np.concatenate(rr)
        js = np.concatenate(ss)
        gp = np.maximum(0.0, np.maximum(bS[js, :3] - bR[r_rep, 3:], bR[r_rep, :3] - bS[js, 3:]))
        keep = np.sqrt(np.sum(gp * gp, -1)) <= gap
        r_k, s_k = r_rep[keep], js[keep]
        o = np.lexsort((s_k, r_k))
        cr.append(r_k[o])
        cso.append(s_k[o])
    if not cr:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(cr).astype(np.int64), np.concatenate(cso).astype(np.int64)


def _facets(M, obj, lod):
    """Float32 corners [n, 3, 3] of one object's facets at a LoD."""
    L = M.n_lods
    v = M.verts[M.vert_begin[obj]:M.vert_begin[obj] + M.vert_count[obj]]
    t = M.tris[M.tri_begin[obj * L + lod]:M.tri_begin[obj * L + lod] + M.tri_count[obj * L + lod]]
    return v[t]


def cpu_baseline(R, S, seconds, gap=5.0, per_pair=1 << 16):
    """The oracle's facet-pair rate on a bounded sample of the workload: its
    triangle-pair routine (exact meet test and FP64 distance, the step the
    brute-force join repeats for every facet pair) on facet pairs drawn from
    random MBB candidate pairs (box gap <= gap) at the finest LoD, in
    batches of 2^20 over the host's threads until `seconds` have passed.
    Only the oracle calls are timed (drawing the pairs is not)."""
    import numpy as np
    import oracle
    O_R, O_S = oracle.OSet(R), oracle.OSet(S)
    rng = np.random.default_rng(0)
    cr, cs = sample_candidates(oracle, O_R, O_S, gap)
    order = rng.permutation(len(cr))
    threads = oracle.lib().oracle_num_threads()
    L = R.n_lods
    evals, el, k = 0, 0.0, 0
    while el < seconds and k < len(order):
        T1, T2 = [], []
        while sum(len(x) for x in T1) < (1 << 20) and k < len(order):
            FR, FS = _facets(R, cr[order[k]], L - 1), _facets(S, cs[order[k]], L - 1)
            a = rng.integers(0, len(FR), per_pair)
            b = rng.integers(0, len(FS), per_pair)
            T1.append(FR[a])
            T2.append(FS[b])
            k += 1
        T1, T2 = np.concatenate(T1), np.concatenate(T2)
        t0 = time.time()
        oracle.tri_tri_batch(T1, T2, threads=threads)
        el += time.time() - t0
        evals += len(T1)
    return dict(value=evals / el, unit="facet-pair evals/s", cores=threads, kind="oracle",
                sample=(f"oracle triangle-pair routine (exact meet test + FP64 distance) on {evals:.3e} facet "
                        f"pairs drawn from {k} random MBB candidate pairs (box gap <= {gap}) of the same workload "
                        f"at the finest LoD, {el:.1f} s of oracle time"))


def cpu_join_baseline(R, S, tau, single_seconds=10.0):
    """The oracle's join itself on the workload: every MBB candidate (box gap
    <= tau, found by a sweep over the oracle's FP64 boxes) decided by its
    culled finest-LoD scan, over all host threads (wall time of the whole
    join); then the same scan on one thread over the first candidates until
    `single_seconds` have passed (per-core rate, whole-join time
    extrapolated).  value = facet pairs the scan evaluated per second."""
    import numpy as np
    import oracle
    O_R, O_S = oracle.OSet(R), oracle.OSet(S)
    threads = oracle.lib().oracle_num_threads()
    t0 = time.time()
    cr, cs = sample_candidates(oracle, O_R, O_S, tau, max_r=R.n_objects)
    t_sweep = time.time() - t0
    t0 = time.time()
    d, hit, ev = oracle.pair_distances_counted(O_R, O_S, cr, cs, threads=threads)
    t_all = time.time() - t0
    n_res = int(np.sum(hit if tau == 0.0 else d <= tau))
    # single thread on a prefix of the candidates (random order)
    perm = np.random.default_rng(0).permutation(len(cr))
    done, ev1, t1 = 0, 0, 0.0
    while t1 < single_seconds and done < len(cr):
        blk = perm[done:done + 8]
        t0 = time.time()
        _, _, e = oracle.pair_distances_counted(O_R, O_S, cr[blk], cs[blk], threads=1)
        t1 += time.time() - t0
        ev1 += int(e.sum())
        done += len(blk)
    per_core = ev1 / t1 if t1 > 0 else 0.0
    return dict(value=float(ev.sum()) / t_all, unit="facet-pair evals/s", cores=threads, kind="oracle",
                join_wall_s=t_all + t_sweep, join_scan_s=t_all, sweep_s=t_sweep, candidates=int(len(cr)),
                results=n_res, facet_pairs_evaluated=int(ev.sum()),
                single_thread={"value": per_core, "candidates": int(done), "seconds": t1,
                               "join_s_extrapolated": t1 * len(cr) / max(done, 1)},
                sample=(f"the oracle's whole join on this workload: all {len(cr)} MBB candidates (box gap <= {tau}) "
                        f"decided by its culled FP64 finest-LoD scan (exact meet test) on {threads} threads in "
                        f"{t_all:.2f} s plus a {t_sweep:.2f} s box sweep; single-threaded on {done} random "
                        f"candidates in {t1:.1f} s ({per_core:.3e} facet pairs/s per core, whole join "
                        f"extrapolated to {t1 * len(cr) / max(done, 1):.1f} s)"))


# Workloads.  "large" is the default line (the largest configuration, and the
# one the end-to-end speedup over the plain schedule is stated on); the
# timed steps run on HBM-resident sets and the 32 GB-capped host-resident
# variant ("capped") is timed beside them.
WORKLOADS = {
    "large": dict(builder="config_large", taus=(0.0,), ctx={}, cpu="join",
                  capped=dict(host_resident=True, mem_cap_bytes=32 << 30),
                  desc="large intersection join: {nr} blobs (80..5120 triangles) x {ns} tubes (336..20496 "
                       "triangles), 20000^3 box, tau = 0; timed on HBM-resident mesh sets, with the same join on "
                       "host-resident sets under a 32 GB device cap reported beside it"),
    # capped: host-resident sets under a 256 MB device cap, so that every LoD
    # round streams in many chunks (the overlap study of the chunk pipeline)
    "multilod": dict(builder="config_multilod", taus=TAUS, ctx={}, cpu_gap=5.0,
                     capped=dict(host_resident=True, mem_cap_bytes=256 << 20),
                     desc="multilod within-tau join: {nr} blobs (80/320/1280/5120 triangles) x {ns} tubes "
                          "(336..20496 triangles), 500^3 box, tau in {{0, 5, 20}} per step"),
    "learned": dict(builder="config_learned", taus=(10.0,), ctx={}, cpu_gap=10.0,
                    desc="learned-skip within-tau join: {nr} blobs (80..5120 triangles) x {ns} tubes "
                         "(336..20496 triangles), 5000^3 box, tau = 10"),
    "knn": dict(builder="config_knn", taus=(), k=3, ctx={}, cpu_gap=5.0,
                desc="batched k-NN join, k = 3: {nr} x {ns} blob/tube mix (finest 1k..50k triangles, 4 LoDs), "
                     "50 Gaussian clusters (sigma 30) in a 2000^3 box"),
}


def timed_steps(ctx, gR, gS, taus, kk, steps, warmup, verbose=True):
    """warmup untimed steps, then `steps` timed ones bracketed by device
    synchronisation; returns (per-step totals, wall seconds)."""
    import torch
    for w in range(warmup):
        run_step(ctx, gR, gS, taus, k=kk)
    torch.cuda.synchronize()
    out = []
    t_start = time.time()
    for k in range(steps):
        ts = time.time()
        tot = run_step(ctx, gR, gS, taus, verbose=verbose and k == steps - 1, k=kk)
        torch.cuda.synchronize()
        tot["ms"] = (time.time() - ts) * 1e3
        out.append(tot)
    torch.cuda.synchronize()
    return out, time.time() - t_start


def kernel_roofline(steps, workload):
    kms = sum(s["kms"] for s in steps)
    launches = sum(s["launches"] for s in steps)
    p32 = sum(s["pairs"] for s in steps)
    achieved = (p32 * FLOP_PER_PAIR) / (kms * 1e-3) / 1e12 if kms > 0 else 0.0
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS, "traffic": measured_traffic(workload),
            "kernel": "k_refine_f32", "launches": launches, "avg_launch_ms": kms / max(launches, 1),
            "kernel_ms_per_step": kms / max(len(steps), 1),
            "facet_pairs_per_launch": p32 / max(launches, 1), "flop_per_pair": FLOP_PER_PAIR,
            "single_issue_fma_peak": SINGLE_ISSUE_FP32_TFLOPS}


def variants(pj, stream, gR, gS, taus, kk, base_ms, base_digest, tune, wctx, timed, ablations=True, plain=True):
    """The ablations, one change of the timed configuration `timed` at a
    time (no learned skip; no voxel filter; neither, nor block and facet
    culling), and the plain GPU schedule (FP64, one workgroup per pair and
    LoD, from LoD 0, no voxels), one step each on the same ingested sets;
    each reports whether its results equal the timed run's."""
    abl = {}
    todo = []
    if ablations:
        todo += [("no_learned_skip", dict({k: v for k, v in timed.items() if k not in ("learned_skip", "model_path")},
                                          **tune, **wctx))]
        if timed.get("voxels"):
            todo += [("no_voxels", dict(dict(timed, voxels=False), **tune, **wctx))]
        todo += [("no_learned_no_voxels_no_cull", dict(tile_cull=False, **tune, **wctx))]
    if plain:
        todo += [("plain_gpu_schedule", dict(schedule="plain", precision="fp64", **wctx))]
    for name, cfg in todo:
        # the plain FP64 schedule takes seconds per step and has no first-use
        # costs to speak of; the others get one warmup step
        t = one_step(pj, stream, gR, gS, taus, k=kk, warmup=0 if name == "plain_gpu_schedule" else 1, **cfg)
        a = {"ms": t["ms"], "facet_pairs": t["pairs"] + t["pairsc"] + t["pairs64"],
             "planned_facet_pairs": t["planned"], "items": t["items"], "results": t["results"],
             "results_match": t["digest"] == base_digest, "speedup_of_timed_run": t["ms"] / base_ms}
        if name == "plain_gpu_schedule":
            a["kernel_ms"] = t["kms64"]
            if t["kms64"] > 0:
                a["fp64_kernel_facet_pair_evals_per_s"] = t["pairs64"] / (t["kms64"] * 1e-3)
        elif t["kms"] > 0:
            ach = t["pairs"] * FLOP_PER_PAIR / (t["kms"] * 1e-3) / 1e12
            a.update(kernel_ms=t["kms"], kernel_tflops=ach, kernel_frac=ach / PEAK_FP32_TFLOPS)
        abl[name] = a
        log(f"{name}: {t['ms']:.1f} ms, results match: {a['results_match']}")
    return abl


def measure_side(pj, stream, name, R, S, gen_s, timed, workdir, steps):
    """A workload other than the headline: HBM-resident sets, a few timed
    steps, the ablations and the plain schedule."""
    import torch
    wl = WORKLOADS[name]
    tune = dict(autotune=True, autotune_path=os.path.join(workdir, f"shapes_{name}.txt"))
    ctx = pj.Context(stream=stream.cuda_stream, **timed, **tune)
    t0 = time.time()
    gR, gS = ctx.meshes(R), ctx.meshes(S)
    torch.cuda.synchronize()
    ing = time.time() - t0
    kk = wl.get("k")
    st, wall = timed_steps(ctx, gR, gS, wl["taus"], kk, steps, 1, verbose=False)
    ms = wall * 1e3 / steps
    pairs = sum(s["pairs"] + s["pairsc"] + s["pairs64"] for s in st)
    # the k-NN workload's plain FP64 schedule would evaluate ~1e13 facet pairs:
    # not run; its comparisons are the candidate generation (grid against all
    # pairs) and the pruning rule on host threads against the GPU kernel
    abl = variants(pj, stream, gR, gS, wl["taus"], kk, ms, st[-1]["digest"], tune, {}, timed,
                   ablations=kk is None, plain=kk is None)
    if kk is not None:
        for name_v, cfg in (("all_pairs_candidates", dict(filter_mode="pairs")),
                            ("pruning_on_host", dict(knn_prune_host=True))):
            c2 = pj.Context(stream=stream.cuda_stream, **timed, **tune, **cfg)
            run_step(c2, gR, gS, (), k=kk)
            torch.cuda.synchronize()
            ts = time.time()
            t = run_step(c2, gR, gS, (), k=kk)
            torch.cuda.synchronize()
            s2 = c2.stats()
            abl[name_v] = {"ms": (time.time() - ts) * 1e3, "filter_ms": s2["t_filter_ms"],
                           "prune_ms": s2["t_prune_ms"], "results_match": t["digest"] == st[-1]["digest"]}
            log(f"{name}/{name_v}: {abl[name_v]['ms']:.1f} ms (filter {s2['t_filter_ms']:.1f}, "
                f"pruning {s2['t_prune_ms']:.1f})")
        s1 = ctx.stats()
        abl["timed_run_phases"] = {"filter_ms": s1["t_filter_ms"], "prune_ms": s1["t_prune_ms"],
                                   "grid_cells": s1["knn_grid_cells"], "candidates": s1["candidates"]}
    out = {"workload": wl["desc"].format(nr=R.n_objects, ns=S.n_objects), "steps": steps, "ms_per_step": ms,
           "facet_pair_evals_per_s": pairs / wall, "ingest_s": ing, "generate_s": gen_s,
           "results_per_step": st[-1]["results"], "roofline": kernel_roofline(st, name), "ablations": abl}
    if "plain_gpu_schedule" in abl:
        out["speedup_vs_plain"] = abl["plain_gpu_schedule"]["ms"] / ms
    log(f"{name}: {ms:.2f} ms per step" +
        (f", {out['speedup_vs_plain']:.0f}x vs plain" if "speedup_vs_plain" in out else ""))
    del gR, gS, ctx
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="large")
    ap.add_argument("--plain", type=int, default=1, help="run the plain FP64 schedule once for comparison")
    ap.add_argument("--ablations", type=int, default=1, help="one step each without the learned skip / culling")
    ap.add_argument("--capped-steps", type=int, default=5,
                    help="timed steps on host-resident sets under the workload's device cap (large: 32 GB, "
                         "multilod: 256 MB), then the overlap study (0: skip)")
    ap.add_argument("--side", default="multilod,learned,knn",
                    help="large: other workloads measured in the same run (comma list, or 'none')")
    ap.add_argument("--side-steps", type=int, default=3)
    ap.add_argument("--voxels", type=int, default=1, help="voxel-pair filtering in the timed configuration")
    ap.add_argument("--storage-dir", default="none",
                    help="large: also time the capped join with the sets' facet data in files here (out-of-core "
                         "residency); 'auto' uses the temp directory when it has room, 'none' skips it")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--n-r", type=int, default=None)
    ap.add_argument("--n-s", type=int, default=None)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1"}))
        sys.exit(2)
    import meshgen as mg

    wl = WORKLOADS[args.workload]
    taus = wl["taus"]
    kk = wl.get("k")
    size = {}
    if args.n_r:
        size["n_r"] = args.n_r
    if args.n_s:
        size["n_s"] = args.n_s
    # generated before anything touches the GPU (the large sets are built by
    # forked worker processes)
    t0 = time.time()
    R, S = getattr(mg, wl["builder"])(progress=lambda m: log(f"generating: {m}"), **size)
    gen_s = time.time() - t0
    log(f"generated {R.n_objects} x {S.n_objects} objects in {gen_s:.1f} s")
    side_sets = {}
    if args.workload == "large" and args.side != "none":
        for name in [x for x in args.side.split(",") if x]:
            t0 = time.time()
            side_sets[name] = getattr(mg, WORKLOADS[name]["builder"])() + (time.time() - t0,)
            log(f"generated the {name} workload in {side_sets[name][2]:.1f} s")
    import torch
    import paper_2604_19982_amd as pj
    stream = torch.cuda.current_stream()
    import tempfile
    workdir = tempfile.mkdtemp(prefix="pj_bench_")
    t0 = time.time()
    vox = dict(voxels=True) if args.voxels else {}
    model, train_loss, n_rec = train_model(pj, mg, stream, workdir, **vox)
    log(f"LoD model trained on {n_rec} logged pairs in {time.time() - t0:.1f} s, final loss {train_loss:.3f}")
    timed = dict(learned_skip=True, model_path=model, **vox)
    # launch shapes come from the autotuner (it times candidates during the
    # warmup step and caches them for the ablation contexts)
    tune = dict(autotune=True, autotune_path=os.path.join(workdir, "shapes.txt"))
    ctx = pj.Context(stream=stream.cuda_stream, **timed, **tune, **wl["ctx"])
    t0 = time.time()
    gR = ctx.meshes(R)
    log(f"ingested R in {time.time() - t0:.1f} s")
    gS = ctx.meshes(S)
    torch.cuda.synchronize()
    ingest_s = time.time() - t0
    log(f"ingested in {ingest_s:.2f} s")
    fma_tflops = max(ctx.probe_fma(False) for _ in range(2)) / 1e3
    copy_gbps = ctx.probe_copy(1 << 30)
    log(f"probes: scalar FP32 FMA {fma_tflops:.1f} TFLOP/s, copy {copy_gbps:.0f} GB/s")
    steps, wall = timed_steps(ctx, gR, gS, taus, kk, args.steps, args.warmup)
    ms_per_step = wall * 1e3 / args.steps
    log(f"timed: {ms_per_step:.2f} ms per step over {args.steps} steps")
    # every facet pair evaluated: bulk FP32 rounds, the recheck's FP32 collect pass, FP64
    pairs = sum(s["pairs"] + s["pairsc"] + s["pairs64"] for s in steps)
    value = pairs / wall
    st = ctx.stats()
    shapes = open(tune["autotune_path"]).read().split("\n") if os.path.exists(tune["autotune_path"]) else []
    roof = kernel_roofline(steps, args.workload)
    roof.update(fma_probe_measured=fma_tflops, copy_probe_gbps=copy_gbps)
    digest = steps[-1]["digest"]
    out = {
        "metric": "facet-pair evals/s; end-to-end join time, learned+batched vs plain GPU",
        "value": value,
        "unit": "facet-pair evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["desc"].format(nr=R.n_objects, ns=S.n_objects),
                   "facet_pairs_per_step": pairs / args.steps,
                   "planned_facet_pairs_per_step": steps[-1]["planned"],
                   "results_per_step": steps[-1]["results"],
                   "results_digest": digest,
                   "band_pairs_per_step": steps[-1]["band"],
                   "candidates_last_join": st["candidates"],
                   "generate_s": gen_s,
                   "ingest_s": ingest_s,
                   "mode": ("voxel-pair filtering + " if args.voxels else "") +
                           "learned LoD skip + batched persistent tiles + FP32 with FP64 guard band + chunk and "
                           "facet culling + hipGraph rounds",
                   "lod_model": {"train_pairs": n_rec, "final_loss": train_loss},
                   "fp32_kernel_facet_pair_evals_per_s": (sum(s["pairs"] for s in steps) /
                                                          (sum(s["kms"] for s in steps) * 1e-3)
                                                          if sum(s["kms"] for s in steps) > 0 else 0.0),
                   "tuned_shapes": [ln for ln in shapes if ln.strip()]},
        "roofline": roof,
    }
    abl = variants(pj, stream, gR, gS, taus, kk, ms_per_step, digest, tune, wl["ctx"], timed, args.ablations,
                   args.plain)
    if "plain_gpu_schedule" in abl:
        out["config"]["plain_ms_per_step"] = abl["plain_gpu_schedule"]["ms"]
        out["config"]["speedup_vs_plain"] = abl["plain_gpu_schedule"]["ms"] / ms_per_step
    out["config"]["ablations"] = abl
    if wl.get("capped") and args.capped_steps > 0:
        # the configuration's 32 GB device cap: the same join on host-resident
        # sets, each refinement chunk's facets staged and uploaded while the
        # previous chunk computes (PCIe-inclusive; never the headline value)
        del gR, gS
        ctx.close()
        torch.cuda.synchronize()
        cctx = pj.Context(stream=stream.cuda_stream, **timed, **tune, **wl["capped"])
        t0 = time.time()
        hR, hS = cctx.meshes(R), cctx.meshes(S)
        torch.cuda.synchronize()
        ing_h = time.time() - t0
        log(f"ingested host-resident in {ing_h:.1f} s")
        cst, cwall = timed_steps(cctx, hR, hS, taus, kk, args.capped_steps, 1)
        cms = cwall * 1e3 / args.capped_steps
        cab = variants(pj, stream, hR, hS, taus, kk, cms, digest, tune, wl["capped"], timed, ablations=False,
                       plain=args.plain)
        cst_last = cctx.stats()
        # streaming overlap: the same capped join with one staging set (gather,
        # upload, compute and download of each chunk one after another), two
        # and three sets (the next chunks gathered and uploaded while one
        # computes).  Each set gets the room one set has under the
        # configuration's cap with its two sets (the cap scales with the
        # sets), so the chunks are the same and only the overlap differs.
        overlap = {}
        for sets in (1, 2, 3):
            cap = wl["capped"]["mem_cap_bytes"] * sets // 2
            t = one_step(pj, stream, hR, hS, taus, k=kk, mark=f"capped stage_sets={sets}",
                         **dict(wl["capped"], stage_sets=sets, mem_cap_bytes=cap), **timed, **tune)
            overlap[f"stage_sets_{sets}"] = {"mem_cap_bytes": cap, "ms": t["ms"], "refine_ms": t["refine_ms"],
                                             "kernel_ms": t["kms"],
                                             "prep_ms": t["prep_ms"], "chunks": t["chunks"],
                                             "staged_bytes": t["staged"], "peak_device_bytes": t["peak"],
                                             "results_match": t["digest"] == digest}
            log(f"capped, {sets} staging set(s): {t['ms']:.2f} ms, refine {t['refine_ms']:.2f} ms, "
                f"kernel {t['kms']:.2f} ms, prep {t['prep_ms']:.2f} ms, {t['chunks']} chunks")
        out["config"]["capped_host_resident"] = {
            "mem_cap_bytes": wl["capped"]["mem_cap_bytes"], "steps": args.capped_steps, "ms_per_step": cms,
            "results_match": cst[-1]["digest"] == digest, "ingest_s": ing_h,
            "staged_bytes_per_step": cst[-1]["staged"], "chunks_per_step": cst[-1]["chunks"],
            "peak_device_bytes": cst_last["peak_device_bytes"],
            "speedup_vs_plain": (cab["plain_gpu_schedule"]["ms"] / cms) if "plain_gpu_schedule" in cab else None,
            "plain_gpu_schedule": cab.get("plain_gpu_schedule"), "overlap": overlap}
        log(f"capped host-resident: {cms:.2f} ms per step")
        del hR, hS
        cctx.close()
        # out of core: the same capped join with the facet data in files
        sdir = args.storage_dir
        if sdir == "auto":
            import shutil
            sdir = tempfile.gettempdir()
            need = 2 * (R.nbytes() + S.nbytes())
            if shutil.disk_usage(sdir).free < need:
                log(f"out-of-core run skipped: {shutil.disk_usage(sdir).free / 1e9:.0f} GB free in {sdir}, "
                    f"{need / 1e9:.0f} GB wanted")
                sdir = "none"
        if sdir != "none":
            fdir = tempfile.mkdtemp(prefix="pj_facets_", dir=sdir)
            fctx = pj.Context(stream=stream.cuda_stream, **timed, **tune,
                              **dict(wl["capped"], host_resident=False, stage_sets=3), storage_dir=fdir)
            t0 = time.time()
            fR, fS = fctx.meshes(R), fctx.meshes(S)
            torch.cuda.synchronize()
            ing_f = time.time() - t0
            fst, fwall = timed_steps(fctx, fR, fS, taus, kk, max(1, args.capped_steps), 1, verbose=False)
            fms = fwall * 1e3 / max(1, args.capped_steps)
            out["config"]["capped_file_resident"] = {
                "storage": "files under the temp directory, written once at ingest and read back through a "
                           "mapping (pages dropped from the page cache after writing)",
                "ms_per_step": fms, "ingest_s": ing_f, "results_match": fst[-1]["digest"] == digest,
                "prep_ms_per_step": fst[-1]["prep_ms"], "staged_bytes_per_step": fst[-1]["staged"]}
            log(f"capped file-resident: {fms:.2f} ms per step, ingest {ing_f:.1f} s")
            del fR, fS
            fctx.close()
    if side_sets:
        side = {}
        for name, (sR, sS, sg) in list(side_sets.items()):
            side[name] = measure_side(pj, stream, name, sR, sS, sg, timed, workdir, args.side_steps)
            del side_sets[name]
        out["config"]["other_workloads"] = side
    if args.cpu_seconds > 0:
        if wl.get("cpu") == "join":
            out["cpu_baseline"] = cpu_join_baseline(R, S, taus[0], single_seconds=args.cpu_seconds)
        else:
            out["cpu_baseline"] = cpu_baseline(R, S, args.cpu_seconds, gap=wl["cpu_gap"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
