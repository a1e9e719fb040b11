#!/usr/bin/env python
"""Benchmark of the progressive polyhedral within-tau join on one MI355X.

A step is one pass of the whole hot path over the multi-LoD workload:
within-tau joins at tau = 0, 5 and 20 of 10k blob objects (LoDs of
80/320/1280/5120 triangles) against 2k tube objects (336..20,496 triangles)
in a 500^3 box (MBB filter, progressive LoD refinement, guard-band recheck).
Inputs are ingested into HBM before the timed region.

Prints ONE JSON line (rank 0) with the metric, a roofline entry for the
dominant kernel (FP32 tile refinement, timed with HIP events by the library
on its stream), the plain GPU schedule on the same inputs, and the CPU
oracle timed on a bounded sample.
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
COUNTERS = os.path.join(ROOT, "profiles", "k_refine_f32_multilod_counters.json")


def measured_traffic(workload="multilod"):
    """HBM bytes per launch from the committed counter runs, or None when the
    kernel sources changed since they were taken (or for another workload)."""
    if workload != "multilod":
        return None
    import hashlib
    try:
        rec = json.load(open(COUNTERS))
        sha = hashlib.sha256(b"".join(open(os.path.join(ROOT, s), "rb").read() for s in rec["sources"])).hexdigest()
        return rec["traffic_bytes_per_launch"] if sha == rec["source_sha256"] else None
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_step(ctx, gR, gS, taus, verbose=False, k=None):
    """One pass of the hot path: a within-tau join per tau, or one k-NN join."""
    tot = dict(pairs=0, pairs64=0, pairsc=0, kms=0.0, launches=0, results=0, band=0, ms=0.0, kms64=0.0)
    for tau in (taus if k is None else [None]):
        if k is None:
            res = ctx.join_within(gR, gS, tau)
        else:
            kn = ctx.join_knn(gR, gS, k)
            res = {"r": kn["s"][kn["s"] >= 0]}
        st = ctx.stats()
        if verbose:
            log(f"  {'tau=' + str(tau) if k is None else 'k=' + str(k)}: {st['t_total_ms']:.1f} ms (filter {st['t_filter_ms']:.1f}, refine {st['t_refine_ms']:.1f}, "
                f"band {st['t_band_ms']:.1f}), kernel {st['refine_kernel_ms']:.1f} ms, cand {st['candidates']}, "
                f"pairs {st['facet_pairs']:.3e}+{st['facet_pairs_fp64']:.3e}, band {st['band_pairs']}, "
                f"resolved/lod {st['resolved_at_lod'][:4]}, results {len(res['r'])}")
            log(f"    per LoD: items {st['lod_items'][:4]}, tiles {st['lod_tiles'][:4]}, "
                f"pairs {[f'{x:.2e}' for x in st['lod_pairs'][:4]]}, "
                f"kernel ms {[round(x, 2) for x in st['lod_kernel_ms'][:4]]}, chunks culled {st['tiles_culled']}")
        tot["pairs"] += st["facet_pairs"]
        tot["pairs64"] += st["facet_pairs_fp64"]
        tot["pairsc"] += st["collect_pairs"]
        tot["kms"] += st["refine_kernel_ms"]
        tot["kms64"] += st["band_kernel_ms"]
        tot["launches"] += st["refine_launches"]
        tot["results"] += len(res["r"])
        tot["band"] += st["band_pairs"]
    return tot


def train_model(pj, mg, stream, workdir):
    """LoD model for the learned skip, trained on resolution logs of a
    held-out workload of the same shape (seed 101, 2k x 400 in 300^3)."""
    log = os.path.join(workdir, "resolution.log")
    model = os.path.join(workdir, "lod.model")
    if os.path.exists(log):
        os.remove(log)
    R, S = mg.config_multilod(seed=101, n_r=2000, n_s=400, box=300.0)
    c = pj.Context(log_path=log, stream=stream.cuda_stream)
    gR, gS = c.meshes(R), c.meshes(S)
    for tau in (0.0, 2.0, 5.0, 10.0, 20.0):
        c.join_within(gR, gS, tau)
    loss = c.train_lod_model(log, model, epochs=40, batch=1024, lr=3e-3, seed=1)
    return model, loss, os.path.getsize(log) // 72


def one_step(pj, stream, gR, gS, taus, k=None, **cfg):
    """One step on another context over the already ingested mesh sets (a
    mesh set may be shared by contexts on its device)."""
    import torch
    c = pj.Context(stream=stream.cuda_stream, **cfg)
    torch.cuda.synchronize()
    ts = time.time()
    tot = run_step(c, gR, gS, taus, k=k)
    torch.cuda.synchronize()
    tot["ms"] = (time.time() - ts) * 1e3
    return tot


def sample_candidates(oracle, O_R, O_S, gap, max_r=20000, seed=0):
    """MBB candidate pairs (box gap <= gap) of up to max_r random R objects,
    found by an x-sorted sweep over S with the oracle's boxes."""
    import numpy as np
    bR, _ = oracle.mbbs(O_R)
    bS, _ = oracle.mbbs(O_S)
    rng = np.random.default_rng(seed)
    rs = np.sort(rng.permutation(len(bR))[:max_r])
    order = np.argsort(bS[:, 0], kind="stable")
    xs = bS[order, 0]
    wmax = float(np.max(bS[:, 3] - bS[:, 0])) if len(bS) else 0.0
    cr, cs = [], []
    for r in rs:
        lo = np.searchsorted(xs, bR[r, 0] - gap - wmax, "left")
        hi = np.searchsorted(xs, bR[r, 3] + gap, "right")
        js = order[lo:hi]
        if len(js) == 0:
            continue
        md = oracle.mindist(bR[r:r + 1], bS[js])[0]
        js = js[md <= gap]
        cr.append(np.full(len(js), r))
        cs.append(js)
    if not cr:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(cr), np.concatenate(cs)


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


# Workloads: the default is the multi-LoD join the metric is quoted on; the
# other two are the learned-skip join (10x the objects, sparser) and the
# large intersection join with host-resident meshes under a 32 GB device cap.
WORKLOADS = {
    "multilod": dict(builder="config_multilod", taus=TAUS, ctx={}, cpu_gap=5.0,
                     desc="multilod within-tau join: {nr} blobs (80/320/1280/5120 triangles) x {ns} tubes "
                          "(336..20496 triangles), 500^3 box, tau in {{0, 5, 20}} per step"),
    "learned": dict(builder="config_learned", taus=(10.0,), ctx={}, cpu_gap=10.0,
                    desc="learned-skip within-tau join: {nr} blobs (80..5120 triangles) x {ns} tubes "
                         "(336..20496 triangles), 5000^3 box, tau = 10"),
    "knn": dict(builder="config_knn", taus=(), k=3, ctx={}, cpu_gap=5.0,
                desc="batched k-NN join, k = 3: {nr} x {ns} blob/tube mix (finest 1k..50k triangles, 4 LoDs), "
                     "50 Gaussian clusters (sigma 30) in a 2000^3 box"),
    "large": dict(builder="config_large", taus=(0.0,), ctx=dict(host_resident=True, mem_cap_bytes=32 << 30),
                  cpu_gap=5.0,
                  desc="large intersection join: {nr} blobs (80..5120 triangles) x {ns} tubes (336..20496 "
                       "triangles), 20000^3 box, tau = 0, meshes host-resident, 32 GB device cap"),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="multilod")
    ap.add_argument("--plain", type=int, default=1, help="run the plain FP64 schedule once for comparison")
    ap.add_argument("--ablations", type=int, default=1, help="one step each without the learned skip / culling")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--n-r", type=int, default=None)
    ap.add_argument("--n-s", type=int, default=None)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1"}))
        sys.exit(2)
    import torch
    import meshgen as mg
    import paper_2604_19982_amd as pj

    wl = WORKLOADS[args.workload]
    taus = wl["taus"]
    kk = wl.get("k")
    size = {}
    if args.n_r:
        size["n_r"] = args.n_r
    if args.n_s:
        size["n_s"] = args.n_s
    t0 = time.time()
    R, S = getattr(mg, wl["builder"])(progress=lambda m: log(f"generating: {m}"), **size)
    log(f"generated {R.n_objects} x {S.n_objects} objects in {time.time() - t0:.1f} s")
    stream = torch.cuda.current_stream()
    import tempfile
    workdir = tempfile.mkdtemp(prefix="pj_bench_")
    t0 = time.time()
    model, train_loss, n_rec = train_model(pj, mg, stream, workdir)
    log(f"LoD model trained on {n_rec} logged pairs in {time.time() - t0:.1f} s, final loss {train_loss:.3f}")
    # launch shapes come from the autotuner (it times candidates during the
    # warmup step and caches them for the ablation contexts)
    tune = dict(autotune=True, autotune_path=os.path.join(workdir, "shapes.txt"))
    ctx = pj.Context(stream=stream.cuda_stream, learned_skip=True, model_path=model, **tune, **wl["ctx"])
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
    for w in range(args.warmup):
        run_step(ctx, gR, gS, taus, k=kk)
        log(f"warmup step {w} done")
    torch.cuda.synchronize()
    steps = []
    t_start = time.time()
    for k in range(args.steps):
        ts = time.time()
        tot = run_step(ctx, gR, gS, taus, verbose=True, k=kk)
        torch.cuda.synchronize()
        tot["ms"] = (time.time() - ts) * 1e3
        steps.append(tot)
        log(f"step {k}: {tot['ms']:.1f} ms, {tot['pairs']:.3e} FP32 + {tot['pairs64']:.3e} FP64 facet pairs, "
            f"{tot['results']} results")
    torch.cuda.synchronize()
    wall = time.time() - t_start
    ms_per_step = wall * 1e3 / args.steps
    # every facet pair evaluated: bulk FP32 rounds, the recheck's FP32 collect pass, FP64
    pairs = sum(s["pairs"] + s["pairsc"] + s["pairs64"] for s in steps)
    value = pairs / wall
    kms = sum(s["kms"] for s in steps)
    launches = sum(s["launches"] for s in steps)
    p32 = sum(s["pairs"] for s in steps)
    achieved = (p32 * FLOP_PER_PAIR) / (kms * 1e-3) / 1e12 if kms > 0 else 0.0
    st = ctx.stats()
    shapes = open(tune["autotune_path"]).read().split("\n") if os.path.exists(tune["autotune_path"]) else []
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
                   "results_per_step": steps[-1]["results"],
                   "band_pairs_per_step": steps[-1]["band"],
                   "ingest_s": ingest_s,
                   "chunks_last_join": st["chunks"],
                   "staged_bytes_last_join": st["staged_bytes"],
                   "mode": "learned LoD skip + batched persistent tiles + FP32 with FP64 guard band + chunk and "
                           "facet culling + hipGraph rounds",
                   "lod_model": {"train_pairs": n_rec, "final_loss": train_loss},
                   # evaluated FP32 facet pairs per second of refinement-kernel time
                   "fp32_kernel_facet_pair_evals_per_s": p32 / (kms * 1e-3) if kms > 0 else 0.0,
                   "tuned_shapes": [ln for ln in shapes if ln.strip()]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": measured_traffic(args.workload),
                     "kernel": "k_refine_f32", "launches": launches, "avg_launch_ms": kms / max(launches, 1),
                     "flop_per_pair": FLOP_PER_PAIR, "single_issue_fma_peak": SINGLE_ISSUE_FP32_TFLOPS,
                     "fma_probe_measured": fma_tflops, "copy_probe_gbps": copy_gbps},
    }
    abl = {}
    if args.ablations:
        for name, cfg in (("no_learned_skip", {}), ("no_learned_no_cull", dict(tile_cull=False))):
            t = one_step(pj, stream, gR, gS, taus, k=kk, **cfg, **tune, **wl["ctx"])
            abl[name] = {"ms": t["ms"], "facet_pairs": t["pairs"] + t["pairsc"] + t["pairs64"], "results": t["results"]}
            if t["kms"] > 0:
                # the same kernel without culling: every facet pair of every visited item is evaluated
                ach = t["pairs"] * FLOP_PER_PAIR / (t["kms"] * 1e-3) / 1e12
                abl[name]["kernel_ms"] = t["kms"]
                abl[name]["kernel_tflops"] = ach
                abl[name]["kernel_frac"] = ach / PEAK_FP32_TFLOPS
            log(f"ablation {name}: {t['ms']:.1f} ms")
    if args.plain:
        t = one_step(pj, stream, gR, gS, taus, k=kk, schedule="plain", precision="fp64", **wl["ctx"])
        abl["plain_gpu_schedule"] = {"ms": t["ms"], "facet_pairs": t["pairs"] + t["pairsc"] + t["pairs64"],
                                     "results": t["results"], "kernel_ms": t["kms64"]}
        if t["kms64"] > 0:
            # the plain FP64 kernel's facet pairs per second of its kernel time
            abl["plain_gpu_schedule"]["fp64_kernel_facet_pair_evals_per_s"] = t["pairs64"] / (t["kms64"] * 1e-3)
        log(f"plain schedule step: {t['ms']:.1f} ms")
        out["config"]["plain_ms_per_step"] = t["ms"]
        out["config"]["speedup_vs_plain"] = t["ms"] / ms_per_step
    for name, a in abl.items():
        a["results_match"] = a["results"] == steps[-1]["results"]
    out["config"]["ablations"] = abl
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(R, S, args.cpu_seconds, gap=wl["cpu_gap"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
