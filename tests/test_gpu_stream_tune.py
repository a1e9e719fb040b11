"""GPU: chunked streaming of the bulk rounds and the launch-shape autotuner.

Neither may change a result: the per-item minima are merged over chunks and
are independent of tiling and grid size, so every variant is compared pair
set for pair set (and kNN list for list) with the oracle or the default
launch."""
import os

import numpy as np
import pytest

import meshgen as mg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pj():
    import paper_2604_19982_amd as pj
    return pj


@pytest.fixture(scope="module")
def mid():
    return mg.config_multilod(seed=1, n_r=400, n_s=80, box=150.0, n_seg=1280)


@pytest.mark.parametrize("tau", [0.0, 5.0, 20.0])
def test_streamed_chunks_match_oracle(orc, pj, mid, tau):
    """A few tiles per chunk: items are split over many chunks, uploaded on
    one stream, computed on the join stream and read back on a third."""
    R, S = mid
    c = pj.Context(chunk_tiles=37)
    got = c.join_within(c.meshes(R), c.meshes(S), tau)
    st = c.stats()
    ref = orc.join_within(orc.OSet(R), orc.OSet(S), tau)
    assert ref["near_ties"] == 0
    assert np.array_equal(got["r"], ref["r"]) and np.array_equal(got["s"], ref["s"])
    assert st["chunks"] > st["rounds"]


@pytest.mark.parametrize("use_graph", [False, True])
def test_streamed_chunks_match_single_chunk(pj, mid, use_graph):
    R, S = mid
    one = pj.Context(use_graph=use_graph)
    many = pj.Context(use_graph=use_graph, chunk_tiles=101)
    oR, oS = one.meshes(R), one.meshes(S)
    mR, mS = many.meshes(R), many.meshes(S)
    for tau in (5.0, 0.0, 20.0):
        a = one.join_within(oR, oS, tau)
        b = many.join_within(mR, mS, tau)
        assert np.array_equal(a["r"], b["r"]) and np.array_equal(a["s"], b["s"]), tau
        assert many.stats()["chunks"] > one.stats()["chunks"]


def test_streamed_chunks_knn(orc, pj):
    R, S = mg.config_knn(seed=3, n_r=40, n_s=40, n_clusters=2, box=200.0, sigma=12.0, f_median=2000)
    base = pj.Context()
    many = pj.Context(chunk_tiles=13)
    a = base.join_knn(base.meshes(R), base.meshes(S), 3)
    b = many.join_knn(many.meshes(R), many.meshes(S), 3)
    assert np.array_equal(a["s"], b["s"]) and np.array_equal(a["count"], b["count"])
    assert np.array_equal(a["dist"], b["dist"])
    assert many.stats()["chunks"] > base.stats()["chunks"]


def test_mem_cap_too_small_is_an_error(pj, mid):
    R, S = mid
    c = pj.Context(mem_cap_bytes=4096)
    gR, gS = c.meshes(R), c.meshes(S)
    with pytest.raises(pj.PJError) as e:
        c.join_within(gR, gS, 5.0)
    assert e.value.status == 2  # PJ_ERR_OUT_OF_MEMORY


def test_mem_cap_streams_under_budget(pj, mid):
    """Caps below the uncapped high-water mark: the bulk rounds stream in
    more chunks, the FP64 recheck list shrinks, results stay the same and
    the work buffers stay under the cap (or the join says it cannot fit)."""
    R, S = mid
    free = pj.Context()
    ref = free.join_within(free.meshes(R), free.meshes(S), 5.0)
    peak = free.stats()["peak_device_bytes"]
    streamed = 0
    for frac in (0.5, 0.2, 0.08):
        cap = int(peak * frac)
        c = pj.Context(mem_cap_bytes=cap)
        gR, gS = c.meshes(R), c.meshes(S)
        try:
            got = c.join_within(gR, gS, 5.0)
        except pj.PJError as e:
            assert e.status == 2 and frac < 0.5, (frac, str(e))
            continue
        st = c.stats()
        assert np.array_equal(got["r"], ref["r"]) and np.array_equal(got["s"], ref["s"]), frac
        assert st["peak_device_bytes"] <= cap, frac
        streamed += st["chunks"] > st["rounds"]
    assert streamed


def test_autotune_picks_cached_shape(pj, mid, tmp_path):
    R, S = mid
    path = str(tmp_path / "tune.txt")
    base = pj.Context()
    ref = base.join_within(base.meshes(R), base.meshes(S), 5.0)
    t1 = pj.Context(autotune=True, autotune_path=path)
    a = t1.join_within(t1.meshes(R), t1.meshes(S), 5.0)
    s1 = t1.stats()
    assert np.array_equal(a["r"], ref["r"]) and np.array_equal(a["s"], ref["s"])
    assert s1["t_tune_ms"] > 0.0
    assert s1["tile_s_used"] in (1024, 2048, 4096, 8192, 16384)
    assert s1["waves_per_cu_used"] in (4, 8, 12)
    lines = open(path).read().split("\n")
    rows = [ln.split() for ln in lines if ln.strip()]
    assert rows and all(len(r) == 4 for r in rows)
    # a second context reads the cache and does not tune again
    t2 = pj.Context(autotune=True, autotune_path=path)
    b = t2.join_within(t2.meshes(R), t2.meshes(S), 5.0)
    s2 = t2.stats()
    assert np.array_equal(b["r"], ref["r"]) and np.array_equal(b["s"], ref["s"])
    assert s2["t_tune_ms"] == 0.0
    assert s2["tile_s_used"] == s1["tile_s_used"] and s2["waves_per_cu_used"] == s1["waves_per_cu_used"]
    # explicit shapes win over the cache
    t3 = pj.Context(autotune=True, autotune_path=path, tile_s=512, waves_per_cu=8)
    t3.join_within(t3.meshes(R), t3.meshes(S), 5.0)
    s3 = t3.stats()
    assert (s3["tile_s_used"], s3["waves_per_cu_used"]) == (512, 8)
    assert os.path.getsize(path) > 0


# ---------------------------------------------------------------------------
# host-resident mesh sets: facet data gathered per chunk into pinned staging
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def dev_ref(pj, mid):
    R, S = mid
    c = pj.Context()
    gR, gS = c.meshes(R), c.meshes(S)
    return {tau: c.join_within(gR, gS, tau) for tau in (0.0, 5.0, 20.0)}


def test_host_resident_ingest_matches_device(pj, mid):
    R, S = mid
    d = pj.Context()
    h = pj.Context(host_resident=True, mem_cap_bytes=1 << 20)  # ingest in many object batches
    for ms in (R, S):
        gd, gh = d.meshes(ms), h.meshes(ms)
        bd, bh = gd.boxes(), gh.boxes()
        for a, b in zip(bd, bh):
            assert np.array_equal(a, b)
        for obj in (0, ms.n_objects // 2, ms.n_objects - 1):
            for lod in range(ms.n_lods):
                hd1, ph1 = gd.hdph(obj, lod)
                hd2, ph2 = gh.hdph(obj, lod)
                assert np.array_equal(hd1, hd2) and np.array_equal(ph1, ph2)


@pytest.mark.parametrize("sets", [2, 3])
@pytest.mark.parametrize("cap", [0, 6 << 20])
def test_host_resident_join_matches_device(pj, mid, dev_ref, sets, cap):
    R, S = mid
    c = pj.Context(host_resident=True, stage_sets=sets, mem_cap_bytes=cap)
    gR, gS = c.meshes(R), c.meshes(S)
    for tau in (0.0, 5.0, 20.0):
        got = c.join_within(gR, gS, tau)
        st = c.stats()
        ref = dev_ref[tau]
        assert np.array_equal(got["r"], ref["r"]) and np.array_equal(got["s"], ref["s"]), tau
        assert st["staged_bytes"] > 0
        if cap:
            assert st["chunks"] > st["rounds"] and st["peak_device_bytes"] <= cap


def test_host_resident_join_vs_oracle(orc, pj):
    R, S = mg.config_small(seed=4, n_r=60, n_s=60, box=10.0)
    c = pj.Context(host_resident=True, want_dist=True)
    got = c.join_within(c.meshes(R), c.meshes(S), 0.5)
    ref = orc.join_within(orc.OSet(R), orc.OSet(S), 0.5)
    assert np.array_equal(got["r"], ref["r"]) and np.array_equal(got["s"], ref["s"])
    assert np.all(np.abs(got["dist"] - ref["d"]) <= np.maximum(1e-5 * ref["d"], 1e-12 * 10.0))


@pytest.mark.parametrize("mode", ["fp64", "plain"])
def test_host_resident_fp64_paths(pj, mid, dev_ref, mode):
    R, S = mid
    c = pj.Context(host_resident=True, precision="fp64", schedule="plain" if mode == "plain" else "batched",
                   mem_cap_bytes=16 << 20)
    got = c.join_within(c.meshes(R), c.meshes(S), 5.0)
    assert np.array_equal(got["r"], dev_ref[5.0]["r"]) and np.array_equal(got["s"], dev_ref[5.0]["s"])


def test_host_resident_knn(pj):
    R, S = mg.config_knn(seed=3, n_r=40, n_s=40, n_clusters=2, box=200.0, sigma=12.0, f_median=2000)
    d = pj.Context()
    h = pj.Context(host_resident=True, mem_cap_bytes=8 << 20, stage_sets=3)
    a = d.join_knn(d.meshes(R), d.meshes(S), 3)
    b = h.join_knn(h.meshes(R), h.meshes(S), 3)
    assert np.array_equal(a["s"], b["s"]) and np.array_equal(a["count"], b["count"])
    assert np.array_equal(a["dist"], b["dist"])
    assert h.stats()["staged_bytes"] > 0


def parallel_grids(n):
    """Two n x n unit grids (2 n^2 triangles each), the second one unit above
    the first: each facet of one lies at distance exactly 1 from the dozen
    facets of the other that touch its projection, so the k-NN recheck keeps
    about 12 facet pairs per facet."""
    g = np.arange(n + 1, dtype=np.float32)
    X, Y = np.meshgrid(g, g, indexing="ij")
    v = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size, np.float32)], 1)
    idx = np.arange((n + 1) ** 2).reshape(n + 1, n + 1)
    a, b, c, d = idx[:-1, :-1].ravel(), idx[1:, :-1].ravel(), idx[1:, 1:].ravel(), idx[:-1, 1:].ravel()
    tri = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)])
    return mg.single_object(v, [tri]), mg.single_object(v + np.float32([0.0, 0.0, 1.0]), [tri])


def test_knn_recheck_overflow_redo(pj):
    """Memory caps small enough that the recheck's collect list overflows
    (the parallel grids offer about 1.5M pairs for their one item, 24 MB of
    list): the item is recomputed by the tiled FP64 kernel over all its
    finest facet pairs, and the list and distance must equal the uncapped
    join's (both take the minimum of the same FP64 pair distance over a set
    holding the minimising pair; here exactly 1)."""
    R, S = parallel_grids(250)
    d = pj.Context()
    ref = d.join_knn(d.meshes(R), d.meshes(S), 1)
    assert d.stats()["collect_overflow"] == 0 and ref["dist"][0][0] == 1.0
    overflowed = []
    for cap in (32 << 20, 24 << 20, 16 << 20, 12 << 20, 8 << 20):
        h = pj.Context(host_resident=True, mem_cap_bytes=cap, stage_sets=2)
        try:
            got = h.join_knn(h.meshes(R), h.meshes(S), 1)
        except pj.PJError as e:  # a cap below what one chunk or the recheck needs
            assert pj.STATUS_NAMES[e.status] == "OUT_OF_MEMORY", (cap, e)
            print(cap, "out of memory")
            continue
        st = h.stats()
        print(cap, st["collected_pairs"], st["collect_regrow"], st["collect_overflow"])
        assert np.array_equal(got["s"], ref["s"]) and np.array_equal(got["count"], ref["count"]), cap
        assert np.array_equal(got["dist"], ref["dist"]), cap
        if st["collect_overflow"] > 0:
            overflowed.append(cap)
    assert overflowed, "no cap made the collect list overflow"


def test_knn_recheck_list_grows_to_need(pj):
    """The parallel grids' recheck offers about 1.5M pairs, more than its
    first list (2^20 pairs for one item) holds.  The pass runs once more with
    a list of the offered size: no item falls back to the full FP64 pass,
    and the distance is exact."""
    R, S = parallel_grids(250)
    ctx = pj.Context()
    res = ctx.join_knn(ctx.meshes(R), ctx.meshes(S), 1)
    st = ctx.stats()
    print(st["collected_pairs"], st["collect_regrow"], st["collect_overflow"])
    assert res["count"][0] == 1 and res["s"][0].tolist()[:1] == [0]
    assert res["dist"][0][0] == 1.0
    assert st["collect_regrow"] >= 1 and st["collect_overflow"] == 0
    assert st["collected_pairs"] > (1 << 20)


def test_host_resident_pair_bounds(pj, mid):
    R, S = mid
    d = pj.Context()
    h = pj.Context(host_resident=True)
    dR, dS, hR, hS = d.meshes(R), d.meshes(S), h.meshes(R), h.meshes(S)
    rng = np.random.default_rng(5)
    rr = rng.integers(0, R.n_objects, 64)
    ss = rng.integers(0, S.n_objects, 64)
    for lod in range(R.n_lods):
        a = d.pair_bounds(dR, dS, rr, ss, lod)
        b = h.pair_bounds(hR, hS, rr, ss, lod)
        for x, y in zip(a, b):
            assert np.array_equal(x, y), lod


# ---------------------------------------------------------------------------
# MBB filter: x sweep against all pairs
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["sweep", "grid"])
@pytest.mark.parametrize("tau", [0.0, 5.0, 20.0, 400.0])
def test_sweep_filter_matches_all_pairs(pj, mid, tau, mode):
    R, S = mid
    out = {}
    for m in ("pairs", mode):
        c = pj.Context(filter_mode=m)
        res = c.join_within(c.meshes(R), c.meshes(S), tau)
        out[m] = (res, c.stats())
    a, b = out["pairs"][0], out[mode][0]
    assert np.array_equal(a["r"], b["r"]) and np.array_equal(a["s"], b["s"])
    assert out["pairs"][1]["candidates"] == out[mode][1]["candidates"] > 0
    assert out["pairs"][1]["confirmed_filter"] == out[mode][1]["confirmed_filter"]


def test_sweep_filter_ties_and_edges(orc, pj):
    # many boxes with equal xmin (a lattice in y and z), touching boxes, empty sides
    A = mg.objects([mg.cube_mesh([0, y, z], [1, y + 1, z + 1]) for y in range(4) for z in range(4)])
    B = mg.objects([mg.cube_mesh([1, y + 0.5, z], [2, y + 1.5, z + 1]) for y in range(4) for z in range(3)]
                   + [mg.cube_mesh([1.25, 0, 0], [2, 1, 1]), mg.cube_mesh([-3, 0, 0], [-1.0, 1, 1])])
    ref = orc.join_within(orc.OSet(A), orc.OSet(B), 0.0)
    for tau in (0.0, 0.25, 1.0, 3.0):
        got = {}
        for mode in ("pairs", "sweep", "grid"):
            c = pj.Context(filter_mode=mode)
            r = c.join_within(c.meshes(A), c.meshes(B), tau)
            got[mode] = set(zip(r["r"].tolist(), r["s"].tolist()))
        assert got["pairs"] == got["sweep"] == got["grid"], tau
        if tau == 0.0:
            assert got["sweep"] == set(zip(ref["r"].tolist(), ref["s"].tolist()))
    for mode in ("sweep", "grid"):
        c = pj.Context(filter_mode=mode)
        gA, gE = c.meshes(A), c.meshes(A.subset([]))
        assert len(c.join_within(gA, gE, 1.0)["r"]) == 0
        assert len(c.join_within(gE, gA, 1.0)["r"]) == 0
    assert len(c.join_within(gE, gA, 1.0)["r"]) == 0


# ---------------------------------------------------------------------------
# Out-of-core residency: facet data in an (unlinked) file under storage_dir,
# read back through a mapping by the chunk prep thread.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cap", [0, 6 << 20])
def test_file_resident_join_matches_device(pj, mid, dev_ref, tmp_path, cap):
    R, S = mid
    c = pj.Context(storage_dir=str(tmp_path), stage_sets=3, mem_cap_bytes=cap)
    gR, gS = c.meshes(R), c.meshes(S)
    assert os.listdir(tmp_path) == []  # the files are unlinked at once
    for tau in (0.0, 5.0, 20.0):
        got = c.join_within(gR, gS, tau)
        st = c.stats()
        ref = dev_ref[tau]
        assert np.array_equal(got["r"], ref["r"]) and np.array_equal(got["s"], ref["s"]), tau
        assert st["staged_bytes"] > 0 and st["t_prep_ms"] > 0.0
        if cap:
            assert st["chunks"] > st["rounds"] and st["peak_device_bytes"] <= cap
    d = pj.Context()
    for ms, g in ((R, gR), (S, gS)):
        gd = d.meshes(ms)
        for obj in (0, ms.n_objects - 1):
            for lod in range(ms.n_lods):
                assert all(np.array_equal(a, b) for a, b in zip(gd.hdph(obj, lod), g.hdph(obj, lod)))


def test_file_resident_knn_and_oracle(orc, pj, tmp_path):
    R, S = mg.config_small(seed=4, n_r=60, n_s=60, box=10.0)
    c = pj.Context(storage_dir=str(tmp_path), want_dist=True, mem_cap_bytes=4 << 20)
    gR, gS = c.meshes(R), c.meshes(S)
    got = c.join_within(gR, gS, 0.5)
    ref = orc.join_within(orc.OSet(R), orc.OSet(S), 0.5)
    assert np.array_equal(got["r"], ref["r"]) and np.array_equal(got["s"], ref["s"])
    assert np.all(np.abs(got["dist"] - ref["d"]) <= np.maximum(1e-5 * ref["d"], 1e-12 * 10.0))
    d = pj.Context()
    a = d.join_knn(d.meshes(R), d.meshes(S), 3)
    b = c.join_knn(gR, gS, 3)
    assert np.array_equal(a["s"], b["s"]) and np.array_equal(a["dist"], b["dist"])


def test_file_residency_needs_a_directory(pj):
    with pytest.raises(pj.PJError):
        c = pj.Context(storage_dir="")
        c.meshes(mg.config_small(seed=0, n_r=2, n_s=2)[0])
    c = pj.Context(storage_dir="/nonexistent/dir")
    with pytest.raises(pj.PJError) as e:
        c.meshes(mg.config_small(seed=0, n_r=2, n_s=2)[0])
    assert e.value.status == 1
