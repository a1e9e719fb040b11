"""CPU checks of the boundary: the library loads and exports every symbol
declared in include/pj.h (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "pj.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pj_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_join_calls():
    names = declared_symbols()
    for must in ("pj_join_within", "pj_join_intersect", "pj_join_knn", "pj_meshes_create", "pj_context_create"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2604_19982_amd as pj
    assert os.path.exists(pj.LIB_PATH), "build the library first (__graft_entry__.build())"
    L = ctypes.CDLL(pj.LIB_PATH)
    missing = [n for n in declared_symbols() if not hasattr(L, n)]
    assert not missing, missing
    assert set(pj.EXPORTS) <= set(declared_symbols())


def test_config_default_is_host_only():
    import paper_2604_19982_amd as pj
    c = pj.Config()
    pj.lib().pj_config_default(ctypes.byref(c))
    assert c.precision == 0 and c.schedule == 0 and c.tile_cull == 1 and c.mem_cap_bytes == 0


def test_struct_sizes_match_header_layout():
    import paper_2604_19982_amd as pj
    assert ctypes.sizeof(pj.Config) == 4 * 16 + 8 + 8 * 4 + 8 * 3 + 8 + 8
    assert ctypes.sizeof(pj.MeshDesc) == 8 + 8 + 8 + 8 * 10
    assert ctypes.sizeof(pj.Pairs) == 32
    assert ctypes.sizeof(pj.Stats) == 7 * 8 + 8 * 8 + 8 * 8 + 16 + 4 * 8 + 8 + 8 + 4 * 64 + 24 + 16 + 64 + 8 + 16 + 40 + 8 + 8


def test_product_path_does_not_import_oracle():
    src = open(os.path.join(ROOT, "paper_2604_19982_amd", "__init__.py")).read()
    assert "import oracle" not in src and "from oracle" not in src
    for f in os.listdir(os.path.join(ROOT, "paper_2604_19982_amd", "csrc")):
        assert "oracle" not in open(os.path.join(ROOT, "paper_2604_19982_amd", "csrc", f)).read().lower()


def test_every_launch_fits_a_dispatch():
    """A dispatch counts its grid in 32-bit work-items per dimension; a larger
    grid would run only part of the work.  Each kernel launch either checks its
    grid (PJ_GRID_CHECK), strides over its list with a capped grid
    (kStrideBlocks), or has a grid bounded by construction (listed here: one
    block, the persistent CU-sized grids, the model kernels over int counts of
    at most 128 per block, and the probes)."""
    import re
    bounded = {"k_scan", "k_init_round", "k_refine_f32", "k_collect_f32", "k_mlp_fwd_bwd", "k_mlp_wgrad",
               "k_mlp_adam", "k_mlp_start", "k_fma_probe", "k_copy_probe"}
    csrc = os.path.join(ROOT, "paper_2604_19982_amd", "csrc")
    seen = set()
    for f in sorted(os.listdir(csrc)):
        if not f.endswith(".hip"):
            continue
        src = open(os.path.join(csrc, f)).read()
        for m in re.finditer(r"hipLaunchKernelGGL\((\w+)", src):
            name = m.group(1)
            seen.add(name)
            start = src.rfind("hipError_t launch_", 0, m.start())
            end = src.index(";", m.start())
            span = src[start:end]
            assert name in bounded or "PJ_GRID_CHECK" in span or "kStrideBlocks" in span, (f, name)
    assert {"k_refine_f64_tiles", "k_refine_f64_plain", "k_pairs_f64", "k_hd", "k_ph"} <= seen


def test_one_hip_runtime_with_torch():
    """The library and torch share one HIP runtime (torch's copy is loaded
    first), so torch streams and device memory can be handed to it."""
    import subprocess
    import sys
    code = ("import paper_2604_19982_amd as pj; pj.lib(); import torch; "
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"
