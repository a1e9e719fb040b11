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
    assert ctypes.sizeof(pj.Config) == 4 * 16 + 8 + 8 * 4
    assert ctypes.sizeof(pj.MeshDesc) == 8 + 8 + 8 + 8 * 10
    assert ctypes.sizeof(pj.Pairs) == 32
    assert ctypes.sizeof(pj.Stats) == 7 * 8 + 8 * 8 + 8 * 8 + 16 + 4 * 8 + 8 + 8 + 4 * 64 + 24 + 16


def test_product_path_does_not_import_oracle():
    src = open(os.path.join(ROOT, "paper_2604_19982_amd", "__init__.py")).read()
    assert "import oracle" not in src and "from oracle" not in src
    for f in os.listdir(os.path.join(ROOT, "paper_2604_19982_amd", "csrc")):
        assert "oracle" not in open(os.path.join(ROOT, "paper_2604_19982_amd", "csrc", f)).read().lower()
