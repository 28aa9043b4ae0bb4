"""The C-ABI library loads and exports every function include/pmc.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pmc.h")
LIB = os.path.join(ROOT, "paper_1302_6256_amd", "libpmc.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pmc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for want in ("pmc_core_numbers", "pmc_heuristic", "pmc_max_clique", "pmc_max_clique_batch",
                 "pmc_prune_orient", "pmc_status_string", "pmc_last_error"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpmc.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpmc.so not built")
def test_binding_loads_and_matches_header():
    from paper_1302_6256_amd import pmc
    lib = pmc.load()
    assert set(pmc.EXPORTS) <= set(declared())
    assert lib.pmc_status_string(3).decode() == "capacity too small"
    assert ctypes.sizeof(pmc.Options) > 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpmc.so not built")
def test_tuning_roundtrip_and_validation():
    from paper_1302_6256_amd import pmc
    pmc.load()
    pmc.set_tuning(None)
    d = pmc.get_tuning()
    assert d["search_blocks_per_cu"] == [32, 32, 16, 16, 2, 2, 2]
    assert d["heuristic_chunk"] == [4, 64]
    assert d["heuristic_waves_per_cu"] == [4, 16]
    assert d["search_split_min"] == 32
    assert d["search_split_depth"] == 1
    cfg = {"search_blocks_per_cu": [8, 8, 4, 4, 1, 1, 1], "heuristic_waves_per_cu": [4, 2],
           "search_graph": 1, "heuristic_chunk": [1, 32], "search_split_min": -1,
           "search_split_depth": 3, "search_sweep_nodes": 16, "learned_min_open": 8,
           "batch_peel": -1}
    pmc.set_tuning(cfg)
    assert pmc.get_tuning() == cfg
    with pytest.raises(pmc.PmcError):
        pmc.set_tuning({"heuristic_chunk": [65, 1]})
    with pytest.raises(pmc.PmcError):
        pmc.set_tuning({"search_blocks_per_cu": [99] * 7})
    with pytest.raises(pmc.PmcError):
        pmc.set_tuning({"search_split_depth": 9})
    pmc.set_tuning(None)
    assert pmc.get_tuning() == d


def test_product_path_does_not_load_the_oracle():
    """The oracle is test infrastructure: nothing under the package imports,
    links or runs it (the product path has no CPU fallback)."""
    import glob
    import re
    pkg = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_1302_6256_amd")
    pat = re.compile(r"^\s*(import\s+oracle|from\s+oracle\b|.*oracle\.cpp|.*liboracle)", re.M)
    for path in glob.glob(os.path.join(pkg, "**", "*.py"), recursive=True) + \
            glob.glob(os.path.join(pkg, "csrc", "*")):
        with open(path, errors="replace") as f:
            assert not pat.search(f.read()), path
