"""Host logic of bench.py: the bytes models and the traffic figures it takes
from the committed counter summaries (used only while the profiled sources
are unchanged, else reported as null)."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_counter_summaries_parse():
    b = _bench()
    for kernel in ("k_peel", "k_orient"):
        path = os.path.join(ROOT, "profiles", f"{kernel}_c2_counters.md")
        keys = {}
        with open(path) as fh:
            for line in fh:
                for k in ("traffic_bytes_per_launch", "source_hash"):
                    if line.startswith(f"{k} {kernel}:"):
                        keys[k] = line.split(":", 1)[1].strip()
        assert int(keys["traffic_bytes_per_launch"]) > 0
        assert len(keys["source_hash"]) == 16
        t = b.profiled_traffic(kernel)  # None once the kernel's sources changed
        assert t is None or t == float(keys["traffic_bytes_per_launch"])
    assert b.profiled_traffic("k_search") is None  # no summary of that form


def test_bytes_models():
    b = _bench()
    assert b.peel_bytes(1_000_000, 12_003_017) == 8 * 1_000_001 + 24 * 12_003_017 + 12 * 1_000_000
    assert b.orient_bytes(10, 2, 3) == 2 * (16 * 2 + 8 * 10) + 4 * 3
