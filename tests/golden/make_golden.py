"""Writes the stored expected values of tests/golden/ from the CPU oracle.

Calls only the oracle (and the shared input generators).  Run:
    python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402


def main():
    g = gg.c2_graph()
    t = time.time()
    w, cl, st = oracle.max_clique(g.offsets, g.indices)
    out = {
        "workload": g.name,
        "source": "oracle.max_clique (CPU oracle), written by tests/golden/make_golden.py",
        "n": g.n, "m": g.m, "omega": w, "kmax": st["kmax"], "nrounds": st["nrounds"],
        "heuristic": st["heuristic"], "survivors": st["survivors"],
        "clique": cl.tolist(), "oracle_seconds": round(time.time() - t, 2),
    }
    with open(os.path.join(HERE, "c2.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k != "clique"}))


if __name__ == "__main__":
    main()
