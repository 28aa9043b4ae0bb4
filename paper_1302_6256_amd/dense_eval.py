"""Dense random graphs: InitialBranch's neighbourhood-core test, and the
split of the search into tasks.

The paper asks whether its neighbourhood-core bounds (InitialBranch) help on the
dense DIMACS instances as well as on sparse networks, and reports that they
usually do.  The DIMACS graphs are not available here; seeded G(n, p) graphs
with n = 100..1,000 and p = 0.5..0.9 stand in for them.  For each graph this
runs pmc_max_clique with and without the neighbourhood-core test (same GPU,
interleaved, best of `reps` calls) and reports time-to-certified omega, branch
nodes and roots branched; then with the split depth at 1 (only the roots'
level-0 branches become tasks) and 3, and with the split off (every branched
root searched by one wave), to show what splitting the branches of big
subproblems across waves buys on these few-root, deep-search instances.

  python -m paper_1302_6256_amd.dense_eval --json dense.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

CASES = ((200, 0.5), (300, 0.5), (500, 0.5), (1000, 0.5), (200, 0.7), (300, 0.7), (150, 0.8),
         (100, 0.9), (120, 0.9))


def _solve(pmc, off, idx, reps, **kw):
    import torch
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        w, _, st = pmc.max_clique(off, idx, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        if best is None or dt < best[0]:
            best = (dt, w, st)
    return best


def evaluate(cases=CASES, reps=3, seed=7, log=print):
    import torch
    import graphgen
    from . import pmc
    pmc.load()
    dev = torch.device("cuda:0")
    rows = []
    for n, p in cases:
        g = graphgen.gnp(n, p, seed)
        off, idx = torch.from_numpy(g.offsets).to(dev), torch.from_numpy(g.indices).to(dev)
        pmc.max_clique(off, idx)  # warm-up
        t1, w1, s1 = _solve(pmc, off, idx, reps)
        t0, w0, s0 = _solve(pmc, off, idx, reps, use_neighborhood_cores=0)
        if w0 != w1:
            raise SystemExit(f"omega differs with and without neighbourhood cores: {w1} {w0}")
        tun = pmc.get_tuning()
        alt = {}
        for key, over in (("depth1", {"search_split_depth": 1}), ("depth3", {"search_split_depth": 3}),
                          ("no_split", {"search_split_min": -1})):
            pmc.set_tuning(dict(tun, **over))
            try:
                alt[key] = _solve(pmc, off, idx, max(1, reps - 2))
            finally:
                pmc.set_tuning(tun)
            if alt[key][1] != w1:
                raise SystemExit(f"omega differs with {over}: {w1} {alt[key][1]}")
        row = {"n": n, "p": p, "m": g.m, "omega": w1, "heuristic": s1["heuristic"],
               "roots": s1["roots"], "ms_nc": round(1000 * t1, 3), "ms_no_nc": round(1000 * t0, 3),
               "nodes_nc": s1["nodes"], "nodes_no_nc": s0["nodes"],
               "branched_nc": s1["roots_branched"], "branched_no_nc": s0["roots_branched"]}
        for key, (t, _, st) in alt.items():
            row["ms_" + key] = round(1000 * t, 3)
            row["nodes_" + key] = st["nodes"]
        rows.append(row)
        log(json.dumps(row))
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    rows = evaluate(reps=a.reps, log=lambda s: print(s, flush=True))
    if a.json:
        with open(a.json, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
