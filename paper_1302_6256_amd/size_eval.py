"""Size sweep: time to a certified omega on the benchmark's Chung-Lu family
(exponent 2.1, mean degree 24, w_max = sqrt(24 n), planted cliques of 20 and
40 vertices) from n = 10^3 to 10^7 vertices, the synthetic counterpart of the
paper's near-linear runtime scaling over networks of 10^3 to 10^8 vertices
(Sec. 3, Fig. 1).  Each size: the graph resident in HBM, one warm-up, then the
median of `reps` pmc_max_clique calls.

  python -m paper_1302_6256_amd.size_eval --json size.json
"""
from __future__ import annotations

import argparse
import json
import statistics
import sys
import time


def evaluate(sizes=(1_000, 10_000, 100_000, 1_000_000, 10_000_000), reps=5, log=print,
             budget=0, sweep=0):
    import torch

    import graphgen as gg
    from . import pmc
    pmc.load()
    d = torch.device("cuda:0")
    rows = []
    for n in sizes:
        t = time.perf_counter()
        g = gg.c2_graph(n=n)
        log(f"# n={n}: generated m={g.m} in {time.perf_counter() - t:.1f} s")
        off, idx = torch.from_numpy(g.offsets).to(d), torch.from_numpy(g.indices).to(d)
        kw = {"node_budget": budget, "allow_budget": True} if budget > 0 else {}
        if sweep > 0:
            kw["tune_table"] = {"search_sweep_nodes": sweep}
        t = time.perf_counter()
        pmc.max_clique(off, idx, **kw)
        torch.cuda.synchronize()
        log(f"# n={n}: warm-up solve {time.perf_counter() - t:.2f} s")
        times, st = [], None
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            w, _, st = pmc.max_clique(off, idx, **kw)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
        ms = 1000 * statistics.median(times)
        row = {"n": g.n, "m": g.m, "omega": w, "certified": bool(st["certified"]),
               "kmax": st["kmax"], "heuristic": st["heuristic"], "nodes": st["nodes"],
               "roots": st["roots"], "roots_open_after_sweep": st["roots_second_pass"],
               "nrounds": st["nrounds"], "ms": round(ms, 3),
               "edges_per_s": round(g.m / (ms / 1000.0)),
               "stage_ms": {k: round(st[k], 3) for k in ("ms_peel", "ms_heuristic", "ms_prune",
                                                          "ms_search", "ms_sweep")}}
        rows.append(row)
        log(json.dumps(row))
        del off, idx
        torch.cuda.empty_cache()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--sizes", type=int, nargs="*",
                    default=[1_000, 10_000, 100_000, 1_000_000, 10_000_000])
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--json", default=None)
    ap.add_argument("--budget", type=int, default=0,
                    help="Branch-node budget per solve (0: none; with one, omega may be uncertified)")
    ap.add_argument("--sweep", type=int, default=0,
                    help="sweep every root first with this many Branch nodes each (0: off)")
    a = ap.parse_args(argv)
    rows = evaluate(a.sizes, a.reps, log=lambda s: print(s, flush=True), budget=a.budget,
                    sweep=a.sweep)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
