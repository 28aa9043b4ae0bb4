"""The scale workload: R-MAT scale 27 (about 1.85 billion undirected edges,
the size of the paper's largest network), generated on the device, and the
stages of the method on it at full size.

For each scale given (default 22, 24, 27): generation time, pmc_core_numbers
(K, rounds, time), then pmc_max_clique under a node budget (0: none), optionally
with the sweep first (R-MAT with these
quadrant probabilities has a dense core: omega is about 200 at scale 22 and 289
at scale 24, whose exact search already takes about 35 s; at scale 27 the run
reports the heuristic clique, the stage times and "not certified" once the
budget is spent).

  python -m paper_1302_6256_amd.scale_eval --json scale.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def evaluate(scales=(22, 24, 27), budget=1_000_000, log=print, core_only=False, sweep=0):
    import torch
    from graphgen import device as gd
    from . import pmc
    pmc.load()
    d = torch.device("cuda:0")
    rows = []
    for scale in scales:
        torch.cuda.reset_peak_memory_stats()
        t = time.perf_counter()
        off, idx, n, m, planted = gd.c5_csr(scale, 14, device=d)
        torch.cuda.synchronize()
        t_gen = time.perf_counter() - t
        gen_peak = torch.cuda.max_memory_allocated()
        pmc.core_numbers(off, idx)  # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, _, _, km, nr = pmc.core_numbers(off, idx)
        torch.cuda.synchronize()
        t_core = time.perf_counter() - t
        if core_only:
            row = {"scale": scale, "n": n, "m": m, "K": km, "rounds": nr,
                   "core_numbers_ms": round(1000 * t_core, 1),
                   "core_numbers_edges_per_s": round(m / t_core)}
            rows.append(row)
            log(json.dumps(row))
            del off, idx
            torch.cuda.empty_cache()
            continue
        t = time.perf_counter()
        table = {"search_sweep_nodes": sweep} if sweep > 0 else None
        w, cl, st = pmc.max_clique(off, idx, node_budget=budget, allow_budget=True,
                                   tune_table=table)
        torch.cuda.synchronize()
        t_mc = time.perf_counter() - t
        row = {"scale": scale, "n": n, "m": m, "gen_s": round(t_gen, 2),
               "gen_peak_gib": round(gen_peak / 2**30, 1), "K": km, "rounds": nr,
               "core_numbers_ms": round(1000 * t_core, 1),
               "core_numbers_edges_per_s": round(m / t_core),
               "node_budget": budget, "omega": w, "heuristic": st["heuristic"],
               "certified": bool(st["certified"]), "roots": st["roots"],
               "sweep_nodes": sweep, "roots_open_after_sweep": st["roots_second_pass"],
               "roots_branched": st["roots_branched"], "nodes": st["nodes"],
               "max_clique_ms": round(1000 * t_mc, 1),
               "stage_ms": {k: round(v, 2) for k, v in st.items()
                            if k.startswith("ms_") and not k.startswith("ms_k_")}}
        rows.append(row)
        log(json.dumps(row))
        del off, idx, cl
        torch.cuda.empty_cache()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--scales", type=int, nargs="*", default=[22, 24, 27])
    ap.add_argument("--budget", type=int, default=1_000_000)
    ap.add_argument("--json", default=None)
    ap.add_argument("--core-only", action="store_true",
                    help="time pmc_core_numbers only (no maximum-clique solve)")
    ap.add_argument("--sweep", type=int, default=0,
                    help="sweep every root first with this many Branch nodes each (0: off)")
    a = ap.parse_args(argv)
    rows = evaluate(a.scales, a.budget, log=lambda s: print(s, flush=True), core_only=a.core_only,
                    sweep=a.sweep)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
