"""Largest temporal strong components (Sec. 6.1) on synthetic temporal
networks shaped like the paper's Table 2 rows.

The contact, interaction and retweet networks of the paper are not available;
seeded synthetic sequences from graphgen.temporal_contacts stand in for them
(group structure with within-group contacts; symmetric contacts for the
contact / interaction rows, mostly one-way edges for the retweet rows).  For
each: the strong-reachability graph on the GPU (pmc_strong_reachability), then
its maximum clique (pmc_max_clique), with a node budget so an intractable case
reports "not certified" instead of running on.

  python -m paper_1302_6256_amd.temporal_eval --json temporal.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

# name, people, contacts, groups, p_within, seed, directed fraction
WORKLOADS = (("infect-hyper stand-in", 113, 10000, 3, 0.7, 21, 0.0),
             ("infect-dublin stand-in", 11000, 150000, 3000, 0.9995, 22, 0.0),
             ("fb-messages stand-in", 1900, 10000, 200, 0.95, 23, 0.3),
             ("reality stand-in", 6800, 40000, 400, 0.995, 24, 0.0),
             ("retweet stand-in", 18000, 120000, 300, 0.9, 25, 0.9),
             ("twitter-copen stand-in", 8600, 45000, 400, 0.97, 26, 0.8))


def evaluate(budget=50_000_000, log=print):
    import torch
    import graphgen
    from . import pmc
    pmc.load()
    dev = torch.device("cuda:0")
    rows = []
    for name, n, contacts, groups, pw, seed, dfrac in WORKLOADS:
        src, dst = graphgen.temporal_contacts(n, contacts, groups, pw, seed, directed_frac=dfrac)
        s = torch.tensor(src, device=dev)
        t = torch.tensor(dst, device=dev)
        pmc.strong_reachability(n, s, t)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        off, idx = pmc.strong_reachability(n, s, t)
        torch.cuda.synchronize()
        t_reach = time.perf_counter() - t0
        t0 = time.perf_counter()
        try:
            pmc.max_clique(off, idx, node_budget=budget, allow_budget=True)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            w, cl, st = pmc.max_clique(off, idx, node_budget=budget, allow_budget=True)
        except pmc.PmcError as e:  # e.g. a neighbourhood beyond the search's 4,096 vertices
            log(json.dumps({"graph": name, "error": str(e)}))
            continue
        torch.cuda.synchronize()
        t_clique = time.perf_counter() - t0
        deg = np.diff(off.cpu().numpy())
        row = {"graph": name, "temporal_edges": int(src.shape[0]), "n": n,
               "reach_vertices": int((deg > 0).sum()), "reach_edges": int(idx.numel() // 2),
               "K": st["kmax"], "heuristic": st["heuristic"], "omega": w,
               "certified": bool(st["certified"]), "certified_early": bool(st["certified_early"]),
               "ms_reach": round(1000 * t_reach, 2), "ms_clique": round(1000 * t_clique, 2)}
        rows.append(row)
        log(json.dumps(row))
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--json", default=None)
    ap.add_argument("--budget", type=int, default=50_000_000)
    a = ap.parse_args(argv)
    rows = evaluate(a.budget, log=lambda s: print(s, flush=True))
    if a.json:
        with open(a.json, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
