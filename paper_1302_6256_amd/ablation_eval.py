"""The paper's ablations on sparse social-network-like graphs (Sec. 5: pmc, pmc
without neighbourhood cores, pmc in native order), on seeded Chung-Lu graphs:
the small parity workload (n = 2,000), two mid sizes and the benchmark graph
(n = 10^6, 12 M edges).

Variants, each timed as the best of `reps` pmc_max_clique calls on the same
GPU with the graph resident in HBM (omega must agree):

* default: degeneracy order, neighbourhood-core test on;
* no neighbourhood cores: InitialBranch's core test off;
* pmc-native: roots searched in input (vertex-id) order, each root's reduced
  neighbourhood its neighbours of larger id (the option native_order), with
  only the k-core pruning (neighbourhood cores off), as the paper's variant;
  without the degeneracy bound a subproblem may exceed the 4,096-vertex
  limit, which is then reported instead of a time;
* native dispatch only: orientation by degeneracy rank, roots and heuristic
  seeds visited in input order (a score of minus the vertex id).

  python -m paper_1302_6256_amd.ablation_eval --json ablation.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def _best(pmc, off, idx, reps, **kw):
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


def workloads():
    import graphgen
    return (("chung-lu n=2,000 (parity workload)", lambda: graphgen.c1_graph()),
            ("chung-lu n=100,000 g=2.1 d=24 plant 25",
             lambda: graphgen.chung_lu(100000, 2.1, 24.0, 1549.0, 31, plants=(25,))),
            ("chung-lu n=300,000 g=2.2 d=30 plant 30",
             lambda: graphgen.chung_lu(300000, 2.2, 30.0, 3000.0, 32, plants=(30,))),
            ("chung-lu n=10^6 g=2.1 d=24 plants 20+40 (benchmark)", lambda: graphgen.c2_graph()))


def evaluate(reps=5, log=print):
    import torch
    from . import pmc
    pmc.load()
    dev = torch.device("cuda:0")
    rows = []
    for name, make in workloads():
        g = make()
        off, idx = torch.from_numpy(g.offsets).to(dev), torch.from_numpy(g.indices).to(dev)
        native = -torch.arange(g.n, dtype=torch.float32, device=dev)
        pmc.max_clique(off, idx)  # warm-up
        t0, w0, s0 = _best(pmc, off, idx, reps)
        t1, w1, s1 = _best(pmc, off, idx, reps, use_neighborhood_cores=0)
        t2, w2, s2 = _best(pmc, off, idx, reps, score=native)
        try:
            t3, w3, s3 = _best(pmc, off, idx, reps, native_order=1, use_neighborhood_cores=0)
        except pmc.PmcError as e:
            if e.status != pmc.PMC_ERR_CAPACITY:
                raise
            t3, w3, s3 = None, w0, None
        if not (w0 == w1 == w2 == w3):
            raise SystemExit(f"omega differs between variants on {name}: {w0} {w1} {w2} {w3}")
        row = {"graph": name, "n": g.n, "m": g.m, "omega": w0, "heuristic": s0["heuristic"],
               "heuristic_native": s2["heuristic"], "ms_default": round(1000 * t0, 3),
               "ms_no_neighborhood_cores": round(1000 * t1, 3),
               "ms_native_dispatch": round(1000 * t2, 3),
               "ms_pmc_native": round(1000 * t3, 3) if t3 is not None else "capacity (> 4096)",
               "branched_default": s0["roots_branched"], "branched_no_nc": s1["roots_branched"],
               "branched_native_dispatch": s2["roots_branched"],
               "branched_pmc_native": s3["roots_branched"] if s3 else None,
               "nodes_default": s0["nodes"], "nodes_no_nc": s1["nodes"],
               "nodes_native_dispatch": s2["nodes"], "nodes_pmc_native": s3["nodes"] if s3 else None,
               "roots_default": s0["roots"], "roots_pmc_native": s3["roots"] if s3 else None}
        rows.append(row)
        log(json.dumps(row))
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    rows = evaluate(a.reps, log=lambda s: print(s, flush=True))
    if a.json:
        with open(a.json, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
