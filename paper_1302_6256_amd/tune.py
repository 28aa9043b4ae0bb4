"""Autotuner of the launch parameters, and the batch report.

Objective: time-to-certified omega of a batch of the 2,048-graph workload
(graphgen.c3_graph), solved in one pmc_max_clique_batch call.  Searched, one
knob group at a time (a coordinate search): heuristic waves per CU and seeds
claimed per wave for a batch, then workgroups per CU of the search kernel for
the small (64-128 vertex) and medium (256-512) bitset classes, then whether
the search launches run as one captured hipGraph.  The split of big
subproblems (the smallest root that splits its level-0 branches, and the
split depth) only matters on hard dense instances, so it is chosen on four
dense G(n, p) graphs instead; the single-graph heuristic launch (waves per CU
and seeds per claim) on the 10^6-vertex Chung-Lu benchmark graph.  The best
setting is written to
paper_1302_6256_amd/tuning.json with the device name; the binding applies it
when it loads on the same device model.

  python -m paper_1302_6256_amd.tune tune --graphs 2048
  python -m paper_1302_6256_amd.tune batch --graphs 2048
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import sys
import time

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)


# a knob leaves its current value only for a gain above the timing noise: the
# table applies to single-graph calls too, which a batch-only tie should not
# change
MIN_GAIN = 0.02


def _batch(count):
    """The first `count` graphs of the batch workload, generated on host
    threads (the generator's C calls release the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    import graphgen
    t = time.perf_counter()
    with ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1))) as pool:
        gs = list(pool.map(graphgen.c3_graph, range(count)))
    u, vb = graphgen.concat(gs)
    return u, vb, time.perf_counter() - t


def _solve_ms(pmc, off, idx, vb, reps=3):
    import torch
    ts, om = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        o, _, st = pmc.max_clique_batch(off, idx, vb)
        torch.cuda.synchronize()
        ts.append(1000 * (time.perf_counter() - t))
        if om is not None and o != om:
            raise SystemExit("omega changed between runs")
        om = o
    return float(np.median(ts)), om, st


def tune(count=2048, out=None, log=print):
    import torch
    from . import pmc
    os.environ["PMC_NO_TUNING"] = "1"
    pmc.load()
    pmc.set_tuning(None)
    dev = torch.device("cuda:0")
    u, vb, tgen = _batch(count)
    off, idx = torch.from_numpy(u.offsets).to(dev), torch.from_numpy(u.indices).to(dev)
    pmc.max_clique_batch(off, idx, vb)  # warm-up
    base_ms, om0, _ = _solve_ms(pmc, off, idx, vb)
    log(f"default: {base_ms:.2f} ms ({count} graphs, n={u.n}, m={u.m})")
    table = []
    best = [base_ms, pmc.get_tuning()]

    def trial(cfg):
        pmc.set_tuning(cfg)
        ms, om, _ = _solve_ms(pmc, off, idx, vb)
        if om != om0:
            raise SystemExit(f"omega changed under tuning {cfg}")
        table.append({"config": cfg, "ms": round(ms, 3)})
        log(f"{ms:8.2f} ms  {json.dumps(cfg)}")
        if ms < best[0] * (1.0 - MIN_GAIN):
            best[0], best[1] = ms, cfg

    # coordinate search: heuristic launch, then search launch, then graph mode
    base = best[1]
    for hw, chunk in itertools.product((4, 8, 16, 32), (16, 32, 64)):
        trial(dict(base, heuristic_waves_per_cu=[base["heuristic_waves_per_cu"][0], hw],
                   heuristic_chunk=[base["heuristic_chunk"][0], chunk]))
    base = best[1]
    for small, medium in itertools.product((8, 16, 32), (4, 8, 16)):
        trial(dict(base, search_blocks_per_cu=[small, small, medium, medium, 2, 2, 2]))
    # the split of big subproblems matters on hard dense instances, not on
    # this batch: its knobs are chosen on four dense G(n, p) graphs
    base = best[1]
    split = _tune_split(pmc, base, log)
    best[1] = dict(best[1], **split["best"])
    base = best[1]
    single = _tune_single(pmc, base, log)
    best[1] = dict(best[1], **single["best"])
    base = best[1]
    for graph in (0, 1):
        trial(dict(base, search_graph=graph))
    pmc.set_tuning(None)
    res = {"device": torch.cuda.get_device_name(0),
           "workload": f"first {count} graphs of the 2,048-graph batch (n={u.n}, m={u.m})",
           "objective": "median of 3 batch time-to-certified omega (ms)",
           "default_ms": round(base_ms, 3), "best_ms": round(best[0], 3), "best": best[1],
           "table": table, "split": split, "single": single}
    log(json.dumps({k: v for k, v in res.items() if k != "table"}))
    path = out or os.path.join(PKG, "tuning.json")
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    return res


SPLIT_GRAPHS = ((500, 0.5, 7), (300, 0.7, 7), (150, 0.8, 7), (120, 0.9, 7))


def _tune_single(pmc, base, log):
    """Heuristic waves per CU and seeds per claim of a single-graph call, by
    the median of 5 time-to-certified omega calls on the Chung-Lu benchmark
    graph (10^6 vertices): its seeds are claimed in decreasing core order, so
    the claim size trades claim atomics against the serial share of the
    first, largest seeds."""
    import torch
    import graphgen
    g = graphgen.c2_graph()
    dev = torch.device("cuda:0")
    off, idx = torch.from_numpy(g.offsets).to(dev), torch.from_numpy(g.indices).to(dev)

    def total(cfg):
        pmc.set_tuning(cfg)
        pmc.max_clique(off, idx)
        ts, om = [], None
        for _ in range(5):
            torch.cuda.synchronize()
            t = time.perf_counter()
            w, _, _ = pmc.max_clique(off, idx)
            torch.cuda.synchronize()
            ts.append(1000 * (time.perf_counter() - t))
            if om is not None and w != om:
                raise SystemExit("omega changed between runs")
            om = w
        return float(np.median(ts)), om

    cur = {"heuristic_waves_per_cu": base["heuristic_waves_per_cu"],
           "heuristic_chunk": base["heuristic_chunk"]}
    best_ms, om0 = total(dict(base, **cur))
    table = [{"config": cur, "ms": round(best_ms, 3)}]
    best = cur
    for hw, chunk in itertools.product((4, 8, 16), (1, 4, 16)):
        cfg = {"heuristic_waves_per_cu": [hw, base["heuristic_waves_per_cu"][1]],
               "heuristic_chunk": [chunk, base["heuristic_chunk"][1]]}
        ms, om = total(dict(base, **cfg))
        if om != om0:
            raise SystemExit(f"omega changed under single-graph setting {cfg}")
        table.append({"config": cfg, "ms": round(ms, 3)})
        log(f"{ms:8.2f} ms  single graph {json.dumps(cfg)}")
        if ms < best_ms * (1.0 - MIN_GAIN / 2):
            best_ms, best = ms, cfg
    pmc.set_tuning(base)
    return {"objective": "Chung-Lu n=10^6 (the benchmark graph): median of 5 calls (ms)",
            "best": best, "best_ms": round(best_ms, 3), "table": table}


def _tune_split(pmc, base, log):
    """Split threshold and depth by the geometric mean over four dense
    G(n, p) graphs (p = 0.5 to 0.9) of the time-to-certified omega (median of
    3 calls each): splitting helps the deep searches at high p and must not
    cost the shallow ones at p = 0.5."""
    import torch
    import graphgen
    dev = torch.device("cuda:0")
    gs = []
    for n, p, seed in SPLIT_GRAPHS:
        g = graphgen.gnp(n, p, seed)
        gs.append((torch.from_numpy(g.offsets).to(dev), torch.from_numpy(g.indices).to(dev)))

    def total(cfg):
        pmc.set_tuning(cfg)
        logt, oms = 0.0, []
        for off, idx in gs:
            pmc.max_clique(off, idx)  # warm-up
            ts = []
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                w, _, _ = pmc.max_clique(off, idx)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            logt += math.log(1000 * float(np.median(ts)))
            oms.append(w)
        return math.exp(logt / len(gs)), oms

    cur = {"search_split_min": base["search_split_min"], "search_split_depth": base["search_split_depth"]}
    best_ms, om0 = total(dict(base, **cur))
    table = [{"config": cur, "ms": round(best_ms, 3)}]
    best = cur
    for smin, depth in itertools.product((16, 32, 64, -1), (1, 2)):
        if smin < 0 and depth > 1:
            continue
        cfg = {"search_split_min": smin, "search_split_depth": depth}
        ms, om = total(dict(base, **cfg))
        if om != om0:
            raise SystemExit(f"omega changed under split setting {cfg}")
        table.append({"config": cfg, "ms": round(ms, 3)})
        log(f"{ms:8.2f} ms  dense split {json.dumps(cfg)}")
        if ms < best_ms * (1.0 - MIN_GAIN):
            best_ms, best = ms, cfg
    pmc.set_tuning(base)
    return {"objective": "geometric mean over G(500,0.5), G(300,0.7), G(150,0.8), G(120,0.9) "
                         "of the median of 3 calls (ms)",
            "best": best, "best_ms": round(best_ms, 3), "table": table}


def batch_report(count=2048, tuning=None, log=print):
    """Time-to-certified omega of the whole batch in one call (eager and with
    the captured search graph)."""
    import torch
    from . import pmc
    pmc.load()
    if tuning:
        with open(tuning) as f:
            pmc.set_tuning(json.load(f)["best"])
    dev = torch.device("cuda:0")
    u, vb, tgen = _batch(count)
    log(f"generated {count} graphs in {tgen:.1f} s: n={u.n}, m={u.m}")
    off, idx = torch.from_numpy(u.offsets).to(dev), torch.from_numpy(u.indices).to(dev)
    pmc.max_clique_batch(off, idx, vb)
    ms, om, st = _solve_ms(pmc, off, idx, vb)
    cfg = pmc.get_tuning()
    cfg_g = dict(cfg, search_graph=1)
    pmc.set_tuning(cfg_g)
    ms_g, om_g, st_g = _solve_ms(pmc, off, idx, vb)
    pmc.set_tuning(cfg)
    if om_g != om:
        raise SystemExit("graph mode changed omega")
    rep = {"graphs": count, "n": u.n, "m": u.m, "ms_per_batch": round(ms, 3),
           "ms_per_batch_graph_mode": round(ms_g, 3),
           "ms_search_graph_mode": round(st_g["ms_search"], 3),
           "graphs_per_s": count / (ms / 1000),
           "edges_per_s": u.m / (ms / 1000), "stage_ms": {k: round(st[k], 3) for k in st
                                                         if k.startswith("ms_")},
           "roots": st["roots"], "nodes": st["nodes"], "certified": st["certified"],
           "tuning": cfg, "omega_hist": np.bincount(np.asarray(om)).tolist()}
    log(json.dumps(rep))
    return rep


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("tune")
    t.add_argument("--graphs", type=int, default=2048)
    t.add_argument("--out", default=None)
    b = sub.add_parser("batch")
    b.add_argument("--graphs", type=int, default=2048)
    b.add_argument("--tuning", default=None)
    b.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)  # noqa: E731
    if a.cmd == "tune":
        tune(a.graphs, a.out, log)
    else:
        rep = batch_report(a.graphs, a.tuning, log)
        if a.json:
            with open(a.json, "w") as f:
                json.dump(rep, f, indent=1)


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    main()
