"""Writes the stored expected values of tests/golden/ from the CPU oracle
(and, for C2's third pin, from networkx alone).

Calls only the oracle, networkx and the shared input generators.  Run:
    python tests/golden/make_golden.py [c2 | c2nx | c3 | c4 | split] ...
(no argument: all of them).  c2nx is the slow one (networkx on the n = 10^6
benchmark graph: its 40-core and an exact clique search in each oriented
neighbourhood's 39-core).
"""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

SOURCE = "written by tests/golden/make_golden.py from the CPU oracle only"


def _dump(name, out):
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f, indent=1)


def c2():
    g = gg.c2_graph()
    t = time.time()
    w, cl, st = oracle.max_clique(g.offsets, g.indices)
    path = os.path.join(HERE, "c2.json")
    old = json.load(open(path)) if os.path.exists(path) else {}
    out = {
        "workload": g.name,
        "source": "oracle.max_clique (CPU oracle), written by tests/golden/make_golden.py",
        "n": g.n, "m": g.m, "omega": w, "kmax": st["kmax"], "nrounds": st["nrounds"],
        "heuristic": st["heuristic"], "survivors": st["survivors"],
        "clique": cl.tolist(), "oracle_seconds": round(time.time() - t, 2),
    }
    for k in ("omega_networkx", "networkx_source", "networkx_seconds"):
        if k in old:
            out[k] = old[k]
    _dump("c2.json", out)
    print(json.dumps({k: v for k, v in out.items() if k != "clique"}))


def c2nx():
    """A pin of C2's omega independent of the oracle, from networkx alone:
    omega >= 40 because the planted 40-set is pairwise adjacent; omega <= 40
    because a clique of 41 vertices lies in the 40-core and, under any total
    order of its vertices, consists of its first vertex v and 40 pairwise
    adjacent vertices ordered after v among v's neighbours.  For every v of
    the 40-core (order: networkx core number, then id), those later
    neighbours P(v) are checked: a 40-clique in G[P(v)] lies in its 39-core
    (networkx k_core), on which networkx's exact max_weight_clique is run
    whenever that core is not empty."""
    import networkx as nx
    import numpy as np
    g = gg.c2_graph()
    t = time.time()
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    src = np.repeat(np.arange(g.n), np.diff(g.offsets))
    keep = src < g.indices
    G.add_edges_from(zip(src[keep].tolist(), g.indices[keep].tolist()))
    plant = [int(v) for v in g.planted[20:60]]  # the second plant: 40 vertices
    assert len(plant) == 40
    lower = 40 if all(G.has_edge(a, b) for i, a in enumerate(plant) for b in plant[i + 1:]) else 0
    core = nx.core_number(G)
    core40 = nx.k_core(G, 40, core_number=core)
    key = {v: (core[v], v) for v in core40}
    best, exact_runs = 0, 0
    for v in core40:
        P = [u for u in core40.adj[v] if key[u] > key[v]]
        if len(P) < 40:
            continue
        sub = nx.k_core(core40.subgraph(P), 39)
        if sub.number_of_nodes() == 0:
            continue
        exact_runs += 1
        clique, size = nx.max_weight_clique(sub, weight=None)
        best = max(best, size + 1)
    upper = max(best, 40 if lower == 40 else 0)
    w = 40 if lower == 40 and upper <= 40 else -1
    path = os.path.join(HERE, "c2.json")
    out = json.load(open(path))
    out["omega_networkx"] = w
    out["networkx_source"] = (
        "networkx only: the planted 40-set is a clique (omega >= 40); for each of the "
        f"{core40.number_of_nodes()} vertices v of networkx.k_core(G, 40), the 39-core of G[later "
        "neighbours of v] (order: networkx.core_number, then id) is empty or its "
        f"networkx.max_weight_clique has at most 39 vertices ({exact_runs} exact runs; largest "
        f"clique through a first vertex: {best if best else 'none above 40'}), so no 41-clique exists")
    out["networkx_seconds"] = round(time.time() - t, 1)
    _dump("c2.json", out)
    print("c2 networkx omega", w, "exact runs", exact_runs, out["networkx_seconds"], "s")


def _omega(i_kind):
    kind, i = i_kind
    g = gg.c3_graph(i) if kind == "c3" else gg.c4_graph(i)
    t = time.time()
    w, cl, st = oracle.max_clique(g.offsets, g.indices)
    return {"i": i, "name": g.name, "n": g.n, "m": g.m, "omega": w, "kmax": st["kmax"],
            "heuristic": st["heuristic"], "seconds": round(time.time() - t, 3)}


def c3(workers=8):
    with ProcessPoolExecutor(workers) as ex:
        rows = list(ex.map(_omega, [("c3", i) for i in range(2048)], chunksize=8))
    _dump("c3.json", {"workload": "c3 batch of 2,048 graphs (graphgen.c3_graph(0..2047))",
                      "source": SOURCE, "graphs": rows})
    print("c3:", len(rows), "graphs, max omega", max(r["omega"] for r in rows),
          "oracle seconds", round(sum(r["seconds"] for r in rows), 1))


C4_HELD_OUT = [10**6 + i for i in range(8)]


def c4(workers=8):
    with ProcessPoolExecutor(workers) as ex:
        rows = list(ex.map(_omega, [("c4", i) for i in C4_HELD_OUT]))
    _dump("c4_heldout.json", {"workload": "c4 held-out graphs (graphgen.c4_graph(10^6 + i), "
                                          "n = 200,000)", "source": SOURCE, "graphs": rows})
    print("c4:", [(r["i"], r["omega"]) for r in rows])


SPLIT_GRAPHS = [("gnp", 120, 0.9, 3), ("gnp", 300, 0.7, 2)]


def split():
    rows = []
    for kind, n, p, seed in SPLIT_GRAPHS:
        g = gg.gnp(n, p, seed)
        t = time.time()
        w, _, _ = oracle.max_clique_ex(g.offsets, g.indices, threads=os.cpu_count() or 1)
        rows.append({"kind": kind, "n": n, "p": p, "seed": seed, "omega": w,
                     "seconds": round(time.time() - t, 1)})
    _dump("split_graphs.json", {"source": SOURCE + " (threaded mode, or_max_clique_ex)",
                                "graphs": rows})
    print("split:", rows)


if __name__ == "__main__":
    jobs = sys.argv[1:] or ["c2", "c3", "c4", "split", "c2nx"]
    for j in jobs:
        {"c2": c2, "c2nx": c2nx, "c3": c3, "c4": c4, "split": split}[j]()
