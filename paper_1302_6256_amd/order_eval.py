"""Clique-peeling order for compression (Sec. 6.2): how local does it make the
adjacency lists?

The paper permutes two Facebook graphs by the clique-peeling order and
compresses them with bvgraph; neither the graphs nor bvgraph are available
here.  Seeded stand-ins of the same size (n = 42,000 and 36,000, ~1.4-1.6 M
edges, a Chung-Lu background plus many planted cliques for the local density
of a social network, vertex ids shuffled) are permuted three ways: the native
(shuffled) ids, the degeneracy order, and the clique-peeling order computed on
the GPU.  The figure of merit is the log-gap cost that gap-coding compressors
such as bvgraph pay: for every adjacency list in the new numbering, sorted,
the sum over entries of log2(1 + |gap|), the first gap taken from the list's
own vertex, reported in bits per edge (lower is better).

  python -m paper_1302_6256_amd.order_eval --json order.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

WORKLOADS = (("fb-Penn stand-in", 42000, 57.0, 2600, 11),
             ("fb-Texas stand-in", 36000, 79.0, 2300, 12))


def social_graph(n, dbar, cliques, seed):
    import graphgen
    rng = np.random.Generator(np.random.Philox(seed))
    plants = tuple(int(k) for k in rng.integers(4, 24, size=cliques))
    return graphgen.chung_lu(n, 2.4, dbar, float(np.sqrt(n * dbar)), seed, plants=plants)


def log_gap_bits(offsets, indices, pos):
    """Sum over adjacency entries of log2(1 + |gap|) under the numbering pos."""
    n = offsets.shape[0] - 1
    deg = np.diff(offsets)
    src = np.repeat(np.arange(n), deg)
    new_src = pos[src]
    new_dst = pos[indices]
    o = np.lexsort((new_dst, new_src))
    a, b = new_src[o], new_dst[o]
    prev = np.empty_like(b)
    prev[1:] = b[:-1]
    first = np.ones(b.shape[0], dtype=bool)
    first[1:] = a[1:] != a[:-1]
    prev[first] = a[first]
    return float(np.log2(1.0 + np.abs(b.astype(np.int64) - prev.astype(np.int64))).sum())


def evaluate(log=print):
    import torch
    from . import pmc
    pmc.load()
    dev = torch.device("cuda:0")
    rows = []
    for name, n, dbar, cliques, seed in WORKLOADS:
        g = social_graph(n, dbar, cliques, seed)
        off, idx = torch.from_numpy(g.offsets).to(dev), torch.from_numpy(g.indices).to(dev)
        pmc.clique_order(off, idx)  # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        order, block = pmc.clique_order(off, idx)
        torch.cuda.synchronize()
        t_order = time.perf_counter() - t
        _, _, rank, _, _, _ = pmc.core_numbers(off, idx)
        order = order.cpu().numpy()
        pos_clique = np.empty(g.n, dtype=np.int64)
        pos_clique[order] = np.arange(g.n)
        pos_native = np.arange(g.n, dtype=np.int64)
        pos_degen = rank.cpu().numpy().astype(np.int64)
        nnz = g.indices.shape[0]
        bits = {k: log_gap_bits(g.offsets, g.indices, p) / nnz
                for k, p in (("native", pos_native), ("degeneracy", pos_degen),
                             ("clique", pos_clique))}
        sizes = np.diff(block.cpu().numpy())
        row = {"graph": name, "n": g.n, "m": g.m, "blocks": int(sizes.shape[0]),
               "largest_block": int(sizes.max()), "vertices_in_blocks_ge_3": int(sizes[sizes >= 3].sum()),
               "ms_clique_order": round(1000 * t_order, 2),
               "bits_per_edge": {k: round(v, 3) for k, v in bits.items()}}
        rows.append(row)
        log(json.dumps(row))
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    rows = evaluate(log=lambda s: print(s, flush=True))
    if a.json:
        with open(a.json, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
