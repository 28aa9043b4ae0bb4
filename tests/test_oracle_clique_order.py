"""Pins of the clique-peeling order (Sec. 6.2) in the oracle: closed forms on
disjoint cliques, complete and edgeless graphs; on random graphs every block
is a clique that was maximal among the vertices still unplaced, the first
block is the heuristic's largest seed clique (Alg. 1 with C = {v}, every seed,
an independently pinned oracle function) and at most omega."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from refs import adj_sets, bron_kerbosch_omega


def order_of(g):
    _, rnd, _, _ = oracle.peel(g.offsets, g.indices)
    rk, _ = oracle.rank(rnd)
    o, b = oracle.clique_order(g.offsets, g.indices, rk)
    return o, b, rk


def adjsets(g):
    return [set(g.indices[g.offsets[v]:g.offsets[v + 1]].tolist()) for v in range(g.n)]


def test_disjoint_cliques_are_the_blocks():
    sizes = (5, 3, 7, 1, 3, 9)
    g = gg.permuted(gg.disjoint_cliques(sizes), 11)
    o, b, _ = order_of(g)
    adj = adjsets(g)
    assert sorted(o.tolist()) == list(range(g.n))
    got = [int(b[i + 1] - b[i]) for i in range(len(b) - 1)]
    assert got == sorted(sizes, reverse=True)
    for i in range(len(b) - 1):
        blk = o[b[i]:b[i + 1]].tolist()
        for x in blk:  # a whole component
            assert adj[x] == set(blk) - {x}


def test_complete_and_edgeless():
    o, b, _ = order_of(gg.complete(12))
    assert b.tolist() == [0, 12] and sorted(o.tolist()) == list(range(12))
    g = gg.empty(9)
    o, b, rk = order_of(g)
    assert b.tolist() == list(range(10))
    assert o.tolist() == sorted(range(9), key=lambda v: -rk[v])  # keys (1, rank) descending


def test_degree_order_inside_a_block():
    # a 4-clique with pendant vertices of different degrees
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (0, 4), (0, 5), (1, 6)]
    g = gg.from_edges(7, edges)
    o, b, _ = order_of(g)
    first = o[b[0]:b[1]].tolist()
    assert first == [0, 1, 2, 3]  # degrees 5, 4, 3, 3 (ties by id)


@pytest.mark.parametrize("g", [gg.c1_graph(), gg.gnp(120, 0.2, 3), gg.gnp(60, 0.5, 4),
                               gg.chung_lu(1500, 2.2, 10.0, 150.0, 9, plants=(8,)), gg.grid(9, 11)],
                         ids=lambda g: g.name)
def test_blocks_are_maximal_cliques(g):
    o, b, rk = order_of(g)
    adj = adjsets(g)
    assert sorted(o.tolist()) == list(range(g.n))
    pos = np.empty(g.n, dtype=np.int64)
    pos[o] = np.arange(g.n)
    for i in range(len(b) - 1):
        blk = o[b[i]:b[i + 1]].tolist()
        for x in blk:
            assert set(blk) - {x} <= adj[x]
        # maximal among the vertices placed after it (all unplaced at its pass)
        common = set.intersection(*(adj[x] for x in blk))
        assert not any(pos[y] >= b[i + 1] for y in common)
    core, _, _, _ = oracle.peel(g.offsets, g.indices)
    _, rnd, _, _ = oracle.peel(g.offsets, g.indices)
    rk2, od = oracle.rank(rnd)
    h = oracle.heuristic(g.offsets, g.indices, core, rk2, od, frozen_tau=0)
    assert b[1] - b[0] == len(h)
    assert b[1] - b[0] <= bron_kerbosch_omega(adj_sets(g))
