"""Pins of the oracle's heuristic, maximum clique and per-root search.

omega: 2^n brute force (n <= 16), textbook Bron-Kerbosch with pivoting,
networkx.find_cliques (library), closed forms (K_n -> n, C_n -> 2 for n > 3,
Turan T(n,r) -> r, cocktail party on 2r vertices -> r, bipartite -> 2,
edgeless -> 1, empty -> 0), planted cliques (omega >= k), Fact 1's chain
omega~ <= omega <= L <= K+1 <= Delta+1, and pairwise adjacency of the witness.
Per-root values: 1 + omega of the oriented neighbourhood by brute force,
networkx core numbers of the neighbourhood, Fact 1 on each neighbourhood.
"""
import itertools

import networkx as nx
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import graphgen as gg
import oracle
from refs import adj_sets, bron_kerbosch_omega, brute_force_omega, check_greedy_colouring, \
    dense, is_clique


def nx_omega(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    src = np.repeat(np.arange(g.n), np.diff(g.offsets))
    G.add_edges_from(zip(src.tolist(), g.indices.tolist()))
    return max((len(c) for c in nx.find_cliques(G)), default=0)


def tiny_graphs():
    gs = []
    for i, (n, p) in enumerate([(6, 0.5), (9, 0.6), (12, 0.5), (14, 0.7), (16, 0.4), (16, 0.8),
                                (15, 0.9), (13, 0.3)]):
        gs.append(gg.gnp(n, p, 1000 + i))
    return gs


@pytest.mark.parametrize("g", tiny_graphs(), ids=lambda g: g.name)
def test_max_clique_vs_brute_force(g):
    adj = adj_sets(g)
    w, cl, st = oracle.max_clique(g.offsets, g.indices)
    assert w == brute_force_omega(adj)
    assert len(cl) == w and is_clique(adj, cl.tolist())
    w2, _, _ = oracle.max_clique(g.offsets, g.indices, use_neigh_cores=False)
    assert w2 == w


@settings(max_examples=60, deadline=None)
@given(n=st.integers(0, 14), p=st.floats(0.0, 1.0), seed=st.integers(0, 2**31))
def test_max_clique_hypothesis_brute_force(n, p, seed):
    g = gg.gnp(n, p, seed)
    adj = adj_sets(g)
    w, cl, _ = oracle.max_clique(g.offsets, g.indices)
    assert w == brute_force_omega(adj)
    assert len(cl) == w and is_clique(adj, cl.tolist())


def medium_graphs():
    gs = [gg.gnp(n, p, 2000 + i) for i, (n, p) in enumerate(
        [(40, 0.5), (60, 0.6), (80, 0.3), (120, 0.15), (150, 0.5), (200, 0.05), (100, 0.75)])]
    gs += [gg.chung_lu(400, 2.2, 12.0, 100.0, 31, plants=(9,)),
           gg.chung_lu(800, 2.1, 20.0, 200.0, 32, plants=(12, 14)),
           gg.chung_lu(600, 2.5, 8.0, 60.0, 33)]
    return gs


@pytest.mark.parametrize("g", medium_graphs(), ids=lambda g: g.name)
def test_max_clique_vs_bron_kerbosch(g):
    adj = adj_sets(g)
    w, cl, st = oracle.max_clique(g.offsets, g.indices)
    assert w == bron_kerbosch_omega(adj)
    assert len(cl) == w and is_clique(adj, cl.tolist())
    # Fact 1: omega~ <= omega <= L <= K+1 <= Delta+1
    core, rnd, km, _ = oracle.peel(g.offsets, g.indices)
    rk, order = oracle.rank(rnd)
    L, col = oracle.greedy_colour(dense(g), order[::-1].copy())
    delta = int(np.diff(g.offsets).max())
    assert st["heuristic"] <= w <= L <= km + 1 <= delta + 1
    assert st["kmax"] == km


def test_max_clique_c1_networkx():
    g = gg.c1_graph()
    w, cl, st = oracle.max_clique(g.offsets, g.indices)
    assert w == nx_omega(g) == 15
    assert set(cl.tolist()) == set(g.planted.tolist())


@pytest.mark.parametrize("i", range(3))
def test_max_clique_chung_lu_networkx(i):
    g = gg.chung_lu(3000, 2.1, 16.0, 300.0, 4000 + i, plants=(6,))
    w, cl, st = oracle.max_clique(g.offsets, g.indices)
    assert w == nx_omega(g)
    assert is_clique(adj_sets(g), cl.tolist())


def test_closed_forms():
    for n in range(0, 9):
        g = gg.complete(n)
        assert oracle.max_clique(g.offsets, g.indices)[0] == n
    for n in range(4, 12):
        g = gg.cycle(n)
        assert oracle.max_clique(g.offsets, g.indices)[0] == 2
    assert oracle.max_clique(*(lambda g: (g.offsets, g.indices))(gg.cycle(3)))[0] == 3
    for n, r in [(6, 2), (9, 3), (12, 4), (20, 5), (21, 7), (30, 6)]:
        g = gg.turan(n, r)
        assert oracle.max_clique(g.offsets, g.indices)[0] == r
    for r in range(1, 8):
        g = gg.cocktail_party(r)
        assert oracle.max_clique(g.offsets, g.indices)[0] == r
    for a, b in [(1, 1), (2, 5), (4, 4)]:
        g = gg.complete_bipartite(a, b)
        assert oracle.max_clique(g.offsets, g.indices)[0] == 2
    assert oracle.max_clique(*(lambda g: (g.offsets, g.indices))(gg.empty(7)))[0] == 1
    g = gg.empty(0)
    assert oracle.max_clique(g.offsets, g.indices)[0] == 0
    g = gg.grid(5, 6)
    assert oracle.max_clique(g.offsets, g.indices)[0] == 2
    g = gg.disjoint_cliques([3, 7, 5, 7])
    w, cl, _ = oracle.max_clique(g.offsets, g.indices)
    assert w == 7 and is_clique(adj_sets(g), cl.tolist())


@pytest.mark.parametrize("k", [5, 11, 20])
def test_planted(k):
    g = gg.gnp(500, 0.02, 77 + k, plants=(k,))
    w, cl, _ = oracle.max_clique(g.offsets, g.indices)
    assert w >= k
    assert w == k  # the sparse background has no clique near k
    assert set(cl.tolist()) == set(g.planted.tolist())


# ----------------------------------------------------------------- heuristic

@pytest.mark.parametrize("g", tiny_graphs() + medium_graphs(), ids=lambda g: g.name)
def test_heuristic_is_clique_and_below_omega(g):
    core, rnd, km, _ = oracle.peel(g.offsets, g.indices)
    rk, order = oracle.rank(rnd)
    adj = adj_sets(g)
    w = oracle.max_clique(g.offsets, g.indices)[0]
    for tau in (-1, 0, 2):
        h = oracle.heuristic(g.offsets, g.indices, core, rk, order, tau)
        assert is_clique(adj, h.tolist()) and 1 <= len(h) <= w


def test_heuristic_closed_forms():
    def heur(g, tau=-1):
        core, rnd, _, _ = oracle.peel(g.offsets, g.indices)
        rk, order = oracle.rank(rnd)
        return oracle.heuristic(g.offsets, g.indices, core, rk, order, tau)
    for n in (1, 2, 6, 13):
        assert len(heur(gg.complete(n))) == n
    for n, r in [(9, 3), (12, 4), (25, 5)]:
        # every maximal clique of a complete multipartite graph has one vertex per part
        assert len(heur(gg.turan(n, r))) == r
        assert len(heur(gg.turan(n, r), 0)) == r
    h = heur(gg.disjoint_cliques([4, 9, 6]))
    assert len(h) == 9
    assert len(heur(gg.star(8))) == 2
    assert len(heur(gg.empty(4))) == 1


def test_heuristic_frozen_first_fit():
    """Frozen mode: each seed's clique is first-fit over the filtered
    neighbours by decreasing rank, started from {seed}; H is the first seed
    (decreasing rank) reaching the largest size.  Checked by enumerating the
    greedy choices directly on small graphs."""
    for g in tiny_graphs()[:5] + medium_graphs()[:3]:
        core, rnd, _, _ = oracle.peel(g.offsets, g.indices)
        rk, order = oracle.rank(rnd)
        adj = adj_sets(g)
        for tau in (0, 3):
            best, bestC = 0, None
            for v in order[::-1]:
                cand = [u for u in adj[v] if core[u] >= tau]
                cand.sort(key=lambda u: -rk[u])
                C = [v]
                for u in cand:
                    if all(u in adj[c] for c in C):
                        C.append(u)
                if len(C) > best:
                    best, bestC = len(C), sorted(C)
            h = oracle.heuristic(g.offsets, g.indices, core, rk, order, tau)
            assert h.tolist() == bestC


# --------------------------------------------------------- per-root search

@pytest.mark.parametrize("g", tiny_graphs() + medium_graphs()[:4], ids=lambda g: g.name)
def test_root_omega_frozen_zero(g):
    adj = adj_sets(g)
    core, rnd, km, _ = oracle.peel(g.offsets, g.indices)
    rk, order = oracle.rank(rnd)
    r = oracle.root_omega(g.offsets, g.indices, 0)
    w = oracle.max_clique(g.offsets, g.indices)[0]
    assert (r["omega"].max() if g.n else 0) == w  # every clique appears at its lowest-rank member
    for v in range(g.n):
        P = sorted(u for u in adj[v] if rk[u] > rk[v])
        assert r["s"][v] == len(P)
        sub = [adj[u] & set(P) for u in P]
        idx = {u: i for i, u in enumerate(P)}
        sub_l = [{idx[x] for x in s} for s in sub]
        wv = 1 + (bron_kerbosch_omega(sub_l) if P else 0)
        assert r["omega"][v] == wv
        if P:
            G = nx.Graph()
            G.add_nodes_from(range(len(P)))
            G.add_edges_from((i, j) for i in range(len(P)) for j in sub_l[i] if i < j)
            kn = max(nx.core_number(G).values())
        else:
            kn = -1
        assert r["kn"][v] == kn
        # Fact 1 on the neighbourhood: omega <= L <= K + 1
        assert wv - 1 <= r["L"][v] <= kn + 1


def test_root_omega_frozen_bound():
    g = medium_graphs()[7]
    w = oracle.max_clique(g.offsets, g.indices)[0]
    r0 = oracle.root_omega(g.offsets, g.indices, 0)
    for b in (2, w - 1, w):
        r = oracle.root_omega(g.offsets, g.indices, b)
        for v in range(g.n):
            if r0["omega"][v] > b:
                assert r["omega"][v] == r0["omega"][v]
            else:
                assert r["omega"][v] in (0, -1)


# ------------------------------------------------------ local peel / colour

@pytest.mark.parametrize("seed", range(6))
def test_local_peel_and_colouring(seed):
    g = gg.gnp(25 + 5 * seed, 0.2 + 0.1 * seed, 500 + seed)
    a = dense(g)
    kn, lr = oracle.local_peel(a)
    G = nx.from_numpy_array(a)
    ref = nx.core_number(G)
    assert kn.tolist() == [ref[v] for v in range(g.n)]
    adj = adj_sets(g)
    # reverse peel order: by decreasing (round, index); colours <= K + 1 (Fact 1)
    order = sorted(range(g.n), key=lambda v: (-lr[v], -v))
    L, col = oracle.greedy_colour(a, np.array(order, dtype=np.int32))
    assert check_greedy_colouring(adj, order, col) is None
    assert L <= kn.max() + 1
    nat = list(range(g.n))
    L2, col2 = oracle.greedy_colour(a, np.array(nat, dtype=np.int32))
    assert check_greedy_colouring(adj, nat, col2) is None
    assert L2 >= brute_force_omega(adj) if g.n <= 18 else True


def test_colouring_turan_any_order():
    g = gg.turan(12, 4)
    a = dense(g)
    for perm in itertools.islice(itertools.permutations(range(12)), 0, 2000, 97):
        L, col = oracle.greedy_colour(a, np.array(perm, dtype=np.int32))
        assert L == 4  # each part is forced into one colour


def test_c2_stored_omega_pinned_by_networkx():
    """The benchmark graph's stored omega (written from the oracle) agrees
    with the value tests/golden/make_golden.py derived from networkx alone
    (planted 40-set, and an exact networkx clique search in the 39-core of
    every oriented neighbourhood of the 40-core): two independent routes."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "c2.json")) as f:
        gold = json.load(f)
    assert gold["omega_networkx"] == gold["omega"] == 40
    assert "networkx only" in gold["networkx_source"]
    assert len(gold["clique"]) == gold["omega"]
