"""Pins of the oracle's variants and test modes, and of the parts of the
per-root search that were pinned only by Fact 1 before.

* Threaded search (Sec. 4.5: workers on a task queue sharing the bound):
  omega equals brute force / Bron-Kerbosch for every thread count, and the
  witness is a clique.
* Dispatch permutations and scripted bound raises (the CPU stand-in for racing
  workers): omega never changes; a raise below omega still ends with a
  maximum clique; a raise above omega is kept, with no clique larger than it.
* Native order (Sec. 5, "pmc-native"): neighbourhoods oriented by vertex id;
  omega unchanged; per-root sizes and omega_v against definitions written
  here (set comprehension, brute force).
* InitialBranch's colour count L at bounds b > 0 (Alg. 2, InitialBranch;
  Fact 1), recomputed independently in open form: networkx core numbers of
  G[N+(v)], the drop of K_N(x) < b - 1, a level-synchronous peel written here
  and checked by the fixed-point characterisation, and first-fit colouring in
  reverse (round, index) order checked by the first-fit characterisation.
* The production heuristic (Alg. 1 with its seed-skip rule K(v) < max and
  the threshold K(u) >= max, max the running best) re-enumerated here.
"""
import itertools
import random

import networkx as nx
import numpy as np
import pytest

import graphgen as gg
import oracle
from refs import adj_sets, bron_kerbosch_omega, brute_force_omega, check_greedy_colouring, \
    check_peel, is_clique


def tiny():
    return [gg.gnp(n, p, 3000 + i) for i, (n, p) in enumerate(
        [(8, 0.5), (11, 0.6), (13, 0.7), (15, 0.5), (16, 0.85), (14, 0.3)])]


def medium():
    gs = [gg.gnp(n, p, 3100 + i) for i, (n, p) in enumerate(
        [(50, 0.5), (70, 0.6), (120, 0.2), (90, 0.75)])]
    gs += [gg.chung_lu(500, 2.2, 12.0, 100.0, 3150, plants=(9,)),
           gg.chung_lu(900, 2.1, 20.0, 220.0, 3151, plants=(12, 14))]
    return gs


def ref_omega(g):
    adj = adj_sets(g)
    return brute_force_omega(adj) if g.n <= 16 else bron_kerbosch_omega(adj)


# ------------------------------------------------------------ threaded search

@pytest.mark.parametrize("g", tiny() + medium(), ids=lambda g: g.name)
def test_threads_omega(g):
    w0 = ref_omega(g)
    adj = adj_sets(g)
    for T in (1, 2, 4, 8):
        w, cl, st = oracle.max_clique_ex(g.offsets, g.indices, threads=T)
        assert w == w0, T
        assert st["witness"] == w and is_clique(adj, cl.tolist())
        assert st["heuristic"] <= w <= st["kmax"] + 1


def test_threads_closed_forms():
    cases = [(gg.complete(9), 9), (gg.cycle(11), 2), (gg.turan(20, 5), 5),
             (gg.cocktail_party(6), 6), (gg.complete_bipartite(3, 5), 2), (gg.empty(5), 1),
             (gg.empty(0), 0), (gg.disjoint_cliques([4, 8, 6]), 8)]
    for g, w0 in cases:
        for T in (1, 3, 16):
            assert oracle.max_clique_ex(g.offsets, g.indices, threads=T)[0] == w0


def test_threads_c1():
    g = gg.c1_graph()
    for T in (2, 8):
        w, cl, _ = oracle.max_clique_ex(g.offsets, g.indices, threads=T)
        assert w == 15 and set(cl.tolist()) == set(g.planted.tolist())


# ---------------------------------------- dispatch order and bound injection

@pytest.mark.parametrize("g", tiny() + medium(), ids=lambda g: g.name)
def test_dispatch_orders(g):
    w0 = ref_omega(g)
    adj = adj_sets(g)
    core, rnd, _, _ = oracle.peel(g.offsets, g.indices)
    rk, order = oracle.rank(rnd)
    rng = np.random.default_rng(g.n)
    orders = {"reversed": order[::-1].copy(), "ids": np.arange(g.n, dtype=np.int32),
              "random": rng.permutation(g.n).astype(np.int32),
              # adversarial: the largest neighbourhoods first
              "big_first": np.argsort(-np.diff(g.offsets), kind="stable").astype(np.int32)}
    for name, d in orders.items():
        for T in (1, 4):
            w, cl, st = oracle.max_clique_ex(g.offsets, g.indices, threads=T, dispatch=d)
            assert w == w0, (name, T)
            assert st["witness"] == w and is_clique(adj, cl.tolist()), (name, T)


@pytest.mark.parametrize("g", tiny() + medium(), ids=lambda g: g.name)
def test_bound_injection(g):
    w0 = ref_omega(g)
    adj = adj_sets(g)
    rnd = random.Random(g.n * 7 + 1)
    for trial in range(6):
        # raises below omega at random queue positions: the search still ends
        # with a clique of size omega
        inj = [(rnd.randrange(max(g.n, 1)), rnd.randrange(0, max(w0, 1))) for _ in range(3)]
        for T in (1, 4):
            w, cl, st = oracle.max_clique_ex(g.offsets, g.indices, threads=T, inject=inj)
            assert w == w0 and st["witness"] == w0 and is_clique(adj, cl.tolist()), (inj, T)
    if g.n:
        # a raise to omega: the bound is omega (the witness may be smaller);
        # a raise past omega is kept and nothing larger is ever found
        w, cl, st = oracle.max_clique_ex(g.offsets, g.indices, inject=[(0, w0)])
        assert w == w0 and st["witness"] <= w0 and is_clique(adj, cl.tolist())
        # (when the heuristic already certifies omega by Fact 1 no root starts,
        # so nothing is injected)
        w, cl, st = oracle.max_clique_ex(g.offsets, g.indices, inject=[(0, w0 + 3)])
        assert w == (w0 if st["certified_early"] else w0 + 3) and st["witness"] <= w0


# ------------------------------------------------------------- native order

@pytest.mark.parametrize("g", tiny() + medium(), ids=lambda g: g.name)
def test_native_order_omega(g):
    w0 = ref_omega(g)
    adj = adj_sets(g)
    for nc in (True, False):
        for T in (1, 4):
            w, cl, st = oracle.max_clique_ex(g.offsets, g.indices, use_neigh_cores=nc,
                                             native=True, threads=T)
            assert w == w0 and st["witness"] == w and is_clique(adj, cl.tolist())


@pytest.mark.parametrize("g", tiny() + medium()[:2], ids=lambda g: g.name)
def test_native_root_omega(g):
    """Per root under native orientation: s = |{u in N(v): u > v, K(u) >= b}|
    and omega_v = 1 + omega(G[that set]) when it exceeds b (else 0)."""
    adj = adj_sets(g)
    core = oracle.peel(g.offsets, g.indices)[0]
    w0 = ref_omega(g)
    for b in (0, 2, max(w0 - 1, 0)):
        r = oracle.root_omega(g.offsets, g.indices, b, native=True)
        for v in range(g.n):
            if core[v] < b:
                assert r["s"][v] == -1
                continue
            P = sorted(u for u in adj[v] if u > v and core[u] >= b)
            assert r["s"][v] == len(P)
            loc = {u: i for i, u in enumerate(P)}
            sub = [{loc[x] for x in adj[u] if x in loc} for u in P]
            wv = 1 + (brute_force_omega(sub) if len(P) <= 16 else bron_kerbosch_omega(sub))
            assert r["omega"][v] == (wv if wv > b else 0), (v, b)
        if b == 0:
            assert r["omega"].max() == w0


def test_native_orientation_differs():
    """The option changes the subproblems (not only the dispatch): on a graph
    whose ids are not in degeneracy order the per-root sizes differ."""
    g = medium()[4]
    a = oracle.root_omega(g.offsets, g.indices, 0, native=False)["s"]
    b = oracle.root_omega(g.offsets, g.indices, 0, native=True)["s"]
    assert not np.array_equal(a, b)
    assert a.sum() == b.sum() == g.indices.size // 2  # each edge oriented once either way


# ------------------------------------- InitialBranch's L at b > 0, open form

def level_peel(nbrs, s):
    """Level-synchronous peel written out here (the definition of the rounds):
    level k from 0; each round removes every remaining vertex of remaining
    degree <= k; an empty round raises k to the minimum remaining degree."""
    deg = [len(nbrs[i]) for i in range(s)]
    alive = set(range(s))
    core, rnd = [0] * s, [0] * s
    k, r = 0, 0
    while alive:
        R = [x for x in alive if deg[x] <= k]
        if not R:
            k = min(deg[x] for x in alive)
            continue
        for x in R:
            core[x], rnd[x] = k, r
        alive -= set(R)
        for x in R:
            for y in nbrs[x]:
                if y in alive:
                    deg[y] -= 1
        r += 1
    return core, rnd


def first_fit(nbrs, order):
    col = {}
    for x in order:
        used = {col[y] for y in nbrs[x] if y in col}
        c = 1
        while c in used:
            c += 1
        col[x] = c
    return col


def open_form_L(adj, rk, core, v, b):
    """(s, K_N, L) of root v at bound b, with the open neighbourhood
    P = {u in N(v): rank(u) > rank(v), K(u) >= b} in rank order; -1 where the
    size or neighbourhood-core test stops InitialBranch first."""
    P = sorted((u for u in adj[v] if rk[u] > rk[v] and core[u] >= b), key=lambda u: rk[u])
    s = len(P)
    if s + 1 <= b:
        return s, -1, -1
    loc = {u: i for i, u in enumerate(P)}
    nbrs = [{loc[x] for x in adj[u] if x in loc} for u in P]
    G = nx.Graph()
    G.add_nodes_from(range(s))
    G.add_edges_from((i, j) for i in range(s) for j in nbrs[i] if i < j)
    kn = nx.core_number(G)
    KP = max(kn.values(), default=-1)
    if KP + 2 <= b:  # the closed neighbourhood's largest core is K(P) + 1 < b
        return s, KP, -1
    kn2, rounds = level_peel(nbrs, s)
    assert kn2 == [kn[i] for i in range(s)]
    assert check_peel(nbrs, np.array(kn2), np.array(rounds)) is None
    keep = [x for x in range(s) if kn[x] >= b - 1]  # drop K_N(x) + 1 < b
    order = sorted(keep, key=lambda x: (-rounds[x], -x))
    col = first_fit(nbrs, order)
    sub = [nbrs[x] & set(keep) for x in range(s)]
    assert check_greedy_colouring(sub, order, col) is None
    return s, KP, max(col.values(), default=0)


@pytest.mark.parametrize("g", tiny() + medium()[:3] + [gg.chung_lu(400, 2.2, 12.0, 100.0, 31,
                                                                     plants=(9,))],
                         ids=lambda g: g.name)
def test_initial_branch_L_at_positive_bounds(g):
    adj = adj_sets(g)
    core, rnd, km, _ = oracle.peel(g.offsets, g.indices)
    rk, _ = oracle.rank(rnd)
    w0 = ref_omega(g)
    bounds = sorted({1, 2, 3, max(w0 - 2, 1), max(w0 - 1, 1), w0})
    checked = 0
    for b in bounds:
        r = oracle.root_omega(g.offsets, g.indices, b)
        for v in range(g.n):
            if core[v] < b:
                continue
            s, KP, L = open_form_L(adj, rk, core, v, b)
            assert (r["s"][v], r["kn"][v], r["L"][v]) == (s, KP, L), (v, b)
            checked += L > 0
    assert checked > 0


# ------------------------------------------------- the production heuristic

def production_heuristic(adj, core, rk, order):
    """Alg. 1 as written (with C = {v}): seeds by decreasing rank; a seed of
    core below the running maximum is skipped; its candidates are the
    neighbours of core >= the running maximum, by decreasing rank; first fit;
    a strictly larger clique replaces H."""
    mx, H = 0, []
    for v in order[::-1]:
        if core[v] < mx:
            continue
        cand = sorted((u for u in adj[v] if core[u] >= mx), key=lambda u: -rk[u])
        C = [v]
        for u in cand:
            if all(u in adj[c] for c in C):
                C.append(u)
        if len(C) > mx:
            mx, H = len(C), sorted(C)
    return H


@pytest.mark.parametrize("g", tiny() + medium() + [gg.c1_graph()], ids=lambda g: g.name)
def test_production_heuristic_reenumerated(g):
    core, rnd, _, _ = oracle.peel(g.offsets, g.indices)
    rk, order = oracle.rank(rnd)
    h = oracle.heuristic(g.offsets, g.indices, core, rk, order, -1)
    assert h.tolist() == production_heuristic(adj_sets(g), core, rk, order)


def test_production_heuristic_skip_rule_matters():
    """A graph where the skip and threshold rules change which seeds run:
    the frozen (threshold 0, no skip) mode processes every seed, the
    production mode fewer; both stay cliques of size <= omega."""
    g = gg.chung_lu(900, 2.1, 20.0, 220.0, 3151, plants=(12, 14))
    core, rnd, _, _ = oracle.peel(g.offsets, g.indices)
    rk, order = oracle.rank(rnd)
    adj = adj_sets(g)
    mx, seeds = 0, 0
    for v in order[::-1]:
        if core[v] < mx:
            continue
        seeds += 1
        cand = sorted((u for u in adj[v] if core[u] >= mx), key=lambda u: -rk[u])
        C = [v]
        for u in cand:
            if all(u in adj[c] for c in C):
                C.append(u)
        mx = max(mx, len(C))
    assert seeds < g.n
    for tau in (-1, 0):
        h = oracle.heuristic(g.offsets, g.indices, core, rk, order, tau)
        assert is_clique(adj, h.tolist()) and len(h) <= ref_omega(g)
