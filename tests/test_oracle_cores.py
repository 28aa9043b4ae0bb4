"""Pins of the oracle's core numbers, peel rounds, rank and orientation.

Core numbers: networkx (library), closed forms, and agreement of two
independent algorithms (bucket peeling and level-synchronous peeling).
Rounds: closed forms and the fixed-point characterisation in refs.check_peel.
Rank: numpy lexsort (library).  Orientation: set definitions and the
degeneracy bound |N+(v)| <= K(v) (Sec. 3, degeneracy order).
"""
import math

import networkx as nx
import numpy as np
import pytest

import graphgen as gg
import oracle
from refs import adj_sets, check_peel


def nxg(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    src = np.repeat(np.arange(g.n), np.diff(g.offsets))
    G.add_edges_from(zip(src.tolist(), g.indices.tolist()))
    return G


def small_graphs():
    out = [gg.gnp(n, p, 100 + i) for i, (n, p) in enumerate(
        [(1, 0.5), (2, 1.0), (5, 0.5), (12, 0.3), (30, 0.2), (60, 0.1), (80, 0.5), (150, 0.05)])]
    out += [gg.chung_lu(300, 2.2, 6.0, 40.0, 7, plants=(8,)),
            gg.chung_lu(500, 2.5, 10.0, 80.0, 8, plants=(6, 9)),
            gg.gnp(200, 0.02, 9, plants=(7,))]
    return out


@pytest.mark.parametrize("g", small_graphs(), ids=lambda g: g.name)
def test_core_matches_networkx_and_bz(g):
    core, rnd, km, nr = oracle.peel(g.offsets, g.indices)
    bz = oracle.core_bz(g.offsets, g.indices)
    ref = nx.core_number(nxg(g))
    assert [ref[v] for v in range(g.n)] == core.tolist()
    assert (bz == core).all()
    assert km == (core.max() if g.n else 0)
    assert nr == (rnd.max() + 1 if g.n else 0)


def test_core_c1_networkx():
    g = gg.c1_graph()
    core, rnd, km, nr = oracle.peel(g.offsets, g.indices)
    ref = nx.core_number(nxg(g))
    assert [ref[v] for v in range(g.n)] == core.tolist()
    assert km == 14  # the 15-clique plant lies in the 14-core
    assert check_peel(adj_sets(g), core, rnd) is None


@pytest.mark.parametrize("g", small_graphs(), ids=lambda g: g.name)
def test_rounds_characterisation(g):
    core, rnd, _, _ = oracle.peel(g.offsets, g.indices)
    assert check_peel(adj_sets(g), core, rnd) is None


@pytest.mark.parametrize("n", [1, 2, 3, 7, 10])
def test_closed_forms_complete(n):
    g = gg.complete(n)
    core, rnd, km, nr = oracle.peel(g.offsets, g.indices)
    assert (core == n - 1).all() and (rnd == 0).all() and km == n - 1 and nr == 1


@pytest.mark.parametrize("n", [3, 4, 9])
def test_closed_forms_cycle(n):
    g = gg.cycle(n)
    core, rnd, km, nr = oracle.peel(g.offsets, g.indices)
    assert (core == 2).all() and (rnd == 0).all()


@pytest.mark.parametrize("n", [1, 2, 3, 6, 7])
def test_closed_forms_path(n):
    g = gg.path(n)
    core, rnd, _, _ = oracle.peel(g.offsets, g.indices)
    assert (core == min(1, n - 1)).all()
    assert rnd.tolist() == [min(i, n - 1 - i) for i in range(n)]


def test_closed_forms_star_bipartite_grid_empty():
    g = gg.star(6)
    core, rnd, _, _ = oracle.peel(g.offsets, g.indices)
    assert core.tolist() == [1] * 6 and rnd.tolist() == [1, 0, 0, 0, 0, 0]
    g = gg.complete_bipartite(3, 5)
    core, rnd, _, _ = oracle.peel(g.offsets, g.indices)
    assert (core == 3).all() and rnd.tolist() == [1, 1, 1, 0, 0, 0, 0, 0]
    g = gg.grid(4, 5)
    core, _, _, _ = oracle.peel(g.offsets, g.indices)
    assert (core == 2).all()
    g = gg.empty(5)
    core, rnd, km, nr = oracle.peel(g.offsets, g.indices)
    assert (core == 0).all() and (rnd == 0).all() and km == 0 and nr == 1


@pytest.mark.parametrize("n,r", [(6, 2), (7, 3), (10, 4), (12, 5)])
def test_closed_forms_turan(n, r):
    g = gg.turan(n, r)
    core, _, _, _ = oracle.peel(g.offsets, g.indices)
    assert (core == n - math.ceil(n / r)).all()


@pytest.mark.parametrize("g", small_graphs() + [gg.c1_graph()], ids=lambda g: g.name)
def test_rank_and_orientation(g):
    core, rnd, km, _ = oracle.peel(g.offsets, g.indices)
    rk, order = oracle.rank(rnd)
    ref_order = np.lexsort((np.arange(g.n), rnd))
    assert order.tolist() == ref_order.tolist()
    assert (rk[order] == np.arange(g.n)).all()
    # rank is nondecreasing in core (rounds are monotone in the level)
    assert (np.diff(core[order]) >= 0).all()
    adj = adj_sets(g)
    for bound in sorted({0, 1, 2, km // 2, km, km + 1}):
        r0, poff, padj = oracle.prune_orient(g.offsets, g.indices, core, rk, order, bound)
        assert r0 == int((core < bound).sum())
        assert poff.shape[0] == g.n - r0 + 1
        for i in range(g.n - r0):
            v = order[r0 + i]
            row = padj[poff[i]:poff[i + 1]].tolist()
            want = sorted(rk[u] - r0 for u in adj[v] if rk[u] > rk[v])
            assert row == want
            assert len(row) <= core[v]  # degeneracy order bound


def test_validate_rejects():
    g = gg.cycle(5)
    assert oracle.validate(g.offsets, g.indices) == 0
    idx = g.indices.copy()
    idx[0] = 9
    assert oracle.validate(g.offsets, idx) == 2
    idx = g.indices.copy()
    idx[0] = 0
    assert oracle.validate(g.offsets, idx) == 3
    idx = g.indices.copy()
    idx[0], idx[1] = idx[1], idx[0]
    assert oracle.validate(g.offsets, idx) == 4
    # 0-1 present one way only
    off = np.array([0, 1, 1], dtype=np.int64)
    assert oracle.validate(off, np.array([1], dtype=np.int32)) == 5
    off = np.array([0, 2, 1], dtype=np.int64)
    assert oracle.validate(off, np.array([1, 0], dtype=np.int32)) == 1
