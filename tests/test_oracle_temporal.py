"""Pins of the strong-reachability graph (Sec. 6.1) in the oracle: closed forms
on temporal cycles and contacts, and brute-force enumeration of time-respecting
paths on small random temporal networks."""
import itertools

import networkx as nx
import numpy as np
import pytest

import graphgen as gg
import oracle


def csr_sets(off, adj, n):
    return [set(adj[off[v]:off[v + 1]].tolist()) for v in range(n)]


def test_single_pass_cycle_is_a_star():
    k = 6
    src = list(range(k))
    dst = [(i + 1) % k for i in range(k)]
    off, adj = oracle.strong_reach(k, src, dst)
    sets = csr_sets(off, adj, k)
    # i < j: i reaches j forward; j reaches only the later vertices and 0
    assert sets[0] == set(range(1, k))
    for j in range(1, k):
        assert sets[j] == {0}


def test_two_passes_make_a_clique():
    k = 7
    src = list(range(k)) * 2
    dst = [(i + 1) % k for i in range(k)] * 2
    off, adj = oracle.strong_reach(k, src, dst)
    for v, s in enumerate(csr_sets(off, adj, k)):
        assert s == set(range(k)) - {v}


def test_contacts_and_one_way_edges():
    off, adj = oracle.strong_reach(3, [0, 1], [1, 0])  # a contact: both directions
    assert csr_sets(off, adj, 3) == [{1}, {0}, set()]
    off, adj = oracle.strong_reach(3, [0], [1])  # one way only
    assert csr_sets(off, adj, 3) == [set(), set(), set()]
    off, adj = oracle.strong_reach(4, [], [])
    assert off.tolist() == [0, 0, 0, 0, 0]


def brute_reach(n, src, dst):
    """reach[a][b]: a temporal path a -> b exists (edges used in increasing
    position), found by depth-first enumeration of edge sequences."""
    m = len(src)
    reach = [[a == b for b in range(n)] for a in range(n)]

    def walk(a, at, pos):
        for e in range(pos, m):
            if src[e] == at:
                reach[a][dst[e]] = True
                walk(a, dst[e], e + 1)

    for a in range(n):
        walk(a, a, 0)
    return reach


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_paths(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 8))
    m = int(rng.integers(0, 16))
    src = rng.integers(0, n, size=m).tolist()
    dst = rng.integers(0, n, size=m).tolist()
    off, adj = oracle.strong_reach(n, src, dst)
    reach = brute_reach(n, src, dst)
    want = [{b for b in range(n) if b != a and reach[a][b] and reach[b][a]} for a in range(n)]
    assert csr_sets(off, adj, n) == want
    assert np.all(np.diff(adj[off[0]:off[1]]) > 0) if off[1] > 1 else True


def test_synthetic_contacts_symmetric_and_clique_is_tscc():
    src, dst = gg.temporal_contacts(60, 500, 4, 0.8, 3, directed_frac=0.3)
    off, adj = oracle.strong_reach(60, src, dst)
    sets = csr_sets(off, adj, 60)
    for a, s in enumerate(sets):
        for b in s:
            assert a in sets[b]
    w, cl, _ = oracle.max_clique(off, adj)
    G = nx.Graph()
    G.add_nodes_from(range(60))
    G.add_edges_from((a, b) for a, s in enumerate(sets) for b in s)
    assert w == max(len(c) for c in nx.find_cliques(G))
