"""Independent reference routines used to pin the oracle (test side only).

Nothing here is shared with the oracle or the GPU path: brute-force clique
enumeration, a textbook Bron-Kerbosch enumerator, and checkers that verify a
result against a characterisation (rather than recomputing it the same way).
"""
from __future__ import annotations

import itertools

import numpy as np


def adj_sets(g):
    off, idx = g.offsets, g.indices
    return [set(idx[off[v]:off[v + 1]].tolist()) for v in range(g.n)]


def dense(g):
    a = np.zeros((g.n, g.n), dtype=np.uint8)
    for v in range(g.n):
        a[v, g.indices[g.offsets[v]:g.offsets[v + 1]]] = 1
    return a


def is_clique(adj, vs):
    vs = list(vs)
    if len(set(vs)) != len(vs):
        return False
    return all(b in adj[a] for a, b in itertools.combinations(vs, 2))


def brute_force_omega(adj):
    """Largest clique by enumerating all 2^n vertex subsets (n <= ~18)."""
    n = len(adj)
    masks = [0] * n
    for v in range(n):
        for u in adj[v]:
            masks[v] |= 1 << u
    best = 0
    for S in range(1 << n):
        c = bin(S).count("1")
        if c <= best:
            continue
        ok = True
        T = S
        while T:
            v = (T & -T).bit_length() - 1
            T &= T - 1
            if (S & ~(1 << v)) & ~masks[v]:
                ok = False
                break
        if ok:
            best = c
    return best


def bron_kerbosch_omega(adj):
    """Textbook Bron-Kerbosch with pivoting (Tomita et al.): size of the largest maximal clique."""
    best = 0

    def bk(R, P, X):
        nonlocal best
        if not P and not X:
            best = max(best, len(R))
            return
        if len(R) + len(P) <= best:
            return
        pivot = max(P | X, key=lambda u: len(P & adj[u]))
        for v in list(P - adj[pivot]):
            bk(R | {v}, P & adj[v], X & adj[v])
            P = P - {v}
            X = X | {v}

    bk(set(), set(range(len(adj))), set())
    return best


def check_peel(adj, core, rnd):
    """Verify (core, round) against the fixed-point characterisation of the
    level-synchronous peel: for every round r, with A_r = vertices of round >= r
    and k_r their level, the vertices of round r are exactly the members of A_r
    whose degree inside A_r is <= k_r, and k_r is the larger of k_{r-1} and the
    minimum degree inside A_r.  Returns a message or None."""
    n = len(adj)
    core = np.asarray(core)
    rnd = np.asarray(rnd)
    if n == 0:
        return None
    R = int(rnd.max()) + 1
    if sorted(set(rnd.tolist())) != list(range(R)):
        return "rounds are not 0..R-1"
    kprev = 0
    for r in range(R):
        A = set(np.nonzero(rnd >= r)[0].tolist())
        ks = set(core[rnd == r].tolist())
        if len(ks) != 1:
            return f"round {r} mixes levels {ks}"
        k = ks.pop()
        degA = {v: len(adj[v] & A) for v in A}
        if k != max(kprev, min(degA.values())):
            return f"round {r}: level {k} but expected max({kprev}, min deg {min(degA.values())})"
        want = {v for v in A if degA[v] <= k}
        got = set(np.nonzero(rnd == r)[0].tolist())
        if want != got:
            return f"round {r}: removed {sorted(got)[:8]} expected {sorted(want)[:8]}"
        kprev = k
    return None


def check_greedy_colouring(adj, order, colour):
    """A colouring is the greedy (first-fit) colouring of `order` iff it is
    proper, uses colours 1..L, and every vertex of colour c has, earlier in the
    order, a neighbour of each colour 1..c-1.  Returns a message or None."""
    pos = {v: i for i, v in enumerate(order)}
    for v in order:
        c = colour[v]
        if c < 1:
            return f"vertex {v} uncoloured"
        for u in adj[v]:
            if u in pos and colour[u] == c:
                return f"edge {v}-{u} monochromatic"
        earlier = {colour[u] for u in adj[v] if u in pos and pos[u] < pos[v]}
        if any(cc not in earlier for cc in range(1, c)):
            return f"vertex {v} colour {c} not first-fit"
    return None
