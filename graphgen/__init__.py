"""Seeded synthetic graph inputs shared by the oracle tests and the GPU path.

This module holds no arithmetic of the maximum-clique method: only random
graph models (Chung-Lu, G(n,p), R-MAT, planted cliques), closed-form graph
families, and CSR assembly.  The native sampler is ``graphgen.c`` (built with
gcc into ``libgraphgen.so`` next to it).

All graphs are simple, undirected and returned as a symmetric CSR
``(offsets int64[n+1], indices int32[nnz])`` with rows sorted ascending.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")

#: base seed of every workload; graph i of workload c uses seed_for(c, i)
S0 = 0x13026256


def build(force: bool = True) -> str:
    """Compile the sampler with gcc (always, when ``force``)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", _SRC, "-o", tmp, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.gg_chung_lu.restype = ctypes.c_void_p
        lib.gg_chung_lu.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_uint64, i32p, ctypes.c_int32, i32p]
        lib.gg_gnp.restype = ctypes.c_void_p
        lib.gg_gnp.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, i32p,
                               ctypes.c_int32, i32p]
        lib.gg_rmat.restype = ctypes.c_void_p
        lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_uint64, i32p, ctypes.c_int32, i32p]
        lib.gg_from_edges.restype = ctypes.c_void_p
        lib.gg_from_edges.argtypes = [ctypes.c_int64, i32p, ctypes.c_int64]
        lib.gg_n.restype = ctypes.c_int64
        lib.gg_n.argtypes = [ctypes.c_void_p]
        lib.gg_nnz.restype = ctypes.c_int64
        lib.gg_nnz.argtypes = [ctypes.c_void_p]
        lib.gg_copy.restype = None
        lib.gg_copy.argtypes = [ctypes.c_void_p, i64p, i32p]
        lib.gg_free.restype = None
        lib.gg_free.argtypes = [ctypes.c_void_p]
        lib.gg_splitmix64.restype = ctypes.c_uint64
        lib.gg_splitmix64.argtypes = [ctypes.c_uint64]
        lib.gg_chung_lu_weights.restype = ctypes.c_int
        lib.gg_chung_lu_weights.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
        _lib = lib
    return _lib


@dataclass
class Graph:
    """A simple undirected graph in symmetric CSR form (host numpy arrays)."""
    offsets: np.ndarray  # int64[n+1]
    indices: np.ndarray  # int32[nnz]
    planted: np.ndarray | None = None  # planted-clique members, plant after plant
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.indices.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _take(h, planted=None, name="") -> Graph:
    lib = _load()
    if not h:
        raise RuntimeError("graphgen: generation failed (bad parameters or out of memory)")
    try:
        n = lib.gg_n(h)
        nnz = lib.gg_nnz(h)
        off = np.empty(n + 1, dtype=np.int64)
        idx = np.empty(max(nnz, 1), dtype=np.int32)
        lib.gg_copy(h, _ptr(off, ctypes.c_int64), _ptr(idx, ctypes.c_int32))
    finally:
        lib.gg_free(h)
    return Graph(off, idx[:nnz].copy() if nnz else np.empty(0, np.int32), planted, name)


def _plants(plants):
    arr = np.asarray(list(plants), dtype=np.int32)
    tot = int(arr.sum()) if arr.size else 0
    mem = np.empty(max(tot, 1), dtype=np.int32)
    return arr, mem, tot


def seed_for(config: int, i: int) -> int:
    """Seed of graph ``i`` of workload ``config`` (splitmix64 of S0 ^ c<<32 ^ i)."""
    return int(_load().gg_splitmix64((S0 ^ (config << 32) ^ i) & 0xFFFFFFFFFFFFFFFF))


def chung_lu(n, gamma, mean_deg, w_max, seed, plants=()) -> Graph:
    arr, mem, tot = _plants(plants)
    h = _load().gg_chung_lu(n, gamma, mean_deg, w_max, seed, _ptr(arr, ctypes.c_int32),
                            len(arr), _ptr(mem, ctypes.c_int32))
    return _take(h, mem[:tot].copy(), f"chung_lu(n={n},g={gamma},d={mean_deg})")


def chung_lu_weights(n, gamma, mean_deg, w_max) -> np.ndarray:
    w = np.empty(n, dtype=np.float64)
    if _load().gg_chung_lu_weights(n, gamma, mean_deg, w_max, _ptr(w, ctypes.c_double)):
        raise ValueError("bad Chung-Lu parameters")
    return w


def gnp(n, p, seed, plants=()) -> Graph:
    arr, mem, tot = _plants(plants)
    h = _load().gg_gnp(n, p, seed, _ptr(arr, ctypes.c_int32), len(arr), _ptr(mem, ctypes.c_int32))
    return _take(h, mem[:tot].copy(), f"gnp(n={n},p={p:.4g})")


def rmat(scale, edge_factor, a, b, c, seed, plants=()) -> Graph:
    arr, mem, tot = _plants(plants)
    h = _load().gg_rmat(scale, edge_factor, a, b, c, seed, _ptr(arr, ctypes.c_int32), len(arr),
                        _ptr(mem, ctypes.c_int32))
    return _take(h, mem[:tot].copy(), f"rmat(scale={scale},ef={edge_factor})")


def from_edges(n, edges) -> Graph:
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    if e.size == 0:
        e = np.zeros((0, 2), dtype=np.int32)
    h = _load().gg_from_edges(n, _ptr(e, ctypes.c_int32) if e.size else None, e.shape[0])
    if not h:
        raise ValueError("from_edges: vertex id out of range")
    return _take(h, None, f"edges(n={n})")


# ------------------------------------------------------------ closed forms

def _pairs(n):
    i, j = np.triu_indices(n, 1)
    return i.astype(np.int32), j.astype(np.int32)


def complete(n) -> Graph:
    i, j = _pairs(n)
    return from_edges(n, np.stack([i, j], 1))


def cycle(n) -> Graph:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)] if n >= 3 else [])


def path(n) -> Graph:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)])


def empty(n) -> Graph:
    return from_edges(n, [])


def turan(n, r) -> Graph:
    """Complete r-partite graph with parts as equal as possible (part of i = i % r)."""
    i, j = _pairs(n)
    k = (i % r) != (j % r)
    return from_edges(n, np.stack([i[k], j[k]], 1))


def cocktail_party(r) -> Graph:
    """K_{2r} minus a perfect matching: omega = r."""
    n = 2 * r
    i, j = _pairs(n)
    k = j != i + r
    return from_edges(n, np.stack([i[k], j[k]], 1))


def complete_bipartite(a, b) -> Graph:
    i, j = np.meshgrid(np.arange(a, dtype=np.int32), np.arange(b, dtype=np.int32), indexing="ij")
    return from_edges(a + b, np.stack([i.ravel(), a + j.ravel()], 1))


def star(n) -> Graph:
    return from_edges(n, [(0, i) for i in range(1, n)])


def disjoint_cliques(sizes) -> Graph:
    edges, base = [], 0
    for s in sizes:
        edges += [(base + i, base + j) for i in range(s) for j in range(i + 1, s)]
        base += s
    return from_edges(base, edges)


def grid(a, b) -> Graph:
    e = []
    for i in range(a):
        for j in range(b):
            v = i * b + j
            if j + 1 < b:
                e.append((v, v + 1))
            if i + 1 < a:
                e.append((v, v + b))
    return from_edges(a * b, e)


def permuted(g: Graph, seed: int) -> Graph:
    """The same graph with vertex ids relabelled by a seeded permutation."""
    rng = np.random.Generator(np.random.Philox(seed))
    perm = rng.permutation(g.n).astype(np.int32)
    deg = np.diff(g.offsets)
    src = np.repeat(np.arange(g.n, dtype=np.int32), deg)
    e = np.stack([perm[src], perm[g.indices]], axis=1)
    e = e[e[:, 0] < e[:, 1]]
    out = from_edges(g.n, e)
    if g.planted is not None:
        out.planted = perm[g.planted]
    return out


# ------------------------------------------------------------- workloads

def c1_graph(i: int = 0) -> Graph:
    """Chung-Lu, n=2,000, exponent 2.3, mean degree 8, max weight 200, one planted 15-clique."""
    g = chung_lu(2000, 2.3, 8.0, 200.0, seed_for(1, i), plants=(15,))
    g.name = f"chung-lu n=2000 g=2.3 d=8 wmax=200 plant15 #{i}"
    return g


def c2_graph(i: int = 0, n: int = 1_000_000) -> Graph:
    """Chung-Lu, n=10^6, exponent 2.1, mean degree 24, w_max = sqrt(n*d), planted 20 and 40."""
    wmax = math.sqrt(n * 24.0)
    g = chung_lu(n, 2.1, 24.0, wmax, seed_for(2, i), plants=(20, 40))
    g.name = f"chung-lu n={n} g=2.1 d=24 wmax={wmax:.0f} plants20+40 #{i}"
    return g


def c3_params(i: int):
    """Parameters of graph i (0..2047) of the 2,048-graph batch."""
    s = seed_for(3, i)
    rng = np.random.Generator(np.random.Philox(s))
    n = int(math.floor(math.exp(rng.uniform(math.log(64), math.log(20000)))))
    d = float(rng.uniform(6.0, 40.0))
    k = int(rng.integers(5, 61))
    k = min(k, n)
    d = min(d, (n - 1) * 0.9)
    kind = "gnp" if i < 1024 else "chung-lu"
    return dict(kind=kind, n=n, d=d, k=k, seed=s)


def c3_graph(i: int) -> Graph:
    p = c3_params(i)
    if p["kind"] == "gnp":
        g = gnp(p["n"], p["d"] / max(p["n"] - 1, 1), p["seed"], plants=(p["k"],))
    else:
        wmax = min(math.sqrt(p["n"] * p["d"]), p["n"] - 1.0)
        wmax = max(wmax, p["d"])
        g = chung_lu(p["n"], 2.2, p["d"], wmax, p["seed"], plants=(p["k"],))
    g.name = f"{p['kind']} n={p['n']} d={p['d']:.1f} plant{p['k']} #{i}"
    return g


def c4_params(i: int):
    """Graph i of the learned-ordering workload; i >= 10**6 are held-out graphs (n=200,000)."""
    s = seed_for(4, i)
    rng = np.random.Generator(np.random.Philox(s))
    if i >= 10**6:
        n = 200_000
    else:
        n = int(math.floor(math.exp(rng.uniform(math.log(500), math.log(50000)))))
    gamma = float(rng.uniform(2.0, 2.6))
    d = float(rng.uniform(6.0, 40.0))
    k = int(rng.integers(10, 81))
    k = min(k, n)
    return dict(n=n, gamma=gamma, d=d, k=k, seed=s)


def c4_graph(i: int) -> Graph:
    p = c4_params(i)
    wmax = max(min(math.sqrt(p["n"] * p["d"]), p["n"] - 1.0), p["d"])
    g = chung_lu(p["n"], p["gamma"], p["d"], wmax, p["seed"], plants=(p["k"],))
    g.name = f"chung-lu n={p['n']} g={p['gamma']:.2f} d={p['d']:.1f} plant{p['k']} #{i}"
    return g


def c5_graph(scale: int = 27, edge_factor: int = 14) -> Graph:
    """R-MAT (a,b,c,d)=(.57,.19,.19,.05), symmetrised and de-duplicated, planted 50-clique."""
    g = rmat(scale, edge_factor, 0.57, 0.19, 0.19, seed_for(5, 0), plants=(50,))
    g.name = f"rmat scale={scale} ef={edge_factor} plant50"
    return g


def concat(graphs):
    """Disjoint union of graphs in one CSR: (Graph, vertex_base int64[count+1])."""
    offs, idxs, base = [np.zeros(1, np.int64)], [], [0]
    nnz = 0
    for g in graphs:
        offs.append(g.offsets[1:] + nnz)
        idxs.append(g.indices.astype(np.int64) + base[-1])
        nnz += g.nnz
        base.append(base[-1] + g.n)
    off = np.concatenate(offs).astype(np.int64)
    idx = np.concatenate(idxs).astype(np.int32) if idxs else np.zeros(0, np.int32)
    return Graph(off, idx, None, f"batch of {len(graphs)}"), np.asarray(base, dtype=np.int64)


def c3_batch(count: int = 2048):
    """The batch workload: graphs 0..count-1 of c3_graph, concatenated."""
    return concat([c3_graph(i) for i in range(count)])


def temporal_contacts(n, contacts, groups, p_within, seed, directed_frac=0.0):
    """A seeded synthetic temporal contact sequence (stand-in for the paper's
    contact / interaction / retweet networks): n people in `groups` groups of
    Zipf-like sizes; each contact picks a group by size, then two members of it
    (with probability p_within) or two people anywhere.  A contact is symmetric
    (both directions, consecutive in time) unless it falls in the directed
    fraction (one direction only, as a retweet).  Returns (src, dst) int32 arrays
    in time order."""
    rng = np.random.Generator(np.random.Philox(seed))
    perm = rng.permutation(n).astype(np.int32)
    w = 1.0 / np.arange(1, groups + 1) ** 0.8
    sizes = np.maximum(2, np.floor(w / w.sum() * n)).astype(np.int64)
    starts = np.concatenate([[0], np.cumsum(sizes)])
    starts = np.minimum(starts, n)
    src, dst = [], []
    gsel = rng.choice(groups, size=contacts, p=sizes / sizes.sum())
    within = rng.random(contacts) < p_within
    directed = rng.random(contacts) < directed_frac
    for i in range(contacts):
        if within[i]:
            a0, a1 = starts[gsel[i]], max(starts[gsel[i] + 1], starts[gsel[i]] + 1)
            u, v = rng.integers(a0, a1, size=2)
        else:
            u, v = rng.integers(0, n, size=2)
        if u == v:
            continue
        u, v = int(perm[min(u, n - 1)]), int(perm[min(v, n - 1)])
        src.append(u)
        dst.append(v)
        if not directed[i]:
            src.append(v)
            dst.append(u)
    return np.asarray(src, dtype=np.int32), np.asarray(dst, dtype=np.int32)
