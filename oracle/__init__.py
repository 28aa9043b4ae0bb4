"""CPU oracle of the exact maximum-clique method -- TEST INFRASTRUCTURE ONLY.

Thin ctypes binding over ``oracle.cpp`` (built with g++ into ``liboracle.so``).
Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package; the GPU product path never does.  It shares no code with the GPU
library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (always, when ``force``)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", _SRC, "-o",
                        tmp], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        I64, I32 = ctypes.c_int64, ctypes.c_int32
        sig = {
            "or_validate": (ctypes.c_int, [I64, _i64p, _i32p]),
            "or_core_bz": (None, [I64, _i64p, _i32p, _i32p]),
            "or_peel": (I32, [I64, _i64p, _i32p, _i32p, _i32p, _i32p]),
            "or_rank": (None, [I64, _i32p, _i32p, _i32p]),
            "or_heuristic": (I32, [I64, _i64p, _i32p, _i32p, _i32p, _i32p, I32, _i32p]),
            "or_r0": (I32, [I64, _i32p, _i32p, I32]),
            "or_prune_orient": (I32, [I64, _i64p, _i32p, _i32p, _i32p, _i32p, I32, _i64p, _i32p]),
            "or_max_clique": (I32, [I64, _i64p, _i32p, I32, _i32p, _i64p]),
            "or_max_clique_ex": (I32, [I64, _i64p, _i32p, I32, I32, I32, _i32p, I64, _i64p,
                                       _i32p, _i32p, _i64p]),
            "or_root_omega": (None, [I64, _i64p, _i32p, I32, _i32p, _i32p, _i32p, _i32p]),
            "or_root_omega_ex": (None, [I64, _i64p, _i32p, I32, I32, _i32p, _i32p, _i32p,
                                        _i32p]),
            "or_local_peel": (None, [I32, _u8p, _i32p, _i32p]),
            "or_greedy_colour": (I32, [I32, _u8p, _i32p, I32, _i32p]),
            "or_clique_order": (I64, [I64, _i64p, _i32p, _i32p, _i32p, _i64p]),
            "or_strong_reach": (I64, [I64, I64, _i32p, _i32p, _i64p, _i32p, I64]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _csr(offsets, indices):
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    idx = np.ascontiguousarray(indices, dtype=np.int32)
    if idx.size == 0:
        idx = np.zeros(1, dtype=np.int32)
    return off.shape[0] - 1, off, idx


def validate(offsets, indices) -> int:
    n, off, idx = _csr(offsets, indices)
    return int(_load().or_validate(n, _p(off, ctypes.c_int64), _p(idx, ctypes.c_int32)))


def core_bz(offsets, indices) -> np.ndarray:
    n, off, idx = _csr(offsets, indices)
    core = np.zeros(max(n, 1), dtype=np.int32)
    _load().or_core_bz(n, _p(off, ctypes.c_int64), _p(idx, ctypes.c_int32), _p(core, ctypes.c_int32))
    return core[:n]


def peel(offsets, indices):
    """Level-synchronous peel: (core, round, kmax, nrounds)."""
    n, off, idx = _csr(offsets, indices)
    core = np.zeros(max(n, 1), dtype=np.int32)
    rnd = np.zeros(max(n, 1), dtype=np.int32)
    km = np.zeros(1, dtype=np.int32)
    nr = _load().or_peel(n, _p(off, ctypes.c_int64), _p(idx, ctypes.c_int32),
                         _p(core, ctypes.c_int32), _p(rnd, ctypes.c_int32), _p(km, ctypes.c_int32))
    return core[:n], rnd[:n], int(km[0]) if n else 0, int(nr)


def rank(rounds):
    rounds = np.ascontiguousarray(rounds, dtype=np.int32)
    n = rounds.shape[0]
    rk = np.zeros(max(n, 1), dtype=np.int32)
    od = np.zeros(max(n, 1), dtype=np.int32)
    r = rounds if n else np.zeros(1, np.int32)
    _load().or_rank(n, _p(r, ctypes.c_int32), _p(rk, ctypes.c_int32), _p(od, ctypes.c_int32))
    return rk[:n], od[:n]


def heuristic(offsets, indices, core, rk, order, frozen_tau=-1):
    n, off, idx = _csr(offsets, indices)
    core = np.ascontiguousarray(core, dtype=np.int32)
    rk = np.ascontiguousarray(rk, dtype=np.int32)
    order = np.ascontiguousarray(order, dtype=np.int32)
    cap = int(core.max()) + 2 if n else 1
    out = np.zeros(cap, dtype=np.int32)
    if n == 0:
        return out[:0]
    h = _load().or_heuristic(n, _p(off, ctypes.c_int64), _p(idx, ctypes.c_int32),
                             _p(core, ctypes.c_int32), _p(rk, ctypes.c_int32),
                             _p(order, ctypes.c_int32), frozen_tau, _p(out, ctypes.c_int32))
    return out[:h].copy()


def prune_orient(offsets, indices, core, rk, order, bound):
    """Oriented pruned lists: (r0, poff int64[n-r0+1], padj int32[...])."""
    n, off, idx = _csr(offsets, indices)
    core = np.ascontiguousarray(core, dtype=np.int32)
    rk = np.ascontiguousarray(rk, dtype=np.int32)
    order = np.ascontiguousarray(order, dtype=np.int32)
    poff = np.zeros(n + 1, dtype=np.int64)
    padj = np.zeros(max(idx.shape[0], 1), dtype=np.int32)
    r0 = _load().or_prune_orient(n, _p(off, ctypes.c_int64), _p(idx, ctypes.c_int32),
                                 _p(core, ctypes.c_int32), _p(rk, ctypes.c_int32),
                                 _p(order, ctypes.c_int32), bound, _p(poff, ctypes.c_int64),
                                 _p(padj, ctypes.c_int32))
    nn = n - r0
    poff = poff[:nn + 1].copy()
    return int(r0), poff, padj[:int(poff[-1])].copy()


STAT_KEYS = ("kmax", "nrounds", "heuristic", "omega", "certified_early", "survivors",
             "roots_visited", "roots_branched", "nodes", "pruned_size", "pruned_kn",
             "pruned_colour")


def max_clique(offsets, indices, use_neigh_cores=True):
    """Alg. 2: (omega, clique sorted ascending, stats dict)."""
    n, off, idx = _csr(offsets, indices)
    deg = np.diff(off)
    cap = int(deg.max()) + 2 if n else 1
    out = np.zeros(cap, dtype=np.int32)
    st = np.zeros(12, dtype=np.int64)
    w = _load().or_max_clique(n, _p(off, ctypes.c_int64), _p(idx, ctypes.c_int32),
                              1 if use_neigh_cores else 0, _p(out, ctypes.c_int32),
                              _p(st, ctypes.c_int64))
    return int(w), out[:w].copy(), dict(zip(STAT_KEYS, (int(x) for x in st)))


def max_clique_ex(offsets, indices, use_neigh_cores=True, native=False, threads=1,
                  dispatch=None, inject=()):
    """Alg. 2 with the paper's variants and the test modes (see or_max_clique_ex):
    native vertex order, T worker threads sharing the bound (Sec. 4.5), a root
    dispatch permutation, and scripted bound raises ``inject`` = [(queue
    position, bound), ...].  Returns (bound, clique sorted ascending, stats);
    stats["witness"] is the clique's size."""
    n, off, idx = _csr(offsets, indices)
    deg = np.diff(off)
    cap = int(deg.max()) + 2 if n else 1
    out = np.zeros(cap, dtype=np.int32)
    st = np.zeros(13, dtype=np.int64)
    inj = sorted((int(a), int(b)) for a, b in inject)
    ia = np.array([a for a, _ in inj] or [0], dtype=np.int64)
    iv = np.array([b for _, b in inj] or [0], dtype=np.int32)
    disp = None
    if dispatch is not None:
        disp = np.ascontiguousarray(dispatch, dtype=np.int32)
        if disp.shape != (n,) or (n and not np.array_equal(np.sort(disp), np.arange(n))):
            raise ValueError("dispatch must be a permutation of the vertices")
    w = _load().or_max_clique_ex(n, _p(off, ctypes.c_int64), _p(idx, ctypes.c_int32),
                                 1 if use_neigh_cores else 0, 1 if native else 0, int(threads),
                                 _p(disp, ctypes.c_int32) if disp is not None and n else None,
                                 len(inj), _p(ia, ctypes.c_int64), _p(iv, ctypes.c_int32),
                                 _p(out, ctypes.c_int32), _p(st, ctypes.c_int64))
    stats = dict(zip(STAT_KEYS + ("witness",), (int(x) for x in st)))
    return int(w), out[:stats["witness"]].copy(), stats


def root_omega(offsets, indices, b=0, native=False):
    """Per-root frozen-bound search: dict of arrays s, kn, L, omega (by vertex
    id); ``native`` orients the neighbourhoods by vertex id."""
    n, off, idx = _csr(offsets, indices)
    outs = [np.zeros(max(n, 1), dtype=np.int32) for _ in range(4)]
    _load().or_root_omega_ex(n, _p(off, ctypes.c_int64), _p(idx, ctypes.c_int32), b,
                             1 if native else 0, *[_p(o, ctypes.c_int32) for o in outs])
    return dict(zip(("s", "kn", "L", "omega"), (o[:n] for o in outs)))


def local_peel(adj):
    a = np.ascontiguousarray(adj, dtype=np.uint8)
    s = a.shape[0]
    kn = np.zeros(max(s, 1), dtype=np.int32)
    lr = np.zeros(max(s, 1), dtype=np.int32)
    _load().or_local_peel(s, _p(a, ctypes.c_uint8), _p(kn, ctypes.c_int32), _p(lr, ctypes.c_int32))
    return kn[:s], lr[:s]


def greedy_colour(adj, order):
    a = np.ascontiguousarray(adj, dtype=np.uint8)
    s = a.shape[0]
    o = np.ascontiguousarray(order, dtype=np.int32)
    col = np.zeros(max(s, 1), dtype=np.int32)
    L = _load().or_greedy_colour(s, _p(a, ctypes.c_uint8), _p(o, ctypes.c_int32), o.shape[0],
                                 _p(col, ctypes.c_int32))
    return int(L), col[:s]


def clique_order(offsets, indices, rk):
    """Clique-peeling compression order (Sec. 6.2): (order int32[n], block
    starts int64[nb + 1])."""
    n, off, idx = _csr(offsets, indices)
    rk = np.ascontiguousarray(rk, dtype=np.int32)
    order = np.zeros(max(n, 1), dtype=np.int32)
    block = np.zeros(n + 1, dtype=np.int64)
    if n == 0:
        return order[:0], block[:1]
    nb = _load().or_clique_order(n, _p(off, ctypes.c_int64), _p(idx, ctypes.c_int32),
                                 _p(rk, ctypes.c_int32), _p(order, ctypes.c_int32),
                                 _p(block, ctypes.c_int64))
    return order[:n].copy(), block[:nb + 1].copy()


def strong_reach(n, src, dst):
    """Strong-reachability graph of the temporal edges src[e] -> dst[e] (in time
    order), Sec. 6.1: (offsets int64[n+1], indices int32)."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = src.shape[0]
    off = np.zeros(n + 1, dtype=np.int64)
    cap = max(1, n * (n - 1))
    adj = np.zeros(min(cap, 1 << 26), dtype=np.int32)
    s_ = src if m else np.zeros(1, np.int32)
    d_ = dst if m else np.zeros(1, np.int32)
    k = _load().or_strong_reach(n, m, _p(s_, ctypes.c_int32), _p(d_, ctypes.c_int32),
                                _p(off, ctypes.c_int64), _p(adj, ctypes.c_int32), adj.shape[0])
    if k > adj.shape[0]:
        raise ValueError("strong-reachability graph too large for the oracle buffer")
    return off, adj[:k].copy()
