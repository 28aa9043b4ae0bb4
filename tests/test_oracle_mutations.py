"""Mutation check of the oracle's pins (CPU).

Each mutation below is a plausible mistake in writing the oracle from the
paper (an off-by-one in a bound test, a dropped term, a wrong comparison or
orientation).  The test compiles the oracle with the mutation applied, runs
a battery of the independent pins on it (omega against brute force and
Bron-Kerbosch, core numbers against networkx, peel rounds against the
fixed-point characterisation, InitialBranch's L at positive bounds against
the open-form recomputation, the production heuristic against its
re-enumeration), and asserts that at least one pin fails.  A mutation that
survived would be a gap in the pins.
"""
import ctypes
import os
import subprocess
import tempfile

import networkx as nx
import numpy as np
import pytest

import graphgen as gg
import oracle
from refs import adj_sets, bron_kerbosch_omega, brute_force_omega, check_peel, is_clique
from test_oracle_modes import open_form_L, production_heuristic

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.cpp")

# (name, text in oracle.cpp (must occur once), replacement)
MUTATIONS = [
    ("colour test prunes one too many",
     "if (L <= bound()) { st.pruned_colour++; return; }",
     "if (L <= bound() + 1) { st.pruned_colour++; return; }"),
    ("Branch loop bound off by one",
     "while (!P.empty() && (int64_t)(P.size() + C.size()) > bound()) {",
     "while (!P.empty() && (int64_t)(P.size() + C.size()) > bound() + 1) {"),
    ("neighbourhood-core drop too strict",
     "if (!use_neigh_cores || kn[i] >= b1) keep.push_back(i);",
     "if (!use_neigh_cores || kn[i] > b1) keep.push_back(i);"),
    ("peel crossing test",
     "if (deg[u] == k) next.push_back(u);",
     "if (deg[u] == k - 1) next.push_back(u);"),
    ("seed missing from its own clique",
     "std::vector<int32_t> C{v};  // (R1)",
     "std::vector<int32_t> C;  // (R1)"),
    ("colouring ignores adjacency",
     "if (colour[y] > 0 && G.adj(x, y)) used[colour[y]] = 1;",
     "if (colour[y] > 0) used[colour[y]] = 1;"),
    ("bucket comparison in the core algorithm",
     "if (deg[u] > deg[v]) {",
     "if (deg[u] >= deg[v]) {"),
    ("implicit removal too strict",
     "if (G.adj(u, e.first) && core[ids[e.first]] >= hsize) Pn.push_back(e.first);",
     "if (G.adj(u, e.first) && core[ids[e.first]] > hsize) Pn.push_back(e.first);"),
    ("neighbourhood oriented the wrong way",
     "if (key(u) > key(v) && core[u] >= b0) P.push_back(u);",
     "if (key(u) < key(v) && core[u] >= b0) P.push_back(u);"),
    ("colouring in forward peel order",
     "if (lround[a] != lround[b]) return lround[a] > lround[b];",
     "if (lround[a] != lround[b]) return lround[a] < lround[b];"),
    ("heuristic candidate threshold off by one",
     "if (core[g.idx[e]] >= tau) S.push_back(g.idx[e]);",
     "if (core[g.idx[e]] > tau) S.push_back(g.idx[e]);"),
    ("level jump to the maximum degree",
     "kmin = std::min(kmin, deg[v]);",
     "kmin = std::max(kmin == INT64_MAX ? 0 : kmin, deg[v]);"),
]


def _graphs():
    tiny = [gg.gnp(n, p, 5000 + i) for i, (n, p) in enumerate(
        [(9, 0.6), (12, 0.5), (13, 0.75), (14, 0.45), (15, 0.85), (11, 0.3), (14, 0.6)])]
    medium = [gg.gnp(60, 0.5, 5100), gg.gnp(80, 0.75, 5101), gg.gnp(120, 0.2, 5102),
              gg.chung_lu(500, 2.2, 12.0, 100.0, 5103, plants=(9,)), gg.turan(40, 5),
              gg.cocktail_party(9),
              # maximum cliques whose members have core omega - 1
              gg.disjoint_cliques([4, 6, 5]),
              # a heuristic clique of 5 in high cores first, then a K_6 of core 5
              gg.concat([gg.turan(40, 5), gg.complete(6)])[0]]
    return tiny, medium


@pytest.fixture(scope="module")
def battery_refs():
    tiny, medium = _graphs()
    refs = []
    for g in tiny + medium:
        adj = adj_sets(g)
        w = brute_force_omega(adj) if g.n <= 16 else bron_kerbosch_omega(adj)
        G = nx.Graph()
        G.add_nodes_from(range(g.n))
        G.add_edges_from((v, u) for v in range(g.n) for u in adj[v] if v < u)
        core = nx.core_number(G)
        refs.append((g, adj, w, np.array([core[v] for v in range(g.n)])))
    return refs


def _bind(path):
    lib = ctypes.CDLL(path)
    i32p, i64p = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
    I64, I32 = ctypes.c_int64, ctypes.c_int32
    lib.or_max_clique.restype = I32
    lib.or_max_clique.argtypes = [I64, i64p, i32p, I32, i32p, i64p]
    lib.or_peel.restype = I32
    lib.or_peel.argtypes = [I64, i64p, i32p, i32p, i32p, i32p]
    lib.or_core_bz.restype = None
    lib.or_core_bz.argtypes = [I64, i64p, i32p, i32p]
    lib.or_rank.restype = None
    lib.or_rank.argtypes = [I64, i32p, i32p, i32p]
    lib.or_heuristic.restype = I32
    lib.or_heuristic.argtypes = [I64, i64p, i32p, i32p, i32p, i32p, I32, i32p]
    lib.or_root_omega.restype = None
    lib.or_root_omega.argtypes = [I64, i64p, i32p, I32, i32p, i32p, i32p, i32p]
    return lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _failures(lib, refs):
    """Names of the pins the library fails (stops at the first few)."""
    fails = []
    c32, c64 = ctypes.c_int32, ctypes.c_int64
    for g, adj, w0, core0 in refs:
        n = g.n
        off = np.ascontiguousarray(g.offsets, dtype=np.int64)
        idx = np.ascontiguousarray(g.indices if g.nnz else np.zeros(1, np.int32), dtype=np.int32)
        out = np.zeros(n + 2, np.int32)
        st = np.zeros(12, np.int64)
        w = lib.or_max_clique(n, _p(off, c64), _p(idx, c32), 1, _p(out, c32), _p(st, c64))
        if w != w0 or not is_clique(adj, out[:w].tolist()):
            fails.append(f"omega {g.name}")
        bz = np.zeros(n, np.int32)
        lib.or_core_bz(n, _p(off, c64), _p(idx, c32), _p(bz, c32))
        core = np.zeros(n, np.int32)
        rnd = np.zeros(n, np.int32)
        km = np.zeros(1, np.int32)
        lib.or_peel(n, _p(off, c64), _p(idx, c32), _p(core, c32), _p(rnd, c32), _p(km, c32))
        if not np.array_equal(bz, core0):
            fails.append(f"bucket cores {g.name}")
        if not np.array_equal(core, core0) or check_peel(adj, core, rnd) is not None:
            fails.append(f"peel {g.name}")
            continue  # the checks below build on a correct peel
        rk = np.zeros(n, np.int32)
        order = np.zeros(n, np.int32)
        lib.or_rank(n, _p(rnd, c32), _p(rk, c32), _p(order, c32))
        h = np.zeros(n + 2, np.int32)
        hs = lib.or_heuristic(n, _p(off, c64), _p(idx, c32), _p(core, c32), _p(rk, c32),
                              _p(order, c32), -1, _p(h, c32))
        if h[:hs].tolist() != production_heuristic(adj, core, rk, order):
            fails.append(f"heuristic {g.name}")
        for b in sorted({2, max(w0 - 1, 1)}):
            outs = [np.zeros(n, np.int32) for _ in range(4)]
            lib.or_root_omega(n, _p(off, c64), _p(idx, c32), b, *[_p(o, c32) for o in outs])
            for v in range(n):
                if core[v] < b:
                    continue
                if (outs[0][v], outs[1][v], outs[2][v]) != open_form_L(adj, rk, core, v, b):
                    fails.append(f"root report {g.name} b={b}")
                    break
                # omega_v = 1 + omega of the oriented neighbourhood, when > b
                P = [u for u in adj[v] if rk[u] > rk[v] and core[u] >= b]
                loc = {u: i for i, u in enumerate(P)}
                sub = [{loc[x] for x in adj[u] if x in loc} for u in P]
                wv = 1 + (brute_force_omega(sub) if len(P) <= 16 else bron_kerbosch_omega(sub))
                if outs[3][v] != (wv if wv > b else 0):
                    fails.append(f"root omega {g.name} b={b}")
                    break
        if len(fails) >= 3:
            break
    return fails


def test_unmutated_oracle_passes_the_battery(battery_refs):
    assert _failures(_bind(oracle.build(force=False)), battery_refs) == []


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(battery_refs, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {old}"
    with tempfile.TemporaryDirectory() as d:
        cpp = os.path.join(d, "mutant.cpp")
        so = os.path.join(d, "mutant.so")
        with open(cpp, "w") as f:
            f.write(src.replace(old, new))
        subprocess.run(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-pthread", cpp, "-o", so],
                       check=True)
        fails = _failures(_bind(so), battery_refs)
    assert fails, f"mutation '{name}' passed every pin"
