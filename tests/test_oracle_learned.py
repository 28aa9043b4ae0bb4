"""Pins of the learned-ordering reference (oracle/learned.py): gradients against
central finite differences, triangle counts against networkx, the neighbour
statistics against explicit per-vertex sets, and Adam against its closed form
on a quadratic."""
import networkx as nx
import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import learned as L


def test_gradients_finite_differences():
    rng = np.random.Generator(np.random.Philox(3))
    X = rng.normal(size=(37, L.F_IN))
    y = rng.normal(size=37)
    p = L.init_params(5)
    p[L.N_PARAMS - 1] = 0.3  # nonzero output bias
    loss, g = L.loss_and_grad(p, X, y)
    h = 1e-5
    idx = list(range(0, L.N_PARAMS, 53)) + [L.N_PARAMS - 1, 512, 513, 600]
    for i in idx:
        e = np.zeros(L.N_PARAMS)
        e[i] = h
        num = (L.loss_and_grad(p + e, X, y)[0] - L.loss_and_grad(p - e, X, y)[0]) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(num)), (i, num, g[i])


def test_triangles_networkx():
    for g in (gg.gnp(120, 0.1, 4), gg.chung_lu(500, 2.2, 10.0, 80.0, 5, plants=(7,)),
              gg.complete(6), gg.empty(3)):
        G = nx.Graph()
        G.add_nodes_from(range(g.n))
        src = np.repeat(np.arange(g.n), np.diff(g.offsets))
        G.add_edges_from(zip(src.tolist(), g.indices.tolist()))
        t = nx.triangles(G)
        assert L.triangles(g.offsets, g.indices).tolist() == [float(t[v]) for v in range(g.n)]


def test_feature_definitions():
    g = gg.chung_lu(300, 2.2, 8.0, 60.0, 6, plants=(6,))
    core, _, km, _ = oracle.peel(g.offsets, g.indices)
    X = L.features(g.offsets, g.indices, core)
    adj = [set(g.indices[g.offsets[v]:g.offsets[v + 1]].tolist()) for v in range(g.n)]
    K = max(km, 1)
    for v in range(g.n):
        d = len(adj[v])
        assert X[v, 0] == pytest.approx(np.log1p(d))
        assert X[v, 1] == pytest.approx(np.log1p(core[v]))
        assert X[v, 2] == pytest.approx(core[v] / K)
        if d:
            cs = [core[u] for u in adj[v]]
            assert X[v, 4] == pytest.approx(sum(cs) / d / K)
            assert X[v, 5] == pytest.approx(max(cs) / K)
            assert X[v, 6] == pytest.approx(min(cs) / K)
            assert X[v, 7] == pytest.approx(sum(c >= core[v] for c in cs) / d)
        else:
            assert (X[v, 4:] == 0).all()


def test_adam_closed_form():
    # first step of Adam moves every coordinate by lr * sign(grad) (bias-corrected)
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    p1, m, v = L.adam(p, np.zeros(3), np.zeros(3), g, 1, 0.01)
    assert np.allclose(p1, p - 0.01 * np.sign(g), atol=1e-6)
    # on f(x) = x^2 / 2 Adam converges to 0
    x, m, v = np.array([2.0]), np.zeros(1), np.zeros(1)
    for t in range(1, 3001):
        x, m, v = L.adam(x, m, v, x.copy(), t, 0.01)
    assert abs(x[0]) < 1e-2


def test_flat_layout():
    assert L.N_PARAMS == 8 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 4801
    p = L.init_params(1)
    assert np.array_equal(L.flatten(L.unflatten(p)), p)
