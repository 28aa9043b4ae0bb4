"""GPU parity of the batch entry point: every graph of a disjoint-union batch
gets the omega the oracle computes for it alone, a valid clique inside its
own id range, and frozen-bound per-root reports equal to the oracle's."""
import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def pmc():
    from paper_1302_6256_amd import pmc as p
    p.load()
    return p


def batch_graphs():
    gs = []
    for i in range(12):
        gs.append(gg.gnp(50 + 37 * i, 0.05 + 0.03 * (i % 5), 700 + i, plants=(3 + i,)))
    for i in range(10):
        gs.append(gg.chung_lu(300 + 211 * i, 2.2, 6.0 + 2 * i, 80.0 + 10 * i, 800 + i,
                              plants=(5 + 2 * i,)))
    gs += [gg.empty(1), gg.empty(5), gg.complete(9), gg.cycle(7), gg.cocktail_party(40),
           gg.turan(120, 6), gg.path(30), gg.star(20), gg.complete(70), gg.gnp(180, 0.5, 3)]
    return gs


@pytest.fixture(scope="module")
def batch():
    gs = batch_graphs()
    u, vb = gg.concat(gs)
    refs = [oracle.max_clique(g.offsets, g.indices)[0] for g in gs]
    return gs, u, vb, refs


def check_cliques(gs, u, vb, om, out):
    out = out.cpu().numpy()
    for g_i, g in enumerate(gs):
        cl = out[vb[g_i]:vb[g_i] + om[g_i]]
        assert list(cl) == sorted(cl)
        assert all(vb[g_i] <= v < vb[g_i + 1] for v in cl)
        rows = {v: set(u.indices[u.offsets[v]:u.offsets[v + 1]].tolist()) for v in cl}
        assert all(b in rows[a] for a in cl for b in cl if a != b)


def test_batch_omega_matches_oracle(pmc, batch):
    gs, u, vb, refs = batch
    d = dev()
    off = torch.from_numpy(u.offsets).to(d)
    idx = torch.from_numpy(u.indices).to(d)
    om, out, st = pmc.max_clique_batch(off, idx, vb, validate=True)
    assert om == refs
    check_cliques(gs, u, vb, om, out)
    for kw in ({"skip_heuristic": 1}, {"use_neighborhood_cores": 0},
               {"score": torch.rand(u.n, generator=torch.Generator().manual_seed(1)).to(d)}):
        om2, out2, _ = pmc.max_clique_batch(off, idx, vb, **kw)
        assert om2 == refs, kw
        check_cliques(gs, u, vb, om2, out2)


def test_batch_frozen_reports(pmc, batch):
    gs, u, vb, refs = batch
    d = dev()
    off = torch.from_numpy(u.offsets).to(d)
    idx = torch.from_numpy(u.indices).to(d)
    rep = torch.full((4 * u.n,), -7, dtype=torch.int32, device=d)
    om, out, st = pmc.max_clique_batch(off, idx, vb, frozen_bound=0, root_report=rep)
    rep = rep.cpu().numpy().reshape(-1, 4)
    for g_i, g in enumerate(gs):
        ref = oracle.root_omega(g.offsets, g.indices, 0)
        part = rep[vb[g_i]:vb[g_i + 1]]
        for j, key in enumerate(("s", "kn", "L", "omega")):
            assert np.array_equal(part[:, j], ref[key]), (g_i, key)
    assert om == refs


def test_batch_equals_single_solves(pmc, batch):
    gs, u, vb, refs = batch
    d = dev()
    for g, w in zip(gs[:8], refs[:8]):
        w1, _, _ = pmc.max_clique(torch.from_numpy(g.offsets).to(d),
                                  torch.from_numpy(g.indices).to(d))
        assert w1 == w


def test_batch_rejects_cross_edges(pmc):
    a, b = gg.complete(4), gg.complete(3)
    u, vb = gg.concat([a, b])
    d = dev()
    with pytest.raises(pmc.PmcError) as e:
        # claim the first graph has 3 vertices: vertex 3's edges cross graphs
        pmc.max_clique_batch(torch.from_numpy(u.offsets).to(d), torch.from_numpy(u.indices).to(d),
                             [0, 3, 7], validate=True)
    assert e.value.status == 2


def test_single_graph_batch(pmc):
    g = gg.c1_graph()
    d = dev()
    om, out, _ = pmc.max_clique_batch(torch.from_numpy(g.offsets).to(d),
                                      torch.from_numpy(g.indices).to(d), [0, g.n])
    assert om == [15]


def test_graph_mode_replays_match_eager(pmc, batch):
    """The search stage captured as one hipGraph: several solves in a row, with
    eager work and synchronisations between them, each equal to eager mode."""
    gs, u, vb, refs = batch
    d = dev()
    off = torch.from_numpy(u.offsets).to(d)
    idx = torch.from_numpy(u.indices).to(d)
    saved = pmc.get_tuning()
    try:
        pmc.set_tuning(dict(saved, search_graph=1))
        for rep in range(4):
            om, out, st = pmc.max_clique_batch(off, idx, vb)
            assert om == refs, rep
            check_cliques(gs, u, vb, om, out)
            x = torch.arange(1000, device=d).sum()  # eager work between replays
            torch.cuda.synchronize()
            assert int(x) == 499500
            w, _, _ = pmc.max_clique(off, idx)  # the union as one graph, eager path
            assert w == max(refs)
    finally:
        pmc.set_tuning(saved)


def test_graph_array_entry_point(pmc, batch):
    """pmc_max_clique_graphs: the same graphs as separate device CSRs (32- and
    64-bit offsets mixed), solved in one call; every omega equals the
    oracle's and every clique, in the graph's own ids, is a clique of it."""
    gs, _, _, refs = batch
    d = dev()
    parts = []
    for i, g in enumerate(gs):
        bits = np.int32 if i % 2 else np.int64
        parts.append((torch.from_numpy(g.offsets.astype(bits)).to(d),
                      torch.from_numpy(g.indices if g.nnz else np.zeros(0, np.int32)).to(d)))
    om, cls, st = pmc.max_clique_graphs(parts, validate=True)
    assert om == refs
    for g, cl in zip(gs, cls):
        cl = cl.cpu().tolist()
        assert cl == sorted(cl) and all(0 <= v < g.n for v in cl)
        rows = {v: set(g.indices[g.offsets[v]:g.offsets[v + 1]].tolist()) for v in cl}
        assert all(b in rows[a] for a in cl for b in cl if a != b)
    assert st["certified"] == 1
