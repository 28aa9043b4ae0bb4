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
    """The search stage captured as one hipGraph and kept for replay: several
    solves in a row (back to back, where the kept graph is replayed, and with
    eager work, synchronisations and a solve of another shape between them,
    which replaces it), each equal to eager mode."""
    gs, u, vb, refs = batch
    d = dev()
    off = torch.from_numpy(u.offsets).to(d)
    idx = torch.from_numpy(u.indices).to(d)
    saved = pmc.get_tuning()
    try:
        pmc.set_tuning(dict(saved, search_graph=1))
        for rep in range(4):
            replays = 0
            for again in range(3):
                om, out, st = pmc.max_clique_batch(off, idx, vb)
                assert om == refs, (rep, again)
                check_cliques(gs, u, vb, om, out)
                replays += st["search_graph_replays"]
            # back to back, the scratch comes back at the same addresses and
            # the kept graph is replayed
            assert replays >= 1, rep
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


def peel_batch_graphs():
    """The batch above plus graphs on both sides of the per-graph peel's
    4,096-vertex split and one of 32,768 vertices, its largest graph."""
    return batch_graphs() + [gg.gnp(4096, 0.002, 901), gg.gnp(4097, 0.003, 902),
                             gg.chung_lu(12000, 2.1, 12.0, 400.0, 903, plants=(25,)),
                             gg.gnp(32768, 0.0004, 904, plants=(7,))]


def test_core_numbers_batch_vs_oracle(pmc):
    """pmc_core_numbers_batch: every graph's core numbers and rounds equal the
    oracle's peel of that graph alone, K and the round count per graph too;
    the union's rank is the (round, id) order, so within each graph it orders
    the vertices as the graph's own rank does."""
    gs = peel_batch_graphs()
    u, vb = gg.concat(gs)
    d = dev()
    off, idx = torch.from_numpy(u.offsets).to(d), torch.from_numpy(u.indices).to(d)
    core, rnd, rank, order, km, nr = pmc.core_numbers_batch(off, idx, vb)
    core, rnd, rank, order = (t.cpu().numpy() for t in (core, rnd, rank, order))
    n = u.n
    assert np.array_equal(order, np.lexsort((np.arange(n), rnd)))
    assert np.array_equal(rank[order], np.arange(n))
    for i, g in enumerate(gs):
        c0, r0, k0, n0 = oracle.peel(g.offsets, g.indices)
        lo, hi = vb[i], vb[i + 1]
        assert np.array_equal(core[lo:hi], c0), i
        assert np.array_equal(rnd[lo:hi], r0), i
        assert (km[i], nr[i]) == (k0, n0), i
        rk0, _ = oracle.rank(r0)
        assert np.array_equal(np.argsort(rank[lo:hi]), np.argsort(rk0)), i


def test_batch_peel_per_graph_and_union_agree(pmc, batch):
    """max_clique_batch gives the oracle's omegas and valid cliques whether
    the batch is peeled one workgroup per graph or as one union."""
    gs, u, vb, refs = batch
    d = dev()
    off, idx = torch.from_numpy(u.offsets).to(d), torch.from_numpy(u.indices).to(d)
    for mode in (1, -1):
        om, out, st = pmc.max_clique_batch(off, idx, vb, tune_table={"batch_peel": mode})
        assert om == refs, mode
        check_cliques(gs, u, vb, om, out)


def test_batch_with_a_graph_beyond_the_per_graph_peel(pmc):
    """A graph of more than 32,768 vertices: pmc_core_numbers_batch refuses
    the batch (capacity) before any work; max_clique_batch peels the union
    and still gets every graph's omega."""
    gs = [gg.gnp(40000, 0.0002, 905, plants=(6,)), gg.complete(5), gg.gnp(300, 0.1, 906)]
    u, vb = gg.concat(gs)
    d = dev()
    off, idx = torch.from_numpy(u.offsets).to(d), torch.from_numpy(u.indices).to(d)
    with pytest.raises(pmc.PmcError) as e:
        pmc.core_numbers_batch(off, idx, vb)
    assert e.value.status == pmc.PMC_ERR_CAPACITY
    om, out, _ = pmc.max_clique_batch(off, idx, vb)
    assert om == [oracle.max_clique(g.offsets, g.indices)[0] for g in gs]
    check_cliques(gs, u, vb, om, out)
