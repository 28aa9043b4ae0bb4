"""Oracle parity of the workloads at their stated sizes, through the C ABI.

* The 2,048-graph batch (n log-uniform in [64, 20,000], half G(n,p), half
  Chung-Lu, planted cliques of 5..60) in one pmc_max_clique_batch call under
  the installed tuning table: every graph's omega equals the oracle's
  (tests/golden/c3.json, written by the oracle only) and every returned
  clique is a clique of its own graph.
* Held-out graphs of the learned-ordering workload (n = 200,000): omega under
  core order and under the trained model's order equals the oracle's
  (tests/golden/c4_heldout.json).
* R-MAT scale 27 (134 M vertices, 1.85 billion edges): every core number
  from pmc_core_numbers equals the oracle's bucket algorithm run on the host
  (linear time; about a minute), and every core number and peel round the
  oracle's level-synchronous peel.
"""
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def pmc():
    from paper_1302_6256_amd import pmc as p
    p.load()
    return p


def clique_ok(off, idx, cl):
    """cl (numpy int ids) is a set of distinct, pairwise adjacent vertices."""
    cl = np.asarray(cl, dtype=np.int64)
    if np.unique(cl).size != cl.size:
        return False
    for v in cl:
        row = idx[off[v]:off[v + 1]]
        if np.count_nonzero(np.isin(cl, row)) != cl.size - 1:
            return False
    return True


def test_c3_batch_full_vs_oracle(pmc):
    ref = json.load(open(os.path.join(GOLDEN, "c3.json")))["graphs"]
    assert len(ref) == 2048
    u, vb = gg.c3_batch(2048)
    d = dev()
    off, idx = torch.from_numpy(u.offsets).to(d), torch.from_numpy(u.indices).to(d)
    om, out, st = pmc.max_clique_batch(off, idx, vb)
    torch.cuda.synchronize()
    want = [r["omega"] for r in ref]
    bad = [i for i in range(2048) if om[i] != want[i]]
    assert not bad, [(i, om[i], want[i]) for i in bad[:10]]
    out = out.cpu().numpy()
    for i in range(2048):
        cl = out[vb[i]:vb[i] + om[i]]
        assert np.all((cl >= vb[i]) & (cl < vb[i + 1])), i
        assert clique_ok(u.offsets, u.indices, cl), i
    assert st["certified"] == 1


@pytest.fixture(scope="module")
def trained(pmc):
    from paper_1302_6256_amd import learn
    w = learn.load_weights()
    if w is None:
        pytest.skip("no trained weights")
    return torch.tensor(np.asarray(w, dtype=np.float32), device=dev())


@pytest.mark.parametrize("row", json.load(open(os.path.join(GOLDEN, "c4_heldout.json")))["graphs"],
                         ids=lambda r: f"c4-{r['i']}")
def test_c4_heldout_vs_oracle(pmc, trained, row):
    g = gg.c4_graph(row["i"])
    assert (g.n, g.m) == (row["n"], row["m"])
    d = dev()
    off, idx = torch.from_numpy(g.offsets).to(d), torch.from_numpy(g.indices).to(d)
    for opts in ({}, {"mlp": trained}):
        w, cl, st = pmc.max_clique(off, idx, **opts)
        assert w == row["omega"], (opts.keys(), w, row["omega"])
        assert clique_ok(g.offsets, g.indices, cl.cpu().numpy())
        assert st["heuristic"] <= w <= st["kmax"] + 1


@pytest.mark.timeout(1100)
def test_c5_core_numbers_vs_oracle(pmc):
    """All 134 M core numbers against the oracle's bucket algorithm, then the
    core numbers and peel rounds against the oracle's level-synchronous peel
    (both on the host; the peel takes about a minute here)."""
    from graphgen import device as gd
    d = dev()
    off, idx, n, m, _ = gd.c5_csr(27, 14, device=d)
    print(f"c5: generated n={n} m={m}", flush=True)
    core, rnd, _, _, km, nr = pmc.core_numbers(off, idx)
    torch.cuda.synchronize()
    core_gpu = core.cpu().numpy()
    rnd_gpu = rnd.cpu().numpy()
    del core, rnd
    off_h = off.cpu().numpy()
    del off
    idx_h = idx.cpu().numpy()
    del idx
    torch.cuda.empty_cache()
    ref = oracle.core_bz(off_h, idx_h)
    print("c5: bucket algorithm done", flush=True)
    assert ref.shape == core_gpu.shape == (n,)
    assert int(ref.max()) == km
    mism = np.count_nonzero(ref != core_gpu)
    assert mism == 0, mism
    del ref
    c0, r0, km0, nr0 = oracle.peel(off_h, idx_h)
    print("c5: level-synchronous peel done", flush=True)
    assert (km0, nr0) == (km, nr)
    assert np.count_nonzero(c0 != core_gpu) == 0
    assert np.count_nonzero(r0 != rnd_gpu) == 0
