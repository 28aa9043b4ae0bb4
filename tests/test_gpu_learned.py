"""GPU parity of the learned ordering against the float64 reference
(oracle/learned.py): features, the BF16-MFMA forward, the hand-written
backward, Adam, training progress, and omega invariance under learned order.

Tolerances.  Features are fp32 arithmetic on exact integers: relative 1e-5.
The MLP rounds X, W1, H1 and W2 to bf16 (unit roundoff u = 2^-8) and
accumulates in fp32; with ReLU 1-Lipschitz, every output error is at most
about (number of roundings on the path) * u times the same network evaluated
on absolute values (|X|, |W|), so forward scores are checked against
6 u * s_abs.  Gradients pass through the same roundings plus bf16 dZ2/dZ1:
checked as relative L2 error <= 3e-2 and cosine >= 0.999.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import learned as L

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


GRAPHS = [gg.c1_graph(), gg.chung_lu(20000, 2.1, 20.0, 500.0, 7, plants=(10,)),
          gg.gnp(700, 0.3, 4), gg.complete(30), gg.empty(5), gg.star(40)]


@pytest.mark.parametrize("g", GRAPHS, ids=lambda g: g.name)
def test_features_exact(pmc, g):
    d = dev()
    f = pmc.vertex_features(torch.from_numpy(g.offsets).to(d), torch.from_numpy(g.indices).to(d))
    core, _, _, _ = oracle.peel(g.offsets, g.indices)
    ref = L.features(g.offsets, g.indices, core)
    assert np.allclose(f.cpu().numpy(), ref, rtol=1e-5, atol=1e-6)


def random_batch(n, seed):
    rng = np.random.Generator(np.random.Philox(seed))
    X = np.abs(rng.normal(size=(n, L.F_IN))) * rng.uniform(0.1, 3.0, size=L.F_IN)
    y = rng.uniform(0, 1, size=n)
    return X, y


@pytest.mark.parametrize("n", [1, 15, 16, 17, 1000, 50000])
def test_forward_within_bf16_bound(pmc, n):
    d = dev()
    X, _ = random_batch(n, n)
    p = L.init_params(11)
    p[L.N_PARAMS - 1] = 0.25
    s = pmc.mlp_forward(torch.tensor(p, dtype=torch.float32, device=d),
                        torch.tensor(X, dtype=torch.float32, device=d)).cpu().numpy()
    ref, _ = L.forward(p, X)
    s_abs, _ = L.forward(np.abs(p), np.abs(X))
    u = 2.0 ** -8
    assert np.all(np.abs(s - ref) <= 6 * u * s_abs + 1e-6)


@pytest.mark.parametrize("n", [16, 333, 20000])
def test_gradient_matches_reference(pmc, n):
    d = dev()
    X, y = random_batch(n, 100 + n)
    p = L.init_params(12)
    pt = torch.tensor(p, dtype=torch.float32, device=d)
    z = torch.zeros_like(pt)
    loss, g = pmc.mlp_train_step(pt, z.clone(), z.clone(), 1, 0.0,
                                 torch.tensor(X, dtype=torch.float32, device=d),
                                 torch.tensor(y, dtype=torch.float32, device=d), want_grad=True)
    ref_loss, ref_g = L.loss_and_grad(p, X, y)
    g = g.cpu().numpy().astype(np.float64)
    assert abs(loss - ref_loss) <= 3e-2 * ref_loss + 1e-6
    rel = np.linalg.norm(g - ref_g) / np.linalg.norm(ref_g)
    cos = g @ ref_g / (np.linalg.norm(g) * np.linalg.norm(ref_g))
    assert rel <= 3e-2 and cos >= 0.999, (rel, cos)
    # every parameter block carries gradient
    for name, (a, b) in {"W1": (0, 512), "b1": (512, 576), "W2": (576, 4672), "b2": (4672, 4736),
                         "w3": (4736, 4800), "b3": (4800, 4801)}.items():
        rb = np.linalg.norm(g[a:b] - ref_g[a:b]) / max(np.linalg.norm(ref_g[a:b]), 1e-12)
        assert rb <= 5e-2, name


def test_adam_step_matches_reference(pmc):
    d = dev()
    X, y = random_batch(4000, 7)
    p = L.init_params(13)
    pt = torch.tensor(p, dtype=torch.float32, device=d)
    m = torch.zeros_like(pt)
    v = torch.zeros_like(pt)
    Xt = torch.tensor(X, dtype=torch.float32, device=d)
    yt = torch.tensor(y, dtype=torch.float32, device=d)
    pm, mm, vm = p.copy(), np.zeros_like(p), np.zeros_like(p)
    for step in (1, 2, 3):
        before = pt.cpu().numpy().astype(np.float64)
        _, g = pmc.mlp_train_step(pt, m, v, step, 1e-3, Xt, yt, want_grad=True)
        pm, mm, vm = L.adam(before, mm, vm, g.cpu().numpy().astype(np.float64), step, 1e-3)
        assert np.allclose(pt.cpu().numpy(), pm, rtol=1e-5, atol=1e-7)


def test_training_reduces_loss(pmc):
    d = dev()
    g = gg.chung_lu(20000, 2.2, 12.0, 300.0, 21, plants=(25,))
    off, idx = torch.from_numpy(g.offsets).to(d), torch.from_numpy(g.indices).to(d)
    feat = pmc.vertex_features(off, idx)
    rep = torch.full((4 * g.n,), -1, dtype=torch.int32, device=d)
    w, _, _ = pmc.max_clique(off, idx, frozen_bound=0, root_report=rep)
    label = (rep.view(-1, 4)[:, 3].float() / w).contiguous()
    p = torch.tensor(L.init_params(3), dtype=torch.float32, device=d)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    losses = [pmc.mlp_train_step(p, m, v, t, 3e-3, feat, label)[0] for t in range(1, 201)]
    assert losses[-1] < 0.5 * losses[0]


@pytest.mark.parametrize("g", GRAPHS[:3] + [gg.gnp(200, 0.5, 1)], ids=lambda g: g.name)
def test_learned_order_keeps_omega(pmc, g):
    d = dev()
    off, idx = torch.from_numpy(g.offsets).to(d), torch.from_numpy(g.indices).to(d)
    w0, _, _ = oracle.max_clique(g.offsets, g.indices)
    for seed in (1, 2):
        p = torch.tensor(L.init_params(seed), dtype=torch.float32, device=d)
        w, cl, st = pmc.max_clique(off, idx, mlp=p)
        assert w == w0
    # a model producing NaN scores falls back to the rank order in ties
    p = torch.full((L.N_PARAMS,), float("nan"), dtype=torch.float32, device=d)
    w, _, _ = pmc.max_clique(off, idx, mlp=p)
    assert w == w0


def test_trained_network_gain(pmc):
    """What the trained network gains over the method without it, on two
    held-out graphs of the learned-ordering workload (n = 200,000): omega is
    the same under the learned and the core order, and the trained scores rank
    the vertices by omega_v (the largest clique each root holds) clearly better
    than the core numbers do (Spearman correlation).  Time-to-certified omega
    under both orders is measured beside it by learn.evaluate: there the
    feature pass costs more than the better order saves, which the test
    records but does not assert."""
    dev()
    from paper_1302_6256_amd import learn
    summary, rows = learn.evaluate(n_graphs=2, log=lambda s: None)
    assert summary["graphs"] == 2 and len(rows) == 2
    for r in rows:
        assert r["spearman_trained"] > r["spearman_core"] + 0.05
        assert r["t_core_ms"] > 0 and r["t_learned_ms"] > 0
