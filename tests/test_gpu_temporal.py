"""GPU parity of the strong-reachability graph (Sec. 6.1) against the oracle
(CSR compared exactly) and of the largest temporal strong component."""
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


CASES = [(6, list(range(6)), [1, 2, 3, 4, 5, 0]),
         (7, list(range(7)) * 2, [(i + 1) % 7 for i in range(7)] * 2),
         (5, [], []), (1, [], []),
         (130,) + tuple(gg.temporal_contacts(130, 900, 5, 0.8, 1)),
         (64,) + tuple(gg.temporal_contacts(64, 3000, 3, 0.9, 2, directed_frac=0.5)),
         (700,) + tuple(gg.temporal_contacts(700, 6000, 12, 0.85, 3, directed_frac=0.3)),
         (2000,) + tuple(gg.temporal_contacts(2000, 20000, 40, 0.8, 4, directed_frac=0.2)),
         (4, [0, 1, 1, 2, 3, 3], [1, 1, 2, 0, 3, 2]),  # self-loops change nothing
         # 32-, 16- and 8-bit column slices of the reach matrix
         (20000,) + tuple(gg.temporal_contacts(20000, 30000, 2000, 0.9, 5, directed_frac=0.3)),
         (40000,) + tuple(gg.temporal_contacts(40000, 40000, 4000, 0.9, 6, directed_frac=0.3)),
         (70000,) + tuple(gg.temporal_contacts(70000, 50000, 7000, 0.9, 7, directed_frac=0.3))]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c[0]}_m{len(c[1])}")
def test_strong_reachability_exact(pmc, case):
    n, src, dst = case
    d = dev()
    s = torch.tensor(np.asarray(src, dtype=np.int32), device=d)
    t = torch.tensor(np.asarray(dst, dtype=np.int32), device=d)
    off, idx = pmc.strong_reachability(n, s, t)
    off0, adj0 = oracle.strong_reach(n, src, dst)
    assert np.array_equal(off.cpu().numpy(), off0)
    assert np.array_equal(idx.cpu().numpy(), adj0)
    if 1 < n <= 130:  # larger contact graphs are nearly complete: hard for any search
        w, cl = pmc.temporal_strong_component(n, s, t)
        w0, _, _ = oracle.max_clique(off0, adj0)
        assert w == w0
        members = cl.cpu().tolist()
        assert len(members) == w
        for a in members:
            row = set(adj0[off0[a]:off0[a + 1]].tolist())
            assert set(members) - {a} <= row


def test_strong_reachability_errors(pmc):
    d = dev()
    s = torch.tensor([0, 5], dtype=torch.int32, device=d)
    t = torch.tensor([1, 0], dtype=torch.int32, device=d)
    with pytest.raises(pmc.PmcError):
        pmc.strong_reachability(3, s, t)  # endpoint out of range


def _standins():
    from paper_1302_6256_amd.temporal_eval import WORKLOADS
    return WORKLOADS


@pytest.mark.parametrize("w", _standins(), ids=lambda w: w[0].split()[0])
def test_temporal_standins_vs_oracle(pmc, w):
    """The six Table 2 stand-ins of temporal_eval: the strong-reachability
    CSR equals the oracle's, and the largest temporal strong component (the
    maximum clique of that graph) has the oracle's size."""
    name, n, contacts, groups, pw, seed, dfrac = w
    src, dst = gg.temporal_contacts(n, contacts, groups, pw, seed, directed_frac=dfrac)
    d = dev()
    s = torch.tensor(np.asarray(src, dtype=np.int32), device=d)
    t = torch.tensor(np.asarray(dst, dtype=np.int32), device=d)
    off, idx = pmc.strong_reachability(n, s, t)
    off0, adj0 = oracle.strong_reach(n, src, dst)
    assert np.array_equal(off.cpu().numpy(), off0)
    assert np.array_equal(idx.cpu().numpy(), adj0)
    w_gpu, cl, st = pmc.max_clique(off, idx)
    w0, _, _ = oracle.max_clique_ex(off0, adj0, threads=8)
    assert w_gpu == w0 and st["certified"] == 1
    members = cl.cpu().tolist()
    for a in members:
        row = set(adj0[off0[a]:off0[a + 1]].tolist())
        assert set(members) - {a} <= row
