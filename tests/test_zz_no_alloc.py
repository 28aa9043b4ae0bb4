"""The allocation-free entry point pmc_core_numbers_noalloc against
pmc_core_numbers, through the C ABI: core numbers, peel rounds, ranks, order,
K and the round count identical, on two calls in a row (the second on a
smaller graph, over the fixed scratch the first one left behind), plus the
documented rejection of a graph too large for the fixed scratch."""
import numpy as np
import pytest

import graphgen as gg
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pmc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1302_6256_amd import pmc as p
    p.load()
    return p


def _dev(g, bits=64):
    d = torch.device("cuda:0")
    off = torch.from_numpy(g.offsets.astype(np.int64 if bits == 64 else np.int32)).to(d)
    idx = torch.from_numpy(g.indices if g.nnz else np.zeros(0, np.int32)).to(d)
    return off, idx


def test_noalloc_matches_core_numbers(pmc):
    graphs = [gg.chung_lu(200_000, 2.1, 16.0, 2000.0, gg.seed_for(71, 0), plants=(25,)),
              gg.chung_lu(3_000, 2.3, 8.0, 200.0, gg.seed_for(71, 1), plants=(12,))]
    for i, g in enumerate(graphs):
        for bits in (64, 32):
            off, idx = _dev(g, bits)
            ref = pmc.core_numbers(off, idx)
            got = pmc.core_numbers(off, idx, noalloc=True)
            torch.cuda.synchronize()
            for a, b in zip(ref[:4], got[:4]):
                assert torch.equal(a, b), (i, bits)
            assert ref[4:] == got[4:], (i, bits)
        if i == 1:  # the small one also against the oracle
            core, rnd, km, nr = oracle.peel(g.offsets, g.indices)
            assert np.array_equal(got[0].cpu().numpy(), core)
            assert np.array_equal(got[1].cpu().numpy(), rnd)
            assert (got[4], got[5]) == (km, nr)


def test_noalloc_rejects_oversized_graph(pmc):
    # a valid edgeless graph of 10^7 vertices: its scratch bound (52 bytes per
    # vertex and more) exceeds the fixed 256 MiB, so the call refuses it
    n = 10_000_000
    d = torch.device("cuda:0")
    off = torch.zeros(n + 1, dtype=torch.int64, device=d)
    idx = torch.zeros(1, dtype=torch.int32, device=d)[:0]
    with pytest.raises(pmc.PmcError) as e:
        pmc.core_numbers(off, idx, noalloc=True)
    assert e.value.status == 3
    assert "fixed buffer" in str(e.value)
