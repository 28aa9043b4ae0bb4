"""The scale workload at full size: R-MAT scale 27 (134,217,728 vertices,
about 1.85 billion edges, a 15 GB CSR with int64 offsets), generated on the
device.  The oracle cannot run at this size, so the checks are properties
that hold at any size:

* core numbers and rounds satisfy the level-synchronous peel's per-vertex
  characterisation on sampled vertices (every round has one level, levels
  never decrease; a vertex of round r has at most k_r neighbours of round
  >= r, and more than k_{r-1} neighbours of round >= r-1);
* a node-budgeted solve returns a clique (pairwise adjacent, distinct ids)
  at least as large as the planted one and at most K + 1."""
import pytest

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


def rows_of(off, idx, vs):
    """Flattened neighbour lists of the vertices vs: (segment id, neighbour)."""
    lens = off[vs + 1] - off[vs]
    seg = torch.repeat_interleave(torch.arange(vs.numel(), device=vs.device), lens)
    start = torch.repeat_interleave(off[vs], lens)
    first = torch.repeat_interleave(torch.cumsum(lens, 0) - lens, lens)
    pos = start + torch.arange(seg.numel(), device=vs.device) - first
    return seg, idx[pos].long()


def test_c5_full_size(pmc):
    from graphgen import device as gd
    d = dev()
    off, idx, n, m, planted = gd.c5_csr(27, 14, device=d)
    assert n == 1 << 27 and off.numel() == n + 1 and idx.numel() == 2 * m
    assert m > 1_700_000_000
    core, rnd, rank, order, km, nr = pmc.core_numbers(off, idx)
    core, rnd = core.long(), rnd.long()
    assert 0 <= int(rnd.min()) and int(rnd.max()) == nr - 1
    assert int(core.max()) == km
    # every round has one level; levels never decrease
    lev_hi = torch.full((nr,), -1, dtype=torch.long, device=d).scatter_reduce_(0, rnd, core, "amax")
    lev_lo = torch.full((nr,), 1 << 40, dtype=torch.long, device=d).scatter_reduce_(0, rnd, core, "amin")
    assert torch.equal(lev_hi, lev_lo)
    assert bool((lev_hi[1:] >= lev_hi[:-1]).all())
    # per-vertex conditions on sampled vertices (and the planted clique)
    g = torch.Generator(device="cpu").manual_seed(5)
    vs = torch.cat([torch.randint(0, n, (4096,), generator=g),
                    torch.tensor(planted[0], dtype=torch.long)]).to(d)
    seg, nb = rows_of(off, idx, vs)
    rv = rnd[vs]
    ge = torch.zeros(vs.numel(), dtype=torch.long, device=d).index_add_(
        0, seg, (rnd[nb] >= rv[seg]).long())
    ge_prev = torch.zeros(vs.numel(), dtype=torch.long, device=d).index_add_(
        0, seg, (rnd[nb] >= rv[seg] - 1).long())
    assert bool((ge <= core[vs]).all())
    later = rv >= 1
    assert bool((ge_prev[later] > lev_hi[rv[later] - 1]).all())
    del seg, nb, core, rnd, rank, order
    # budgeted solve: a valid clique, at least the planted size, at most K + 1
    w, cl, st = pmc.max_clique(off, idx, node_budget=1_000_000, allow_budget=True)
    assert len(planted[0]) <= w <= km + 1
    members = cl.long()
    assert members.numel() == w and torch.unique(members).numel() == w
    assert bool(((members >= 0) & (members < n)).all())
    seg, nb = rows_of(off, idx, members)
    hits = torch.zeros(w, dtype=torch.long, device=d).index_add_(
        0, seg, torch.isin(nb, members).long())
    assert bool((hits == w - 1).all())
    del off, idx, cl, members, seg, nb
    torch.cuda.empty_cache()
