"""Seeded R-MAT graphs generated on a device with PyTorch, for sizes where the
host generator takes minutes (R-MAT scale 27: 1.9 billion samples).

Same recipe as ``graphgen.rmat``: edge_factor * 2^scale samples, each choosing
one of the four quadrants per level with probabilities (a, b, c, 1-a-b-c);
symmetrised, self-loops dropped, duplicates removed, cliques planted on
disjoint uniformly chosen vertex sets.  The random stream is torch's seeded
device generator, so the instance differs from the host generator's for the
same seed (it is reproducible for a given seed, device type and PyTorch
build).  Input generation only: nothing here computes any part of the method.
Work is split into buckets by the top bits of a key so that no sort handles
more than about a billion keys.
"""
from __future__ import annotations

BUCKET_BITS = 4


def _bucket_of(keys, shift):
    return (keys >> shift).to(dtype=keys.dtype)


def rmat_csr(scale, edge_factor, a, b, c, seed, plants=(), device="cuda:0", chunk=1 << 27):
    """Returns (offsets int64 [n+1], indices int32 [2m], n, m, planted) with
    rows sorted ascending; `planted` lists the vertex sets of the planted
    cliques."""
    import torch
    n = 1 << scale
    samples = edge_factor << scale
    nb = 1 << BUCKET_BITS
    kshift = 2 * scale - BUCKET_BITS  # bucket = top bits of the key = top bits of its row
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    ab, abc = a + b, a + b + c
    buckets = [[] for _ in range(nb)]

    def add(keys):
        bk = _bucket_of(keys, kshift)
        order = torch.argsort(bk)
        keys, bk = keys[order], bk[order]
        counts = torch.bincount(bk, minlength=nb).tolist()
        pos = 0
        for i, cnt in enumerate(counts):
            if cnt:
                buckets[i].append(keys[pos:pos + cnt].clone())
            pos += cnt

    done = 0
    while done < samples:
        cnt = min(chunk, samples - done)
        u = torch.zeros(cnt, dtype=torch.int64, device=device)
        v = torch.zeros(cnt, dtype=torch.int64, device=device)
        for _ in range(scale):
            r = torch.rand(cnt, generator=gen, device=device)
            u.mul_(2).add_((r >= ab).to(torch.int64))                        # quadrants c, d
            v.mul_(2).add_((((r >= a) & (r < ab)) | (r >= abc)).to(torch.int64))  # b, d
            del r
        lo, hi = torch.minimum(u, v), torch.maximum(u, v)
        del u, v
        keep = lo != hi
        add((lo[keep] << scale) | hi[keep])
        del lo, hi, keep
        done += cnt
    planted = []
    if plants:
        perm = torch.randperm(n, generator=gen, device=device)
        pos = 0
        for k in plants:
            vs = torch.sort(perm[pos:pos + k]).values
            pos += k
            i, j = torch.triu_indices(k, k, 1, device=device)
            add((vs[i] << scale) | vs[j])
            planted.append(vs.cpu().tolist())
        del perm
    # undirected edges: sorted and unique per bucket (buckets follow key order)
    und = []
    for i in range(nb):
        if buckets[i]:
            und.append(torch.unique(torch.cat(buckets[i]), sorted=True))
        buckets[i] = None
    m = int(sum(x.numel() for x in und))
    # both directions, bucketed by row, sorted per bucket
    buckets = [[] for _ in range(nb)]
    for x in und:
        lo, hi = x >> scale, x & (n - 1)
        add(x)
        add((hi << scale) | lo)
        del lo, hi
    del und
    counts = torch.zeros(n, dtype=torch.int64, device=device)
    cols = []
    for i in range(nb):
        if not buckets[i]:
            continue
        d = torch.sort(torch.cat(buckets[i])).values
        buckets[i] = None
        counts += torch.bincount(d >> scale, minlength=n)
        cols.append((d & (n - 1)).to(torch.int32))
        del d
    offsets = torch.zeros(n + 1, dtype=torch.int64, device=device)
    torch.cumsum(counts, 0, out=offsets[1:])
    del counts
    indices = torch.cat(cols) if cols else torch.zeros(0, dtype=torch.int32, device=device)
    return offsets, indices, n, m, planted


def c5_csr(scale: int = 27, edge_factor: int = 14, device="cuda:0"):
    """The scale workload on a device: R-MAT (a,b,c,d)=(.57,.19,.19,.05),
    symmetrised and de-duplicated, planted 50-clique."""
    from . import seed_for
    return rmat_csr(scale, edge_factor, 0.57, 0.19, 0.19, seed_for(5, 0), plants=(50,), device=device)
