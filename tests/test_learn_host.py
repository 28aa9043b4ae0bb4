"""Host logic of the learned ordering: the training target (each vertex's
percentile in its graph's omega_v order, ties sharing their mean position),
checked against its definition written out with sorting."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def reference(w):
    w = np.asarray(w, dtype=np.int64)
    n = w.size
    if n < 2:
        return np.zeros(n)
    order = np.argsort(w, kind="stable")
    pos = np.empty(n)
    pos[order] = np.arange(n)
    out = np.empty(n)
    for v in np.unique(w):
        sel = w == v
        out[sel] = pos[sel].mean()
    return out / (n - 1)


@pytest.mark.parametrize("w", [[3, 1, 1, 5, 3, 0], [7], [], [2, 2, 2, 2], [0, 1, 2, 3, 4],
                               list(np.random.default_rng(3).integers(0, 40, size=500))])
def test_percentile_target(w):
    from paper_1302_6256_amd import learn
    got = learn.percentile(np.asarray(w, dtype=np.float32))
    assert got.shape == (len(w),)
    assert np.allclose(got, reference(w), atol=1e-6)
    if len(w) >= 2:
        assert got.min() >= 0.0 and got.max() <= 1.0


def test_percentile_clamps_unlabelled():
    """Vertices without a label (-1) rank with omega_v = 0."""
    from paper_1302_6256_amd import learn
    got = learn.percentile(np.array([-1.0, 0.0, 2.0]))
    assert np.allclose(got, reference([0, 0, 2]))
