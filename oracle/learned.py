"""Reference of the learned vertex ordering -- TEST INFRASTRUCTURE ONLY.

Plain numpy float64 definitions of what the GPU computes for the learned
ordering (an extension of the method: it only reorders the heuristic seeds and
the search roots, it never changes omega):

  features  eight per vertex: log1p(degree), log1p(core), core / K,
            log1p(triangles through v), mean / max / min core of the
            neighbours divided by K, and the fraction of neighbours whose core
            is at least the vertex's own (0 for an isolated vertex); K is the
            largest core number (at least 1).
  mlp       8 -> 64 -> 64 -> 1, ReLU hidden layers, linear output:
            Z1 = X W1 + b1, H1 = relu(Z1), Z2 = H1 W2 + b2, H2 = relu(Z2),
            s = H2 w3 + b3; loss = mean((s - y)^2).
  adam      Kingma and Ba (2015) with bias correction.

The flat parameter layout is shared with the GPU binding: W1 (8x64, row-major,
W1[k, j]), b1 (64), W2 (64x64, W2[k, j]), b2 (64), w3 (64), b3 (1): 4801 floats.
"""
from __future__ import annotations

import numpy as np

F_IN, HID = 8, 64
SIZES = (("W1", (F_IN, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
         ("w3", (HID,)), ("b3", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unflatten(flat):
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(flat[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def flatten(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SIZES])


def init_params(seed=0):
    """He-style initial weights (the same draw feeds both sides as an input)."""
    rng = np.random.Generator(np.random.Philox(seed))
    p = {"W1": rng.normal(0, np.sqrt(2.0 / F_IN), (F_IN, HID)), "b1": np.zeros(HID),
         "W2": rng.normal(0, np.sqrt(2.0 / HID), (HID, HID)), "b2": np.zeros(HID),
         "w3": rng.normal(0, np.sqrt(1.0 / HID), HID), "b3": np.zeros(1)}
    return flatten(p)


def triangles(offsets, indices):
    """Triangles through each vertex: diag(A^3) / 2 (library sparse product)."""
    import scipy.sparse as sp
    n = offsets.shape[0] - 1
    A = sp.csr_matrix((np.ones(indices.shape[0]), indices, offsets), shape=(n, n))
    return np.asarray((A @ A).multiply(A).sum(axis=1)).ravel() / 2.0


def features(offsets, indices, core):
    n = offsets.shape[0] - 1
    core = np.asarray(core, dtype=np.float64)
    K = max(core.max() if n else 1.0, 1.0)
    deg = np.diff(offsets).astype(np.float64)
    tri = triangles(offsets, indices)
    X = np.zeros((n, F_IN))
    X[:, 0] = np.log1p(deg)
    X[:, 1] = np.log1p(core)
    X[:, 2] = core / K
    X[:, 3] = np.log1p(tri)
    for v in range(n):
        nb = indices[offsets[v]:offsets[v + 1]]
        if nb.size == 0:
            continue
        c = core[nb]
        X[v, 4] = c.mean() / K
        X[v, 5] = c.max() / K
        X[v, 6] = c.min() / K
        X[v, 7] = np.count_nonzero(c >= core[v]) / nb.size
    return X


def forward(flat, X):
    p = unflatten(flat)
    Z1 = X @ p["W1"] + p["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ p["W2"] + p["b2"]
    H2 = np.maximum(Z2, 0.0)
    s = H2 @ p["w3"] + p["b3"][0]
    return s, (X, Z1, H1, Z2, H2)


def loss_and_grad(flat, X, y):
    """Mean squared error and its gradient (flat, same layout)."""
    s, (X, Z1, H1, Z2, H2) = forward(flat, X)
    p = unflatten(flat)
    B = X.shape[0]
    r = s - y
    loss = float(np.mean(r * r))
    dS = 2.0 * r / B
    g = {"w3": H2.T @ dS, "b3": np.array([dS.sum()])}
    dZ2 = np.outer(dS, p["w3"]) * (Z2 > 0)
    g["W2"] = H1.T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ p["W2"].T) * (Z1 > 0)
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return loss, flatten(g)


def adam(flat, m, v, grad, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (flat, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v
