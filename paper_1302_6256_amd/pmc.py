"""Python binding of the gfx950 maximum-clique library (``libpmc.so``).

Argument marshalling only: every step runs in the HIP kernels behind the C ABI
declared in ``include/pmc.h``.  Tensors live on the GPU; PyTorch supplies
device memory and the current stream.  There is no CPU fallback: if the
library is missing the import of the binding fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpmc.so")

PMC_OK = 0
PMC_ERR_CAPACITY = 3
PMC_ERR_BUDGET = 6
STATUS = {0: "ok", 1: "invalid argument", 2: "invalid graph", 3: "capacity too small",
          4: "out of memory", 5: "device error", 6: "node budget exhausted"}
PMC_GRAPH_VALIDATE = 1
PMC_ORDER_CORE = 0
PMC_ORDER_SCORE = 1


class PmcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("offsets", ctypes.c_void_p),
                ("offsets_bits", ctypes.c_int32), ("indices", ctypes.c_void_p),
                ("flags", ctypes.c_uint32)]


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("order", ctypes.c_int32),
                ("score", ctypes.c_void_p), ("use_neighborhood_cores", ctypes.c_int32),
                ("rebuild_on_bound_gain", ctypes.c_int32), ("frozen_threshold", ctypes.c_int32),
                ("frozen_bound", ctypes.c_int32), ("skip_heuristic", ctypes.c_int32),
                ("node_budget", ctypes.c_int64), ("root_report", ctypes.c_void_p),
                ("wave_roots", ctypes.c_int32), ("mlp", ctypes.c_void_p),
                ("native_order", ctypes.c_int32), ("tune_table", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("kmax", ctypes.c_int32), ("nrounds", ctypes.c_int32),
                ("heuristic", ctypes.c_int32), ("omega", ctypes.c_int32),
                ("certified", ctypes.c_int32), ("certified_early", ctypes.c_int32),
                ("survivors", ctypes.c_int64), ("oriented_nnz", ctypes.c_int64),
                ("roots", ctypes.c_int64), ("roots_branched", ctypes.c_int64),
                ("nodes", ctypes.c_int64), ("rebuilds", ctypes.c_int32),
                ("search_graph_replays", ctypes.c_int32),
                ("ms_peel", ctypes.c_float), ("ms_rank", ctypes.c_float),
                ("ms_heuristic", ctypes.c_float), ("ms_prune", ctypes.c_float),
                ("ms_queue", ctypes.c_float), ("ms_search", ctypes.c_float),
                ("ms_total", ctypes.c_float),
                ("ms_k_peel", ctypes.c_float), ("ms_k_heuristic", ctypes.c_float),
                ("ms_k_orient", ctypes.c_float), ("ms_k_search", ctypes.c_float),
                ("heuristic_seeds", ctypes.c_int64), ("roots_second_pass", ctypes.c_int64),
                ("ms_sweep", ctypes.c_float), ("learned_used", ctypes.c_int32),
                ("gbps_peel", ctypes.c_float), ("gbps_orient", ctypes.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if not k.startswith("reserved")}


class Batch(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("offsets", ctypes.c_void_p),
                ("offsets_bits", ctypes.c_int32), ("indices", ctypes.c_void_p),
                ("count", ctypes.c_int32), ("vertex_base", ctypes.POINTER(ctypes.c_int64)),
                ("flags", ctypes.c_uint32)]


class Tuning(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("search_blocks_per_cu", ctypes.c_int32 * 7),
                ("heuristic_waves_per_cu", ctypes.c_int32 * 2), ("search_graph", ctypes.c_int32),
                ("heuristic_chunk", ctypes.c_int32 * 2), ("search_split_min", ctypes.c_int32),
                ("search_split_depth", ctypes.c_int32), ("search_sweep_nodes", ctypes.c_int32),
                ("learned_min_open", ctypes.c_int32), ("batch_peel", ctypes.c_int32)]


EXPORTS = ("pmc_core_numbers", "pmc_core_numbers_noalloc", "pmc_core_numbers_batch", "pmc_heuristic", "pmc_prune_orient", "pmc_max_clique",
           "pmc_max_clique_batch", "pmc_max_clique_graphs", "pmc_default_options", "pmc_status_string", "pmc_last_error",
           "pmc_vertex_features", "pmc_mlp_forward", "pmc_mlp_train_step", "pmc_get_tuning",
           "pmc_set_tuning", "pmc_clique_order", "pmc_strong_reachability")
MLP_PARAMS = 4801

_lib = None


def load():
    """Load libpmc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I32, I64 = ctypes.c_int32, ctypes.c_int64
    GP = ctypes.POINTER(Graph)
    OP = ctypes.POINTER(Options)
    lib.pmc_core_numbers.restype = ctypes.c_int
    lib.pmc_core_numbers.argtypes = [GP, P, P, P, P, ctypes.POINTER(I32), ctypes.POINTER(I32), P]
    lib.pmc_core_numbers_noalloc.restype = ctypes.c_int
    lib.pmc_core_numbers_noalloc.argtypes = lib.pmc_core_numbers.argtypes
    lib.pmc_core_numbers_batch.restype = ctypes.c_int
    lib.pmc_core_numbers_batch.argtypes = [ctypes.POINTER(Batch), P, P, P, P, ctypes.POINTER(I32),
                                           ctypes.POINTER(I32), P]
    lib.pmc_heuristic.restype = ctypes.c_int
    lib.pmc_heuristic.argtypes = [GP, P, P, P, OP, P, I32, ctypes.POINTER(I32), P]
    lib.pmc_prune_orient.restype = ctypes.c_int
    lib.pmc_prune_orient.argtypes = [GP, P, P, P, I32, P, P, I64, ctypes.POINTER(I32),
                                     ctypes.POINTER(I64), P]
    lib.pmc_max_clique.restype = ctypes.c_int
    lib.pmc_max_clique.argtypes = [GP, OP, P, I32, ctypes.POINTER(I32), ctypes.POINTER(Stats), P]
    lib.pmc_max_clique_graphs.restype = ctypes.c_int
    lib.pmc_max_clique_graphs.argtypes = [ctypes.POINTER(Graph), ctypes.c_int32, OP, P,
                                          ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(Stats), P]
    lib.pmc_max_clique_batch.restype = ctypes.c_int
    lib.pmc_max_clique_batch.argtypes = [ctypes.POINTER(Batch), OP, P, ctypes.POINTER(I32),
                                         ctypes.POINTER(Stats), P]
    FP = ctypes.c_void_p
    lib.pmc_vertex_features.restype = ctypes.c_int
    lib.pmc_vertex_features.argtypes = [GP, FP, P]
    lib.pmc_clique_order.restype = ctypes.c_int
    lib.pmc_clique_order.argtypes = [GP, P, P, ctypes.POINTER(I64), P]
    lib.pmc_strong_reachability.restype = ctypes.c_int
    lib.pmc_strong_reachability.argtypes = [I64, I64, P, P, P, P, I64, ctypes.POINTER(I64), P]
    lib.pmc_mlp_forward.restype = ctypes.c_int
    lib.pmc_mlp_forward.argtypes = [FP, FP, I64, FP, P]
    lib.pmc_mlp_train_step.restype = ctypes.c_int
    lib.pmc_mlp_train_step.argtypes = [FP, FP, FP, I64, ctypes.c_float, FP, FP, I64,
                                       ctypes.POINTER(ctypes.c_float), FP, P]
    lib.pmc_get_tuning.restype = ctypes.c_int
    lib.pmc_get_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.pmc_set_tuning.restype = ctypes.c_int
    lib.pmc_set_tuning.argtypes = [ctypes.POINTER(Tuning)]
    lib.pmc_default_options.restype = None
    lib.pmc_default_options.argtypes = [OP]
    lib.pmc_status_string.restype = ctypes.c_char_p
    lib.pmc_status_string.argtypes = [ctypes.c_int]
    lib.pmc_last_error.restype = ctypes.c_char_p
    lib.pmc_last_error.argtypes = []
    _lib = lib
    _apply_tuning_table()
    return lib


def _check(status):
    if status != PMC_OK:
        raise PmcError(status, load().pmc_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _graph(offsets: torch.Tensor, indices: torch.Tensor, validate: bool):
    if not (offsets.is_cuda and indices.is_cuda):
        raise ValueError("offsets and indices must be device tensors")
    if offsets.dtype not in (torch.int32, torch.int64) or indices.dtype != torch.int32:
        raise ValueError("offsets must be int32/int64 and indices int32")
    if not (offsets.is_contiguous() and indices.is_contiguous()):
        raise ValueError("tensors must be contiguous")
    g = Graph()
    g.n = offsets.numel() - 1
    g.nnz = indices.numel()
    g.offsets = offsets.data_ptr()
    g.offsets_bits = 32 if offsets.dtype == torch.int32 else 64
    g.indices = indices.data_ptr() if indices.numel() else None
    g.flags = PMC_GRAPH_VALIDATE if validate else 0
    return g


def default_options() -> Options:
    o = Options()
    load().pmc_default_options(ctypes.byref(o))
    return o


def _options(**kw) -> Options:
    o = default_options()
    score = kw.pop("score", None)
    report = kw.pop("root_report", None)
    mlp = kw.pop("mlp", None)
    table = kw.pop("tune_table", None)
    for k, v in kw.items():
        if v is None:
            continue
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, int(v))
    if score is not None:
        o.order = PMC_ORDER_SCORE
        o.score = score.data_ptr()
    if mlp is not None:
        o.mlp = mlp.data_ptr()
    if report is not None:
        o.root_report = report.data_ptr()
    if table is not None:
        o._table = _tuning_struct(table)  # kept alive with the options
        o.tune_table = ctypes.addressof(o._table)
    return o


def core_numbers(offsets, indices, validate=False, noalloc=False):
    """k-core peel: (core, round, rank, order) int32 device tensors, kmax, nrounds.
    ``noalloc`` calls the allocation-free entry point (the outputs are still
    allocated here, by the caller of the library)."""
    n = offsets.numel() - 1
    dev = offsets.device
    core = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    rnd = torch.empty_like(core)
    rank = torch.empty_like(core)
    order = torch.empty_like(core)
    km, nr = ctypes.c_int32(0), ctypes.c_int32(0)
    g = _graph(offsets, indices, validate)
    fn = load().pmc_core_numbers_noalloc if noalloc else load().pmc_core_numbers
    _check(fn(ctypes.byref(g), _ptr(core), _ptr(rnd), _ptr(rank), _ptr(order), ctypes.byref(km),
              ctypes.byref(nr), _stream()))
    return core[:n], rnd[:n], rank[:n], order[:n], km.value, nr.value


def heuristic(offsets, indices, core=None, rank=None, order=None, frozen_threshold=-1, score=None,
              capacity=None, validate=False):
    """Alg. 1 heuristic clique: int32 device tensor (sorted ids)."""
    n = offsets.numel() - 1
    if capacity is None:
        capacity = max(n, 1)
    out = torch.empty(max(capacity, 1), dtype=torch.int32, device=offsets.device)
    size = ctypes.c_int32(0)
    o = _options(frozen_threshold=frozen_threshold, score=score)
    g = _graph(offsets, indices, validate)
    _check(load().pmc_heuristic(ctypes.byref(g), _ptr(core), _ptr(rank), _ptr(order),
                                ctypes.byref(o), _ptr(out), capacity, ctypes.byref(size),
                                _stream()))
    return out[:size.value]


def prune_orient(offsets, indices, core, rank, order, bound, validate=False):
    """Pruned oriented graph: (r0, poff int64, padj int32) device tensors."""
    n = offsets.numel() - 1
    cap = indices.numel() // 2 + 1
    poff = torch.empty(n + 1, dtype=torch.int64, device=offsets.device)
    padj = torch.empty(cap, dtype=torch.int32, device=offsets.device)
    r0, nnz = ctypes.c_int32(0), ctypes.c_int64(0)
    g = _graph(offsets, indices, validate)
    _check(load().pmc_prune_orient(ctypes.byref(g), _ptr(core), _ptr(rank), _ptr(order), bound,
                                   _ptr(poff), _ptr(padj), cap, ctypes.byref(r0),
                                   ctypes.byref(nnz), _stream()))
    return r0.value, poff[:n - r0.value + 1], padj[:nnz.value]


def max_clique(offsets, indices, capacity=None, validate=False, allow_budget=False, **options):
    """Alg. 2 exact maximum clique: (omega, clique int32 device tensor, stats dict).

    options: use_neighborhood_cores, rebuild_on_bound_gain, frozen_threshold,
    frozen_bound, skip_heuristic, node_budget, score (float32 device tensor),
    root_report (int32 device tensor of 4n entries), wave_roots.
    """
    n = offsets.numel() - 1
    if capacity is None:
        capacity = max(n, 1)
    out = torch.empty(max(capacity, 1), dtype=torch.int32, device=offsets.device)
    om = ctypes.c_int32(0)
    st = Stats()
    o = _options(**options)
    g = _graph(offsets, indices, validate)
    s = load().pmc_max_clique(ctypes.byref(g), ctypes.byref(o), _ptr(out), capacity,
                              ctypes.byref(om), ctypes.byref(st), _stream())
    if not (allow_budget and s == PMC_ERR_BUDGET):
        _check(s)
    return om.value, out[:om.value], st.as_dict()


def _batch(offsets, indices, vertex_base, validate):
    import numpy as np
    vb = np.ascontiguousarray(np.asarray(vertex_base, dtype=np.int64))
    g = _graph(offsets, indices, validate)
    b = Batch()
    b.n, b.nnz, b.offsets, b.offsets_bits, b.indices = g.n, g.nnz, g.offsets, g.offsets_bits, \
        g.indices
    b.count = vb.shape[0] - 1
    b.vertex_base = vb.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    b.flags = g.flags
    return b, vb


def core_numbers_batch(offsets, indices, vertex_base, validate=False):
    """Every graph of a batch peeled on its own: (core, round, rank, order)
    int32 device tensors over the union (rounds per graph; rank over the
    union in (round, id) order), and per-graph lists kmax, nrounds."""
    b, vb = _batch(offsets, indices, vertex_base, validate)
    n, count = int(b.n), int(b.count)
    dev = offsets.device
    core = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    rnd, rank, order = torch.empty_like(core), torch.empty_like(core), torch.empty_like(core)
    km = (ctypes.c_int32 * count)()
    nr = (ctypes.c_int32 * count)()
    _check(load().pmc_core_numbers_batch(ctypes.byref(b), _ptr(core), _ptr(rnd), _ptr(rank),
                                         _ptr(order), km, nr, _stream()))
    del vb
    return core[:n], rnd[:n], rank[:n], order[:n], list(km), list(nr)


def max_clique_batch(offsets, indices, vertex_base, validate=False, allow_budget=False, **options):
    """Exact maximum clique of every graph of a batch (the disjoint union in one
    CSR; graph g owns ids [vertex_base[g], vertex_base[g+1])).

    Returns (omegas list, cliques int32 device tensor of n entries -- graph g's
    clique at [vertex_base[g], vertex_base[g] + omegas[g]) -- and stats dict).
    """
    import numpy as np
    vb = np.ascontiguousarray(np.asarray(vertex_base, dtype=np.int64))
    count = vb.shape[0] - 1
    g = _graph(offsets, indices, validate)
    b = Batch()
    b.n, b.nnz, b.offsets, b.offsets_bits, b.indices = g.n, g.nnz, g.offsets, g.offsets_bits, \
        g.indices
    b.count = count
    b.vertex_base = vb.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    b.flags = g.flags
    out = torch.empty(max(g.n, 1), dtype=torch.int32, device=offsets.device)
    om = (ctypes.c_int32 * count)()
    st = Stats()
    o = _options(**options)
    s = load().pmc_max_clique_batch(ctypes.byref(b), ctypes.byref(o), _ptr(out), om,
                                    ctypes.byref(st), _stream())
    if not (allow_budget and s == PMC_ERR_BUDGET):
        _check(s)
    return list(om), out, st.as_dict()


def max_clique_graphs(graphs, validate=False, allow_budget=False, **options):
    """Exact maximum clique of every graph of a list of separate device CSRs
    [(offsets, indices), ...] in one call (pmc_max_clique_graphs).  Returns
    (omegas list, list of per-graph clique tensors in the graphs' own ids,
    stats dict)."""
    import numpy as np
    count = len(graphs)
    arr = (Graph * count)()
    keep = []
    for i, (off, idx) in enumerate(graphs):
        arr[i] = _graph(off, idx, validate)
        keep.append((off, idx))
    sizes = [max(int(off.numel()) - 1, 0) for off, _ in graphs]
    coff = np.zeros(count + 1, dtype=np.int64)
    coff[1:] = np.cumsum(sizes)
    dev = graphs[0][0].device
    out = torch.empty(max(int(coff[-1]), 1), dtype=torch.int32, device=dev)
    om = (ctypes.c_int32 * count)()
    st = Stats()
    o = _options(**options)
    s = load().pmc_max_clique_graphs(arr, count, ctypes.byref(o), _ptr(out),
                                     coff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), om,
                                     ctypes.byref(st), _stream())
    if not (allow_budget and s == PMC_ERR_BUDGET):
        _check(s)
    oms = list(om)
    return oms, [out[coff[i]:coff[i] + oms[i]] for i in range(count)], st.as_dict()


def strong_reachability(n, src, dst):
    """Strong-reachability graph (Sec. 6.1) of the temporal edges src[e] ->
    dst[e] (int32 device tensors, time order): (offsets int64, indices int32)
    device tensors, ready for max_clique."""
    m = src.numel()
    dev = src.device if m else torch.device("cuda:0")
    offsets = torch.empty(n + 1, dtype=torch.int64, device=dev)
    nnz = ctypes.c_int64(0)
    s = load().pmc_strong_reachability(n, m, _ptr(src) if m else None, _ptr(dst) if m else None,
                                       _ptr(offsets), None, 0, ctypes.byref(nnz), _stream())
    if s not in (0, PMC_ERR_CAPACITY):
        _check(s)
    indices = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=dev)
    _check(load().pmc_strong_reachability(n, m, _ptr(src) if m else None,
                                          _ptr(dst) if m else None, _ptr(offsets), _ptr(indices),
                                          nnz.value, ctypes.byref(nnz), _stream()))
    return offsets, indices[:nnz.value]


def temporal_strong_component(n, src, dst):
    """Largest temporal strong component (Sec. 6.1): (size, vertex ids)."""
    off, idx = strong_reachability(n, src, dst)
    w, cl, _ = max_clique(off, idx)
    return w, cl


def clique_order(offsets, indices, validate=False):
    """Clique-peeling compression order (Sec. 6.2): (order int32 device tensor of
    n vertex ids, block int64 device tensor of first positions, nblocks + 1
    entries)."""
    n = offsets.numel() - 1
    dev = offsets.device
    order = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    block = torch.empty(n + 1, dtype=torch.int64, device=dev)
    nb = ctypes.c_int64(0)
    g = _graph(offsets, indices, validate)
    _check(load().pmc_clique_order(ctypes.byref(g), _ptr(order), _ptr(block), ctypes.byref(nb),
                                   _stream()))
    return order[:n], block[:nb.value + 1]


def vertex_features(offsets, indices, validate=False):
    """Eight features per vertex: float32 device tensor (n, 8)."""
    n = offsets.numel() - 1
    feat = torch.empty((max(n, 1), 8), dtype=torch.float32, device=offsets.device)
    g = _graph(offsets, indices, validate)
    _check(load().pmc_vertex_features(ctypes.byref(g), _ptr(feat), _stream()))
    return feat[:n]


def mlp_forward(params, features):
    """Scores of the 8->64->64->1 MLP (bf16 MFMA, fp32 accumulation)."""
    n = features.shape[0]
    score = torch.empty(max(n, 1), dtype=torch.float32, device=features.device)
    _check(load().pmc_mlp_forward(_ptr(params), _ptr(features), n, _ptr(score), _stream()))
    return score[:n]


def mlp_train_step(params, adam_m, adam_v, step, lr, features, label, want_grad=False):
    """One full-batch Adam step in place; returns (loss before the step, grad or None)."""
    n = features.shape[0]
    loss = ctypes.c_float(0.0)
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=features.device) if want_grad \
        else None
    _check(load().pmc_mlp_train_step(_ptr(params), _ptr(adam_m), _ptr(adam_v), step, lr,
                                     _ptr(features), _ptr(label), n, ctypes.byref(loss),
                                     _ptr(grad), _stream()))
    return loss.value, grad


TUNING_TABLE = os.path.join(_PKG, "tuning.json")


def get_tuning() -> dict:
    t = Tuning()
    _check(load().pmc_get_tuning(ctypes.byref(t)))
    return {"search_blocks_per_cu": list(t.search_blocks_per_cu),
            "heuristic_waves_per_cu": list(t.heuristic_waves_per_cu), "search_graph": t.search_graph,
            "heuristic_chunk": list(t.heuristic_chunk), "search_split_min": t.search_split_min,
            "search_split_depth": t.search_split_depth,
            "search_sweep_nodes": t.search_sweep_nodes, "learned_min_open": t.learned_min_open,
            "batch_peel": t.batch_peel}


def set_tuning(cfg: dict | None):
    """Apply launch parameters (None restores the defaults)."""
    if cfg is None:
        _check(load().pmc_set_tuning(None))
        return
    _check(load().pmc_set_tuning(ctypes.byref(_tuning_struct(cfg))))


def _tuning_struct(cfg: dict) -> Tuning:
    t = Tuning()
    t.struct_size = ctypes.sizeof(Tuning)
    for i, v in enumerate(cfg.get("search_blocks_per_cu", [0] * 7)):
        t.search_blocks_per_cu[i] = int(v)
    for i, v in enumerate(cfg.get("heuristic_waves_per_cu", [0, 0])):
        t.heuristic_waves_per_cu[i] = int(v)
    t.search_graph = int(cfg.get("search_graph", 0))
    for i, v in enumerate(cfg.get("heuristic_chunk", [0, 0])):
        t.heuristic_chunk[i] = int(v)
    t.search_split_min = int(cfg.get("search_split_min", 0))
    t.search_split_depth = int(cfg.get("search_split_depth", 0))
    t.search_sweep_nodes = int(cfg.get("search_sweep_nodes", 0))
    t.learned_min_open = int(cfg.get("learned_min_open", 0))
    t.batch_peel = int(cfg.get("batch_peel", 0))
    return t


def _apply_tuning_table():
    """Apply the autotuner's table when it was made on this device model."""
    import json
    if not os.path.exists(TUNING_TABLE) or os.environ.get("PMC_NO_TUNING"):
        return
    try:
        with open(TUNING_TABLE) as f:
            tab = json.load(f)
        if torch.cuda.is_available() and tab.get("device") == torch.cuda.get_device_name(0):
            set_tuning(tab["best"])
    except (OSError, ValueError, KeyError):
        pass
