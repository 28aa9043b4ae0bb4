// pmc_capi.hip -- the C ABI (include/pmc.h): argument checks, the pipeline of
// MaxClique (Alg. 2 of the paper) on the device, error conversion.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <exception>
#include <string>
#include <vector>

#include "common.h"
#include "graph.h"
#include "pmc.h"
#include "search.h"

namespace pmc {
void max_degree(const GraphView &g, int32_t *out, hipStream_t s);
}

using namespace pmc;

namespace {

thread_local std::string g_last_error;

pmc_status fail(int st, const std::string &m) {
  g_last_error = m;
  return (pmc_status)st;
}

GraphView make_view(const pmc_graph *g) {
  if (!g) throw Error{PMC_ERR_INVALID_ARG, "graph is NULL"};
  if (g->n < 0 || g->nnz < 0) throw Error{PMC_ERR_INVALID_ARG, "negative n or nnz"};
  if (g->n >= (int64_t)1 << 31) throw Error{PMC_ERR_INVALID_ARG, "n must be < 2^31"};
  if (g->offsets_bits != 32 && g->offsets_bits != 64)
    throw Error{PMC_ERR_INVALID_ARG, "offsets_bits must be 32 or 64"};
  if (g->offsets_bits == 32 && g->nnz >= (int64_t)1 << 31)
    throw Error{PMC_ERR_INVALID_ARG, "nnz does not fit 32-bit offsets"};
  if (!g->offsets) throw Error{PMC_ERR_INVALID_ARG, "offsets is NULL"};
  if (g->nnz > 0 && !g->indices) throw Error{PMC_ERR_INVALID_ARG, "indices is NULL"};
  GraphView v;
  v.n = g->n;
  v.nnz = g->nnz;
  v.off = g->offsets;
  v.bits = g->offsets_bits;
  v.idx = g->indices;
  return v;
}

void maybe_validate(const pmc_graph *g, const GraphView &v, Scratch &sc) {
  if (!(g->flags & PMC_GRAPH_VALIDATE) || v.n == 0) return;
  int code = validate_graph(v, sc);
  static const char *what[] = {"", "offsets are not a valid prefix array", "vertex id out of range",
                               "self-loop", "row not strictly increasing (unsorted or duplicate)",
                               "adjacency not symmetric"};
  if (code) throw Error{PMC_ERR_INVALID_GRAPH, std::string("invalid graph: ") + what[code]};
}

pmc_options defaults() {
  pmc_options o;
  std::memset(&o, 0, sizeof(o));
  o.struct_size = sizeof(pmc_options);
  o.order = PMC_ORDER_CORE;
  o.use_neighborhood_cores = 1;
  o.rebuild_on_bound_gain = 1;
  o.frozen_threshold = -1;
  o.frozen_bound = -1;
  return o;
}

pmc_options read_options(const pmc_options *opt) {
  pmc_options o = defaults();
  if (!opt) return o;
  if (opt->struct_size < sizeof(pmc_options))
    throw Error{PMC_ERR_INVALID_ARG, "pmc_options.struct_size too small"};
  o = *opt;
  if (o.order != PMC_ORDER_CORE && o.order != PMC_ORDER_SCORE)
    throw Error{PMC_ERR_INVALID_ARG, "unknown order"};
  if (o.order == PMC_ORDER_SCORE && !o.score)
    throw Error{PMC_ERR_INVALID_ARG, "PMC_ORDER_SCORE needs score"};
  if (o.node_budget < 0) throw Error{PMC_ERR_INVALID_ARG, "negative node_budget"};
  return o;
}

template <typename F>
pmc_status guarded(F &&f) {
  try {
    f();
    return PMC_OK;
  } catch (const Error &e) {
    (void)hipGetLastError();
    return fail(e.status, e.msg);
  } catch (const std::exception &e) {
    return fail(PMC_ERR_DEVICE, e.what());
  } catch (...) {
    return fail(PMC_ERR_DEVICE, "unknown failure");
  }
}

struct Timer {
  hipStream_t s;
  hipEvent_t e;
  explicit Timer(hipStream_t st) : s(st) {
    PMC_HIP(hipEventCreate(&e));
    PMC_HIP(hipEventRecord(e, s));
  }
  ~Timer() { (void)hipEventDestroy(e); }
  float lap() {  // ms since the last lap (synchronises)
    hipEvent_t e2;
    PMC_HIP(hipEventCreate(&e2));
    PMC_HIP(hipEventRecord(e2, s));
    PMC_HIP(hipEventSynchronize(e2));
    float ms = 0;
    PMC_HIP(hipEventElapsedTime(&ms, e, e2));
    (void)hipEventDestroy(e);
    e = e2;
    return ms;
  }
};

// Seeds by decreasing score, ties by decreasing rank; non-finite scores last.
__global__ void k_seed_keys(int n, const int32_t *order, const float *score, uint32_t *keys,
                            int32_t *vals) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int v = order[n - 1 - p];
  float f = score[v];
  uint32_t k;
  if (!isfinite(f)) {
    k = 0xffffffffu;
  } else {
    uint32_t b = __float_as_uint(f);
    uint32_t asc = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    k = ~asc;
    if (k == 0xffffffffu) k = 0xfffffffeu;
  }
  keys[p] = k;
  vals[p] = v;
}

__global__ void k_state_init(CliqueState *st, int bound) {
  st->bound = bound;
  st->err = 0;
  st->best_packed = 0;
  st->nodes = 0;
  st->roots_branched = 0;
  st->seed_next = 0;
  st->budget_hit = 0;
  st->seeds_done = 0;
}

struct Pipeline {
  GraphView g;
  Scratch &sc;
  int32_t *core = nullptr, *rnd = nullptr, *rank = nullptr, *order = nullptr;
  int32_t kmax = 0, nrounds = 0;
  Pipeline(const GraphView &gv, Scratch &s) : g(gv), sc(s) {}

  PeelResult peel(int32_t *ucore, int32_t *urnd) {
    core = ucore ? ucore : sc.get<int32_t>(g.n);
    rnd = urnd ? urnd : sc.get<int32_t>(g.n);
    PeelResult pr = run_peel(g, core, rnd, sc);
    kmax = pr.kmax;
    nrounds = pr.nrounds;
    return pr;
  }
  void ranks(int32_t *urank, int32_t *uorder) {
    rank = urank ? urank : sc.get<int32_t>(g.n);
    order = uorder ? uorder : sc.get<int32_t>(g.n);
    run_rank(g.n, rnd, nrounds, rank, order, sc);
  }
  void cores(int32_t *ucore, int32_t *urnd, int32_t *urank, int32_t *uorder, bool need_rank) {
    peel(ucore, urnd);
    if (need_rank) ranks(urank, uorder);
  }
};

void copy_sorted_clique(const int32_t *slot, int size, int32_t *dst, hipStream_t s) {
  std::vector<int32_t> h(size);
  if (size) {
    PMC_HIP(hipMemcpyAsync(h.data(), slot, sizeof(int32_t) * size, hipMemcpyDeviceToHost, s));
    PMC_HIP(hipStreamSynchronize(s));
  }
  std::sort(h.begin(), h.end());
  if (size) {
    PMC_HIP(hipMemcpyAsync(dst, h.data(), sizeof(int32_t) * size, hipMemcpyHostToDevice, s));
    PMC_HIP(hipStreamSynchronize(s));
  }
}

}  // namespace

extern "C" {

void pmc_default_options(pmc_options *opt) {
  if (opt) *opt = defaults();
}

const char *pmc_status_string(pmc_status s) {
  switch (s) {
    case PMC_OK: return "ok";
    case PMC_ERR_INVALID_ARG: return "invalid argument";
    case PMC_ERR_INVALID_GRAPH: return "invalid graph";
    case PMC_ERR_CAPACITY: return "capacity too small";
    case PMC_ERR_OUT_OF_MEMORY: return "out of memory";
    case PMC_ERR_DEVICE: return "device error";
    case PMC_ERR_BUDGET: return "node budget exhausted";
  }
  return "unknown status";
}

const char *pmc_last_error(void) { return g_last_error.c_str(); }

pmc_status pmc_core_numbers(const pmc_graph *g, int32_t *core, int32_t *round, int32_t *rank,
                            int32_t *order, int32_t *kmax, int32_t *nrounds, void *stream) {
  return guarded([&] {
    GraphView v = make_view(g);
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(s);
    maybe_validate(g, v, sc);
    if (v.n == 0) {
      if (kmax) *kmax = 0;
      if (nrounds) *nrounds = 0;
      return;
    }
    Pipeline p(v, sc);
    p.cores(core, round, rank, order, rank || order);
    PMC_HIP(hipStreamSynchronize(s));
    if (kmax) *kmax = p.kmax;
    if (nrounds) *nrounds = p.nrounds;
  });
}

pmc_status pmc_heuristic(const pmc_graph *g, const int32_t *core, const int32_t *rank,
                         const int32_t *order, const pmc_options *opt, int32_t *clique,
                         int32_t capacity, int32_t *size, void *stream) {
  return guarded([&] {
    GraphView v = make_view(g);
    pmc_options o = read_options(opt);
    if (!clique || !size) throw Error{PMC_ERR_INVALID_ARG, "clique and size are required"};
    if ((core == nullptr) != (rank == nullptr) || (core == nullptr) != (order == nullptr))
      throw Error{PMC_ERR_INVALID_ARG, "core, rank and order must all be given or all be NULL"};
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(s);
    maybe_validate(g, v, sc);
    if (v.n == 0) {
      *size = 0;
      return;
    }
    Pipeline p(v, sc);
    int32_t km = 0;
    if (!core) {
      p.cores(nullptr, nullptr, nullptr, nullptr, true);
      km = p.kmax;
    } else {
      p.core = const_cast<int32_t *>(core);
      p.rank = const_cast<int32_t *>(rank);
      p.order = const_cast<int32_t *>(order);
      // K(G) is the core of the last vertex in rank order
      int32_t last = 0;
      PMC_HIP(hipMemcpyAsync(&last, order + (v.n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
      PMC_HIP(hipStreamSynchronize(s));
      if (last < 0 || last >= v.n) throw Error{PMC_ERR_INVALID_ARG, "order is not a permutation"};
      PMC_HIP(hipMemcpyAsync(&km, core + last, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      PMC_HIP(hipStreamSynchronize(s));
    }
    CliqueState *st = sc.get<CliqueState>(1);
    k_state_init<<<1, 1, 0, s>>>(st, 0);
    int32_t *slots = sc.get<int32_t>((size_t)(km + 2) * (km + 1));
    int32_t *seeds = nullptr;
    if (o.order == PMC_ORDER_SCORE) {
      uint32_t *k1 = sc.get<uint32_t>(v.n), *k2 = sc.get<uint32_t>(v.n);
      int32_t *v1 = sc.get<int32_t>(v.n);
      seeds = sc.get<int32_t>(v.n);
      k_seed_keys<<<(int)((v.n + 255) / 256), 256, 0, s>>>((int)v.n, p.order, o.score, k1, v1);
      radix_sort_pairs(k1, v1, k2, seeds, v.n, 32, sc);
    }
    run_heuristic(v, p.core, p.rank, p.order, seeds, km, o.frozen_threshold, st, slots, sc);
    CliqueState h;
    PMC_HIP(hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, s));
    PMC_HIP(hipStreamSynchronize(s));
    *size = h.bound;
    if (capacity < h.bound)
      throw Error{PMC_ERR_CAPACITY, "clique capacity " + std::to_string(capacity) + " < " +
                                        std::to_string(h.bound)};
    copy_sorted_clique(slots + (size_t)h.bound * (km + 1), h.bound, clique, s);
  });
}

pmc_status pmc_prune_orient(const pmc_graph *g, const int32_t *core, const int32_t *rank,
                            const int32_t *order, int32_t bound, int64_t *poff, int32_t *padj,
                            int64_t capacity, int32_t *r0, int64_t *out_nnz, void *stream) {
  return guarded([&] {
    GraphView v = make_view(g);
    if (!core || !rank || !order || !poff || (!padj && capacity > 0) || !r0 || !out_nnz)
      throw Error{PMC_ERR_INVALID_ARG, "missing argument"};
    if (bound < 0 || capacity < 0) throw Error{PMC_ERR_INVALID_ARG, "negative bound or capacity"};
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(s);
    maybe_validate(g, v, sc);
    if (v.n == 0) {
      PMC_HIP(hipMemsetAsync(poff, 0, sizeof(int64_t), s));
      PMC_HIP(hipStreamSynchronize(s));
      *r0 = 0;
      *out_nnz = 0;
      return;
    }
    // r0 = number of vertices with core < bound (ranks are nondecreasing in core)
    int32_t last = 0, km = 0;
    PMC_HIP(hipMemcpyAsync(&last, order + (v.n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PMC_HIP(hipStreamSynchronize(s));
    PMC_HIP(hipMemcpyAsync(&km, core + last, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PMC_HIP(hipStreamSynchronize(s));
    int32_t *r0tab = sc.get<int32_t>(km + 2);
    run_r0_table(v.n, core, order, km, r0tab, sc);
    int32_t r = 0;
    int c = std::min(bound, km + 1);
    PMC_HIP(hipMemcpyAsync(&r, r0tab + c, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PMC_HIP(hipStreamSynchronize(s));
    if (bound > km + 1) r = (int32_t)v.n;
    *r0 = r;
    *out_nnz = run_prune_orient(v, rank, order, r, poff, padj, capacity, km, sc);
    PMC_HIP(hipStreamSynchronize(s));
  });
}

pmc_status pmc_max_clique(const pmc_graph *g, const pmc_options *opt, int32_t *clique,
                          int32_t capacity, int32_t *omega, pmc_stats *stats, void *stream) {
  pmc_status budget_status = PMC_OK;
  pmc_status st_ret = guarded([&] {
    auto t_start = std::chrono::steady_clock::now();
    GraphView v = make_view(g);
    pmc_options o = read_options(opt);
    if (!omega) throw Error{PMC_ERR_INVALID_ARG, "omega is required"};
    if (!clique && capacity > 0) throw Error{PMC_ERR_INVALID_ARG, "clique is NULL"};
    pmc_stats S;
    std::memset(&S, 0, sizeof(S));
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(s);
    maybe_validate(g, v, sc);
    if (v.n == 0) {
      *omega = 0;
      S.certified = 1;
      if (stats) *stats = S;
      return;
    }
    Timer tm(s);
    Pipeline p(v, sc);
    PeelResult pr0 = p.peel(nullptr, nullptr);
    S.ms_k_peel = pr0.ms;
    S.ms_peel = tm.lap();
    p.ranks(nullptr, nullptr);
    S.ms_rank = tm.lap();
    S.kmax = p.kmax;
    S.nrounds = p.nrounds;
    const int km = p.kmax;
    const int stride = km + 1;
    CliqueState *st = sc.get<CliqueState>(1);
    int32_t *slots = sc.get<int32_t>((size_t)(km + 2) * stride);
    int32_t *r0tab = sc.get<int32_t>(km + 2);
    run_r0_table(v.n, p.core, p.order, km, r0tab, sc);
    const bool frozen = o.frozen_bound >= 0;
    int b0 = 0;
    k_state_init<<<1, 1, 0, s>>>(st, 0);
    PMC_HIP(hipGetLastError());
    if (frozen) {
      b0 = o.frozen_bound;
    } else if (!o.skip_heuristic) {
      int32_t *seeds = nullptr;
      if (o.order == PMC_ORDER_SCORE) {
        uint32_t *k1 = sc.get<uint32_t>(v.n), *k2 = sc.get<uint32_t>(v.n);
        int32_t *v1 = sc.get<int32_t>(v.n);
        seeds = sc.get<int32_t>(v.n);
        k_seed_keys<<<(int)((v.n + 255) / 256), 256, 0, s>>>((int)v.n, p.order, o.score, k1, v1);
        radix_sort_pairs(k1, v1, k2, seeds, v.n, 32, sc);
      }
      S.ms_k_heuristic =
          run_heuristic(v, p.core, p.rank, p.order, seeds, km, o.frozen_threshold, st, slots, sc);
      CliqueState hs;
      PMC_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
      PMC_HIP(hipStreamSynchronize(s));
      b0 = hs.bound;
      S.heuristic_seeds = (int64_t)hs.seeds_done;
    }
    S.ms_heuristic = tm.lap();
    S.heuristic = frozen ? 0 : b0;
    std::vector<int32_t> r0h(km + 2);
    PMC_HIP(hipMemcpyAsync(r0h.data(), r0tab, sizeof(int32_t) * (km + 2), hipMemcpyDeviceToHost, s));
    PMC_HIP(hipStreamSynchronize(s));
    int omega_v = b0;
    if (!frozen && b0 == km + 1) {
      S.certified_early = 1;  // Fact 1: nothing larger than K(G) + 1 exists
    } else {
      int r0 = b0 > km + 1 ? (int)v.n : r0h[b0];
      int nn = (int)(v.n - r0);
      S.survivors = nn;
      int64_t cap = v.nnz / 2 + 1;
      int64_t *poff = sc.get<int64_t>((size_t)nn + 1);
      int32_t *padj = sc.get<int32_t>((size_t)cap);
      int64_t onnz =
          run_prune_orient(v, p.rank, p.order, r0, poff, padj, cap, km, sc, &S.ms_k_orient);
      S.oriented_nnz = onnz;
      S.ms_prune = tm.lap();
      int32_t *queue = sc.get<int32_t>((size_t)std::max(nn, 1));
      QueueResult q = run_queue(nn, r0, poff, p.order, frozen ? 0 : b0,
                                o.order == PMC_ORDER_SCORE ? o.score : nullptr, queue, sc);
      S.roots = q.total;
      S.ms_queue = tm.lap();
      if (q.count[SEARCH_CLASSES] > 0)
        throw Error{PMC_ERR_CAPACITY, "a subproblem exceeds 4096 vertices"};
      SearchArgs a;
      a.nn = nn;
      a.r0 = r0;
      a.poff = poff;
      a.padj = padj;
      a.r0tab = r0tab;
      a.kmax = km;
      a.order = p.order;
      a.st = st;
      a.slots = slots;
      a.slot_stride = stride;
      a.frozen_bound = o.frozen_bound;
      a.use_nc = o.use_neighborhood_cores;
      a.root_report = frozen ? o.root_report : nullptr;
      a.node_budget = o.node_budget;
      if (a.root_report)
        PMC_HIP(hipMemsetAsync(a.root_report, 0xff, sizeof(int32_t) * 4 * v.n, s));
      if (!frozen) {
        // the heuristic clique is the current bound
        k_state_init<<<1, 1, 0, s>>>(st, b0);
      } else {
        k_state_init<<<1, 1, 0, s>>>(st, 0);
      }
      PMC_HIP(hipGetLastError());
      for (int c = 0; c < SEARCH_CLASSES; c++)
        if (q.count[c]) S.ms_k_search += run_search_class(c, a, queue + q.start[c], q.count[c], sc);
      S.ms_search = tm.lap();
      CliqueState h;
      PMC_HIP(hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, s));
      PMC_HIP(hipStreamSynchronize(s));
      if (h.err) throw Error{PMC_ERR_CAPACITY, "search capacity exceeded (code " +
                                                   std::to_string(h.err) + ")"};
      omega_v = std::max(h.bound, frozen ? 0 : b0);
      S.nodes = (int64_t)h.nodes;
      S.roots_branched = (int64_t)h.roots_branched;
      if (h.budget_hit) budget_status = PMC_ERR_BUDGET;
    }
    S.omega = omega_v;
    S.certified = budget_status == PMC_OK ? 1 : 0;
    *omega = omega_v;
    if (capacity < omega_v)
      throw Error{PMC_ERR_CAPACITY, "clique capacity " + std::to_string(capacity) + " < omega " +
                                        std::to_string(omega_v)};
    if (omega_v > 0) copy_sorted_clique(slots + (size_t)omega_v * stride, omega_v, clique, s);
    PMC_HIP(hipStreamSynchronize(s));
    S.ms_total = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() -
                                                          t_start).count();
    if (stats) *stats = S;
  });
  if (st_ret == PMC_OK && budget_status != PMC_OK)
    return fail(budget_status, "node budget exhausted; clique not certified");
  return st_ret;
}

}  // extern "C"
