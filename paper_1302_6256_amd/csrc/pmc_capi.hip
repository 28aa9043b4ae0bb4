// pmc_capi.hip -- the C ABI (include/pmc.h): argument checks, the pipeline of
// MaxClique (Alg. 2 of the paper) on the device, error conversion.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "graph.h"
#include "learn.h"
#include "pmc.h"
#include "search.h"
#include "tuning.h"

namespace pmc {
void max_degree(const GraphView &g, int32_t *out, hipStream_t s);
}

namespace pmc {
Tuning &global_tuning() {
  static Tuning t;
  return t;
}
namespace {
thread_local const Tuning *call_tuning = nullptr;
}
const Tuning &tuning() { return call_tuning ? *call_tuning : global_tuning(); }
TuningScope::TuningScope(const Tuning *t) : prev_(call_tuning) {
  if (t) call_tuning = t;
}
TuningScope::~TuningScope() { call_tuning = prev_; }
}  // namespace pmc

namespace {
pmc::Tuning tuning_from(const pmc_tuning *t, pmc::Tuning c);
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
                               "adjacency not symmetric", "an edge joins two graphs of the batch"};
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
  if (o.node_budget < 0) throw Error{PMC_ERR_INVALID_ARG, "negative node_budget"};
  if (o.mlp) o.order = PMC_ORDER_SCORE;
  else if (o.order == PMC_ORDER_SCORE && !o.score)
    throw Error{PMC_ERR_INVALID_ARG, "PMC_ORDER_SCORE needs score"};
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

__global__ void k_state_init(CliqueState *st) {
  st->err = 0;
  st->seed_next = 0;
  st->budget_hit = 0;
  st->nodes = 0;
  st->roots_branched = 0;
  st->seeds_done = 0;
}

__global__ void k_mark_done(const int32_t *queue, int count, const int32_t *lab_vertex,
                            int32_t *vdone) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) vdone[lab_vertex[queue[i]]] = 1;
}

// Every root of the queue has been searched: mark its vertex.
void mark_done(const int32_t *queue, int count, const int32_t *lab_vertex, int32_t *vdone,
               hipStream_t s) {
  if (count <= 0) return;
  k_mark_done<<<(count + 255) / 256, 256, 0, s>>>(queue, count, lab_vertex, vdone);
  PMC_HIP(hipGetLastError());
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// vertex -> graph of a batch (binary search over the graph boundaries)
__global__ void k_fill_gid(int64_t n, const int64_t *vbase, int G, int32_t *gid) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int lo = 0, hi = G - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (vbase[mid] <= v) lo = mid; else hi = mid - 1;
  }
  gid[v] = lo;
}

// One graph of a pmc_graph array and its place in the union.
struct UnionPart {
  int64_t vb, eb;       // first vertex / entry in the union
  const void *off;      // its own offsets (bits wide)
  const int32_t *idx;   // its own indices
  int32_t bits;
};

// Last part whose base is <= x (empty parts share a base with the next one,
// which is the part that holds x).
__device__ __forceinline__ int part_of(const int64_t *base, int G, int64_t x) {
  int lo = 0, hi = G - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (base[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The union's offsets: union row v = the part's row, shifted by its entry base.
__global__ void k_union_offsets(int64_t n, const UnionPart *parts, const int64_t *vb, int G,
                                int64_t nnz, int64_t *off) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v > n) return;
  if (v == n) {
    off[n] = nnz;
    return;
  }
  const UnionPart P = parts[part_of(vb, G, v)];
  const int64_t lv = v - P.vb;
  const int64_t o = P.bits == 32 ? (int64_t)((const int32_t *)P.off)[lv] : ((const int64_t *)P.off)[lv];
  off[v] = P.eb + o;
}

// The union's indices: the part's ids shifted by its vertex base.
__global__ void k_union_indices(int64_t nnz, const UnionPart *parts, const int64_t *eb, int G,
                                int32_t *idx) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const UnionPart P = parts[part_of(eb, G, e)];
  idx[e] = (int32_t)(P.vb + P.idx[e - P.eb]);
}

// Graph g's clique (union ids at src + vb[g], omega[g] of them) to the
// caller's layout: dst + coff[g], as the graph's own ids.
__global__ void k_scatter_cliques(const int32_t *src, const int64_t *vb, const int64_t *coff,
                                  const int32_t *omega, int32_t *dst) {
  const int g = blockIdx.x;
  for (int t = threadIdx.x; t < omega[g]; t += blockDim.x)
    dst[coff[g] + t] = (int32_t)(src[vb[g] + t] - vb[g]);
}

// largest core number per graph: each thread folds a run of KMAX_RUN
// consecutive vertices (a graph's vertices are consecutive) and issues one
// atomic per graph it meets, instead of one per vertex on a few addresses
constexpr int KMAX_RUN = 64;
__global__ void k_graph_kmax(int64_t n, const int32_t *gid, const int32_t *core, int32_t *gk) {
  const int64_t v0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * KMAX_RUN;
  if (v0 >= n) return;
  const int64_t v1 = v0 + KMAX_RUN < n ? v0 + KMAX_RUN : n;
  int g = gid[v0], m = core[v0];
  for (int64_t v = v0 + 1; v < v1; v++) {
    const int gv = gid[v];
    if (gv != g) {
      atomicMax(&gk[g], m);
      g = gv;
      m = core[v];
    } else {
      m = max(m, core[v]);
    }
  }
  atomicMax(&gk[g], m);
}

// Copies each graph's maximum clique from its slot to the output range of the
// graph and sorts it (one wave per graph, bitonic network in LDS).
constexpr int OUT_CAP = 4096;
__global__ void __launch_bounds__(PMC_WAVE)
    k_write_cliques(Bounds B, const int64_t *vbase, int32_t *out, int *err) {
  __shared__ int buf[OUT_CAP];
  int g = blockIdx.x;
  int w = B.bound[g];
  if (w <= 0) return;
  if (w > OUT_CAP) {
    if (lane() == 0) atomicExch(err, 4);
    return;
  }
  const int32_t *src = slot_ptr(B, g, w);
  int p = 1;
  while (p < w) p <<= 1;
  for (int t = lane(); t < p; t += PMC_WAVE) buf[t] = t < w ? src[t] : INT_MAX;
  wave_sync();
  for (int k = 2; k <= p; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane(); i < p; i += PMC_WAVE) {
        int x = i ^ j;
        if (x > i) {
          int a = buf[i], b2 = buf[x];
          if ((a > b2) == ((i & k) == 0)) {
            buf[i] = b2;
            buf[x] = a;
          }
        }
      }
      wave_sync();
    }
  for (int t = lane(); t < w; t += PMC_WAVE) out[vbase[g] + t] = buf[t];
}

struct Pipeline {
  GraphView g;
  Scratch &sc;
  int32_t *core = nullptr, *rnd = nullptr, *rank = nullptr, *order = nullptr;
  int32_t kmax = 0, nrounds = 0;
  bool timed = true;  // false: no timing events (the allocation-free entry point)
  Pipeline(const GraphView &gv, Scratch &s) : g(gv), sc(s) {}

  PeelResult peel(int32_t *ucore, int32_t *urnd) {
    core = ucore ? ucore : sc.get<int32_t>(g.n);
    rnd = urnd ? urnd : sc.get<int32_t>(g.n);
    PeelResult pr = run_peel(g, core, rnd, sc, timed);
    kmax = pr.kmax;
    nrounds = pr.nrounds;
    return pr;
  }
  // A batch: every graph peeled alone (one workgroup each) when they all fit
  // and the table allows it, else the union as one graph.  Either way each
  // graph gets its own core numbers and, within the graph, the (round, id)
  // order of its own peel.
  PeelResult peel_batch(const std::vector<int64_t> &vb, std::vector<int32_t> *gkmax = nullptr,
                        std::vector<int32_t> *grounds = nullptr) {
    if (vb.size() <= 2 || tuning().batch_peel < 0 || !peel_graphs_fits(vb))
      return peel(nullptr, nullptr);
    core = sc.get<int32_t>(g.n);
    rnd = sc.get<int32_t>(g.n);
    PeelResult pr = run_peel_graphs(g, vb, core, rnd, sc, timed, gkmax, grounds);
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

// Per-graph state: bounds, frozen-heuristic winners, clique slots.

Bounds make_bounds(int G, const int32_t *gid, const std::vector<int32_t> &gk, Scratch &sc) {
  hipStream_t s = sc.stream();
  Bounds B;
  B.G = G;
  B.gid = gid;
  std::vector<int64_t> base(G);
  std::vector<int32_t> stride(G);
  int64_t tot = 0;
  for (int g = 0; g < G; g++) {
    base[g] = tot;
    stride[g] = gk[g] + 1;
    tot += (int64_t)(gk[g] + 2) * (gk[g] + 1);
  }
  B.slots = sc.get<int32_t>((size_t)std::max<int64_t>(tot, 1));
  int64_t *db = sc.get<int64_t>(G);
  int32_t *ds = sc.get<int32_t>(G);
  PMC_HIP(hipMemcpyAsync(db, base.data(), sizeof(int64_t) * G, hipMemcpyHostToDevice, s));
  PMC_HIP(hipMemcpyAsync(ds, stride.data(), sizeof(int32_t) * G, hipMemcpyHostToDevice, s));
  B.slot_base = db;
  B.slot_stride = ds;
  B.bound = sc.get<int32_t>(G);
  PMC_HIP(hipMemsetAsync(B.bound, 0, sizeof(int32_t) * G, s));
  B.packed = sc.get<unsigned long long>(G);
  PMC_HIP(hipMemsetAsync(B.packed, 0, sizeof(unsigned long long) * G, s));
  return B;
}

int32_t *score_seed_order(int64_t n, const int32_t *order, const float *score, Scratch &sc) {
  hipStream_t s = sc.stream();
  uint32_t *k1 = sc.get<uint32_t>(n), *k2 = sc.get<uint32_t>(n);
  int32_t *v1 = sc.get<int32_t>(n);
  int32_t *seeds = sc.get<int32_t>(n);
  k_seed_keys<<<(int)((n + 255) / 256), 256, 0, s>>>((int)n, order, score, k1, v1);
  PMC_HIP(hipGetLastError());
  radix_sort_pairs(k1, v1, k2, seeds, n, 32, sc);
  return seeds;
}

// The whole MaxClique pipeline for a batch of G graphs (G = 1: one graph).
// Fills omegas (host) and, when `out` is given, each graph's sorted clique
// at out + vbase[g] (device).  Returns PMC_ERR_BUDGET when a node budget
// stopped the search.
int solve(const GraphView &v, int G, const std::vector<int64_t> &vbase, const int32_t *gid_in,
          const pmc_options &o, int32_t *out, std::vector<int32_t> &omegas, pmc_stats &S,
          Scratch &sc) {
  hipStream_t s = sc.stream();
  Timer tm(s);
  Pipeline p(v, sc);
  std::vector<int32_t> gk_peel;
  PeelResult pr0 = p.peel_batch(vbase, &gk_peel);
  S.ms_k_peel = pr0.ms;
  if (pr0.ms > 0) {
    // bytes models: the grid peel reads the offsets, each entry once and
    // updates a degree per entry; the per-graph peel keeps the degrees in LDS
    const double bytes = gk_peel.empty() ? 8.0 * (v.n + 1) + 12.0 * v.nnz + 12.0 * v.n
                                         : 24.0 * v.n + 4.0 * v.nnz;
    S.gbps_peel = (float)(bytes / (pr0.ms * 1e6));
  }
  S.ms_peel = tm.lap();
  p.ranks(nullptr, nullptr);
  S.ms_rank = tm.lap();
  S.kmax = p.kmax;
  S.nrounds = p.nrounds;
  // per-graph largest core
  std::vector<int32_t> gk(G, p.kmax);
  const int32_t *gid = gid_in;
  if (G > 1 && (int)gk_peel.size() == G) {
    gk = gk_peel;  // the per-graph peel reports every graph's K
  } else if (G > 1) {
    int32_t *dgk = sc.get<int32_t>(G);
    PMC_HIP(hipMemsetAsync(dgk, 0, sizeof(int32_t) * G, s));
    const int64_t nthr = (v.n + KMAX_RUN - 1) / KMAX_RUN;
    k_graph_kmax<<<(int)((nthr + 255) / 256), 256, 0, s>>>(v.n, gid, p.core, dgk);
    PMC_HIP(hipGetLastError());
    PMC_HIP(hipMemcpyAsync(gk.data(), dgk, sizeof(int32_t) * G, hipMemcpyDeviceToHost, s));
    PMC_HIP(hipStreamSynchronize(s));
  }
  CliqueState *st = sc.get<CliqueState>(1);
  k_state_init<<<1, 1, 0, s>>>(st);
  PMC_HIP(hipGetLastError());
  Bounds B = make_bounds(G, gid, gk, sc);
  const bool frozen = o.frozen_bound >= 0;
  std::vector<int32_t> hb(G, 0);
  pmc_options oo = o;
  if (o.mlp) oo.order = PMC_ORDER_CORE;  // the model's scores come after the heuristic
  if (!frozen && !o.skip_heuristic) {
    int32_t *seeds = oo.order == PMC_ORDER_SCORE ? score_seed_order(v.n, p.order, oo.score, sc)
                                                 : nullptr;
    S.ms_k_heuristic =
        run_heuristic(v, p.core, p.rank, p.order, seeds, p.kmax, o.frozen_threshold, B, st, sc);
    PMC_HIP(hipMemcpyAsync(hb.data(), B.bound, sizeof(int32_t) * G, hipMemcpyDeviceToHost, s));
    unsigned long long seeds_done = 0;
    PMC_HIP(hipMemcpyAsync(&seeds_done, &st->seeds_done, sizeof(seeds_done),
                           hipMemcpyDeviceToHost, s));
    PMC_HIP(hipStreamSynchronize(s));
    S.heuristic_seeds = (int64_t)seeds_done;
  }
  S.ms_heuristic = tm.lap();
  S.heuristic = *std::max_element(hb.begin(), hb.end());
  int open = 0;  // graphs not certified by Fact 1 after the heuristic
  for (int g = 0; g < G; g++) open += frozen || hb[g] != gk[g] + 1;
  S.certified_early = open == 0 ? 1 : 0;
  // Learned order: features and scores on the GPU (timed with the
  // heuristic), only once the heuristic (in degeneracy order) has not
  // certified omega.  A single graph first runs the sweep in degeneracy
  // order, and the model orders only the roots the sweep leaves open (none:
  // no features at all); a batch or a frozen-bound run is scored right away.
  auto learned_scores = [&]() {
    S.learned_used = 1;
    float *feat = sc.get<float>((size_t)v.n * 8);
    float *score = sc.get<float>((size_t)v.n);
    run_features(v, p.core, p.rank, p.order, p.kmax, feat, sc);
    run_mlp_forward(o.mlp, feat, v.n, score, sc);
    oo.score = score;
    oo.order = PMC_ORDER_SCORE;
  };
  const bool learned_after_sweep = o.mlp && open > 0 && G == 1 && !frozen;
  if (o.mlp && open > 0 && !learned_after_sweep) {
    learned_scores();
    S.ms_heuristic += tm.lap();
  }
  int budget = 0;
  if (open > 0) {
    // explicit pruning against the heuristic bound (or the frozen bound)
    const int32_t *prune_bound = B.bound;
    if (frozen) {
      int32_t *fb = sc.get<int32_t>(G);
      k_fill_i32<<<(G + 255) / 256, 256, 0, s>>>(fb, G, o.frozen_bound);
      PMC_HIP(hipGetLastError());
      prune_bound = fb;
    }
    // Roots are searched in waves of consecutive labels (rank order).  Between
    // waves, once the bound of some graph has risen above the one the current
    // oriented graph was pruned with, the pruning is run again (Alg. 2's
    // periodic re-pruning, triggered by the bound rather than by a timer): it
    // drops the vertices whose core fell below the bound and the roots already
    // searched (a rank prefix, never in a later root's higher-ranked P).
    // Automatic wave size: a quarter of the survivors (at least 2^18) for one
    // graph; one wave for a batch, where re-pruning the whole union for the
    // bound gain of a few small graphs costs more than it saves.
    const bool waves_on = !frozen && (G == 1 || o.wave_roots > 0);
    const bool by_score = oo.order == PMC_ORDER_SCORE;
    std::vector<int32_t> hb_prune = hb;
    float msk = 0.f;
    const bool native = o.native_order != 0;
    // a single graph in degeneracy order dispatches each size class from its
    // highest label down (thousands of roots run at once, and starting in the
    // densest part measured faster on single graphs, slower on a batch's
    // union); the subproblems are the same either way, fixed by the
    // orientation
    const bool desc = G == 1 && !native;
    Labels L = run_prune_orient(v, p.core, p.rank, p.order, gid, prune_bound, p.kmax, sc, &msk,
                                nullptr, nullptr, -1, 0, native);
    S.ms_k_orient += msk;
    S.survivors = L.nn;
    S.oriented_nnz = L.nnz;
    if (msk > 0)
      S.gbps_orient = (float)((2.0 * (16.0 * L.nn + 8.0 * L.deg_sum) + 4.0 * L.nnz) / (msk * 1e6));
    S.ms_prune = tm.lap();
    int32_t *queue = sc.get<int32_t>((size_t)std::max(L.nn, 1));
    SearchArgs a;
    a.kmax = p.kmax;
    a.B = B;
    a.st = st;
    a.frozen_bound = o.frozen_bound;
    a.use_nc = o.use_neighborhood_cores;
    a.root_report = frozen ? o.root_report : nullptr;
    a.node_budget = o.node_budget;
    a.native = native;
    if (a.root_report)
      PMC_HIP(hipMemsetAsync(a.root_report, 0xff, sizeof(int32_t) * 4 * v.n, s));
    alloc_split(a, sc);
    int lab_lo = 0;
    CliqueState h;
    const int sweep_nodes =
        learned_after_sweep ? std::max(tuning().search_sweep_nodes, 64) : tuning().search_sweep_nodes;
    const bool sweep_on = !frozen && G == 1 && sweep_nodes > 0 && !by_score;
    auto read_state = [&]() {
      PMC_HIP(hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, s));
      PMC_HIP(hipMemcpyAsync(hb.data(), B.bound, sizeof(int32_t) * G, hipMemcpyDeviceToHost, s));
      PMC_HIP(hipStreamSynchronize(s));
      if (h.err)
        throw Error{PMC_ERR_CAPACITY, "search capacity exceeded (code " + std::to_string(h.err) + ")"};
    };
    if (sweep_on) {
      // Sweep: every root gets InitialBranch's bounds and Branch's first
      // descent plus at most sweep_nodes more nodes; what that settles is
      // done, and every clique it finds raises the bound at once.  Then,
      // after re-pruning against the raised bound, the open roots are
      // searched fully, in degeneracy order.
      int32_t *vdone = sc.get<int32_t>((size_t)v.n);
      float *skey = sc.get<float>((size_t)v.n);
      PMC_HIP(hipMemsetAsync(vdone, 0, sizeof(int32_t) * v.n, s));
      PMC_HIP(hipMemsetAsync(skey, 0, sizeof(float) * v.n, s));
      QueueResult q = run_queue(L, prune_bound, false, nullptr, queue, sc, 0, INT_MAX, nullptr,
                                INT_MAX, desc);
      S.roots += q.total;
      S.ms_queue += tm.lap();
      if (q.count[SEARCH_CLASSES] > 0)
        throw Error{PMC_ERR_CAPACITY, "a subproblem exceeds 4096 vertices"};
      SearchArgs a1 = a;
      a1.L = L;
      a1.sweep_cap = sweep_nodes;
      a1.sweep_key = skey;
      a1.vdone = vdone;
      S.ms_k_search += run_search(a1, queue, q, sc, false, &S.search_graph_replays);
      S.ms_sweep = tm.lap();
      S.ms_search += S.ms_sweep;
      read_state();
      if (!h.budget_hit) {
        if (o.rebuild_on_bound_gain && hb[0] > hb_prune[0]) {
          L = run_prune_orient(v, p.core, p.rank, p.order, gid, prune_bound, p.kmax, sc, &msk,
                               nullptr, nullptr, -1, 0, native);
          S.ms_k_orient += msk;
          S.ms_prune += tm.lap();
          S.rebuilds++;
          hb_prune = hb;
        }
        QueueResult q2 = run_queue(L, prune_bound, false, nullptr, queue, sc, 0, INT_MAX, vdone,
                                   INT_MAX, desc);
        S.roots_second_pass = q2.total;
        S.ms_queue += tm.lap();
        if (learned_after_sweep && q2.total >= tuning().learned_min_open) {
          // the open roots by the model's score (fewer open roots than that are
          // searched in degeneracy order: the order of a handful of roots
          // cannot repay the features of every vertex)
          learned_scores();
          S.ms_heuristic += tm.lap();
          q2 = run_queue(L, prune_bound, false, oo.score, queue, sc, 0, INT_MAX, vdone);
          S.ms_queue += tm.lap();
        }
        a.L = L;
        S.ms_k_search += run_search(a, queue, q2, sc, false, &S.search_graph_replays);
        S.ms_search += tm.lap();
        read_state();
      }
    }
    if (by_score) {
      // Dispatch by score in waves: each wave takes the best-scored roots not
      // searched yet; once the bound has risen the oriented graph is pruned
      // again (by core only: in this order the searched roots are no rank
      // prefix, and a later root's neighbourhood may still hold them).
      int32_t *vdone = sc.get<int32_t>((size_t)v.n);
      PMC_HIP(hipMemsetAsync(vdone, 0, sizeof(int32_t) * v.n, s));
      while (true) {
        int64_t wr = INT_MAX;
        if (waves_on) wr = o.wave_roots > 0 ? o.wave_roots : std::max<int64_t>(1 << 18, L.nn / 4 + 1);
        QueueResult q = run_queue(L, prune_bound, frozen, oo.score, queue, sc, 0, INT_MAX,
                                  vdone, (int)std::min<int64_t>(wr, INT_MAX));
        S.roots += q.total;
        S.ms_queue += tm.lap();
        if (q.total == 0) break;
        if (q.count[SEARCH_CLASSES] > 0)
          throw Error{PMC_ERR_CAPACITY, "a subproblem exceeds 4096 vertices"};
        a.L = L;
        S.ms_k_search += run_search(a, queue, q, sc, false, &S.search_graph_replays);
        mark_done(queue, q.total, L.vertex, vdone, s);
        S.ms_search += tm.lap();
        read_state();
        if (h.budget_hit) break;
        bool gained = false;
        for (int g = 0; g < G; g++) gained |= hb[g] > hb_prune[g];
        if (o.rebuild_on_bound_gain && gained) {
          L = run_prune_orient(v, p.core, p.rank, p.order, gid, prune_bound, p.kmax, sc, &msk,
                               nullptr, nullptr, -1, 0, native);
          S.ms_k_orient += msk;
          S.ms_prune += tm.lap();
          S.rebuilds++;
          hb_prune = hb;
          if (L.nn == 0) break;
        }
      }
    }
    while (!sweep_on && !by_score) {
      int64_t wr = INT_MAX;
      if (waves_on) wr = o.wave_roots > 0 ? o.wave_roots : std::max<int64_t>(1 << 18, L.nn / 4 + 1);
      const int lab_hi = (int)std::min<int64_t>((int64_t)lab_lo + wr, INT_MAX);
      QueueResult q = run_queue(L, prune_bound, frozen, nullptr, queue, sc, lab_lo, lab_hi, nullptr,
                                INT_MAX, desc);
      S.roots += q.total;
      S.ms_queue += tm.lap();
      if (q.count[SEARCH_CLASSES] > 0)
        throw Error{PMC_ERR_CAPACITY, "a subproblem exceeds 4096 vertices"};
      a.L = L;
      S.ms_k_search += run_search(a, queue, q, sc, false, &S.search_graph_replays);
      S.ms_search += tm.lap();
      read_state();
      if (h.budget_hit || lab_hi >= L.nn) break;
      lab_lo = lab_hi;
      bool gained = false;
      for (int g = 0; g < G; g++) gained |= hb[g] > hb_prune[g];
      if (o.rebuild_on_bound_gain && gained) {
        // the first unsearched label's position in the search order: its
        // rank, or in native order its id
        int32_t vfirst = 0, rfirst = 0;
        PMC_HIP(hipMemcpyAsync(&vfirst, L.vertex + lab_lo, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        PMC_HIP(hipStreamSynchronize(s));
        if (native) {
          rfirst = vfirst;
        } else {
          PMC_HIP(hipMemcpyAsync(&rfirst, p.rank + vfirst, sizeof(int32_t), hipMemcpyDeviceToHost, s));
          PMC_HIP(hipStreamSynchronize(s));
        }
        L = run_prune_orient(v, p.core, p.rank, p.order, gid, prune_bound, p.kmax, sc, &msk, nullptr,
                             nullptr, -1, rfirst, native);
        S.ms_k_orient += msk;
        S.ms_prune += tm.lap();
        S.rebuilds++;
        hb_prune = hb;
        lab_lo = 0;
        if (L.nn == 0) break;
      }
    }
    S.nodes = (int64_t)h.nodes;
    S.roots_branched = (int64_t)h.roots_branched;
    budget = h.budget_hit;
  }
  omegas = hb;
  S.omega = *std::max_element(hb.begin(), hb.end());
  S.certified = budget ? 0 : 1;
  if (out && G > 1) {
    int64_t *dvb = sc.get<int64_t>(G + 1);
    PMC_HIP(hipMemcpyAsync(dvb, vbase.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
    int *err = sc.get<int>(1);
    PMC_HIP(hipMemsetAsync(err, 0, sizeof(int), s));
    k_write_cliques<<<G, PMC_WAVE, 0, s>>>(B, dvb, out, err);
    PMC_HIP(hipGetLastError());
    int herr = 0;
    PMC_HIP(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
    PMC_HIP(hipStreamSynchronize(s));
    if (herr) throw Error{PMC_ERR_CAPACITY, "a batch clique exceeds 4096 vertices"};
  } else if (out && hb[0] > 0) {
    std::vector<int64_t> bh(1);
    PMC_HIP(hipMemcpyAsync(bh.data(), B.slot_base, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PMC_HIP(hipStreamSynchronize(s));
    copy_sorted_clique(B.slots + bh[0] + (int64_t)hb[0] * (gk[0] + 1), hb[0], out, s);
  }
  return budget ? PMC_ERR_BUDGET : PMC_OK;
}

// ---- fixed scratch of the allocation-free entry point
//
// One copy of this array exists on every device the library runs on, for the
// life of the process.  In host code its name is a host-side stand-in, not a
// device address: the device address of the current device's copy is looked
// up once per device with hipGetSymbolAddress and only that pointer is used.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

void *noalloc_scratch() {
  static std::mutex mu;
  static std::map<int, void *> ptrs;
  int d = 0;
  PMC_HIP(hipGetDevice(&d));
  std::lock_guard<std::mutex> lock(mu);
  auto it = ptrs.find(d);
  if (it != ptrs.end()) return it->second;
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr) {
    (void)hipGetLastError();
    throw Error{PMC_ERR_DEVICE, std::string("fixed scratch address: ") + hipGetErrorString(e)};
  }
  ptrs[d] = p;
  return p;
}

// An upper bound on the scratch bytes of pmc_core_numbers: the peel's five
// n-word arrays, its tail graph (at most 2^24 entries, 16,385-entry tables,
// one word per thread of the launch), core/round/rank/order when the caller
// passes NULL, the rank's keys and the radix sort's temporaries and
// per-tile histograms, plus alignment and slack.
size_t core_numbers_scratch_bound(int64_t n, int64_t nnz) {
  const size_t w = 4;
  return w * (size_t)n * 13 + (size_t)n / 2 + w * (size_t)std::min<int64_t>(nnz, (int64_t)1 << 24) +
         ((size_t)4 << 20);
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

pmc_status pmc_core_numbers_noalloc(const pmc_graph *g, int32_t *core, int32_t *round,
                                    int32_t *rank, int32_t *order, int32_t *kmax, int32_t *nrounds,
                                    void *stream) {
  return guarded([&] {
    GraphView v = make_view(g);
    const size_t need = core_numbers_scratch_bound(v.n, v.nnz);
    if (need > NOALLOC_SCRATCH_BYTES)
      throw Error{PMC_ERR_CAPACITY, "graph needs up to " + std::to_string(need) +
                                        " bytes of scratch; the fixed buffer holds " +
                                        std::to_string(NOALLOC_SCRATCH_BYTES)};
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(s, noalloc_scratch(), NOALLOC_SCRATCH_BYTES);
    maybe_validate(g, v, sc);
    if (v.n == 0) {
      if (kmax) *kmax = 0;
      if (nrounds) *nrounds = 0;
      return;
    }
    Pipeline p(v, sc);
    p.timed = false;
    p.cores(core, round, rank, order, rank || order);
    PMC_HIP(hipStreamSynchronize(s));
    if (kmax) *kmax = p.kmax;
    if (nrounds) *nrounds = p.nrounds;
  });
}

pmc_status pmc_core_numbers_batch(const pmc_batch *b, int32_t *core, int32_t *round,
                                  int32_t *rank, int32_t *order, int32_t *kmax, int32_t *nrounds,
                                  void *stream) {
  return guarded([&] {
    if (!b) throw Error{PMC_ERR_INVALID_ARG, "batch is NULL"};
    if (b->count < 1 || !b->vertex_base)
      throw Error{PMC_ERR_INVALID_ARG, "count and vertex_base are required"};
    pmc_graph gg{b->n, b->nnz, b->offsets, b->offsets_bits, b->indices, b->flags};
    GraphView v = make_view(&gg);
    const int G = b->count;
    std::vector<int64_t> vb(b->vertex_base, b->vertex_base + G + 1);
    if (vb[0] != 0 || vb[G] != v.n) throw Error{PMC_ERR_INVALID_ARG, "vertex_base must span [0, n]"};
    for (int g = 0; g < G; g++)
      if (vb[g + 1] < vb[g]) throw Error{PMC_ERR_INVALID_ARG, "vertex_base must be nondecreasing"};
    if (!peel_graphs_fits(vb))
      throw Error{PMC_ERR_CAPACITY, "a graph of the batch has more than " +
                                        std::to_string(PEEL_GRAPH_MAX_N) + " vertices"};
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(s);
    if ((gg.flags & PMC_GRAPH_VALIDATE) && v.n > 0) {
      int64_t *dvb = sc.get<int64_t>(G + 1);
      PMC_HIP(hipMemcpyAsync(dvb, vb.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
      int32_t *gid = sc.get<int32_t>(v.n);
      k_fill_gid<<<(int)((v.n + 255) / 256), 256, 0, s>>>(v.n, dvb, G, gid);
      PMC_HIP(hipGetLastError());
      int code = validate_graph(v, sc, gid);
      if (code) throw Error{PMC_ERR_INVALID_GRAPH, "invalid batch (code " + std::to_string(code) + ")"};
    }
    std::vector<int32_t> gk(G, 0), gr(G, 0);
    if (v.n > 0) {
      int32_t *c = core ? core : sc.get<int32_t>(v.n);
      int32_t *r = round ? round : sc.get<int32_t>(v.n);
      PeelResult pr = run_peel_graphs(v, vb, c, r, sc, false, &gk, &gr);
      if (rank || order) {
        int32_t *rk = rank ? rank : sc.get<int32_t>(v.n);
        int32_t *od = order ? order : sc.get<int32_t>(v.n);
        run_rank(v.n, r, pr.nrounds, rk, od, sc);
      }
      PMC_HIP(hipStreamSynchronize(s));
    }
    if (kmax) std::memcpy(kmax, gk.data(), sizeof(int32_t) * G);
    if (nrounds) std::memcpy(nrounds, gr.data(), sizeof(int32_t) * G);
  });
}

pmc_status pmc_heuristic(const pmc_graph *g, const int32_t *core, const int32_t *rank,
                         const int32_t *order, const pmc_options *opt, int32_t *clique,
                         int32_t capacity, int32_t *size, void *stream) {
  return guarded([&] {
    GraphView v = make_view(g);
    pmc_options o = read_options(opt);
    Tuning call_table;
    if (o.tune_table) call_table = tuning_from(o.tune_table, global_tuning());
    TuningScope table_scope(o.tune_table ? &call_table : nullptr);
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
    k_state_init<<<1, 1, 0, s>>>(st);
    std::vector<int32_t> gk(1, km);
    Bounds B = make_bounds(1, nullptr, gk, sc);
    int32_t *seeds =
        o.order == PMC_ORDER_SCORE ? score_seed_order(v.n, p.order, o.score, sc) : nullptr;
    run_heuristic(v, p.core, p.rank, p.order, seeds, km, o.frozen_threshold, B, st, sc);
    int32_t h = 0;
    PMC_HIP(hipMemcpyAsync(&h, B.bound, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PMC_HIP(hipStreamSynchronize(s));
    *size = h;
    if (capacity < h)
      throw Error{PMC_ERR_CAPACITY,
                  "clique capacity " + std::to_string(capacity) + " < " + std::to_string(h)};
    copy_sorted_clique(B.slots + (int64_t)h * (km + 1), h, clique, s);
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
    int32_t km = 0;
    if (v.n > 0) {
      int32_t last = 0;
      PMC_HIP(hipMemcpyAsync(&last, order + (v.n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
      PMC_HIP(hipStreamSynchronize(s));
      if (last < 0 || last >= v.n) throw Error{PMC_ERR_INVALID_ARG, "order is not a permutation"};
      PMC_HIP(hipMemcpyAsync(&km, core + last, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    }
    int32_t *db = sc.get<int32_t>(1);
    PMC_HIP(hipMemcpyAsync(db, &bound, sizeof(int32_t), hipMemcpyHostToDevice, s));
    PMC_HIP(hipStreamSynchronize(s));
    Labels L = run_prune_orient(v, core, rank, order, nullptr, db, km, sc, nullptr, poff, padj,
                                capacity);
    PMC_HIP(hipStreamSynchronize(s));
    *r0 = (int32_t)(v.n - L.nn);  // survivors of one graph are a rank suffix
    *out_nnz = L.nnz;
  });
}

pmc_status pmc_max_clique(const pmc_graph *g, const pmc_options *opt, int32_t *clique,
                          int32_t capacity, int32_t *omega, pmc_stats *stats, void *stream) {
  int rc = PMC_OK;
  pmc_status st_ret = guarded([&] {
    auto t_start = std::chrono::steady_clock::now();
    GraphView v = make_view(g);
    pmc_options o = read_options(opt);
    Tuning call_table;
    if (o.tune_table) call_table = tuning_from(o.tune_table, global_tuning());
    TuningScope table_scope(o.tune_table ? &call_table : nullptr);
    if (!omega) throw Error{PMC_ERR_INVALID_ARG, "omega is required"};
    if (!clique && capacity > 0) throw Error{PMC_ERR_INVALID_ARG, "clique is NULL"};
    pmc_stats S;
    std::memset(&S, 0, sizeof(S));
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(s);
    maybe_validate(g, v, sc);
    *omega = 0;
    if (v.n > 0) {
      std::vector<int32_t> om;
      std::vector<int64_t> vb = {0, v.n};
      // the clique goes to a scratch buffer first: its size is known only at the end
      int32_t *tmp = sc.get<int32_t>((size_t)v.n);
      rc = solve(v, 1, vb, nullptr, o, tmp, om, S, sc);
      *omega = om[0];
      if (capacity < om[0])
        throw Error{PMC_ERR_CAPACITY, "clique capacity " + std::to_string(capacity) +
                                          " < omega " + std::to_string(om[0])};
      if (om[0] > 0)
        PMC_HIP(hipMemcpyAsync(clique, tmp, sizeof(int32_t) * om[0], hipMemcpyDeviceToDevice, s));
      PMC_HIP(hipStreamSynchronize(s));
    } else {
      S.certified = 1;
    }
    S.ms_total = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() -
                                                          t_start).count();
    if (stats) *stats = S;
  });
  if (st_ret == PMC_OK && rc != PMC_OK)
    return fail(rc, "node budget exhausted; clique not certified");
  return st_ret;
}

pmc_status pmc_max_clique_batch(const pmc_batch *b, const pmc_options *opt, int32_t *cliques,
                                int32_t *omegas, pmc_stats *stats, void *stream) {
  int rc = PMC_OK;
  pmc_status st_ret = guarded([&] {
    auto t_start = std::chrono::steady_clock::now();
    if (!b) throw Error{PMC_ERR_INVALID_ARG, "batch is NULL"};
    if (b->count < 1 || !b->vertex_base || !omegas || !cliques)
      throw Error{PMC_ERR_INVALID_ARG, "count, vertex_base, omegas and cliques are required"};
    pmc_graph gg{b->n, b->nnz, b->offsets, b->offsets_bits, b->indices, b->flags};
    GraphView v = make_view(&gg);
    pmc_options o = read_options(opt);
    Tuning call_table;
    if (o.tune_table) call_table = tuning_from(o.tune_table, global_tuning());
    TuningScope table_scope(o.tune_table ? &call_table : nullptr);
    int G = b->count;
    std::vector<int64_t> vb(b->vertex_base, b->vertex_base + G + 1);
    if (vb[0] != 0 || vb[G] != v.n) throw Error{PMC_ERR_INVALID_ARG, "vertex_base must span [0, n]"};
    for (int g = 0; g < G; g++)
      if (vb[g + 1] < vb[g]) throw Error{PMC_ERR_INVALID_ARG, "vertex_base must be nondecreasing"};
    pmc_stats S;
    std::memset(&S, 0, sizeof(S));
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(s);
    int32_t *gid = nullptr;
    if (v.n > 0) {
      int64_t *dvb = sc.get<int64_t>(G + 1);
      PMC_HIP(hipMemcpyAsync(dvb, vb.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
      gid = sc.get<int32_t>(v.n);
      k_fill_gid<<<(int)((v.n + 255) / 256), 256, 0, s>>>(v.n, dvb, G, gid);
      PMC_HIP(hipGetLastError());
    }
    if ((gg.flags & PMC_GRAPH_VALIDATE) && v.n > 0) {
      int code = validate_graph(v, sc, gid);
      if (code) throw Error{PMC_ERR_INVALID_GRAPH, "invalid batch (code " + std::to_string(code) + ")"};
    }
    std::vector<int32_t> om(G, 0);
    if (v.n > 0) rc = solve(v, G, vb, gid, o, cliques, om, S, sc);
    else S.certified = 1;
    std::memcpy(omegas, om.data(), sizeof(int32_t) * G);
    S.ms_total = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() -
                                                          t_start).count();
    if (stats) *stats = S;
  });
  if (st_ret == PMC_OK && rc != PMC_OK)
    return fail(rc, "node budget exhausted; cliques not certified");
  return st_ret;
}

pmc_status pmc_max_clique_graphs(const pmc_graph *graphs, int32_t count, const pmc_options *opt,
                                 int32_t *cliques, const int64_t *clique_offsets,
                                 int32_t *omegas, pmc_stats *stats, void *stream) {
  int rc = PMC_OK;
  pmc_status st_ret = guarded([&] {
    auto t_start = std::chrono::steady_clock::now();
    if (!graphs || count < 1 || !clique_offsets || !omegas || !cliques)
      throw Error{PMC_ERR_INVALID_ARG, "graphs, count >= 1, cliques, clique_offsets and omegas are required"};
    pmc_options o = read_options(opt);
    Tuning call_table;
    if (o.tune_table) call_table = tuning_from(o.tune_table, global_tuning());
    TuningScope table_scope(o.tune_table ? &call_table : nullptr);
    const int G = count;
    std::vector<int64_t> vb(G + 1, 0), eb(G + 1, 0);
    std::vector<UnionPart> parts(G);
    bool validate = false;
    for (int g = 0; g < G; g++) {
      GraphView gv = make_view(&graphs[g]);
      validate |= (graphs[g].flags & PMC_GRAPH_VALIDATE) != 0;
      parts[g] = UnionPart{vb[g], eb[g], gv.off, gv.idx, gv.bits};
      vb[g + 1] = vb[g] + gv.n;
      eb[g + 1] = eb[g] + gv.nnz;
      if (clique_offsets[g + 1] < clique_offsets[g])
        throw Error{PMC_ERR_INVALID_ARG, "clique_offsets must be nondecreasing"};
    }
    if (vb[G] >= (int64_t)1 << 31) throw Error{PMC_ERR_INVALID_ARG, "the batch must hold < 2^31 vertices"};
    const int64_t n = vb[G], nnz = eb[G];
    pmc_stats S;
    std::memset(&S, 0, sizeof(S));
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(s);
    std::vector<int32_t> om(G, 0);
    if (n > 0) {
      // the disjoint union in one CSR (int64 offsets), built on the device
      int64_t *dvb = sc.get<int64_t>(G + 1), *deb = sc.get<int64_t>(G + 1);
      UnionPart *dparts = sc.get<UnionPart>(G);
      PMC_HIP(hipMemcpyAsync(dvb, vb.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
      PMC_HIP(hipMemcpyAsync(deb, eb.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
      PMC_HIP(hipMemcpyAsync(dparts, parts.data(), sizeof(UnionPart) * G, hipMemcpyHostToDevice, s));
      int64_t *uoff = sc.get<int64_t>((size_t)n + 1);
      int32_t *uidx = sc.get<int32_t>((size_t)std::max<int64_t>(nnz, 1));
      k_union_offsets<<<(int)((n + 1 + 255) / 256), 256, 0, s>>>(n, dparts, dvb, G, nnz, uoff);
      PMC_HIP(hipGetLastError());
      if (nnz > 0) {
        k_union_indices<<<(int)((nnz + 255) / 256), 256, 0, s>>>(nnz, dparts, deb, G, uidx);
        PMC_HIP(hipGetLastError());
      }
      pmc_graph ug{n, nnz, uoff, 64, uidx, 0u};
      GraphView v = make_view(&ug);
      int32_t *gid = sc.get<int32_t>((size_t)n);
      k_fill_gid<<<(int)((n + 255) / 256), 256, 0, s>>>(n, dvb, G, gid);
      PMC_HIP(hipGetLastError());
      if (validate) {
        int code = validate_graph(v, sc, gid);
        if (code) throw Error{PMC_ERR_INVALID_GRAPH, "invalid graph in the batch (code " + std::to_string(code) + ")"};
      }
      int32_t *ucl = sc.get<int32_t>((size_t)n);
      rc = solve(v, G, vb, gid, o, ucl, om, S, sc);
      for (int g = 0; g < G; g++)
        if (clique_offsets[g + 1] - clique_offsets[g] < om[g])
          throw Error{PMC_ERR_CAPACITY, "graph " + std::to_string(g) + " has omega " +
                                            std::to_string(om[g]) + " but room for " +
                                            std::to_string(clique_offsets[g + 1] - clique_offsets[g])};
      int64_t *dco = sc.get<int64_t>(G + 1);
      int32_t *dom = sc.get<int32_t>(G);
      PMC_HIP(hipMemcpyAsync(dco, clique_offsets, sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
      PMC_HIP(hipMemcpyAsync(dom, om.data(), sizeof(int32_t) * G, hipMemcpyHostToDevice, s));
      k_scatter_cliques<<<G, 64, 0, s>>>(ucl, dvb, dco, dom, cliques);
      PMC_HIP(hipGetLastError());
      PMC_HIP(hipStreamSynchronize(s));
    } else {
      S.certified = 1;
    }
    std::memcpy(omegas, om.data(), sizeof(int32_t) * G);
    S.ms_total = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() -
                                                          t_start).count();
    if (stats) *stats = S;
  });
  if (st_ret == PMC_OK && rc != PMC_OK)
    return fail(rc, "node budget exhausted; cliques not certified");
  return st_ret;
}

pmc_status pmc_get_tuning(pmc_tuning *t) {
  return guarded([&] {
    if (!t) throw Error{PMC_ERR_INVALID_ARG, "tuning is NULL"};
    const Tuning &c = global_tuning();
    pmc_tuning o;
    std::memset(&o, 0, sizeof(o));
    o.struct_size = sizeof(pmc_tuning);
    for (int i = 0; i < 7; i++) o.search_blocks_per_cu[i] = c.search_blocks_per_cu[i];
    o.heuristic_waves_per_cu[0] = c.heuristic_waves_per_cu[0];
    o.heuristic_waves_per_cu[1] = c.heuristic_waves_per_cu[1];
    o.search_graph = c.search_graph;
    o.heuristic_chunk[0] = c.heuristic_chunk[0];
    o.heuristic_chunk[1] = c.heuristic_chunk[1];
    o.search_split_min = c.search_split_min;
    o.search_split_depth = c.search_split_depth;
    o.search_sweep_nodes = c.search_sweep_nodes;
    o.learned_min_open = c.learned_min_open;
    o.batch_peel = c.batch_peel;
    *t = o;
  });
}

pmc_status pmc_set_tuning(const pmc_tuning *t) {
  return guarded([&] {
    if (!t) {
      global_tuning() = Tuning();
      return;
    }
    global_tuning() = tuning_from(t, Tuning());
  });
}

}  // extern "C"

namespace {
// A pmc_tuning applied over `c`: every nonzero field replaces c's value.
Tuning tuning_from(const pmc_tuning *t, Tuning c) {
    if (t->struct_size < sizeof(pmc_tuning))
      throw Error{PMC_ERR_INVALID_ARG, "pmc_tuning.struct_size too small"};
    for (int i = 0; i < 7; i++) {
      if (t->search_blocks_per_cu[i] < 0 || t->search_blocks_per_cu[i] > 64)
        throw Error{PMC_ERR_INVALID_ARG, "search_blocks_per_cu must be in [0, 64]"};
      if (t->search_blocks_per_cu[i]) c.search_blocks_per_cu[i] = t->search_blocks_per_cu[i];
    }
    for (int i = 0; i < 2; i++) {
      if (t->heuristic_waves_per_cu[i] < 0 || t->heuristic_waves_per_cu[i] > 64)
        throw Error{PMC_ERR_INVALID_ARG, "heuristic_waves_per_cu must be in [0, 64]"};
      if (t->heuristic_waves_per_cu[i]) c.heuristic_waves_per_cu[i] = t->heuristic_waves_per_cu[i];
    }
    if (t->search_graph) c.search_graph = t->search_graph > 0 ? 1 : 0;
    if (t->search_split_min > 4096)
      throw Error{PMC_ERR_INVALID_ARG, "search_split_min must be at most 4096"};
    if (t->search_split_min) c.search_split_min = t->search_split_min;
    if (t->search_split_depth < 0 || t->search_split_depth > 8)
      throw Error{PMC_ERR_INVALID_ARG, "search_split_depth must be in [0, 8]"};
    if (t->search_split_depth) c.search_split_depth = t->search_split_depth;
    if (t->search_sweep_nodes) c.search_sweep_nodes = t->search_sweep_nodes;
    if (t->learned_min_open < 0)
      throw Error{PMC_ERR_INVALID_ARG, "learned_min_open must be >= 0"};
    if (t->learned_min_open) c.learned_min_open = t->learned_min_open;
    if (t->batch_peel != 0 && t->batch_peel != 1 && t->batch_peel != -1)
      throw Error{PMC_ERR_INVALID_ARG, "batch_peel must be 1, -1 or 0"};
    if (t->batch_peel) c.batch_peel = t->batch_peel;
    for (int i = 0; i < 2; i++) {
      if (t->heuristic_chunk[i] < 0 || t->heuristic_chunk[i] > 64)
        throw Error{PMC_ERR_INVALID_ARG, "heuristic_chunk must be in [0, 64]"};
      if (t->heuristic_chunk[i]) c.heuristic_chunk[i] = t->heuristic_chunk[i];
    }
    return c;
}
}  // namespace

extern "C" {

pmc_status pmc_strong_reachability(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                                   int64_t *offsets, int32_t *indices, int64_t capacity,
                                   int64_t *nnz, void *stream) {
  return guarded([&] {
    if (n < 0 || m < 0 || capacity < 0) throw Error{PMC_ERR_INVALID_ARG, "negative size"};
    if (n > 131072) throw Error{PMC_ERR_INVALID_ARG, "at most 131072 vertices"};
    if (!offsets || !nnz) throw Error{PMC_ERR_INVALID_ARG, "offsets and nnz are required"};
    if (m > 0 && (!src || !dst)) throw Error{PMC_ERR_INVALID_ARG, "src and dst are required"};
    if (capacity > 0 && !indices) throw Error{PMC_ERR_INVALID_ARG, "indices is NULL"};
    Scratch sc((hipStream_t)stream);
    *nnz = run_strong_reach(n, m, src, dst, offsets, indices, capacity, sc);
    if (*nnz > capacity)
      throw Error{PMC_ERR_CAPACITY, "indices capacity " + std::to_string(capacity) + " < " +
                                        std::to_string(*nnz)};
  });
}

pmc_status pmc_clique_order(const pmc_graph *g, int32_t *order, int64_t *block, int64_t *nblocks,
                            void *stream) {
  return guarded([&] {
    GraphView v = make_view(g);
    if (!nblocks) throw Error{PMC_ERR_INVALID_ARG, "nblocks is NULL"};
    if (v.n > 0 && (!order || !block)) throw Error{PMC_ERR_INVALID_ARG, "order and block are required"};
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(s);
    maybe_validate(g, v, sc);
    *nblocks = 0;
    if (v.n == 0) {
      if (block) PMC_HIP(hipMemsetAsync(block, 0, sizeof(int64_t), s));
      PMC_HIP(hipStreamSynchronize(s));
      return;
    }
    Pipeline p(v, sc);
    p.cores(nullptr, nullptr, nullptr, nullptr, true);
    *nblocks = run_clique_order(v, p.rank, p.kmax, order, block, sc);
  });
}

pmc_status pmc_vertex_features(const pmc_graph *g, float *features, void *stream) {
  return guarded([&] {
    GraphView v = make_view(g);
    if (!features && v.n > 0) throw Error{PMC_ERR_INVALID_ARG, "features is NULL"};
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(s);
    maybe_validate(g, v, sc);
    if (v.n == 0) return;
    Pipeline p(v, sc);
    p.cores(nullptr, nullptr, nullptr, nullptr, true);
    run_features(v, p.core, p.rank, p.order, p.kmax, features, sc);
    PMC_HIP(hipStreamSynchronize(s));
  });
}

pmc_status pmc_mlp_forward(const float *params, const float *features, int64_t n, float *score,
                           void *stream) {
  return guarded([&] {
    if (n < 0) throw Error{PMC_ERR_INVALID_ARG, "negative n"};
    if (n > 0 && (!params || !features || !score))
      throw Error{PMC_ERR_INVALID_ARG, "params, features and score are required"};
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(s);
    run_mlp_forward(params, features, n, score, sc);
    PMC_HIP(hipStreamSynchronize(s));
  });
}

pmc_status pmc_mlp_train_step(float *params, float *adam_m, float *adam_v, int64_t step, float lr,
                              const float *features, const float *label, int64_t n, float *loss,
                              float *grad, void *stream) {
  return guarded([&] {
    if (n < 1 || step < 1 || !(lr >= 0.f)) throw Error{PMC_ERR_INVALID_ARG, "bad n, step or lr"};
    if (!params || !features || !label || (lr > 0.f && (!adam_m || !adam_v)))
      throw Error{PMC_ERR_INVALID_ARG, "missing argument"};
    hipStream_t s = (hipStream_t)stream;
    Scratch sc(s);
    float l = run_mlp_train_step(params, adam_m, adam_v, step, lr, features, label, n, grad, sc);
    if (loss) *loss = l;
  });
}

}  // extern "C"
