// graph.h -- host-side view of a device CSR graph and launcher declarations
// of the pipeline stages.  Used only inside csrc/.
#pragma once
#include <stdint.h>

#include <vector>

#include "runtime.h"

namespace pmc {

struct GraphView {
  int64_t n = 0, nnz = 0;
  const void *off = nullptr;
  int bits = 64;
  const int32_t *idx = nullptr;
};

#define PMC_DISPATCH_OFF(g, OffT, ...)                          \
  do {                                                          \
    if ((g).bits == 32) {                                       \
      using OffT = int32_t;                                     \
      __VA_ARGS__;                                              \
    } else {                                                    \
      using OffT = int64_t;                                     \
      __VA_ARGS__;                                              \
    }                                                           \
  } while (0)

// ---- graph contract check: returns 0 if valid, else a violation code.
// gid (optional): vertex -> graph of a batch; an edge between graphs is a
// violation (code 6).
int validate_graph(const GraphView &g, Scratch &sc, const int32_t *gid = nullptr);
void max_degree(const GraphView &g, int32_t *out, hipStream_t s);

// ---- k-core peel (level-synchronous) and degeneracy rank
struct PeelResult {
  int32_t kmax = 0, nrounds = 0;
  float ms = 0;
};
// timed = false: no events are created and PeelResult::ms stays 0.
PeelResult run_peel(const GraphView &g, int32_t *core, int32_t *rnd, Scratch &sc,
                    bool timed = true);
void run_rank(int64_t n, const int32_t *rnd, int32_t nrounds, int32_t *rank, int32_t *order,
              Scratch &sc);
// Per-graph peel of a batch (vbase: host, G+1 vertex offsets): every graph
// peeled alone, one workgroup each; rounds are numbered per graph, so the
// rank from run_rank orders each graph as its own peel does.  Applies when
// every graph has at most PEEL_GRAPH_MAX_N vertices (peel_graphs_fits).
// gkmax / grounds (optional) receive each graph's K and round count.
constexpr int64_t PEEL_GRAPH_MAX_N = 32768;
bool peel_graphs_fits(const std::vector<int64_t> &vbase);
PeelResult run_peel_graphs(const GraphView &g, const std::vector<int64_t> &vbase, int32_t *core,
                           int32_t *rnd, Scratch &sc, bool timed = true,
                           std::vector<int32_t> *gkmax = nullptr,
                           std::vector<int32_t> *grounds = nullptr);
// ---- shared clique state on the device
struct CliqueState {
  int32_t err;                   // nonzero: a kernel hit a capacity limit
  int32_t seed_next;             // heuristic seed counter
  int32_t budget_hit;
  int32_t pad;
  unsigned long long nodes;      // branch nodes expanded
  unsigned long long roots_branched;
  unsigned long long seeds_done; // heuristic seeds processed
};

// Per-graph state of a batch (a single graph is a batch of one).  A batch is
// the disjoint union of its graphs; gid maps a vertex to its graph.
//   bound[g]  size of graph g's best clique so far (monotone, device atomics)
//   packed[g] frozen-threshold heuristic winner, (size << 32) | seed rank
//   slots     per graph g, (kmax_g + 2) slots of kmax_g + 1 ids at
//             slots + slot_base[g]; slot s holds the clique that first raised
//             bound[g] to s (one writer per slot)
struct Bounds {
  int G = 1;
  const int32_t *gid = nullptr;  // NULL: one graph
  int32_t *bound = nullptr;
  unsigned long long *packed = nullptr;
  int32_t *slots = nullptr;
  const int64_t *slot_base = nullptr;
  const int32_t *slot_stride = nullptr;
};

__device__ __forceinline__ int graph_of(const int32_t *gid, int v) { return gid ? gid[v] : 0; }
__device__ __forceinline__ int32_t *slot_ptr(const Bounds &B, int g, int size) {
  return B.slots + B.slot_base[g] + (int64_t)size * B.slot_stride[g];
}

// ---- heuristic clique (Alg. 1)
// seed_order: NULL for decreasing rank, else the seeds (vertex ids) in
// visiting order.  Returns the device time of the heuristic kernel (ms).
float run_heuristic(const GraphView &g, const int32_t *core, const int32_t *rank,
                    const int32_t *order, const int32_t *seed_order, int32_t kmax,
                    int32_t frozen_tau, const Bounds &B, CliqueState *st, Scratch &sc);

// ---- pruning and orientation
// Survivors: vertices whose core is >= the bound of their graph.  They get
// labels 0..n'-1 in rank order; the oriented graph keeps, for each survivor,
// its higher-ranked neighbours as labels, rows sorted.  A single graph's
// survivors are a suffix of the ranks, so label = rank - r0 there.
struct Labels {
  int nn = 0;                       // survivors
  int32_t *vertex = nullptr;        // label -> vertex id
  int32_t *core = nullptr;          // label -> core number
  int32_t *gid = nullptr;           // label -> graph (NULL: one graph)
  int64_t *poff = nullptr;          // nn + 1
  int32_t *padj = nullptr;
  int64_t nnz = 0;
  int64_t deg_sum = 0;              // entries of the survivors' input rows
};
// Returns the labelled oriented graph (synchronises).  `bound` is per graph;
// vertices of rank below min_rank (roots already searched) are dropped too.
// native: the search order is the vertex ids instead of the degeneracy rank
// (labels in id order, rows keep the neighbours of larger id that survive,
// min_rank is a vertex id); core is then not monotone along a row.
Labels run_prune_orient(const GraphView &g, const int32_t *core, const int32_t *rank,
                        const int32_t *order, const int32_t *gid, const int32_t *bound,
                        int32_t kmax, Scratch &sc, float *ms_kernels = nullptr,
                        int64_t *poff_out = nullptr, int32_t *padj_out = nullptr,
                        int64_t capacity = -1, int32_t min_rank = 0, bool native = false);

// Clique-peeling order (Sec. 6.2): order[p] = vertex at position p, block[b]
// = first position of the b-th clique (block[nb] = n).  Returns nb.
int64_t run_clique_order(const GraphView &g, const int32_t *rank, int32_t kmax, int32_t *order,
                         int64_t *block, Scratch &sc);

// Strong-reachability graph of the temporal edges src[e] -> dst[e] (device,
// time order), Sec. 6.1: CSR into off[n+1] / adj (written when the entry count
// fits `capacity`).  Returns the entry count.
int64_t run_strong_reach(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                         int64_t *off, int32_t *adj, int64_t capacity, Scratch &sc);

// Device time between two events recorded around launches on one stream.
struct KTimer {
  hipStream_t s;
  hipEvent_t a, b;
  explicit KTimer(hipStream_t st);
  ~KTimer();
  void start();
  float stop();  // synchronises on the end event
};

}  // namespace pmc
