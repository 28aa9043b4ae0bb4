// graph.h -- host-side view of a device CSR graph and launcher declarations
// of the pipeline stages.  Used only inside csrc/.
#pragma once
#include <stdint.h>

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

// ---- graph contract check: returns 0 if valid, else a violation code
int validate_graph(const GraphView &g, Scratch &sc);

// ---- k-core peel (level-synchronous) and degeneracy rank
struct PeelResult {
  int32_t kmax = 0, nrounds = 0;
  float ms = 0;
};
PeelResult run_peel(const GraphView &g, int32_t *core, int32_t *rnd, Scratch &sc);
void run_rank(int64_t n, const int32_t *rnd, int32_t nrounds, int32_t *rank, int32_t *order,
              Scratch &sc);
// r0tab[c] = first rank whose core is >= c, for c in [0, kmax + 2]
void run_r0_table(int64_t n, const int32_t *core, const int32_t *order, int32_t kmax,
                  int32_t *r0tab, Scratch &sc);

// ---- shared clique state on the device
struct CliqueState {
  int32_t bound;                 // size of the best clique so far (monotone)
  int32_t err;                   // nonzero: a kernel hit a capacity limit
  unsigned long long best_packed;// frozen-threshold heuristic: (size << 32) | seed rank
  unsigned long long nodes;      // branch nodes expanded
  unsigned long long roots_branched;
  int32_t seed_next;             // heuristic seed counter
  int32_t budget_hit;
  unsigned long long seeds_done; // heuristic seeds processed
};

// ---- heuristic clique (Alg. 1)
// slots: (kmax + 2) x (kmax + 1) int32; slot s holds the clique that first
// raised the bound to s.  seed_order: NULL for decreasing rank, else the
// list of seeds (vertex ids) in visiting order.
// Returns the device time of the heuristic kernel (ms).
float run_heuristic(const GraphView &g, const int32_t *core, const int32_t *rank,
                    const int32_t *order, const int32_t *seed_order, int32_t kmax,
                    int32_t frozen_tau, CliqueState *st, int32_t *slots, Scratch &sc);

// ---- pruning and orientation: oriented lists of ranks >= r0, relabelled
// rank - r0, rows sorted.  Returns the entry count (synchronises).
int64_t run_prune_orient(const GraphView &g, const int32_t *rank, const int32_t *order,
                         int32_t r0, int64_t *poff, int32_t *padj, int64_t capacity,
                         int32_t kmax, Scratch &sc, float *ms_kernels = nullptr);

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
