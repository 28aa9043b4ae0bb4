// search.h -- root queue and per-root branch-and-bound launchers.  Used only
// inside csrc/.
#pragma once
#include <stdint.h>

#include "graph.h"

namespace pmc {

// Size classes of subproblems: class c uses bitset rows of 2^c 64-bit words
// (up to 64 * 2^c vertices).  Class SEARCH_CLASSES means "too large";
// QCLASS_NONE marks vertices that are not roots.
constexpr int SEARCH_CLASSES = 7;
constexpr int QCLASS_NONE = SEARCH_CLASSES + 1;

struct QueueResult {
  int start[SEARCH_CLASSES + 1] = {0};
  int count[SEARCH_CLASSES + 1] = {0};
  int total = 0;
};

// Roots: labels i with oriented degree >= min_deg, grouped by class, each
// class in dispatch order (increasing label, or decreasing score when
// `score` is given).
QueueResult run_queue(int nn, int r0, const int64_t *poff, const int32_t *order, int min_deg,
                      const float *score, int32_t *queue, Scratch &sc);

struct SearchArgs {
  int nn = 0;             // labels in the oriented graph
  int r0 = 0;             // rank of label 0
  const int64_t *poff = nullptr;
  const int32_t *padj = nullptr;
  const int32_t *r0tab = nullptr;  // first rank with core >= c, c in [0, kmax+2)
  int kmax = 0;
  const int32_t *order = nullptr;  // rank -> vertex id
  CliqueState *st = nullptr;
  int32_t *slots = nullptr;
  int slot_stride = 0;
  int frozen_bound = -1;
  int use_nc = 1;
  int32_t *root_report = nullptr;
  long long node_budget = 0;
};

// Searches the roots queue[0..count) of one class.  Returns kernel ms.
float run_search_class(int cls, const SearchArgs &a, const int32_t *queue, int count, Scratch &sc);

}  // namespace pmc
