// search.h -- root queue and per-root branch-and-bound launchers.  Used only
// inside csrc/.
#pragma once
#include <stdint.h>

#include <climits>

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

// Roots: labels i in [lab_lo, lab_hi) with oriented degree >= the bound of
// their graph (or all such labels when `all`), grouped by class, each class in
// dispatch order (increasing label, or decreasing score when `score` is
// given).
// vdone (optional, per vertex): vertices marked 1 are not roots (and sort
// last by score); a label taken that is too small to be a root gets marked.
// pos_hi: only the first pos_hi positions of the dispatch order are taken.
// desc (no score, pos_hi unused): each class in decreasing label order.
QueueResult run_queue(const Labels &L, const int32_t *bound, bool all, const float *score,
                      int32_t *queue, Scratch &sc, int lab_lo = 0, int lab_hi = INT_MAX,
                      int32_t *vdone = nullptr, int pos_hi = INT_MAX, bool desc = false);

struct SearchArgs {
  Labels L;
  int kmax = 0;
  Bounds B;
  CliqueState *st = nullptr;
  int frozen_bound = -1;
  int use_nc = 1;
  int32_t *root_report = nullptr;
  long long node_budget = 0;
  // first-level split pool (allocated once per call by alloc_split; NULL: the
  // launchers allocate it on first use)
  uint64_t *spool = nullptr;
  unsigned long long *spool_used = nullptr;
  unsigned long long *tasks = nullptr;
  int *task_tail = nullptr;
  // sweep pass (sweep_cap > 0 Branch nodes per root): per vertex, vdone = 1
  // once the root is settled, else sweep_key = its colour bound
  long long sweep_cap = 0;
  float *sweep_key = nullptr;
  int32_t *vdone = nullptr;
  // labels follow vertex ids (the native order), not the degeneracy rank
  bool native = false;
};

// Allocates the first-level split pool into `a` when splitting is enabled.
void alloc_split(SearchArgs &a, Scratch &sc);

// Searches the roots queue[0..count) of one class.  Returns kernel ms.
float run_search_class(int cls, const SearchArgs &a, const int32_t *queue, int count, Scratch &sc);
// Searches every class of the queue: one persistent launch per non-empty class
// over the global (graph, root) queue of that class, optionally captured into
// one hipGraph (tuning().search_graph), kept per (device, stream) and
// replayed while the launches stay identical (`replays`, if given, counts the
// replays).  Classes run smallest first, or largest first when
// `largest_first`.  Returns the device ms of the stage.
float run_search(const SearchArgs &a, const int32_t *queue, const QueueResult &q, Scratch &sc,
                 bool largest_first = false, int32_t *replays = nullptr);

}  // namespace pmc
