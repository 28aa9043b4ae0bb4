// tuning.h -- process-wide launch parameters (set by the C ABI's
// pmc_set_tuning, chosen by the autotuner).  Used only inside csrc/.
#pragma once

namespace pmc {

struct Tuning {
  // workgroups (one wave each) per CU of the search kernel, per size class
  int search_blocks_per_cu[7] = {32, 32, 16, 16, 2, 2, 2};
  // heuristic waves per CU: one graph, batch
  int heuristic_waves_per_cu[2] = {4, 16};
  // 1: the search launches of a call are captured into one hipGraph
  int search_graph = 0;
  // heuristic seeds a wave claims (and tests lane-parallel) per atomic: one
  // graph, batch
  int heuristic_chunk[2] = {4, 64};
  // a branched root of at least this many vertices runs its level-0 branches
  // as separate tasks (first-level split); <= 0: off
  int search_split_min = 32;
  // deepest level whose branches are split up front: 1 splits the roots'
  // level-0 branches only; d > 1 lets a task at depth < d with at least
  // search_split_min vertices in P split its own branches again.  (Deeper
  // levels are also handed out on demand, whenever waves wait for tasks.)
  int search_split_depth = 1;
  // single graphs: Branch nodes per root in the sweep that first settles the
  // roots it can and publishes the cliques it finds; the roots it leaves open
  // are searched afterwards by decreasing colour bound.  <= 0: no sweep.
  int search_sweep_nodes = -1;
  // the learned order scores the roots the sweep leaves open only when at
  // least this many remain (fewer cannot repay the features of every vertex)
  int learned_min_open = 1024;
  // a batch whose graphs all have at most 32,768 vertices is peeled one
  // workgroup per graph (1) or as one union (-1)
  int batch_peel = 1;
};

// The launch parameters in effect for the calling thread: a call's own table
// (pmc_options.tune_table) while a TuningScope is alive, else the
// process-wide table.
const Tuning &tuning();
// The process-wide table (pmc_get_tuning / pmc_set_tuning).
Tuning &global_tuning();

// Makes `t` the calling thread's table until the scope ends (NULL: no change).
class TuningScope {
 public:
  explicit TuningScope(const Tuning *t);
  ~TuningScope();

 private:
  const Tuning *prev_;
};

}  // namespace pmc
