/*
 * pmc.h -- C ABI of the MI355X (gfx950) exact maximum-clique library.
 *
 * Problem (paper: Rossi, Gleich, Gebremedhin, Patwary, "Parallel Maximum
 * Clique Algorithms with Applications to Network Analysis and Storage",
 * arXiv 1302.6256, Sec. 1 and Sec. 4): given a simple undirected graph
 * G = (V, E), find a clique (complete subgraph) of the largest size; omega(G)
 * is that size.
 *
 * Conventions shared by every entry point
 *  - Graphs are passed as a symmetric CSR in DEVICE memory: offsets[n+1]
 *    (32- or 64-bit, offsets[0] = 0, offsets[n] = nnz = 2|E|) and
 *    indices[nnz] (int32).  Rows are sorted ascending, contain no self-loop
 *    and no duplicate, every id is in [0, n), and (u,v) is stored iff (v,u)
 *    is.  n < 2^31.  With PMC_GRAPH_VALIDATE set the library checks all of
 *    this first (O(n + nnz log deg) on the GPU) and returns
 *    PMC_ERR_INVALID_GRAPH on a violation; without it a violating graph gives
 *    an undefined result (never an out-of-bounds access for ids in range).
 *    The paper's restriction to the largest strong component is NOT applied:
 *    results are over the whole input.
 *  - The caller owns every input and output buffer; the library never frees
 *    caller memory.  Scratch memory is allocated on the given stream
 *    (hipMallocAsync) and released before the call returns.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call is
 *    ordered on that stream and synchronises it before returning (host
 *    scalar outputs are written on return; device outputs are complete).
 *  - Vertex ids in outputs are the caller's original ids.
 *  - Errors: the return value is a pmc_status; pmc_last_error() gives a
 *    thread-local message for the last failing call.  No C++ exception
 *    crosses this boundary.
 */
#ifndef PMC_H
#define PMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PMC_OK = 0,
  PMC_ERR_INVALID_ARG = 1,   /* NULL pointer, negative size, bad option value */
  PMC_ERR_INVALID_GRAPH = 2, /* graph contract violated (only with PMC_GRAPH_VALIDATE) */
  PMC_ERR_CAPACITY = 3,      /* output capacity too small; sizes are still reported */
  PMC_ERR_OUT_OF_MEMORY = 4, /* scratch allocation failed; nothing leaked */
  PMC_ERR_DEVICE = 5,        /* a HIP runtime error */
  PMC_ERR_BUDGET = 6         /* node budget exhausted: best clique so far returned, not certified */
} pmc_status;

#define PMC_GRAPH_VALIDATE 1u

typedef struct {
  int64_t n;              /* vertices */
  int64_t nnz;            /* stored adjacency entries = offsets[n] = 2|E| */
  const void *offsets;    /* device, n+1 entries of offsets_bits bits */
  int32_t offsets_bits;   /* 32 or 64 */
  const int32_t *indices; /* device, nnz entries */
  uint32_t flags;         /* PMC_GRAPH_VALIDATE */
} pmc_graph;

struct pmc_tuning; /* launch parameters, declared below */

#define PMC_ORDER_CORE 0  /* the paper's degeneracy order (Sec. 4.3) */
#define PMC_ORDER_SCORE 1 /* dispatch by decreasing caller score; ties by degeneracy rank */

typedef struct {
  uint32_t struct_size;           /* sizeof(pmc_options) */
  int32_t order;                  /* PMC_ORDER_CORE | PMC_ORDER_SCORE */
  const float *score;             /* device, n floats (PMC_ORDER_SCORE); NaN/Inf rank last */
  int32_t use_neighborhood_cores; /* 1 (default): InitialBranch's neighbourhood-core test */
  int32_t rebuild_on_bound_gain;  /* 1 (default): re-prune the oriented graph between
                                     search waves once the bound has risen (Sec. 4.3) */
  int32_t frozen_threshold;       /* heuristic: -1 off; >= 0 fixed core threshold, every seed
                                     processed (deterministic per-seed cliques) */
  int32_t frozen_bound;           /* search: -1 off; >= 0 every root searched against this fixed
                                     bound with no sharing between roots */
  int32_t skip_heuristic;         /* 1: start the search from bound 0 (no heuristic) */
  int64_t node_budget;            /* 0: unlimited; else stop after about this many branch nodes */
  int32_t *root_report;           /* device, optional, 4*n int32 written in frozen-bound mode:
                                     per vertex id (s, K_N, L, omega_v), -1 where not reached */
  int32_t wave_roots;             /* labels per search wave between re-prunes; 0 = automatic
                                     (one graph: a quarter of the survivors, at least 2^18;
                                     a batch: one wave) */
  const float *mlp;               /* device, PMC_MLP_PARAMS floats, optional: the learned order.
                                     Once the heuristic has not certified omega, a single graph
                                     is first swept in degeneracy order (search_sweep_nodes, at
                                     least 64); if learned_min_open (1,024) or more roots are
                                     left open, every vertex
                                     is scored by the model (features + MLP on the GPU) and the
                                     open roots are dispatched by that score, else they are
                                     searched in degeneracy order.  A batch or a frozen-bound run
                                     is scored right after the heuristic (as PMC_ORDER_SCORE) */
  int32_t native_order;           /* 1: the "native order" variant of Sec. 5 -- roots are
                                     searched in vertex-id order and each root's reduced
                                     neighbourhood holds its neighbours of larger id (core >=
                                     bound); 0 (default): degeneracy order.  Without the
                                     degeneracy bound a subproblem can exceed 4096 vertices:
                                     the call then returns PMC_ERR_CAPACITY */
  const struct pmc_tuning *tune_table; /* host, optional: launch parameters for this call
                                     only (an entry of the autotuner's table; zero fields
                                     keep the process-wide values, see pmc_set_tuning);
                                     NULL: the process-wide table */
} pmc_options;

typedef struct {
  int32_t kmax;          /* largest core number K(G) */
  int32_t nrounds;       /* level-synchronous peel rounds (a batch peeled per graph: the
                            largest round count of its graphs) */
  int32_t heuristic;     /* heuristic clique size (omega~) */
  int32_t omega;         /* result */
  int32_t certified;     /* 1: omega proven (always, unless PMC_ERR_BUDGET) */
  int32_t certified_early; /* 1: omega~ = K+1, search skipped (Fact 1) */
  int64_t survivors;     /* vertices with K(v) >= omega~ */
  int64_t oriented_nnz;  /* entries of the pruned oriented graph */
  int64_t roots;         /* roots queued */
  int64_t roots_branched;/* roots that entered Branch */
  int64_t nodes;         /* Branch nodes expanded */
  int32_t rebuilds;      /* re-prunes between waves */
  int32_t search_graph_replays; /* search stages run by replaying the hipGraph kept from an
                            earlier call with identical launches (search_graph on) */
  float ms_peel, ms_rank, ms_heuristic, ms_prune, ms_queue, ms_search, ms_total;
  /* device time of the main kernels alone (HIP events on the call's stream
     around each launch): peel, heuristic, orientation (count + fill), and the
     search kernels summed over size classes */
  float ms_k_peel, ms_k_heuristic, ms_k_orient, ms_k_search;
  int64_t heuristic_seeds; /* seeds the heuristic processed */
  int64_t roots_second_pass; /* roots the sweep left open (search_sweep_nodes > 0) */
  float ms_sweep;          /* time of the sweep (part of ms_search) */
  int32_t learned_used;    /* 1: the learned model's scores ordered (some of) the search */
  /* algorithmic HBM rate of the streaming passes, bytes moved by the method
     over the kernel time (GB/s; 8 TB/s is the device's peak): the k-core
     peel, 8(n+1) + 24m + 12n bytes (offsets; each entry read once, one degree
     read-modify-write per entry; degree, core and round words; a batch peeled
     per graph: 24n + 8m, its degrees living in LDS), and the
     first pruning and orientation, 2(16 n' + 8 D) + 4 m' bytes (n'
     survivors, D their input row entries, m' oriented entries) */
  float gbps_peel, gbps_orient;
} pmc_stats;

/* k-core decomposition (Sec. 3; MaxClique's CoreNumbers step).
 * Level-synchronous peeling: at level k every remaining vertex of remaining
 * degree <= k is removed at once (one round); when none is left the level
 * jumps to the minimum remaining degree.
 * Outputs (device, n entries each, any may be NULL): core[v] = K(v);
 * round[v] = peel round; rank[v] = position in (round, id) order (a
 * degeneracy order, nondecreasing in K); order = inverse of rank.
 * Host outputs (may be NULL): *kmax = K(G), *nrounds. */
pmc_status pmc_core_numbers(const pmc_graph *g, int32_t *core, int32_t *round, int32_t *rank,
                            int32_t *order, int32_t *kmax, int32_t *nrounds, void *stream);

/* pmc_core_numbers for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, outputs and results as pmc_core_numbers; the
 * call allocates and frees nothing: its scratch is a fixed 256 MiB device
 * array that the library holds on every device it runs on until the process
 * ends, and no timing events are created.  A graph whose scratch could exceed
 * it returns PMC_ERR_CAPACITY before any work is queued (scratch bound:
 * 52 n + n/2 + 4 min(nnz, 2^24) bytes + 4 MiB, so up to about 3.5 million
 * vertices at any nnz).  Every call on a device shares that device's array
 * and it keeps the previous call's contents (the kernels initialise what they
 * read): calls that overlap on one device, on any streams or threads, race
 * and must not be issued. */
pmc_status pmc_core_numbers_noalloc(const pmc_graph *g, int32_t *core, int32_t *round,
                                    int32_t *rank, int32_t *order, int32_t *kmax,
                                    int32_t *nrounds, void *stream);

/* Greedy heuristic clique (Alg. 1, Sec. 4.1), seeds in decreasing
 * degeneracy rank, each seed's clique started from the seed itself.
 * core/rank/order: device outputs of pmc_core_numbers, or all NULL to compute
 * them here.  opt may be NULL (defaults; frozen_threshold and order/score
 * are read).  clique: device, capacity entries; receives the clique sorted
 * ascending.  *size (host) = its size; PMC_ERR_CAPACITY if capacity < size.
 * With PMC_ORDER_SCORE the seeds are visited by decreasing score instead. */
pmc_status pmc_heuristic(const pmc_graph *g, const int32_t *core, const int32_t *rank,
                         const int32_t *order, const pmc_options *opt, int32_t *clique,
                         int32_t capacity, int32_t *size, void *stream);

/* Explicit pruning and orientation (MaxClique's removal of K(v) < |H|,
 * Sec. 4.2, and the reduced neighbourhoods N_R of Sec. 4.3): for every
 * vertex of core >= bound, in rank order, the list of its higher-ranked
 * neighbours relabelled to rank - r0 (r0 = first rank with core >= bound),
 * sorted ascending.  poff: device, n+1 int64 (n - r0 + 1 written);
 * padj: device, capacity entries (nnz/2 always suffices).  Host outputs:
 * *r0, *out_nnz.  core/rank/order as from pmc_core_numbers (not NULL). */
pmc_status pmc_prune_orient(const pmc_graph *g, const int32_t *core, const int32_t *rank,
                            const int32_t *order, int32_t bound, int64_t *poff, int32_t *padj,
                            int64_t capacity, int32_t *r0, int64_t *out_nnz, void *stream);

/* Exact maximum clique (Alg. 2, Secs. 4.2-4.5).  opt may be NULL (defaults).
 * clique: device, capacity entries, receives one maximum clique sorted
 * ascending; *omega (host) its size.  capacity >= K(G)+1 always suffices
 * (Fact 1); if capacity < omega the call returns PMC_ERR_CAPACITY with
 * *omega set.  stats (host) optional.  n = 0 gives omega = 0; an edgeless
 * graph with n >= 1 gives omega = 1. */
pmc_status pmc_max_clique(const pmc_graph *g, const pmc_options *opt, int32_t *clique,
                          int32_t capacity, int32_t *omega, pmc_stats *stats, void *stream);

/* A batch: the disjoint union of `count` graphs in one CSR.  Graph g owns
 * the vertex ids [vertex_base[g], vertex_base[g+1]) and every edge stays inside
 * one graph (checked with PMC_GRAPH_VALIDATE).  offsets/indices follow the
 * pmc_graph conventions for the union; vertex_base is a HOST array of count+1
 * entries, vertex_base[0] = 0, vertex_base[count] = n. */
typedef struct {
  int64_t n;              /* vertices of the union */
  int64_t nnz;            /* stored entries of the union */
  const void *offsets;    /* device, n+1 entries of offsets_bits bits */
  int32_t offsets_bits;   /* 32 or 64 */
  const int32_t *indices; /* device, nnz entries (union ids) */
  int32_t count;          /* graphs in the batch */
  const int64_t *vertex_base; /* host, count+1 entries */
  uint32_t flags;         /* PMC_GRAPH_VALIDATE */
} pmc_batch;

/* Core numbers of every graph of a batch in one call (Sec. 3, applied to
 * each graph alone): each graph is peeled on its own, one workgroup per
 * graph, so core and round are exactly what pmc_core_numbers gives for that
 * graph by itself (rounds numbered from 0 in every graph).  rank/order are
 * over the union: the position in (round, id) order, which within each graph
 * is that graph's own degeneracy order.  Outputs (device, union-sized, may be
 * NULL): core, round, rank, order; host (count entries each, may be NULL):
 * kmax[g] = K(G_g), nrounds[g].  Every graph must have at most 32,768
 * vertices (its degrees and queue live in LDS), else PMC_ERR_CAPACITY before
 * any work is queued.  The batch follows pmc_max_clique_batch's conventions
 * (PMC_GRAPH_VALIDATE checks every graph and that no edge leaves its graph). */
pmc_status pmc_core_numbers_batch(const pmc_batch *b, int32_t *core, int32_t *round,
                                  int32_t *rank, int32_t *order, int32_t *kmax, int32_t *nrounds,
                                  void *stream);

/* Exact maximum clique of every graph of a batch in one pass of the pipeline
 * (Alg. 2 per graph; Sec. 4.5's task queue becomes one device queue of
 * (graph, root) work with a bound per graph).  cliques: device, n entries;
 * graph g's maximum clique is written sorted ascending at
 * cliques[vertex_base[g] .. vertex_base[g] + omegas[g]) (its id range always
 * has room).  omegas: host, count entries.  opt as for pmc_max_clique
 * (frozen_bound applies to every graph; root_report is indexed by union id).
 * stats (host, optional) aggregates the batch; stats->omega is the largest
 * omega. */
pmc_status pmc_max_clique_batch(const pmc_batch *b, const pmc_options *opt, int32_t *cliques,
                                int32_t *omegas, pmc_stats *stats, void *stream);

/* The same batch given as `count` separate graphs (graphs[g] each with its
 * own device CSR, 32- or 64-bit offsets, ids local to the graph).  The
 * library builds their disjoint union on the device and solves it as
 * pmc_max_clique_batch does.  clique_offsets (host, count+1 entries,
 * nondecreasing): graph g's maximum clique is written, sorted ascending in
 * its own ids, to cliques[clique_offsets[g] .. clique_offsets[g] + omegas[g])
 * (cliques: device); room for n_g, or for K(G_g)+1 (Fact 1), always
 * suffices, and a graph with less room than its omega gives
 * PMC_ERR_CAPACITY.  omegas: host, count entries.  With PMC_GRAPH_VALIDATE
 * on any graph every graph is checked.  At most 2^31 - 1 vertices in all. */
pmc_status pmc_max_clique_graphs(const pmc_graph *graphs, int32_t count, const pmc_options *opt,
                                 int32_t *cliques, const int64_t *clique_offsets, int32_t *omegas,
                                 pmc_stats *stats, void *stream);

/* Strong-reachability graph of a temporal network (Sec. 6.1: the largest
 * temporal strong component is the maximum clique of this graph).  Temporal
 * edges src[e] -> dst[e], e < m (device int32, vertex ids in [0, n)), are
 * given in time order; a temporal path uses edges in increasing position of
 * that order (increasing times; equal times are ordered by position).  Two
 * vertices are joined when each has a temporal path to the other.  Outputs
 * (device): offsets[n+1] (int64) and indices[capacity] (int32, rows sorted
 * ascending, symmetric, no self-loops); *nnz (host) = entries needed; when
 * nnz > capacity the indices are not written and PMC_ERR_CAPACITY is
 * returned.  n <= 131,072 (the reachability bit matrix and its transpose take
 * n^2/4 bytes).  Pass the result to pmc_max_clique. */
pmc_status pmc_strong_reachability(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                                   int64_t *offsets, int32_t *indices, int64_t capacity,
                                   int64_t *nnz, void *stream);

/* Clique-peeling vertex order for compression (Sec. 6.2: remove large
 * heuristic cliques one after another and number their vertices
 * consecutively).  In each pass every remaining vertex v grows its greedy
 * clique H(v) (v, then first fit over its remaining neighbours in decreasing
 * degeneracy rank, as Alg. 1 with C = {v}); every clique whose key
 * (|H(v)|, rank(v)) is the largest among the cliques sharing one of its
 * vertices is taken (the pass's largest clique always is; taken cliques are
 * disjoint), placed by decreasing key, its vertices by decreasing degree (ties
 * by id), and removed.  Outputs (device): order[p] = vertex at position p
 * (n entries), block[b] = first position of clique b, block[nb] = n (n+1
 * entries); *nblocks (host) = nb.  Deterministic. */
pmc_status pmc_clique_order(const pmc_graph *g, int32_t *order, int64_t *block, int64_t *nblocks,
                            void *stream);

/* ---- Learned vertex ordering (an extension: it reorders the heuristic's
 * seeds and the search's roots and never changes omega). */
#define PMC_MLP_PARAMS 4801 /* W1 (8x64, W1[k][j] row-major), b1 (64), W2 (64x64), b2 (64),
                               w3 (64), b3 (1): fp32 master weights, one flat array */

/* Eight features per vertex, row-major n x 8 floats (device): log1p(deg),
 * log1p(core), core/K, log1p(triangles), mean/max/min neighbour core over K,
 * fraction of neighbours with core >= own (K = largest core, at least 1). */
pmc_status pmc_vertex_features(const pmc_graph *g, float *features, void *stream);

/* score[i] = MLP(features[i]) for i < n: relu(relu(x W1 + b1) W2 + b2) w3 + b3
 * with bf16 operands and fp32 accumulation.  All pointers device. */
pmc_status pmc_mlp_forward(const float *params, const float *features, int64_t n, float *score,
                           void *stream);

/* One full-batch training step on mean((score - label)^2): hand-written
 * backward kernels, then Adam (beta 0.9/0.999, eps 1e-8, bias-corrected with
 * `step` >= 1) on the fp32 params when lr > 0.  params, adam_m, adam_v:
 * device, PMC_MLP_PARAMS floats each, updated in place.  *loss (host) = the
 * loss before the step; grad (device, optional) receives the gradient. */
pmc_status pmc_mlp_train_step(float *params, float *adam_m, float *adam_v, int64_t step, float lr,
                              const float *features, const float *label, int64_t n, float *loss,
                              float *grad, void *stream);

/* ---- Launch tuning (process-wide; chosen by the autotuner,
 * paper_1302_6256_amd/tune.py).  Zero fields keep the default. */
typedef struct pmc_tuning {
  uint32_t struct_size;            /* sizeof(pmc_tuning) */
  int32_t search_blocks_per_cu[7]; /* search workgroups (one wave) per CU, per bitset class
                                      (64, 128, ..., 4096 vertices); default 32,32,16,16,2,2,2 */
  int32_t heuristic_waves_per_cu[2]; /* heuristic waves per CU for one graph and for a
                                        batch; default 4, 16 */
  int32_t search_graph;            /* 1: a call's search launches run as one captured hipGraph,
                                      kept per stream and replayed by later calls whose
                                      launches are identical; -1: off; 0 keeps the current
                                      value */
  int32_t heuristic_chunk[2];      /* heuristic seeds claimed per wave at once, 1..64, for one
                                      graph and for a batch; default 4, 64 (one graph: at most
                                      n / (64 x heuristic waves), so small graphs claim one) */
  int32_t search_split_min;        /* a root that reaches Branch with at least this many
                                      vertices runs each level-0 branch as its own task on
                                      another wave (first-level split), and a running Branch
                                      hands the untaken branches of its shallowest open level
                                      to waves that wait for tasks; default 32; < 0: both off */
  int32_t search_split_depth;      /* split tasks at depth < this whose P still holds at least
                                      search_split_min vertices split their own branches
                                      again; 1..8, default 1 (the roots' level-0 branches
                                      only); 0 keeps the current value */
  int32_t search_sweep_nodes;      /* single graphs: the search first sweeps every root
                                      (InitialBranch's bounds, then at most this many Branch
                                      nodes, publishing what it finds), then searches the
                                      roots it left open in degeneracy order; < 0: off (one
                                      pass in degeneracy order); 0 keeps the default */
  int32_t learned_min_open;        /* the learned order scores the roots the sweep leaves open
                                      only when at least this many remain; default 1024; 0
                                      keeps the current value */
  int32_t batch_peel;              /* 1: a batch whose graphs all have at most 32,768 vertices
                                      is peeled one workgroup per graph (each graph's own
                                      rounds); -1: as one union graph; 0 keeps the current
                                      value */
} pmc_tuning;
pmc_status pmc_get_tuning(pmc_tuning *t);
/* NULL restores the defaults; not thread-safe against concurrent solves. */
pmc_status pmc_set_tuning(const pmc_tuning *t);

/* Default option values (struct_size set). */
void pmc_default_options(pmc_options *opt);

const char *pmc_status_string(pmc_status s);
const char *pmc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PMC_H */
