// search.hip -- per-root branch and bound (InitialBranch and Branch of Alg. 2,
// Secs. 4.3-4.5 of the paper) with the shared bound of the parallel search.
//
// Work unit: one root, the label i of the oriented graph.  Its subproblem is
// P = N+(i) restricted to labels whose core is >= the current bound (the
// reduced neighbourhood: lower-ranked, already searched vertices and vertices
// removed by the core bound are excluded), with the root itself as the first
// clique member C = {i}.  (The paper states InitialBranch on the closed set
// {i} + P and Branch({}, P); keeping the root in C and P open is the same
// search with every size shifted by one: a vertex adjacent to all of P
// raises every core number and the colour count by exactly one.)
//
// Steps per root, with b the current bound (size of the best clique):
//   size test        |P| + 1 <= b                      -> done
//   neighbourhood cores K_N of G[P] (level-synchronous peel on bitsets)
//   core test        max K_N + 2 <= b                  -> done
//   drop             x with K_N(x) + 1 < b
//   colouring        greedy, in reverse local peel order (a degeneracy
//                    order, so at most max K_N + 1 colours)
//   colouring test   L + 1 <= b                        -> done
//   Branch           depth-first over P in decreasing colour order; a child
//                    P' = P & row(u) is coloured greedily in decreasing local
//                    index (class by class, bit-parallel) and entered only if
//                    |C'| + L(P') > b; an empty P' with |C'| > b is a new
//                    clique.  A branch vertex whose colour c has |C| + c <= b
//                    ends its level (every later one has a colour <= c).
//   publish          atomicMax on the shared bound of the root's graph; the
//                    wave that raised it to s writes its clique to slot s.
//                    Raising the bound also removes, implicitly, every vertex
//                    of core < bound from the remaining subproblems: along a
//                    sorted row the core is nondecreasing (rank order), so the
//                    removed vertices are always a prefix of P.
//
// GPU mapping: one wavefront (a 64-thread workgroup) per root, roots claimed
// from the class's queue by a device counter (a persistent grid; a wave of a
// class of many small roots claims several at once), the 64- and 128-vertex
// classes in one launch when the smaller holds only a few roots per wave.  The
// subproblem's adjacency is an s x W-word bitset matrix in LDS (W = 1..8
// words) or in a per-wave global buffer (W = 16..64); lane j owns word j of a
// bitset, so an AND, a ballot and a popcount act on the whole set.  The DFS
// stack (P and the colour-ordered branch list of every level) lives in a
// per-wave global slab.  The shared bound is polled with relaxed loads at
// every node.
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "common.h"
#include "search.h"
#include "tuning.h"

namespace pmc {
namespace {

struct KArgs {
  int nn;
  const int64_t *poff;
  const int32_t *padj;
  const int32_t *lab_core;    // label -> core number
  const int32_t *lab_gid;     // label -> graph (NULL: one graph)
  const int32_t *lab_vertex;  // label -> vertex id
  int kmax;
  Bounds B;
  CliqueState *st;
  int frozen_bound;
  int use_nc;
  int32_t *root_report;
  long long node_budget;
  const int32_t *queue;
  int count;
  int *qhead;
  int claim;  // most roots per queue claim
  uint64_t *slab;
  long long slab_words;
  int levels;
  int level_words;
  uint64_t *grows;
  // split of big subproblems: a branched root of at least split_min vertices
  // writes a record (its matrix, P, level-0 branch list) to spool and one
  // task per level-0 branch vertex; waves that run out of roots run the
  // tasks.  A task at depth d < split_depth whose P still holds split_min
  // vertices splits its own branch list the same way (a record with the
  // path, P and the list; labels and matrix stay in the root's record).
  // split_min 0: off.
  int split_min;
  int split_depth;
  uint64_t *spool;
  long long spool_words;
  unsigned long long *spool_used;
  unsigned long long *tasks;  // slot value: (record offset << 16 | branch index) + 1; 0 = empty
  int task_cap;
  int *task_tail;   // slots reserved
  int *task_head;   // slots claimed
  int *waves_done;  // waves past their roots
  int *task_pend;   // tasks reserved and not yet finished
  // sweep (first pass over all roots): InitialBranch's bounds for every root
  // and at most sweep_cap Branch nodes each.  A root that this settles
  // (pruned by a test, or its Branch finished) gets vdone[vertex] = 1; any
  // other keeps vdone = 0 and sweep_key[vertex] = its colour bound L for the
  // second pass.  sweep_cap 0: an ordinary search.
  long long sweep_cap;
  float *sweep_key;
  int32_t *vdone;
  // labels and local indices follow vertex ids (the native order) rather
  // than the degeneracy rank: the core is not monotone along a row
  int native;
};

template <int W>
__host__ __device__ constexpr int smax() { return 64 * W; }

template <int W, bool RL>
__host__ __device__ constexpr size_t lds_bytes() {
  return (RL ? (size_t)smax<W>() * W * 8 : 0) + ((size_t)8 * smax<W>() + 2) * 4 + (size_t)5 * W * 8;
}

// First position in the sorted label list a[0..len) whose core is >= b.
// Within one graph the core is nondecreasing along labels (rank order), so
// the vertices removed by a bound b are always a prefix.
__device__ __forceinline__ int core_cut(const int32_t *a, int len, const int32_t *lab_core, int b) {
  int lo = 0, hi = len;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (lab_core[a[mid]] < b) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Mask of word j keeping local indices >= cut.
__device__ __forceinline__ uint64_t keep_mask(int j, int cut) {
  int lo = j * 64;
  if (cut <= lo) return ~0ull;
  if (cut >= lo + 64) return 0ull;
  return ~0ull << (cut - lo);
}

// This lane's word of the set of local vertices whose core is >= b (lane j
// < W holds word j): the vertices a bound b has not removed.  In degeneracy
// order they are a suffix of P (one binary search); in native order each
// lane tests its 64 vertices.
template <int W>
__device__ __forceinline__ uint64_t core_keep(const KArgs &a, const int *plist, int s, int b) {
  const int l = lane();
  if (!a.native) return l < W ? keep_mask(l, core_cut(plist, s, a.lab_core, b)) : 0ull;
  uint64_t m = 0ull;
  if (l < W)
    for (int t = 0; t < 64; t++) {
      const int x = l * 64 + t;
      if (x < s && a.lab_core[plist[x]] >= b) m |= 1ull << t;
    }
  return m;
}

// Greedy colouring of the set U (lane j < W holds word j) in decreasing local
// index, i.e. decreasing degeneracy rank (the highest-ranked vertices first),
// one colour class at a time: class c is built by repeatedly taking the
// highest uncoloured vertex still allowed and removing its neighbours
// (identical to first-fit colouring in that order).  Vertices of colour >
// kmin are appended to `list` as (colour << 16 | vertex), ascending colour
// and, within a colour, descending index.  Returns the number of colours;
// *cnt receives the list length.
template <int W>
__device__ __forceinline__ int colour_classes(uint64_t Uj, const uint64_t *rows, int kmin, uint32_t *list,
                              int *cnt) {
  const int l = lane();
  int c = 0, n = 0;
  while (ballot(Uj != 0)) {
    c++;
    uint64_t Qj = Uj;
    while (true) {
      uint64_t nz = ballot(Qj != 0);
      if (!nz) break;
      int jj = 63 - __clzll((long long)nz);
      uint64_t qw = shfl64(Qj, jj);
      int bit = 63 - __clzll((long long)qw);
      int x = jj * 64 + bit;
      uint64_t rx = l < W ? rows[(size_t)x * W + l] : 0ull;
      Qj &= ~rx;
      if (l == jj) {
        uint64_t m = ~(1ull << bit);
        Qj &= m;
        Uj &= m;
      }
      if (c > kmin) {
        if (l == 0) list[n] = ((uint32_t)c << 16) | (uint32_t)x;
        n++;
      }
    }
  }
  *cnt = n;
  return c;
}

// Reserves `words` of the split pool and `ntasks` task slots (lane 0 does the
// claims, the result is broadcast) and counts the tasks as pending before
// any of them can be claimed.  false: either does not fit, nothing reserved
// but possibly pool words (the pool only grows within a launch).
__device__ __forceinline__ bool reserve_split(const KArgs &a, long long words, int ntasks, long long &off,
                              int &t0) {
  const int l = lane();
  off = -1;
  t0 = -1;
  if (l == 0) {
    unsigned long long used =
        __hip_atomic_load(a.spool_used, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (used + (unsigned long long)words <= (unsigned long long)a.spool_words) {
      if (__hip_atomic_compare_exchange_strong(a.spool_used, &used, used + words, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        off = (long long)used;
        break;
      }
    }
    if (off >= 0) {
      int tt = ld_relaxed(a.task_tail);
      while (tt + ntasks <= a.task_cap) {
        if (__hip_atomic_compare_exchange_strong(a.task_tail, &tt, tt + ntasks, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          t0 = tt;
          break;
        }
      }
      if (t0 >= 0) atomic_add(a.task_pend, ntasks);
    }
  }
  off = (long long)shfl64((uint64_t)off, 0);
  t0 = shfl(t0, 0);
  return t0 >= 0;
}

// Publishes the tasks of a written record: one slot per branch index.
__device__ __forceinline__ void post_tasks(const KArgs &a, long long off, int t0, int ntasks) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // the record before its tasks
  for (int i = lane(); i < ntasks; i += PMC_WAVE)
    __hip_atomic_store(&a.tasks[t0 + i], (((unsigned long long)off << 16) | (unsigned long long)i) + 1ull,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Split records.  Header words: [1] s, [2] branch list length, [3] root core,
// [4] graph, [5] root vertex, [6] depth d (branch vertices chosen before the
// list), [7] offset of the root's depth-0 record.  Then P at that depth (W
// words), the chosen local vertices Cl[0..d) (int32, two per word), the
// branch list (uint32 colour << 16 | local index, two per word); a record
// that is its own base ([7] = its offset) continues with the labels (s int32)
// and the bitset matrix (s x W), which the records based on it share.
template <int W>
__device__ __forceinline__ void write_header(uint64_t *rec, int root, int s, int nb, int croot,
                                             int gr, int vroot, int d, long long base) {
  if (lane() == 0) {
    rec[0] = (uint64_t)root;
    rec[1] = (uint64_t)s;
    rec[2] = (uint64_t)nb;
    rec[3] = (uint64_t)croot;
    rec[4] = (uint64_t)gr;
    rec[5] = (uint64_t)vroot;
    rec[6] = (uint64_t)d;
    rec[7] = (uint64_t)base;
  }
}

// Work donation: level j of a running Branch (path Cl[0..j), P at level j
// without the branch vertices already taken, the untaken rest of its branch
// list) becomes a record with one task per untaken branch vertex, and the
// level is emptied so its owner moves on.  The first donation of a Branch
// that has no base record yet writes one (labels and matrix); later ones
// share it.  false: the pool or the task slots are full (nothing changes).
template <int W>
__device__ __forceinline__ bool donate_level(const KArgs &a, uint64_t *lv, int j, const int *Cl, int s, int croot,
                             int gr, int vroot, const int *plist, const uint64_t *rows,
                             long long &base_off) {
  const int l = lane();
  const int cnt = (int)lv[W];
  const bool self = base_off < 0;
  const long long words = 8 + W + (j + 1) / 2 + (cnt + 1) / 2 +
                          (self ? (s + 1) / 2 + (long long)s * W : 0ll);
  long long off;
  int t0;
  if (!reserve_split(a, words, cnt, off, t0)) return false;
  uint64_t *rec = a.spool + off;
  write_header<W>(rec, -1, s, cnt, croot, gr, vroot, j, self ? off : base_off);
  if (l < W) rec[8 + l] = lv[l];
  int *path = (int *)(rec + 8 + W);
  for (int i = l; i < j; i += PMC_WAVE) path[i] = Cl[i];
  uint32_t *lst = (uint32_t *)(rec + 8 + W + (j + 1) / 2);
  const uint32_t *src = (const uint32_t *)(lv + W + 1);
  for (int i = l; i < cnt; i += PMC_WAVE) lst[i] = src[i];
  if (self) {
    int *pl = (int *)(rec + 8 + W + (j + 1) / 2 + (cnt + 1) / 2);
    for (int i = l; i < s; i += PMC_WAVE) pl[i] = plist[i];
    uint64_t *rw = rec + 8 + W + (j + 1) / 2 + (cnt + 1) / 2 + (s + 1) / 2;
    for (int i = l; i < s * W; i += PMC_WAVE) rw[i] = rows[i];
    base_off = off;
  }
  post_tasks(a, off, t0, cnt);
  if (l == 0) lv[W] = 0ull;
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  wave_sync();
  return true;
}

// Node budget: each wave adds its branch-node count to the shared total every
// PUB_STEP nodes (and the rest when it ends), so the budget sees the work of
// every wave in flight, overshooting by less than PUB_STEP nodes per wave.
// Returns true (and raises budget_hit) once the total reaches the budget.
constexpr unsigned long long PUB_STEP = 1ull << 10;
__device__ __forceinline__ bool publish_nodes(const KArgs &a, unsigned long long delta) {
  int hit = 0;
  if (lane() == 0) {
    unsigned long long old = atomic_add_u64(&a.st->nodes, delta);
    hit = (long long)(old + delta) >= a.node_budget;
    if (hit) atomicExch(&a.st->budget_hit, 1);
  }
  return shfl(hit, 0) != 0;
}

// Branch (depth first) from level dmin of `slab` (C = the root plus Cl[0..dmin)
// and the vertices taken on the way): pop the branch vertex of largest
// colour, skip it and the rest of its level when |C| + colour <= b or
// |C| + |P| <= b, else take it and recurse on P & N(x) coloured greedily in
// increasing local index; an empty P' with |C'| > b is a new clique.  Returns
// when the levels are exhausted, the root's core falls below the bound, or a
// capacity or node budget is hit; returns true only when it stopped after
// `cap` nodes (cap > 0) with levels left.
template <int W>
__device__ __forceinline__ bool branch_dfs(const KArgs &a, uint64_t *slab, const uint64_t *rows,
                                           const int *plist, int *Cl, int s, int dmin, int &b,
                                           int &best, int croot, int *gbound, int gr, int vroot,
                                           unsigned long long &nodes,
                                           unsigned long long nodes_total,
                                           unsigned long long &pub, long long &base_off,
                                           unsigned long long cap = 0) {
  const int l = lane();
  const bool frozen = a.frozen_bound >= 0;
  const int LW = a.level_words;
  uint64_t cm = core_keep<W>(a, plist, s, b);  // local vertices of core >= b
  int d = dmin;
  unsigned tick = 0;
  while (d >= dmin) {
    // waves waiting for tasks (claims past the reserved slots): hand them the
    // shallowest level that still has untaken branch vertices
    if (a.split_min > 0 && (++tick & 31u) == 0u) {
      int hungry = 0;
      if (l == 0) hungry = ld_relaxed(a.task_head) > ld_relaxed(a.task_tail);
      if (shfl(hungry, 0)) {
        int j = dmin;
        while (j <= d && slab[(size_t)j * LW + W] == 0ull) j++;
        if (j <= d)
          donate_level<W>(a, slab + (size_t)j * LW, j, Cl, s, croot, gr, vroot, plist, rows,
                          base_off);
      }
    }
    if (!frozen) {
      int bn = ld_relaxed(gbound);
      if (bn > b) {
        b = bn;
        if (croot < b) return false;
        cm = core_keep<W>(a, plist, s, b);
      }
    }
    uint64_t *lv = slab + (size_t)d * LW;
    uint32_t *lst = (uint32_t *)(lv + W + 1);
    int cnt = (int)lv[W];
    if (cnt == 0) { d--; continue; }
    if (cap > 0 && nodes >= cap) return true;
    uint32_t e = lst[cnt - 1];
    int x = (int)(e & 0xffffu), cx = (int)(e >> 16);
    int csz = d + 1;
    if (csz + cx <= b) { d--; continue; }  // colour cut-off
    uint64_t Pj = l < W ? lv[l] : 0ull;
    int psz = wave_sum(__popcll(Pj));
    if (csz + psz <= b) { d--; continue; }  // |C| + |P| <= b
    // take x: remove it from P, recurse on P & N(x)
    if (l == (x >> 6)) Pj &= ~(1ull << (x & 63));
    if (l < W) lv[l] = Pj;
    if (l == 0) {
      lv[W] = (uint64_t)(cnt - 1);
      Cl[d] = x;
    }
    nodes++;
    if (a.node_budget > 0 && nodes_total + nodes - pub >= PUB_STEP) {
      const unsigned long long delta = nodes_total + nodes - pub;
      pub = nodes_total + nodes;
      if (publish_nodes(a, delta)) return false;
    }
    uint64_t Pn = l < W ? (Pj & rows[(size_t)x * W + l] & cm) : 0ull;
    if (!ballot(Pn != 0ull)) {
      int size = csz + 1;
      if (size > b) {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        wave_sync();
        int old = 0;
        if (l == 0) old = atomic_max(gbound, size);
        old = shfl(old, 0);
        if (old < size) {
          int32_t *dst = slot_ptr(a.B, gr, size);
          for (int q = l; q < size; q += PMC_WAVE)
            dst[q] = q == 0 ? vroot : a.lab_vertex[plist[Cl[q - 1]]];
        }
        b = size;
        best = max(best, size);
        if (croot < b) return false;
        cm = core_keep<W>(a, plist, s, b);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
      continue;
    }
    if (d + 1 >= a.levels) {
      if (l == 0) atomicExch(&a.st->err, 3);
      return false;
    }
    uint64_t *nl = slab + (size_t)(d + 1) * LW;
    uint32_t *nlst = (uint32_t *)(nl + W + 1);
    int ncnt = 0;
    int kmin = b - (csz + 1);
    int Lc = colour_classes<W>(Pn, rows, kmin, nlst, &ncnt);
    (void)Lc;
    if (ncnt > 0) {
      if (l < W) nl[l] = Pn;
      if (l == 0) nl[W] = (uint64_t)ncnt;
      d++;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    wave_sync();
  }
  return false;
}

// Split of a branched root: a depth-0 record and one task per level-0 branch
// vertex.  Returns false (nothing written) when the pool or the task slots
// are full; the root then runs its own Branch.
template <int W>
__device__ __forceinline__ bool emit_split(const KArgs &a, int root, int s, int n0, int croot, int gr, int vroot,
                           const uint64_t *P0, const uint32_t *list0, const int *plist,
                           const uint64_t *rows) {
  const int l = lane();
  const long long words = 8 + W + (n0 + 1) / 2 + (s + 1) / 2 + (long long)s * W;
  long long off;
  int t0;
  if (!reserve_split(a, words, n0, off, t0)) return false;
  uint64_t *rec = a.spool + off;
  write_header<W>(rec, root, s, n0, croot, gr, vroot, 0, off);
  if (l < W) rec[8 + l] = P0[l];
  uint32_t *lst = (uint32_t *)(rec + 8 + W);
  for (int i = l; i < n0; i += PMC_WAVE) lst[i] = list0[i];
  int *pl = (int *)(rec + 8 + W + (n0 + 1) / 2);
  for (int i = l; i < s; i += PMC_WAVE) pl[i] = plist[i];
  uint64_t *rw = rec + 8 + W + (n0 + 1) / 2 + (s + 1) / 2;
  for (int i = l; i < s * W; i += PMC_WAVE) rw[i] = rows[i];
  post_tasks(a, off, t0, n0);
  return true;
}

// Split of a task's subproblem at depth d >= 1 (the path Cl[0..d), P and
// its branch list at that depth): a record without labels or matrix.
template <int W>
__device__ __forceinline__ bool emit_deeper(const KArgs &a, const uint64_t *parent, int d, const int *Cl,
                            const uint64_t *P, const uint32_t *list, int nb) {
  const int l = lane();
  const long long words = 8 + W + (d + 1) / 2 + (nb + 1) / 2;
  long long off;
  int t0;
  if (!reserve_split(a, words, nb, off, t0)) return false;
  uint64_t *rec = a.spool + off;
  write_header<W>(rec, (int)parent[0], (int)parent[1], nb, (int)parent[3], (int)parent[4],
                  (int)parent[5], d, (long long)parent[7]);
  if (l < W) rec[8 + l] = P[l];
  int *path = (int *)(rec + 8 + W);
  for (int i = l; i < d; i += PMC_WAVE) path[i] = Cl[i];
  uint32_t *lst = (uint32_t *)(rec + 8 + W + (d + 1) / 2);
  for (int i = l; i < nb; i += PMC_WAVE) lst[i] = list[i];
  post_tasks(a, off, t0, nb);
  return true;
}

// One split task: branch vertex ci of a record at depth d.  P at that depth
// loses the branch vertices after ci in the list (they were taken, and
// removed, before it in the sequential Branch); x = the list's entry ci is
// taken, P' = P & N(x) is coloured, and the rest of the subtree runs as
// Branch from depth d + 1, unless it is split once more.
template <int W, bool RL>
__device__ __forceinline__ void run_task(const KArgs &a, unsigned long long task, uint64_t *slab,
                                         uint64_t *rows, int *plist, int *Cl, uint64_t *A,
                                         unsigned long long &nodes_total,
                                         unsigned long long &pub) {
  const int l = lane();
  const bool frozen = a.frozen_bound >= 0;
  const int LW = a.level_words;
  if (a.node_budget > 0 &&
      (long long)__hip_atomic_load(&a.st->nodes, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) +
              (long long)(nodes_total - pub) >= a.node_budget) {
    if (l == 0) atomicExch(&a.st->budget_hit, 1);
    return;  // drain (and clear) the remaining slots without searching
  }
  const uint64_t *rec = a.spool + (task >> 16);
  const int ci = (int)(task & 0xffffull);
  const int s = (int)rec[1], nb = (int)rec[2], croot = (int)rec[3], gr = (int)rec[4];
  const int vroot = (int)rec[5], d = (int)rec[6];
  const uint64_t *base = a.spool + rec[7];
  const long long lab_at = 8 + W + ((long long)base[6] + 1) / 2 + ((long long)base[2] + 1) / 2;
  int *gbound = &a.B.bound[gr];
  int b = frozen ? a.frozen_bound : ld_relaxed(gbound);
  if (croot < b) return;
  const int *path = (const int *)(rec + 8 + W);
  const uint32_t *lst = (const uint32_t *)(rec + 8 + W + (d + 1) / 2);
  const uint32_t e = lst[ci];
  const int x = (int)(e & 0xffffu), cx = (int)(e >> 16);
  const int csz = d + 1;                // |C| before x: the root and the path
  if (csz + cx <= b) return;            // colour cut-off
  if (l < W) A[l] = rec[8 + l];
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  wave_sync();
  for (int j = ci + 1 + l; j < nb; j += PMC_WAVE) {
    const int xj = (int)(lst[j] & 0xffffu);
    atomicAnd((unsigned long long *)&A[xj >> 6], ~(1ull << (xj & 63)));
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  wave_sync();
  uint64_t Pj = l < W ? A[l] : 0ull;
  const int psz = wave_sum(__popcll(Pj));
  if (csz + psz <= b) return;  // |C| + |P| <= b
  if (d + 1 >= a.levels) {
    if (l == 0) atomicExch(&a.st->err, 3);
    return;
  }
  const int *pl = (const int *)(base + lab_at);
  const uint64_t *rw = base + lab_at + (s + 1) / 2;
  for (int t = l; t < s; t += PMC_WAVE) plist[t] = pl[t];
  const uint64_t *crow = rw;
  if (RL) {
    for (int t = l; t < s * W; t += PMC_WAVE) rows[t] = rw[t];
    crow = rows;
  }
  for (int t = l; t < d; t += PMC_WAVE) Cl[t] = path[t];
  if (l == 0) Cl[d] = x;
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  wave_sync();
  int32_t *rep = a.root_report ? a.root_report + 4 * (size_t)vroot : nullptr;
  int best = b;
  const uint64_t cm = core_keep<W>(a, plist, s, b);
  if (l == (x >> 6)) Pj &= ~(1ull << (x & 63));
  const uint64_t Pn = l < W ? (Pj & crow[(size_t)x * W + l] & cm) : 0ull;
  nodes_total++;
  if (!ballot(Pn != 0ull)) {
    const int size = csz + 1;  // the root, the path and x
    if (size > b) {
      int old = 0;
      if (l == 0) old = atomic_max(gbound, size);
      old = shfl(old, 0);
      if (old < size) {
        int32_t *dst = slot_ptr(a.B, gr, size);
        for (int q = l; q < size; q += PMC_WAVE)
          dst[q] = q == 0 ? vroot : a.lab_vertex[plist[Cl[q - 1]]];
      }
      best = size;
    }
  } else {
    uint64_t *nl = slab + (size_t)(d + 1) * LW;
    uint32_t *nlst = (uint32_t *)(nl + W + 1);
    int ncnt = 0;
    colour_classes<W>(Pn, crow, b - (csz + 1), nlst, &ncnt);
    if (ncnt > 0) {
      if (l < W) nl[l] = Pn;
      if (l == 0) nl[W] = (uint64_t)ncnt;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
      wave_sync();
      bool split = false;
      if (d + 1 < a.split_depth && ncnt >= 2 && wave_sum(__popcll(Pn)) >= a.split_min)
        split = emit_deeper<W>(a, rec, d + 1, Cl, nl, nlst, ncnt);
      if (!split) {
        unsigned long long nodes = 0;
        long long base_off = (long long)rec[7];
        branch_dfs<W>(a, slab, crow, plist, Cl, s, d + 1, b, best, croot, gbound, gr, vroot, nodes,
                      nodes_total, pub, base_off);
        nodes_total += nodes;
      }
    }
  }
  if (rep && l == 0 && best > a.frozen_bound) atomic_max(&rep[3], best);
}

// A root the sweep has settled: no clique larger than the bound can remain in
// it (the bound only grows), so the second pass skips it.
__device__ __forceinline__ void settle(const KArgs &a, int vroot) {
  if (a.vdone && lane() == 0) a.vdone[vroot] = 1;
}

template <int W, bool RL>
__global__ void __launch_bounds__(PMC_WAVE) k_search(KArgs a) {
  constexpr int SM = smax<W>();
  extern __shared__ uint64_t lds[];
  uint64_t *rows = RL ? lds : a.grows + (size_t)blockIdx.x * SM * W;
  int *plist = (int *)(lds + (RL ? (size_t)SM * W : 0));
  int *kn = plist + SM;
  int *lr = kn + SM;
  int *dg = lr + SM;
  int *col = dg + SM;
  int *ordv = col + SM;
  int *pre = ordv + SM;  // prefix of row lengths (row build)
  int *Cl = pre + SM;    // chosen local vertex per level (SM + 2)
  uint64_t *A = (uint64_t *)(Cl + SM + 2);  // alive (peel)
  uint64_t *Rw = A + W;                     // removed this round
  uint64_t *K0 = Rw + W;                    // kept after the core drop
  uint64_t *CB = K0 + W;                    // coloured so far
  uint64_t *US = CB + W;                    // colours used by neighbours
  const int l = lane();
  const bool frozen = a.frozen_bound >= 0;
  uint64_t *slab = a.slab + (size_t)blockIdx.x * a.slab_words;
  const int LW = a.level_words;
  unsigned long long nodes_total = 0, branched = 0, pub = 0;


  // roots are claimed a.claim at a time and run one after another (see
  // prepare_class)
  int qnext = 0, qend = 0;
  while (true) {
    if (qnext >= qend) {
      qnext = atomic_add_wave(a.qhead, a.claim);
      if (qnext >= a.count) break;
      qend = min(qnext + a.claim, a.count);
    }
    const int qi = qnext++;
    if (a.node_budget > 0 &&
        (long long)__hip_atomic_load(&a.st->nodes, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) +
                (long long)(nodes_total - pub) >= a.node_budget) {
      if (l == 0) atomicExch(&a.st->budget_hit, 1);
      break;
    }
    const int root = a.queue[qi];
    const int vroot = a.lab_vertex[root];
    const int gr = a.lab_gid ? a.lab_gid[root] : 0;
    int *gbound = &a.B.bound[gr];
    int b = frozen ? a.frozen_bound : ld_relaxed(gbound);
    const int croot = a.lab_core[root];
    int32_t *rep = a.root_report ? a.root_report + 4 * (size_t)vroot : nullptr;
    if (croot < b) {  // the root itself fell below the core bound
      settle(a, vroot);
      continue;
    }
    // ---- P: the oriented row restricted to vertices of core >= b (a suffix
    // of the row in degeneracy order; compacted in native order)
    const int64_t ps = a.poff[root], pe = a.poff[root + 1];
    int s;
    if (!a.native) {
      const int64_t p0 = ps + core_cut(a.padj + ps, (int)(pe - ps), a.lab_core, b);
      s = (int)(pe - p0);
      if (s <= SM)
        for (int t = l; t < s; t += PMC_WAVE) plist[t] = a.padj[p0 + t];
    } else {
      s = 0;
      for (int64_t jb = ps; jb < pe; jb += PMC_WAVE) {
        const int64_t j = jb + l;
        const int x = j < pe ? a.padj[j] : 0;
        const bool keep = j < pe && a.lab_core[x] >= b;
        const uint64_t m = ballot(keep);
        const int at = s + __popcll(m & lanemask_lt());
        if (keep && at < SM) plist[at] = x;
        s += __popcll(m);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
      wave_sync();
    }
    if (rep && l == 0) {
      rep[0] = s;
      rep[3] = 0;
    }
    if (s + 1 <= b) {  // size test
      settle(a, vroot);
      continue;
    }
    if (s > SM) {
      if (l == 0) atomicExch(&a.st->err, 1);
      continue;
    }
    for (int t = l; t < s * W; t += PMC_WAVE) rows[t] = 0ull;
    // build-only scratch: row starts (int64, over kn/lr), an open-addressing
    // hash of P's labels to local indices (over col/ordv, H >= 2s slots; a slot
    // holds a local index, the key is plist[slot value]) and a one-hash
    // membership filter of 8H bits (over dg): most row entries are not in P,
    // and the filter rejects about 15 of 16 of them with one LDS read
    int64_t *rs = (int64_t *)kn;
    int *htab = col;
    uint32_t *filt = (uint32_t *)dg;
    int hbits = 6;
    while ((1 << hbits) < 2 * s) hbits++;
    const int H = 1 << hbits;
    const int fbits = hbits + 3;
    for (int t = l; t < H; t += PMC_WAVE) htab[t] = -1;
    for (int t = l; t < (1 << fbits) / 32; t += PMC_WAVE) filt[t] = 0u;
    // row lengths: a row that fills at least half of one pass of the wave
    // (LONG_ROW entries) is "long" and listed in Cl (free until Branch); the
    // short rows get a prefix of their lengths (for a flattened,
    // lane-balanced pass over them)
    constexpr int UB = 8;
    constexpr int LONG_ROW = PMC_WAVE * UB / 2;
    int run = 0, nlong = 0;
    int *lrows = Cl;
    for (int tb = 0; tb < s; tb += PMC_WAVE) {
      int t = tb + l;
      int len = 0;
      if (t < s) {
        int lab = plist[t];
        int64_t st = a.poff[lab];
        len = (int)(a.poff[lab + 1] - st);
        rs[t] = st;
      }
      const bool lng = len >= LONG_ROW;
      const uint64_t lm = ballot(lng);
      if (lng) lrows[nlong + __popcll(lm & lanemask_lt())] = t;
      nlong += __popcll(lm);
      const int slen = lng ? 0 : len;
      const int inc = wave_incl_scan(slen);
      if (t < s) pre[t] = run + inc - slen;
      run += __builtin_amdgcn_readlane(inc, PMC_WAVE - 1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    wave_sync();
    for (int t = l; t < s; t += PMC_WAVE) {
      const unsigned key = (unsigned)plist[t];
      unsigned h = (key * 2654435761u) >> (32 - hbits);
      while (atomicCAS(&htab[h], -1, t) != -1) h = (h + 1) & (unsigned)(H - 1);
      const unsigned fh = (key * 2246822519u) >> (32 - fbits);
      atomicOr(&filt[fh >> 5], 1u << (fh & 31));
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    wave_sync();
    // ---- bitset adjacency of G[P]: for every a in P and x in N+(a) with x in
    // P, set both bits (N+ only holds higher labels, so each edge once).  x is
    // tested against P's label range and a one-hash membership filter, then
    // looked up in the hash of P's labels.
    const int pmin = s > 0 ? plist[0] : 0, pmax = s > 0 ? plist[s - 1] : -1;
    auto add_entries = [&](const int *xs, const int *ais) {
      bool maybe[UB];
#pragma unroll
      for (int q = 0; q < UB; q++) {
        const unsigned fh = ((unsigned)xs[q] * 2246822519u) >> (32 - fbits);
        maybe[q] = xs[q] >= pmin && xs[q] <= pmax && ((filt[fh >> 5] >> (fh & 31)) & 1u);
      }
#pragma unroll
      for (int q = 0; q < UB; q++) {
        const int x = xs[q];
        if (!maybe[q]) continue;
        unsigned h = ((unsigned)x * 2654435761u) >> (32 - hbits);
        int pos = -1;
        while (true) {
          int t = htab[h];
          if (t < 0) break;
          if (plist[t] == x) {
            pos = t;
            break;
          }
          h = (h + 1) & (unsigned)(H - 1);
        }
        if (pos >= 0) {
          const int ai = ais[q];
          atomicOr((unsigned long long *)&rows[(size_t)ai * W + (pos >> 6)], 1ull << (pos & 63));
          atomicOr((unsigned long long *)&rows[(size_t)pos * W + (ai >> 6)], 1ull << (ai & 63));
        }
      }
    };
    // long rows: the whole wave on one row at a time, UB loads per lane in
    // flight, no search for the row of an entry
    for (int r = 0; r < nlong; r++) {
      const int ai = lrows[r];
      const int64_t st = rs[ai];
      const int len = (int)(a.poff[plist[ai] + 1] - st);
      for (int jb = 0; jb < len; jb += PMC_WAVE * UB) {
        int xs[UB], ais[UB];
#pragma unroll
        for (int q = 0; q < UB; q++) {
          const int j = jb + q * PMC_WAVE + l;
          xs[q] = j < len ? a.padj[st + j] : -1;
          ais[q] = ai;
        }
        add_entries(xs, ais);
      }
    }
    // short rows laid end to end: a lane takes entries f, f + 64, ... of a
    // chunk and finds its row by binary search within the chunk's row range
    int ai_base = 0;
    for (int fb = 0; fb < run; fb += PMC_WAVE * UB) {
      const int flast = min(run, fb + PMC_WAVE * UB) - 1;
      int lo = ai_base, hi = s - 1;  // last row whose prefix is <= fb
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= fb) lo = mid; else hi = mid - 1;
      }
      ai_base = lo;
      hi = s - 1;  // last row whose prefix is <= flast
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= flast) lo = mid; else hi = mid - 1;
      }
      const int ai_last = lo;
      int xs[UB], ais[UB];
      // the lane's row for its first entry by binary search; its later
      // entries lie 64 further on each, usually in the same or the next row
      int it = ai_base;
      if (fb + l <= flast) {
        int r1 = ai_last;
        while (it < r1) {
          int mid = (it + r1 + 1) >> 1;
          if (pre[mid] <= fb + l) it = mid; else r1 = mid - 1;
        }
      }
#pragma unroll
      for (int q = 0; q < UB; q++) {
        const int f = fb + q * PMC_WAVE + l;
        xs[q] = -1;
        ais[q] = 0;
        if (f <= flast) {
          while (it < ai_last && pre[it + 1] <= f) it++;
          ais[q] = it;
          xs[q] = a.padj[rs[it] + (f - pre[it])];
        }
      }
      add_entries(xs, ais);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    wave_sync();
    // ---- neighbourhood core numbers by level-synchronous peeling
    for (int t = 0; t < W; t++) {
      int x = t * 64 + l;
      if (x < s) {
        int d = 0;
        for (int j = 0; j < W; j++) d += __popcll(rows[(size_t)x * W + j]);
        dg[x] = d;
      }
      if (l == 0) {
        int lo = t * 64;
        A[t] = s >= lo + 64 ? ~0ull : (s <= lo ? 0ull : (~0ull >> (64 - (s - lo))));
      }
    }
    wave_sync();
    int k = 0, r = 0, rem = s;
    while (rem > 0) {
      uint64_t any = 0;
      for (int t = 0; t < W; t++) {
        int x = t * 64 + l;
        bool pr = x < s && ((A[t] >> l) & 1ull) && dg[x] <= k;
        uint64_t m = ballot(pr);
        if (l == 0) Rw[t] = m;
        any |= m;
        if (pr) {
          kn[x] = k;
          lr[x] = r;
        }
      }
      if (!any) {
        int mn = INT_MAX;
        for (int t = 0; t < W; t++) {
          int x = t * 64 + l;
          if (x < s && ((A[t] >> l) & 1ull)) mn = min(mn, dg[x]);
        }
        k = wave_min(mn);
        continue;
      }
      wave_sync();
      int gone = 0;
      for (int t = 0; t < W; t++) gone += __popcll(Rw[t]);
      if (l == 0)
        for (int t = 0; t < W; t++) A[t] &= ~Rw[t];
      wave_sync();
      rem -= gone;
      for (int t = 0; t < W; t++) {
        int x = t * 64 + l;
        if (x < s && ((A[t] >> l) & 1ull)) {
          int dec = 0;
          for (int j = 0; j < W; j++) dec += __popcll(rows[(size_t)x * W + j] & Rw[j]);
          dg[x] -= dec;
        }
      }
      wave_sync();
      r++;
    }
    const int nrounds_local = r;
    int kmN = -1;
    for (int t = 0; t < W; t++) {
      int x = t * 64 + l;
      if (x < s) kmN = max(kmN, kn[x]);
    }
    kmN = wave_max(kmN);
    if (rep && l == 0) rep[1] = kmN;
    if (a.use_nc && kmN + 2 <= b) {  // neighbourhood core test
      settle(a, vroot);
      continue;
    }
    // ---- keep K_N(x) + 1 >= b, colour in reverse local peel order
    for (int t = 0; t < W; t++) {
      int x = t * 64 + l;
      bool keep = x < s && (!a.use_nc || kn[x] + 1 >= b);
      uint64_t m = ballot(keep);
      if (l == 0) {
        K0[t] = m;
        CB[t] = 0ull;
        US[t] = 0ull;
      }
    }
    wave_sync();
    int L = 0, nk = 0;
    for (int rr = nrounds_local - 1; rr >= 0; rr--) {
      for (int t = W - 1; t >= 0; t--) {
        int x = t * 64 + l;
        bool pr = x < s && ((K0[t] >> l) & 1ull) && lr[x] == rr;
        uint64_t m = ballot(pr);
        while (m) {
          int bit = 63 - __clzll((long long)m);
          m &= ~(1ull << bit);
          int xx = t * 64 + bit;
          // colours of already coloured neighbours -> US, then the first gap
          if (l < W) {
            uint64_t nb = rows[(size_t)xx * W + l] & CB[l];
            while (nb) {
              int y = l * 64 + __ffsll((unsigned long long)nb) - 1;
              nb &= nb - 1;
              int cy = col[y] - 1;  // colour c is bit c - 1
              atomicOr((unsigned long long *)&US[cy >> 6], 1ull << (cy & 63));
            }
          }
          wave_sync();
          uint64_t freew = l < W ? ~US[l] : 0ull;
          uint64_t fz = ballot(freew != 0ull);
          int fj = __ffsll((unsigned long long)fz) - 1;
          int c = fj * 64 + __ffsll((unsigned long long)shfl64(freew, fj));
          wave_sync();
          if (l < W) US[l] = 0ull;
          if (l == 0) {
            col[xx] = c;
            ordv[nk] = xx;
            CB[xx >> 6] |= 1ull << (xx & 63);
          }
          wave_sync();
          nk++;
          L = max(L, c);
        }
      }
    }
    if (rep && l == 0) rep[2] = L;
    if (L + 1 <= b) {  // colouring test
      settle(a, vroot);
      continue;
    }
    int best = b;  // local best (frozen) / last seen bound
    if (b < 1) {
      // bound 0 (no heuristic): the root alone is a clique of size 1
      int old = 0;
      if (l == 0) old = atomic_max(gbound, 1);
      old = shfl(old, 0);
      if (old < 1 && l == 0) slot_ptr(a.B, gr, 1)[0] = vroot;
      b = 1;
      best = 1;
    }
    // ---- level 0 of the DFS: P0 = K0, branch list = colours > b - 1
    branched++;
    uint64_t *lv0 = slab;
    uint32_t *list0 = (uint32_t *)(lv0 + W + 1);
    int kmin0 = b - 1, n0 = 0;
    for (int c = kmin0 + 1; c <= L; c++) {
      for (int pb = 0; pb < nk; pb += PMC_WAVE) {
        int p = pb + l;
        int x = p < nk ? ordv[p] : 0;
        bool pr = p < nk && col[x] == c;
        uint64_t m = ballot(pr);
        if (pr) list0[n0 + __popcll(m & lanemask_lt())] = ((uint32_t)c << 16) | (uint32_t)x;
        n0 += __popcll(m);
      }
    }
    if (l < W) lv0[l] = K0[l];
    if (l == 0) lv0[W] = (uint64_t)n0;
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    wave_sync();
    if (a.split_min > 0 && s >= a.split_min && n0 >= 2 &&
        emit_split<W>(a, root, s, n0, croot, gr, vroot, K0, list0, plist, rows)) {
      // the level-0 branches run as separate tasks, possibly already running:
      // they and the root combine omega_v with atomic maxima
      if (rep && l == 0) atomic_max(&rep[3], best > a.frozen_bound ? best : 0);
      continue;
    }
    unsigned long long nodes = 0;
    long long base_off = -1;
    // (in the sweep the first descent always reaches a leaf: it takes at
    // most s nodes, and sweep_cap more are allowed after those)
    const bool capped = branch_dfs<W>(
        a, slab, rows, plist, Cl, s, 0, b, best, croot, gbound, gr, vroot, nodes, nodes_total,
        pub, base_off, a.sweep_cap > 0 ? (unsigned long long)(a.sweep_cap + s) : 0ull);
    nodes_total += nodes;
    if (capped) {
      if (l == 0) a.sweep_key[vroot] = (float)L;  // left for the second pass
    } else {
      settle(a, vroot);
    }
    if (rep && l == 0) atomic_max(&rep[3], best > a.frozen_bound ? best : 0);  // donated parts too
  }
  if (a.split_min > 0) {
    // ---- split tasks.  Waves that ran out of roots claim task slots in
    // order; a slot is filled (nonzero) once its record is written.  Every
    // reserved task counts as pending until it has finished, and a task that
    // splits again counts its children first, so once every wave is past its
    // roots and nothing is pending no slot will be filled any more (the
    // claimed slot then lies past every reserved one) and the claims end.
    atomic_add_wave(a.waves_done, 1);
    while (true) {
      const int t = atomic_add_wave(a.task_head, 1);
      unsigned long long task = 0;
      bool over = false;
      int nap = 1;  // backoff: a waiting wave polls less and less often
      while (true) {
        if (t < a.task_cap)
          task = __hip_atomic_load(&a.tasks[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (task) break;
        if (ld_relaxed(a.waves_done) == (int)gridDim.x) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          if (ld_relaxed(a.task_pend) == 0) {
            over = true;
            break;
          }
        }
        for (int z = 0; z < nap; z++) __builtin_amdgcn_s_sleep(8);
        nap = min(nap * 2, 64);
      }
      if (over) break;
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (l == 0) __hip_atomic_store(&a.tasks[t], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      run_task<W, RL>(a, task - 1, slab, rows, plist, Cl, A, nodes_total, pub);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // children before the count drops
      atomic_add_wave(a.task_pend, -1);
    }
  }
  if (l == 0) {
    atomic_add_u64(&a.st->nodes, nodes_total - pub);
    atomic_add_u64(&a.st->roots_branched, branched);
  }
}

__global__ void k_zero(int *p) { *p = 0; }
__global__ void k_reset_split(int *counters, unsigned long long *spool_used) {
  counters[0] = 0;  // task_tail
  counters[1] = 0;  // task_head
  counters[2] = 0;  // waves_done
  counters[3] = 0;  // task_pend
  *spool_used = 0ull;
}

// Split pool shared by the classes of a call (they run one after another):
// 64 MiB of records and up to 2^20 tasks.
constexpr long long SPLIT_POOL_WORDS = 8ll << 20;
constexpr int SPLIT_TASKS = 1 << 20;

// One persistent search launch of a size class: function, grid and arguments
// (scratch allocated up front, so the launch itself can be captured).
struct ClassLaunch {
  const void *fn;
  int blocks;
  size_t lds;
  int words;
  KArgs args;
};

bool search_trace() {
  static const bool on = [] {
    const char *e = std::getenv("PMC_SEARCH_TRACE");
    return e && e[0] == '1';
  }();
  return on;
}

template <int W, bool RL>
ClassLaunch prepare_class(int cls, const KArgs &base, const int32_t *queue, int count,
                          Scratch &sc) {
  ClassLaunch L{};
  KArgs a = base;
  const DevInfo &di = dev_info();
  size_t lb = lds_bytes<W, RL>();
  if (lb > (size_t)di.max_lds) throw Error{5, "search tile does not fit in LDS"};
  if (lb > 65536)
    PMC_HIP(hipFuncSetAttribute((const void *)k_search<W, RL>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lb));
  // the grid below is sized to be resident all at once (waves past their
  // roots wait for split tasks until every wave has finished); the occupancy
  // query does not see a limit that per-lane scratch would add, so a kernel
  // built with scratch is refused rather than risk a grid that cannot drain
  {
    hipFuncAttributes fa;
    PMC_HIP(hipFuncGetAttributes(&fa, (const void *)k_search<W, RL>));
    if (fa.localSizeBytes > 0)
      throw Error{5, "search kernel built with scratch memory; its persistent grid could not "
                     "be guaranteed resident"};
  }
  int per_cu = 0;
  PMC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_search<W, RL>, PMC_WAVE, lb));
  if (per_cu < 1) per_cu = 1;
  int cap = std::max(1, tuning().search_blocks_per_cu[cls]);
  constexpr int SM = smax<W>();
  int levels = std::min(SM, a.kmax + 1) + 1;
  int LW = W + 1 + SM / 2;
  // with the first-level split on, up to 16 waves per root are launched (the
  // waves without a root run the split tasks), as long as their DFS stacks and
  // matrices fit the slab budget: a quarter of the free device memory, at most
  // 16 GiB (the big subproblems of a few hard roots take tens of MB of stack
  // per wave).  Not more: on a small dense graph, thousands of waves without a
  // root make every running Branch hand out its levels as tiny tasks.
  const int64_t full = (int64_t)di.cus * std::min(per_cu, cap);
  const int64_t per_block = ((int64_t)levels * LW + (RL ? 0 : (int64_t)SM * W)) * 8;
  int64_t want = count;
  if (base.split_min > 0) {
    size_t free_b = 0, total_b = 0;
    PMC_HIP(hipMemGetInfo(&free_b, &total_b));
    const int64_t slab_budget =
        std::max<int64_t>((int64_t)256 << 20, std::min<int64_t>((int64_t)16 << 30, free_b / 4));
    want = std::max<int64_t>(count, std::min<int64_t>((int64_t)count * 16,
                                                       slab_budget / per_block));
  }
  int nblocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, full));
  a.levels = levels;
  a.level_words = LW;
  a.slab_words = (long long)levels * LW;
  a.slab = sc.get<uint64_t>((size_t)nblocks * a.slab_words);
  a.grows = RL ? nullptr : sc.get<uint64_t>((size_t)nblocks * SM * W);
  a.qhead = sc.get<int>(1);
  a.queue = queue;
  a.count = count;
  // Roots per queue claim.  Every claim is one atomic on the class's queue
  // head, which the memory side serves at about one per 10 ns: a class of a
  // million small roots that mostly settle at once kept the waves waiting on
  // the head at one root per claim (the search of a 2,048-graph batch took
  // 15.3 ms; 6.0 ms with claims of an eighth of a wave's even share, at most
  // 64).  Roots with rows in global memory (over 512 vertices) and the roots
  // of a sweep (each runs InitialBranch and part of Branch) are never that
  // cheap, and consecutive roots of the queue are alike, so a claim of tens
  // of them put a run of hard roots on one wave (the sweep of R-MAT scale 27
  // took 53 instead of 29 s): those keep one root per claim.
  const int64_t share8 = (int64_t)count / ((int64_t)nblocks * 8);
  a.claim = (RL && a.sweep_cap <= 0) ? (int)std::max<int64_t>(1, std::min<int64_t>(64, share8)) : 1;
  L.fn = (const void *)k_search<W, RL>;
  L.words = W;
  L.blocks = nblocks;
  L.lds = lb;
  L.args = a;
  return L;
}

ClassLaunch prepare(int cls, const KArgs &a, const int32_t *queue, int count, Scratch &sc) {
  switch (cls) {
    case 0: return prepare_class<1, true>(cls, a, queue, count, sc);
    case 1: return prepare_class<2, true>(cls, a, queue, count, sc);
    case 2: return prepare_class<4, true>(cls, a, queue, count, sc);
    case 3: return prepare_class<8, true>(cls, a, queue, count, sc);
    case 4: return prepare_class<16, false>(cls, a, queue, count, sc);
    case 5: return prepare_class<32, false>(cls, a, queue, count, sc);
    case 6: return prepare_class<64, false>(cls, a, queue, count, sc);
    default: throw Error{3, "a subproblem exceeds 4096 vertices"};
  }
}

// Resets the class's queue head (and split counters) with kernels (not
// memset nodes, which must stay out of captured graphs) and launches the
// persistent search (whose waves run the split tasks once the roots are
// gone).
void enqueue(ClassLaunch &L, hipStream_t s) {
  k_zero<<<1, 1, 0, s>>>(L.args.qhead);
  PMC_HIP(hipGetLastError());
  if (L.args.split_min > 0) {
    k_reset_split<<<1, 1, 0, s>>>(L.args.task_tail, L.args.spool_used);
    PMC_HIP(hipGetLastError());
  }
  void *args[] = {&L.args};
  PMC_HIP(hipLaunchKernel(L.fn, dim3(L.blocks), dim3(PMC_WAVE), args, L.lds, s));
}

KArgs base_args(SearchArgs sa, Scratch &sc) {
  KArgs a{};
  const int sm = tuning().search_split_min;
  if (sm > 0) {
    if (!sa.spool) alloc_split(sa, sc);
    a.split_min = sm;
    a.spool_words = SPLIT_POOL_WORDS;
    a.spool = sa.spool;
    a.spool_used = sa.spool_used;
    a.task_cap = SPLIT_TASKS;
    a.tasks = sa.tasks;
    a.task_tail = sa.task_tail;
    a.task_head = sa.task_tail + 1;
    a.waves_done = sa.task_tail + 2;
    a.task_pend = sa.task_tail + 3;
    a.split_depth = tuning().search_split_depth;
  }
  a.nn = sa.L.nn;
  a.poff = sa.L.poff;
  a.padj = sa.L.padj;
  a.lab_core = sa.L.core;
  a.lab_gid = sa.L.gid;
  a.lab_vertex = sa.L.vertex;
  a.kmax = sa.kmax;
  a.B = sa.B;
  a.st = sa.st;
  a.frozen_bound = sa.frozen_bound;
  a.use_nc = sa.use_nc;
  a.root_report = sa.root_report;
  a.node_budget = sa.node_budget;
  a.native = sa.native ? 1 : 0;
  if (sa.sweep_cap > 0) {
    a.sweep_cap = sa.sweep_cap;
    a.sweep_key = sa.sweep_key;
    a.vdone = sa.vdone;
    a.split_min = 0;  // the sweep never splits: its Branch stops early anyway
  }
  return a;
}

}  // namespace

void alloc_split(SearchArgs &a, Scratch &sc) {
  if (tuning().search_split_min <= 0 || a.spool) return;
  a.spool = sc.get<uint64_t>((size_t)SPLIT_POOL_WORDS);
  a.spool_used = sc.get<unsigned long long>(1);
  a.tasks = sc.get<unsigned long long>((size_t)SPLIT_TASKS);
  a.task_tail = sc.get<int>(4);  // tail, head, waves done, pending
  // task slots start empty; every slot a launch fills is cleared by its claimer
  PMC_HIP(hipMemsetAsync(a.tasks, 0, sizeof(unsigned long long) * SPLIT_TASKS, sc.stream()));
}

float run_search_class(int cls, const SearchArgs &sa, const int32_t *queue, int count,
                       Scratch &sc) {
  if (count <= 0) return 0.f;
  ClassLaunch L = prepare(cls, base_args(sa, sc), queue, count, sc);
  KTimer kt(sc.stream());
  kt.start();
  enqueue(L, sc.stream());
  return kt.stop();
}

namespace {

// The search stage as one hipGraph (tuning().search_graph).  Instantiated
// graphs are kept per (device, stream), up to GRAPH_KEEP of them (a solve that
// searches in waves runs one stage per wave), and replayed by a later call
// whose class launches are byte-identical (kernel, grid, LDS and every
// argument, which includes the scratch addresses the pool hands out), as for a
// repeated batch of one shape; any other call captures and instantiates a new
// one in place of the least recently used.  Capture runs on a private stream
// (the caller's may be the null stream, which cannot be captured); the graph
// holds kernel nodes only.
constexpr size_t GRAPH_KEEP = 8;
struct GraphEntry {
  std::vector<ClassLaunch> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  unsigned long long used = 0;
};
std::mutex graph_mu;
std::map<std::pair<int, hipStream_t>, std::vector<GraphEntry>> &graph_map() {
  static auto *m = new std::map<std::pair<int, hipStream_t>, std::vector<GraphEntry>>();
  return *m;
}

void drop_entry(GraphEntry &e) {
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (e.graph) (void)hipGraphDestroy(e.graph);
  e.exec = nullptr;
  e.graph = nullptr;
  e.key.clear();
}

// Destroys the kept graphs at process exit (registered after the first
// capture, so before the runtime's own teardown), after their streams drain.
void release_graphs() {
  std::lock_guard<std::mutex> lock(graph_mu);
  for (auto &kv : graph_map()) {
    if (hipSetDevice(kv.first.first) != hipSuccess) continue;
    (void)hipDeviceSynchronize();
    for (auto &e : kv.second) drop_entry(e);
  }
  graph_map().clear();
  (void)hipGetLastError();
}

bool same_launches(const std::vector<ClassLaunch> &a, const std::vector<ClassLaunch> &b) {
  if (a.size() != b.size()) return false;
  for (size_t i = 0; i < a.size(); i++) {
    if (a[i].fn != b[i].fn || a[i].blocks != b[i].blocks || a[i].lds != b[i].lds ||
        std::memcmp(&a[i].args, &b[i].args, sizeof(KArgs)) != 0)
      return false;
  }
  return true;
}

float run_graph(std::vector<ClassLaunch> &ls, hipStream_t s, KTimer &kt, int32_t *replays) {
  int dev = 0;
  PMC_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(graph_mu);
  static bool registered = (std::atexit(release_graphs) == 0);
  (void)registered;
  static unsigned long long tick = 0;
  std::vector<GraphEntry> &kept = graph_map()[{dev, s}];
  GraphEntry *ent = nullptr;
  for (auto &e : kept)
    if (same_launches(e.key, ls)) ent = &e;
  if (ent) {
    if (replays) ++*replays;
  } else {
    if (kept.size() < GRAPH_KEEP) {
      kept.emplace_back();
      ent = &kept.back();
    } else {
      ent = &kept[0];
      for (auto &e : kept)
        if (e.used < ent->used) ent = &e;
      // a launch of the evicted graph can only be pending on this same stream
      PMC_HIP(hipStreamSynchronize(s));
      drop_entry(*ent);
    }
    hipStream_t cap;
    PMC_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      try {
        for (auto &L : ls) enqueue(L, cap);
      } catch (...) {
        (void)hipStreamEndCapture(cap, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cap);
        throw;
      }
      e = hipStreamEndCapture(cap, &graph);
    }
    (void)hipStreamDestroy(cap);
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      throw Error{5, std::string("search graph: ") + hipGetErrorString(e)};
    }
    ent->graph = graph;
    ent->exec = exec;
    ent->key = ls;
  }
  ent->used = ++tick;
  kt.start();
  const hipError_t e = hipGraphLaunch(ent->exec, s);
  if (e != hipSuccess) {
    PMC_HIP(hipStreamSynchronize(s));
    drop_entry(*ent);
    throw Error{5, std::string("search graph launch: ") + hipGetErrorString(e)};
  }
  return kt.stop();
}

}  // namespace

float run_search(const SearchArgs &sa, const int32_t *queue, const QueueResult &q, Scratch &sc,
                 bool largest_first, int32_t *replays) {
  hipStream_t s = sc.stream();
  KArgs base = base_args(sa, sc);
  std::vector<ClassLaunch> ls;
  // Each launch ends when its slowest wave does, about one root after the
  // others.  When class 0 holds a few roots per wave of its grid, that tail
  // costs more than running its roots with 2-word rows: classes 0 and 1 (next
  // to each other in the queue) then run as one launch of the 2-word kernel
  // (the search of the 10^6-vertex Chung-Lu benchmark graph: 3.43 -> 3.01
  // ms).  Not with many roots per wave (a 2,048-graph batch, ~120 per wave:
  // the 1-word kernel's cheaper roots win, 5.96 vs 6.37 ms merged), nor with
  // fewer roots than an eighth of the grid's waves: those are the few, often
  // deep searches of small dense graphs, where Branch on 1-word rows is what
  // counts (G(150, 0.8): 8.1 ms, 20.4 ms merged).
  const int64_t waves0 = (int64_t)dev_info().cus * std::max(1, tuning().search_blocks_per_cu[0]);
  const bool merge01 = !largest_first && q.count[0] >= waves0 / 8 && q.count[0] < 8 * waves0;
  if (merge01) ls.push_back(prepare(1, base, queue + q.start[0], q.count[0] + q.count[1], sc));
  for (int i = 0; i < SEARCH_CLASSES; i++) {
    const int c = largest_first ? SEARCH_CLASSES - 1 - i : i;
    if (merge01 && c <= 1) continue;
    if (q.count[c] > 0) ls.push_back(prepare(c, base, queue + q.start[c], q.count[c], sc));
  }
  if (ls.empty()) return 0.f;
  KTimer kt(s);
  if (search_trace()) {
    // PMC_SEARCH_TRACE=1: every class in pieces of at most 1/16 of its roots
    // (1/PMC_SEARCH_TRACE_PIECES), one launch each, timed and reported as it
    // ends
    int pieces = 16;
    if (const char *e = std::getenv("PMC_SEARCH_TRACE_PIECES")) pieces = std::max(1, std::atoi(e));
    float tot = 0.f;
    for (auto &L : ls) {
      const int count = L.args.count;
      const int piece = std::max(1, (count + pieces - 1) / pieces);
      for (int at = 0; at < count; at += piece) {
        ClassLaunch P = L;
        P.args.queue = L.args.queue + at;
        P.args.count = std::min(piece, count - at);
        kt.start();
        enqueue(P, s);
        const float ms = kt.stop();
        tot += ms;
        int bnd = 0;
        CliqueState h;
        PMC_HIP(hipMemcpy(&bnd, sa.B.bound, sizeof(int), hipMemcpyDeviceToHost));
        PMC_HIP(hipMemcpy(&h, sa.st, sizeof(h), hipMemcpyDeviceToHost));
        std::fprintf(stderr,
                     "[pmc search] words %d roots %d..%d of %d blocks %d sweep %lld: %.3f ms, "
                     "bound %d, nodes %llu\n",
                     L.words, at, at + P.args.count, count, L.blocks, (long long)L.args.sweep_cap,
                     ms, bnd, h.nodes);
      }
    }
    return tot;
  }
  if (!tuning().search_graph) {
    kt.start();
    for (auto &L : ls) enqueue(L, s);
    return kt.stop();
  }
  return run_graph(ls, s, kt, replays);
}

}  // namespace pmc
