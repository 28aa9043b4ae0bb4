// peel.hip -- k-core decomposition (Sec. 3 of the paper; the CoreNumbers step
// of MaxClique) by level-synchronous peeling, and the degeneracy rank.
//
// Definition computed: level k starts at 0; in each round every remaining
// vertex whose remaining degree is <= k is removed at once (core = k, round =
// the round counter); when nothing is removable, k jumps to the minimum
// remaining degree.  The rank is the position in (round, id) order; rounds are
// monotone in the level, so the rank is a degeneracy order nondecreasing in
// core and every vertex has at most core(v) higher-ranked neighbours.
//
// GPU design: ONE cooperative persistent launch.  The frontier of each round
// is a contiguous segment of a peel-order list; removing a frontier vertex
// decrements its neighbours' remaining degrees with device atomics, and the
// unique decrement that takes a degree from k+1 to k appends the neighbour to
// the next frontier (wave-aggregated append).  Rounds are separated by a grid
// barrier; every datum exchanged between workgroups is stored and loaded at
// device scope, so the barrier needs no cache flush.  Level jumps compact the
// live list and take its minimum degree.  Frontier items are spread over
// waves (item p -> wave p % waves, lane p / waves, waves numbered so that
// consecutive items sit on different CUs) so a small frontier gets one vertex
// per wave and per CU; a short row is walked by its own lane, a long row by
// the whole wave, with several neighbour loads and atomics in flight per lane.
// The peel is a chain of about one round per (level, sub-round), each costing
// a few dependent device-memory round trips, so on power-law graphs its time
// is set by latency, not bandwidth.  PMC_PEEL_TRACE=1 prints a per-phase
// breakdown (rounds and level jumps) to stderr.
#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "common.h"
#include "graph.h"

namespace pmc {
namespace {

constexpr int PEEL_T = 1024;
constexpr int SMALL_DEG = 16;
constexpr int UNR = 16;  // neighbour loads/atomics kept in flight per lane
static_assert(SMALL_DEG <= 32 && UNR <= 32, "crossing masks are 32-bit");
constexpr int FBUF = 4096;  // per-workgroup LDS buffer of next-frontier vertices
// rounds removing at least this many vertices test the `gone` bitmap before
// each decrement (throughput-bound rounds); smaller ones do not (latency-bound)
constexpr int GONE_MIN_FRONTIER = 16384;

struct FrontierBuf {
  int buf[FBUF];
  int cnt;   // appends this round (may exceed FBUF: the excess went to the list)
  int base;  // list position of the flushed buffer
  int len;   // entries flushed
};

// Appends of one phase (a round, or the frontier scan of a level jump) go to
// porder[fend + cnt[phase % 3]]: after the phase's barrier every block reads
// the same count, and the slot reset for the next phase was read by every
// block two barriers earlier, so no block can see a count still growing.
struct PeelCtrl {
  GridBar bar;
  int cnt[3];        // appends of the current phase, rotating
  int alive_cnt[2];  // sizes of the two live lists
  int kmin[2];       // minimum live degree, alternating per level jump
  int nrounds;
  int kmax;
  int tail_cnt;      // remaining unqueued vertices found when the tail starts
  int tail_ok;       // 1: the tail's compacted graph fits its buffer
  int err;           // nonzero: the tail found an inconsistent state
};

// The tail: once at most TAIL_V vertices are left (unqueued, or queued for
// the round about to run), the rounds are short chains of latency and the
// grid barrier dominates.  The remaining subgraph is then compacted (local
// ids, rows keeping only unqueued neighbours) and workgroup 0 finishes the
// peel alone, with remaining degrees and the peel queue in LDS and
// __syncthreads in place of grid barriers.
// (32,768 was measured too: the extra tail rounds and the longer level-jump
// scans cost more than the grid rounds they replace)
constexpr int TAIL_V = 16384;
static_assert(TAIL_V <= 32768, "tail degrees and ids are 16-bit");
constexpr int TAIL_MARK = 1 << 15;  // added to a local degree when the vertex is queued

__device__ __forceinline__ int tdeg(const uint32_t *deg2, int i) {
  return (int)((deg2[i >> 1] >> ((i & 1) * 16)) & 0xffffu);
}

struct TailBufs {
  int *map;    // [n] global -> local id (valid for the tail's vertices only)
  int *glob;   // [TAIL_V] local -> global id
  int *poff;   // [TAIL_V + 1] compacted row offsets
  int *adj;    // [cap] compacted rows (local ids)
  int cap;
  int *rstart; // [TAIL_V + 1] first queue position of each tail round
  int *rk;     // [TAIL_V + 1] level of each tail round
};

constexpr int TAIL_EPT = 4;  // consecutive row entries per thread per pass

// Local degrees are 16-bit halves of 32-bit LDS words (a local degree is
// below TAIL_V <= 2^15, TAIL_MARK sets bit 15): a decrement subtracts 1 from
// its half with a 32-bit atomic, which never borrows since a degree counts
// only neighbours not yet processed.
struct TailLds {
  uint32_t deg2[TAIL_V / 2];  // remaining degree (+ TAIL_MARK once queued)
  uint16_t queue[TAIL_V];     // local ids in peel order
  int poff[TAIL_V + 1];       // compacted row offsets (a round's first lookup)
  int junk[PEEL_T];     // per-thread target of no-op decrements
  int pre[PEEL_T + 1];  // exclusive prefix of the row lengths of a chunk of items
  int rs[PEEL_T];       // row starts of the chunk's items
  int wtot[PEEL_T / PMC_WAVE + 1];
  int qend;             // queue length
};

__global__ void k_peel_ctrl_init(PeelCtrl *c) {
  for (int g = 0; g < GRID_GROUPS; g++) c->bar.group[g][0] = 0;
  c->bar.top = 0;
  c->cnt[0] = c->cnt[1] = c->cnt[2] = 0;
  c->alive_cnt[0] = 0;
  c->alive_cnt[1] = 0;
  c->kmin[0] = INT_MAX;
  c->kmin[1] = INT_MAX;
  c->nrounds = 0;
  c->kmax = 0;
  c->tail_cnt = 0;
  c->tail_ok = 0;
  c->err = 0;
}

// Removes up to NQ edges per lane of frontier rows: slot q of a lane is row
// entry jb + q (own row) or jb + 64 q + lane (a row shared by the wave).
// Every neighbour's remaining degree drops by one; the decrement that takes
// it from k+1 to k queues it for the next round (round r+1, core k).
// In rounds with a large frontier (check_gone) a neighbour that is already
// queued or removed is skipped: its bit in the `gone` bitmap (one bit per
// vertex, set when it is queued) is read first, so the decrements of an edge
// whose other endpoint went first (half of all row entries over the peel)
// cost a bitmap read instead of an atomic.  A stale read only lets a harmless
// decrement through (that degree is already <= k, so it never crosses from
// k+1 again).  Small rounds are bound by the latency of their dependent
// chain, which the extra read would lengthen, so they decrement blindly.  Skipped slots and slots past the end
// of a row subtract 0 from the lane's own junk word instead of branching
// around the atomic, so the NQ atomics of a lane are issued back to back and
// their latencies overlap.  Called by a whole wave.
template <int NQ>
__device__ __forceinline__ void drop_batch(int64_t s, int64_t len, int64_t jb, bool coop,
                                           const int32_t *idx, int *deg, int *junk, int *rnd,
                                           int *core, int *porder, int *pc, FrontierBuf &fb,
                                           int fend, int k, int r, unsigned *gone,
                                           bool check_gone) {
  const int l = lane();
  int u[NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    int64_t j = coop ? jb + (int64_t)q * PMC_WAVE + l : jb + q;
    u[q] = j < len ? idx[s + j] : -1;
  }
  if (check_gone) {
    unsigned gw[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) gw[q] = u[q] >= 0 ? ld_dev_u32(&gone[u[q] >> 5]) : 0u;
#pragma unroll
    for (int q = 0; q < NQ; q++)
      if (u[q] >= 0 && ((gw[q] >> (u[q] & 31)) & 1u)) u[q] = -1;
  }
  int old[NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    const bool ok = u[q] >= 0;
    old[q] = atomic_sub(ok ? &deg[u[q]] : junk, ok ? 1 : 0);
  }
  unsigned cross = 0;
#pragma unroll
  for (int q = 0; q < NQ; q++)
    if (u[q] >= 0 && old[q] == k + 1) cross |= 1u << q;
  // queue the crossings in the workgroup's LDS buffer (flushed to the
  // frontier list with one atomic per workgroup at the end of the round);
  // what does not fit goes to the list directly
  const int c = __popc(cross);
  const int inc = wave_incl_scan(c);
  const int total = __builtin_amdgcn_readlane(inc, PMC_WAVE - 1);
  if (total == 0) return;
  int lb = 0;
  if (l == 0) lb = atomicAdd(&fb.cnt, total);
  lb = __builtin_amdgcn_readfirstlane(lb);
  int lpos = lb + inc - c;  // this lane's first buffer position
  const int nspill = max(0, lpos + c - max(lpos, FBUF));
  int gpos = fend + wave_append_n(pc, nspill);
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    if (cross >> q & 1u) {
      if (lpos < FBUF) fb.buf[lpos] = u[q];
      else st_dev(&porder[gpos++], u[q]);
      lpos++;
      st_dev(&rnd[u[q]], r + 1);
      core[u[q]] = k;
      atomicOr(&gone[u[q] >> 5], 1u << (u[q] & 31));
    }
  }
}

// Removes the edges of one frontier row [s, e) (`coop`: the wave's shared
// row, 64 * UNR entries per batch) or of every lane's own short row.
__device__ __forceinline__ void drop_edges(int64_t s, int64_t e, bool coop, const int32_t *idx,
                                           int *deg, int *junk, int *rnd, int *core,
                                           int *porder, int *pc, FrontierBuf &fb, int fend, int k,
                                           int r, unsigned *gone, bool check_gone) {
  const int64_t len = e - s;
  if (coop) {
    for (int64_t jb = 0; jb < len; jb += (int64_t)PMC_WAVE * UNR)
      drop_batch<UNR>(s, len, jb, true, idx, deg, junk, rnd, core, porder, pc, fb, fend, k, r,
                      gone, check_gone);
    return;
  }
  const int span = wave_max((int)len);  // <= SMALL_DEG
  if (span == 0) return;
  if (span <= 4)
    drop_batch<4>(s, len, 0, false, idx, deg, junk, rnd, core, porder, pc, fb, fend, k, r,
                  gone, check_gone);
  else if (span <= 8)
    drop_batch<8>(s, len, 0, false, idx, deg, junk, rnd, core, porder, pc, fb, fend, k, r,
                  gone, check_gone);
  else
    drop_batch<SMALL_DEG>(s, len, 0, false, idx, deg, junk, rnd, core, porder, pc, fb, fend, k, r,
                  gone, check_gone);
}

// Level jump, part 1: compact the live list (vertices not yet queued) and
// fold its minimum degree into *kmin.  Whole workgroups take part, so the
// list counter and *kmin see one atomic per workgroup.
__device__ __forceinline__ void compact_live(const int *ain, int *aout, int alen, int *acnt,
                                             int *kmin, const int *rnd, const int *deg,
                                             int *lds) {
  int lmin = INT_MAX;
  for (int base = blockIdx.x * blockDim.x; base < alen; base += gridDim.x * blockDim.x) {
    int i = base + threadIdx.x;
    bool ok = i < alen;
    int v = ok ? ld_dev(&ain[i]) : 0;
    bool live = ok && ld_dev(&rnd[v]) == -1;
    int pos = block_append(acnt, live, lds);
    if (live) {
      st_dev(&aout[pos], v);
      lmin = min(lmin, ld_dev(&deg[v]));
    }
  }
  lmin = block_min(lmin, lds);
  if (threadIdx.x == 0 && lmin != INT_MAX) atomic_min(kmin, lmin);
}

// Level jump, part 2: queue every live vertex of degree <= k (round r).
__device__ __forceinline__ void mark_level(const int *alist, int alen, int k, int r, int fend,
                                           int *pc, int *porder, int *rnd, int *core,
                                           const int *deg, int *lds, unsigned *gone) {
  for (int base = blockIdx.x * blockDim.x; base < alen; base += gridDim.x * blockDim.x) {
    int i = base + threadIdx.x;
    bool ok = i < alen;
    int v = ok ? ld_dev(&alist[i]) : 0;
    bool f = ok && ld_dev(&deg[v]) <= k;
    int pos = fend + block_append(pc, f, lds);
    if (f) {
      st_dev(&porder[pos], v);
      st_dev(&rnd[v], r);
      core[v] = k;
      atomicOr(&gone[v >> 5], 1u << (v & 31));
    }
  }
}

// One round: remove the frontier [head, fend).
template <typename OffT>
__device__ __forceinline__ void run_round(int head, int fend, int k, int r, int *pc,
                                          const OffT *__restrict__ off,
                                          const int32_t *__restrict__ idx, int *deg, int *junk,
                                          int *rnd, int *core, int *porder, FrontierBuf &fb,
                                          int w0, int nw, unsigned *gone) {
  const int l = lane();
  const int F = fend - head;
  const bool check_gone = F >= GONE_MIN_FRONTIER;
  for (int base = 0; base < F; base += PMC_WAVE * nw) {
    int p = base + l * nw + w0;
    bool ok = p < F;
    int v = ok ? ld_dev(&porder[head + p]) : 0;
    int64_t s = ok ? (int64_t)off[v] : 0, e = ok ? (int64_t)off[v + 1] : 0;
    bool small = e - s <= SMALL_DEG;
    drop_edges(s, small ? e : s, false, idx, deg, junk, rnd, core, porder, pc, fb, fend, k, r,
               gone, check_gone);
    uint64_t big = ballot(!small);
    while (big) {
      int src = __ffsll((unsigned long long)big) - 1;
      big &= big - 1;
      int64_t vs = (int64_t)shfl64((uint64_t)s, src);
      int64_t ve = (int64_t)shfl64((uint64_t)e, src);
      drop_edges(vs, ve, true, idx, deg, junk, rnd, core, porder, pc, fb, fend, k, r, gone,
                 check_gone);
    }
  }
  // flush the workgroup's buffered crossings: one atomic per workgroup
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = min(fb.cnt, FBUF);
    fb.base = c ? atomic_add(pc, c) : 0;
    fb.len = c;
    fb.cnt = 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < fb.len; i += blockDim.x) st_dev(&porder[fend + fb.base + i], fb.buf[i]);
}

// Optional phase trace (workgroup 0, thread 0): per phase its kind (0 round,
// 1 level jump), the frontier or live-list size and the realtime clock at its
// end.  trace[0] counts records.
constexpr int TRACE_MAX = 16384;
__device__ __forceinline__ void trace_phase(long long *trace, int kind, int size) {
  if (!trace || blockIdx.x != 0 || threadIdx.x != 0) return;
  long long i = trace[0];
  if (i >= TRACE_MAX) return;
  trace[1 + 3 * i] = kind;
  trace[2 + 3 * i] = size;
  trace[3 + 3 * i] = (long long)wall_clock64();
  trace[0] = i + 1;
}

// Tail set-up, run by every workgroup: local ids (the frontier [head, fend)
// first, in queue order, then the unqueued vertices of the live list), row
// lengths, offsets (workgroup 0), rows.  Returns false (uniformly) when the
// compacted rows exceed the buffer; the grid rounds then continue.
template <typename OffT>
__device__ bool tail_setup(int n, const OffT *__restrict__ off, const int32_t *__restrict__ idx,
                           const int *rnd, const int *porder, int head, int fend,
                           const int *alist, int alen, const TailBufs &T, PeelCtrl *ctrl,
                           int *lds, unsigned long long &gen, int wave_g, int nwaves) {
  const unsigned nb = gridDim.x;
  const int l = lane();
  const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
  const int gsz = gridDim.x * blockDim.x;
  const int F = fend - head;
  for (int p = gtid; p < F; p += gsz) {
    int v = ld_dev(&porder[head + p]);
    st_dev(&T.glob[p], v);
    st_dev(&T.map[v], p);
  }
  for (int base = blockIdx.x * blockDim.x; base < alen; base += gridDim.x * blockDim.x) {
    int i = base + threadIdx.x;
    bool ok = i < alen;
    int v = ok ? ld_dev(&alist[i]) : 0;
    bool un = ok && ld_dev(&rnd[v]) == -1;
    int pos = block_append(&ctrl->tail_cnt, un, lds);
    if (un && F + pos < TAIL_V) {
      st_dev(&T.glob[F + pos], v);
      st_dev(&T.map[v], F + pos);
    }
  }
  grid_sync(&ctrl->bar, nb, gen);
  const int S = min(F + ld_dev(&ctrl->tail_cnt), TAIL_V);
  // row lengths: neighbours still unqueued
  for (int i = wave_g; i < S; i += nwaves) {
    int v = ld_dev(&T.glob[i]);
    int64_t s0 = (int64_t)off[v], e0 = (int64_t)off[v + 1];
    int cnt = 0;
    for (int64_t jb = s0; jb < e0; jb += PMC_WAVE) {
      int64_t j = jb + l;
      bool keep = j < e0 && ld_dev(&rnd[idx[j]]) == -1;
      cnt += __popcll(ballot(keep));
    }
    if (l == 0) st_dev(&T.poff[i + 1], cnt);
  }
  grid_sync(&ctrl->bar, nb, gen);
  if (blockIdx.x == 0) {
    // inclusive scan of poff[1..S] by workgroup 0: each thread a run of S/T
    const int per = (S + blockDim.x - 1) / blockDim.x;
    const int a = min(S, (int)threadIdx.x * per), b = min(S, a + per);
    long long own = 0;
    for (int i = a; i < b; i++) own += ld_dev(&T.poff[i + 1]);
    // workgroup exclusive scan of `own`
    long long inc = own;
    for (int o = 1; o < PMC_WAVE; o <<= 1) {
      long long t = __shfl_up(inc, o, PMC_WAVE);
      if (l >= o) inc += t;
    }
    __shared__ long long wsum[PEEL_T / PMC_WAVE + 1];
    const int w = threadIdx.x / PMC_WAVE, nw = blockDim.x / PMC_WAVE;
    if (l == PMC_WAVE - 1) wsum[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
      long long t = 0;
      for (int i = 0; i < nw; i++) {
        long long c = wsum[i];
        wsum[i] = t;
        t += c;
      }
      wsum[nw] = t;
    }
    __syncthreads();
    long long run = wsum[w] + inc - own;
    for (int i = a; i < b; i++) {
      run += ld_dev(&T.poff[i + 1]);
      st_dev(&T.poff[i + 1], (int)min(run, (long long)INT_MAX));
    }
    if (threadIdx.x == 0) {
      st_dev(&T.poff[0], 0);
      st_dev(&ctrl->tail_ok, wsum[nw] <= (long long)T.cap ? 1 : 0);
    }
  }
  grid_sync(&ctrl->bar, nb, gen);
  if (!ld_dev(&ctrl->tail_ok)) return false;
  for (int i = wave_g; i < S; i += nwaves) {
    int v = ld_dev(&T.glob[i]);
    int64_t s0 = (int64_t)off[v], e0 = (int64_t)off[v + 1];
    int pos = ld_dev(&T.poff[i]);
    for (int64_t jb = s0; jb < e0; jb += PMC_WAVE) {
      int64_t j = jb + l;
      int u = j < e0 ? idx[j] : 0;
      bool keep = j < e0 && ld_dev(&rnd[u]) == -1;
      uint64_t m = ballot(keep);
      if (keep) st_dev(&T.adj[pos + __popcll(m & lanemask_lt())], ld_dev(&T.map[u]));
      pos += __popcll(m);
    }
  }
  grid_sync(&ctrl->bar, nb, gen);
  return true;
}

// One round of the tail: the rows of the items [qh, qe) are laid end to end
// (a workgroup scan of their lengths, in chunks of one item per thread) and
// every thread takes TAIL_EPT consecutive entries, so a round's work is spread
// over all waves whatever its row lengths.  LDS decrements; the decrement from
// k+1 to k marks the vertex and appends it to the LDS queue (one LDS atomic
// per wave).
__device__ __forceinline__ void tail_round(int qh, int qe, int k, const TailBufs &T, TailLds &L) {
  const int t = threadIdx.x, l = lane();
  const int w = t / PMC_WAVE, nw = blockDim.x / PMC_WAVE;
  for (int cb = qh; cb < qe; cb += blockDim.x) {
    const int C = min((int)blockDim.x, qe - cb);
    if (C <= PMC_WAVE) {
      // one wave lays out up to 64 rows: no workgroup scan
      if (w == 0) {
        int st = 0, len = 0;
        if (t < C) {
          int v = L.queue[cb + t];
          st = L.poff[v];
          len = L.poff[v + 1] - st;
        }
        const int inc = wave_incl_scan(len);
        if (t < C) {
          L.pre[t] = inc - len;
          L.rs[t] = st;
        }
        if (t == C - 1) L.pre[C] = inc;
      }
    } else {
      int st = 0, len = 0;
      if (t < C) {
        int v = L.queue[cb + t];
        st = L.poff[v];
        len = L.poff[v + 1] - st;
      }
      const int inc = wave_incl_scan(len);
      if (l == PMC_WAVE - 1) L.wtot[w] = inc;
      __syncthreads();
      int before = 0, all = 0;
      for (int i = 0; i < nw; i++) {
        int c = L.wtot[i];
        before += i < w ? c : 0;
        all += c;
      }
      if (t < C) {
        L.pre[t] = before + inc - len;
        L.rs[t] = st;
      }
      if (t == 0) L.pre[C] = all;
    }
    __syncthreads();
    const int E = L.pre[C];
    for (int eb = 0; eb < E; eb += blockDim.x * TAIL_EPT) {
      const int e0 = eb + t * TAIL_EPT;
      int it = 0;
      if (e0 < E) {  // last item whose first entry is <= e0 (a nonempty row)
        int lo = 0, hi = C - 1;
        while (lo < hi) {
          int mid = (lo + hi + 1) >> 1;
          if (L.pre[mid] <= e0) lo = mid; else hi = mid - 1;
        }
        it = lo;
      }
      int u[TAIL_EPT];
#pragma unroll
      for (int q = 0; q < TAIL_EPT; q++) {
        const int e = e0 + q;
        u[q] = -1;
        if (e < E) {
          while (L.pre[it + 1] <= e) it++;
          u[q] = ld_dev(&T.adj[L.rs[it] + e - L.pre[it]]);
        }
      }
      int old[TAIL_EPT];
#pragma unroll
      for (int q = 0; q < TAIL_EPT; q++) {
        const bool ok = u[q] >= 0;
        const unsigned sh = ok ? (unsigned)(u[q] & 1) * 16u : 0u;
        const unsigned w = atomicSub(ok ? &L.deg2[u[q] >> 1] : (uint32_t *)&L.junk[t],
                                     ok ? 1u << sh : 0u);
        old[q] = (int)((w >> sh) & 0xffffu);
      }
      unsigned cross = 0;
#pragma unroll
      for (int q = 0; q < TAIL_EPT; q++)
        if (u[q] >= 0 && old[q] == k + 1) cross |= 1u << q;
      const int c = __popc(cross);
      const int ci = wave_incl_scan(c);
      const int total = __builtin_amdgcn_readlane(ci, PMC_WAVE - 1);
      if (total) {
        int base = 0;
        if (l == 0) base = atomicAdd(&L.qend, total);
        int pos = __builtin_amdgcn_readfirstlane(base) + ci - c;
#pragma unroll
        for (int q = 0; q < TAIL_EPT; q++) {
          if (cross >> q & 1u) {
            atomicAdd(&L.deg2[u[q] >> 1], (uint32_t)TAIL_MARK << ((u[q] & 1) * 16));
            L.queue[pos++] = (uint16_t)u[q];
          }
        }
      }
    }
    __syncthreads();  // pre / rs are rewritten by the next chunk
  }
}

// The tail, run by workgroup 0 alone.  Starts with the frontier (round r,
// level k) in queue positions [0, F); writes rnd and core of every tail
// vertex at the end from the per-round queue boundaries.
__device__ void tail_run(int S, int F, int k, int r, const int *deg, int *core, int *rnd,
                         const TailBufs &T, TailLds &L, PeelCtrl *ctrl, int *lds,
                         long long *trace) {
  for (int w = threadIdx.x; w < (S + 1) / 2; w += blockDim.x) {
    uint32_t h[2];
    for (int q = 0; q < 2; q++) {
      const int i = 2 * w + q;
      h[q] = i >= S ? 0u : i < F ? (uint32_t)TAIL_MARK : (uint32_t)ld_dev(&deg[ld_dev(&T.glob[i])]);
    }
    L.deg2[w] = h[0] | h[1] << 16;
  }
  for (int i = threadIdx.x; i < F; i += blockDim.x) L.queue[i] = (uint16_t)i;
  for (int i = threadIdx.x; i <= S; i += blockDim.x) L.poff[i] = ld_dev(&T.poff[i]);
  if (threadIdx.x == 0) L.qend = F;
  __syncthreads();
  const int r0 = r;
  int qh = 0, qe = F, tr = 0;
  while (qh < qe || qe < S) {
    if (qh == qe) {
      int m = INT_MAX;
      for (int i = threadIdx.x; i < S; i += blockDim.x) {
        int d = tdeg(L.deg2, i);
        if (d < TAIL_MARK) m = min(m, d);
      }
      m = block_min(m, lds);
      k = max(k, m);
      for (int i = threadIdx.x; i < S; i += blockDim.x) {
        int d = tdeg(L.deg2, i);
        if (d < TAIL_MARK && d <= k) {
          atomicAdd(&L.deg2[i >> 1], (uint32_t)TAIL_MARK << ((i & 1) * 16));
          L.queue[atomicAdd(&L.qend, 1)] = (uint16_t)i;
        }
      }
      __syncthreads();
      qe = L.qend;
      trace_phase(trace, 3, S - qh);
      if (qe == qh) {  // no vertex left to queue: cannot happen with a consistent state
        if (threadIdx.x == 0) ctrl->err = 1;
        break;
      }
    }
    if (threadIdx.x == 0) {
      st_dev(&T.rstart[tr], qh);
      st_dev(&T.rk[tr], k);
    }
    const int Fr = qe - qh;
    tail_round(qh, qe, k, T, L);
    trace_phase(trace, 2, Fr);
    qh = qe;
    qe = L.qend;
    tr++;
    r++;
  }
  // round and core of every tail vertex from the queue boundaries
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int q = threadIdx.x; q < S; q += blockDim.x) {
    int lo = 0, hi = tr - 1;  // last round whose start is <= q
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (ld_dev(&T.rstart[mid]) <= q) lo = mid; else hi = mid - 1;
    }
    int v = ld_dev(&T.glob[L.queue[q]]);
    st_dev(&rnd[v], r0 + lo);
    core[v] = ld_dev(&T.rk[lo]);
  }
  if (threadIdx.x == 0) {
    ctrl->nrounds = r;
    ctrl->kmax = k;
  }
}

template <typename OffT>
__global__ void k_peel_init(int n, const OffT *__restrict__ off, int *deg, int *rnd, int *alive0,
                            unsigned *gone) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) {
    deg[v] = (int)(off[v + 1] - off[v]);
    rnd[v] = -1;
    alive0[v] = v;
    if ((v & 31) == 0) gone[v >> 5] = 0u;
  }
}

template <typename OffT>
__global__ void __launch_bounds__(PEEL_T) k_peel(int n, const OffT *__restrict__ off,
                                                 const int32_t *__restrict__ idx, int *deg,
                                                 int *core, int *rnd, int *porder, int *alive0,
                                                 int *alive1, int *junk, TailBufs T,
                                                 PeelCtrl *ctrl, long long *trace,
                                                 unsigned *gone) {
  __shared__ int lds[PEEL_T / PMC_WAVE + 1];
  __shared__ FrontierBuf fb;
  __shared__ TailLds tl;
  if (threadIdx.x == 0) fb.cnt = 0;
  unsigned long long gen = 0;
  const unsigned nb = gridDim.x;
  const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
  const int gsz = gridDim.x * blockDim.x;
  // frontier item p goes to wave (p % nwaves), waves numbered block-minor, so
  // consecutive items land on different CUs (and XCDs): a CU issues scattered
  // atomics about one lane per clock, so items sharing a CU serialise
  const int wave_g = blockIdx.x + gridDim.x * (threadIdx.x / PMC_WAVE);
  const int nwaves = gsz / PMC_WAVE;

  int head = 0, fend = 0, k = 0, r = 0, acur = 0, alen = n, jump = 0, phase = 0;
  bool tail_tried = T.cap <= 0;
  while (fend < n || head < fend) {
    if (head == fend) {
      const int *ain = acur ? alive1 : alive0;
      int *aout = acur ? alive0 : alive1;
      compact_live(ain, aout, alen, &ctrl->alive_cnt[1 - acur], &ctrl->kmin[jump & 1],
                   rnd, deg, lds);
      grid_sync(&ctrl->bar, nb, gen);
      k = max(k, ld_dev(&ctrl->kmin[jump & 1]));
      acur = 1 - acur;
      alen = ld_dev(&ctrl->alive_cnt[acur]);
      if (gtid == 0) {
        st_dev(&ctrl->alive_cnt[1 - acur], 0);
        st_dev(&ctrl->kmin[(jump + 1) & 1], INT_MAX);
        st_dev(&ctrl->cnt[(phase + 1) % 3], 0);
      }
      int *pc = &ctrl->cnt[phase % 3];
      mark_level(acur ? alive1 : alive0, alen, k, r, fend, pc, porder, rnd, core, deg, lds, gone);
      grid_sync(&ctrl->bar, nb, gen);
      fend += ld_dev(pc);
      trace_phase(trace, 1, alen);
      phase++;
      jump++;
    }
    if (!tail_tried && n - head <= TAIL_V) {
      tail_tried = true;
      if (tail_setup<OffT>(n, off, idx, rnd, porder, head, fend, acur ? alive1 : alive0, alen, T,
                           ctrl, lds, gen, wave_g, nwaves)) {
        if (blockIdx.x == 0) {
          const int S = fend - head + ld_dev(&ctrl->tail_cnt);
          if (S != n - head) {
            if (threadIdx.x == 0) ctrl->err = 2;
            return;
          }
          tail_run(S, fend - head, k, r, deg, core, rnd, T, tl, ctrl, lds, trace);
        }
        return;
      }
    }
    int *pc = &ctrl->cnt[phase % 3];
    if (gtid == 0) st_dev(&ctrl->cnt[(phase + 1) % 3], 0);
    run_round<OffT>(head, fend, k, r, pc, off, idx, deg, junk + gtid, rnd, core, porder, fb,
                    wave_g, nwaves, gone);
    grid_sync(&ctrl->bar, nb, gen);
    trace_phase(trace, 0, fend - head);
    head = fend;
    fend += ld_dev(pc);
    phase++;
    r++;
  }
  if (gtid == 0) {
    ctrl->nrounds = r;
    ctrl->kmax = k;
  }
}

__global__ void k_rank_scatter(int64_t n, const int32_t *order, int32_t *rank) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) rank[order[i]] = (int32_t)i;
}

__global__ void k_iota_keys(int64_t n, const int32_t *rnd, uint32_t *keys) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) keys[i] = (uint32_t)rnd[i];
}


long long *trace_buffer(Scratch &sc) {
  if (!getenv("PMC_PEEL_TRACE")) return nullptr;
  long long *t = sc.get<long long>(1 + 3 * TRACE_MAX);
  PMC_HIP(hipMemsetAsync(t, 0, sizeof(long long), sc.stream()));
  return t;
}

void trace_report(long long *dt, hipStream_t s, long long t_start) {
  std::vector<long long> h(1 + 3 * TRACE_MAX);
  PMC_HIP(hipMemcpyAsync(h.data(), dt, h.size() * sizeof(long long), hipMemcpyDeviceToHost, s));
  PMC_HIP(hipStreamSynchronize(s));
  long long cnt = h[0];
  double tot[4] = {0, 0, 0, 0};
  long long num[4] = {0, 0, 0, 0}, sz[4] = {0, 0, 0, 0};
  long long prev = -1;
  for (long long i = 0; i < cnt; i++) {
    int kind = (int)h[1 + 3 * i];
    long long size = h[2 + 3 * i], t = h[3 + 3 * i];
    if (prev >= 0) {
      tot[kind] += (t - prev) * 0.01;  // 100 MHz realtime clock -> us
    }
    num[kind]++;
    sz[kind] += size;
    prev = t;
  }
  const char *names[4] = {"round", "level jump", "tail round", "tail jump"};
  for (int k = 0; k < 4; k++)
    fprintf(stderr, "[peel trace] %-11s n=%6lld  total %9.1f us  mean %7.2f us  mean size %lld\n",
            names[k], num[k], tot[k], num[k] ? tot[k] / num[k] : 0.0, num[k] ? sz[k] / num[k] : 0);
  // rounds by frontier size: count, total and mean time
  const long long edges[] = {1, 2, 17, 257, 4097, 65537, 1ll << 40};
  for (int b = 0; b + 1 < 7; b++) {
    long long c = 0;
    double t = 0;
    for (long long i = 1; i < cnt; i++) {
      long long size = h[2 + 3 * i];
      if (h[1 + 3 * i] != 0 || size < edges[b] || size >= edges[b + 1]) continue;
      c++;
      t += (h[3 + 3 * i] - h[3 * i]) * 0.01;
    }
    if (c)
      fprintf(stderr, "[peel trace]   frontier [%lld, %lld): %5lld rounds  total %9.1f us  mean %7.2f us\n",
              edges[b], edges[b + 1], c, t, t / c);
  }
  (void)t_start;
}

}  // namespace

PeelResult run_peel(const GraphView &g, int32_t *core, int32_t *rnd, Scratch &sc, bool timed) {
  PeelResult res;
  hipStream_t s = sc.stream();
  if (g.n == 0) return res;
  int n = (int)g.n;
  int *deg = sc.get<int>(n);
  int *porder = sc.get<int>(n);
  int *a0 = sc.get<int>(n);
  int *a1 = sc.get<int>(n);
  unsigned *gone = sc.get<unsigned>(((size_t)n + 31) / 32);
  const DevInfo &di = dev_info();
  // one junk word per thread of the launch (target of no-op decrements)
  int *junk = sc.get<int>((size_t)di.cus * PEEL_T);
  TailBufs T;
  T.map = sc.get<int>(n);
  T.glob = sc.get<int>(TAIL_V);
  T.poff = sc.get<int>(TAIL_V + 1);
  T.cap = (int)std::min<int64_t>(g.nnz, (int64_t)1 << 24);
  T.adj = sc.get<int>(std::max(T.cap, 1));
  T.rstart = sc.get<int>(TAIL_V + 1);
  T.rk = sc.get<int>(TAIL_V + 1);
  if (getenv("PMC_PEEL_NO_TAIL")) T.cap = 0;
  PeelCtrl *ctrl = sc.get<PeelCtrl>(1);
  k_peel_ctrl_init<<<1, 1, 0, s>>>(ctrl);
  PMC_HIP(hipGetLastError());
  int per_cu = 0;
  PMC_DISPATCH_OFF(g, OffT, {
    PMC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_peel<OffT>, PEEL_T, 0));
    if (per_cu < 1) throw Error{5, "peel kernel cannot be made resident"};
    int nblocks = di.cus;
    const OffT *off = (const OffT *)g.off;
    const int32_t *idx = g.idx;
    long long *trace = trace_buffer(sc);
    void *args[] = {&n,     (void *)&off, (void *)&idx, &deg,  &core, &rnd, &porder,
                    &a0,    &a1,          &junk,        &T,    &ctrl, &trace, &gone};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
      PMC_HIP(hipEventCreate(&e0));
      PMC_HIP(hipEventCreate(&e1));
    }
    k_peel_init<OffT><<<(n + 255) / 256, 256, 0, s>>>(n, off, deg, rnd, a0, gone);
    PMC_HIP(hipGetLastError());
    if (timed) PMC_HIP(hipEventRecord(e0, s));
    PMC_HIP(hipLaunchCooperativeKernel((const void *)k_peel<OffT>, dim3(nblocks), dim3(PEEL_T),
                                       args, 0, s));
    if (timed) PMC_HIP(hipEventRecord(e1, s));
    PeelCtrl h;
    PMC_HIP(hipMemcpyAsync(&h, ctrl, sizeof(h), hipMemcpyDeviceToHost, s));
    PMC_HIP(hipStreamSynchronize(s));
    if (timed) {
      PMC_HIP(hipEventElapsedTime(&res.ms, e0, e1));
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
    }
    if (h.err) throw Error{5, "k-core peel reached an inconsistent state"};
    res.kmax = h.kmax;
    res.nrounds = h.nrounds;
    if (trace) trace_report(trace, s, 0);
  });
  return res;
}

void run_rank(int64_t n, const int32_t *rnd, int32_t nrounds, int32_t *rank, int32_t *order,
              Scratch &sc) {
  hipStream_t s = sc.stream();
  if (n == 0) return;
  uint32_t *keys = sc.get<uint32_t>(n);
  uint32_t *kout = sc.get<uint32_t>(n);
  int bits = 1;
  while (bits < 31 && (1u << bits) < (uint32_t)nrounds) bits++;
  int nb = (int)((n + 255) / 256);
  k_iota_keys<<<nb, 256, 0, s>>>(n, rnd, keys);
  radix_sort_pairs(keys, nullptr, kout, order, n, bits, sc);
  k_rank_scatter<<<nb, 256, 0, s>>>(n, order, rank);
  PMC_HIP(hipGetLastError());
}


}  // namespace pmc
