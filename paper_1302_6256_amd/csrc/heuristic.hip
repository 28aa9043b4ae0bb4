// heuristic.hip -- greedy heuristic clique (Alg. 1 and Sec. 4.1 of the paper),
// parallel over seeds as in Sec. 4.5.
//
// Per seed v (visited in decreasing degeneracy rank, i.e. decreasing core):
// skip it when K(v) < max; S = neighbours with K >= max; C = {v}; then every
// u of S in decreasing rank joins C when C + {u} is a clique; a larger C
// becomes H.  Equivalent formulation used here: keep the candidate set
// cand = S intersected with the neighbourhoods of the members added so far;
// the next member is the highest-ranked candidate (any candidate ranked above
// it was already adjacent to every earlier member, so first-fit would have
// taken it), after which cand shrinks to cand intersected with N(u).
//
// GPU design: one wavefront per seed.  A wave claims a chunk of consecutive
// seeds with one atomic and tests them against the running maximum with one
// lane per seed, so skipped seeds cost no claim of their own; the live seeds
// of the chunk are then processed in order.  The row of each new member is
// copied into the wave's LDS slice when it fits (it is searched once per
// candidate, so the copy replaces a dozen dependent global loads per
// candidate by one coalesced pass).  The candidate list lives in a per-wave global buffer (lanes stride over it,
// membership in N(u) by binary search in u's sorted row); the running maximum
// is a device-scope atomicMax read with relaxed loads.  A seed that raises the
// maximum writes its clique into the slot of the new size (only one seed can
// raise it to a given size, so slots are never shared).  With a frozen
// threshold every seed is processed against the same threshold and the
// winner is the packed maximum of (size, seed rank); its clique is rebuilt by
// a one-wave kernel afterwards.
#include "common.h"
#include "graph.h"
#include "tuning.h"

namespace pmc {
namespace {

constexpr int HEU_T = 256;

// Builds the greedy clique of seed v against threshold tau into cl[] and
// returns its size.  Called by a whole wave.
// Neighbourhood bitmaps of the hub_count highest-ranked vertices (bitmap h
// belongs to the vertex of rank n-1-h).  Most seeds pick these vertices first,
// and their rows are the longest, so a candidate's adjacency to one of them
// is one bit instead of a search in a row of thousands.
struct HubMaps {
  const uint64_t *bits;
  int count;
  int64_t words;  // per bitmap
  int n;
};

template <typename OffT>
__global__ void k_hub_bits(const OffT *__restrict__ off, const int32_t *__restrict__ idx,
                           const int *__restrict__ order, int n, int64_t words, uint64_t *bits) {
  const int h = blockIdx.x;
  const int u = order[n - 1 - h];
  uint64_t *bm = bits + (size_t)h * words;
  const int64_t s = (int64_t)off[u], e = (int64_t)off[u + 1];
  for (int64_t j = s + threadIdx.x; j < e; j += blockDim.x) {
    const int x = idx[j];
    atomicOr((unsigned long long *)&bm[x >> 6], 1ull << (x & 63));
  }
}

template <typename OffT>
__device__ int seed_clique(int v, int tau, const OffT *__restrict__ off,
                           const int32_t *__restrict__ idx, const int *__restrict__ core,
                           const int *__restrict__ rank, int *cid, int *crk, int *cl,
                           int *rowc, int rowcap, const HubMaps &hubs, int *lcand,
                           int lcap, int stop_le = -1) {
  const int l = lane();
  int64_t s = (int64_t)off[v], e = (int64_t)off[v + 1];
  // candidate list in the wave's LDS slice when the seed's row fits
  if (e - s <= lcap) {
    cid = lcand;
    crk = lcand + lcap;
  }
  int cnt = 0;
  for (int64_t jb = s; jb < e; jb += PMC_WAVE) {
    int64_t j = jb + l;
    bool ok = j < e;
    int u = ok ? idx[j] : 0;
    bool keep = ok && core[u] >= tau;
    uint64_t m = ballot(keep);
    if (keep) {
      int pos = cnt + __popcll(m & lanemask_lt());
      cid[pos] = u;
      crk[pos] = rank[u];
    }
    cnt += __popcll(m);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  if (l == 0) cl[0] = v;
  int csize = 1;
  // stop_le >= 0: a clique that cannot grow beyond stop_le vertices is of no
  // use to the caller (it only records cliques larger than the running
  // maximum), so the greedy ends as soon as C plus every candidate left is
  // that small; the returned size is then <= stop_le
  while (cnt > 0 && csize + cnt > stop_le) {
    int best = -1, bu = -1;
    for (int i = l; i < cnt; i += PMC_WAVE) {
      int r = crk[i];
      if (r > best) { best = r; bu = cid[i]; }
    }
    int bmax = wave_max(best);
    uint64_t who = ballot(best == bmax);
    int u = shfl(bu, __ffsll((unsigned long long)who) - 1);
    if (l == 0) cl[csize] = u;
    csize++;
    const int hid = hubs.n - 1 - bmax;  // u's rank is bmax
    if (hid < hubs.count) {
      const uint64_t *hm = hubs.bits + (size_t)hid * hubs.words;
      int ncnt = 0;
      for (int ib = 0; ib < cnt; ib += PMC_WAVE) {
        int i = ib + l;
        bool ok = i < cnt;
        int x = ok ? cid[i] : 0;
        int r = ok ? crk[i] : 0;
        bool keep = ok && x != u && ((hm[x >> 6] >> (x & 63)) & 1ull);
        uint64_t m = ballot(keep);
        if (keep) {
          int pos = ncnt + __popcll(m & lanemask_lt());
          cid[pos] = x;
          crk[pos] = r;
        }
        ncnt += __popcll(m);
      }
      cnt = ncnt;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
      continue;
    }
    int64_t us = (int64_t)off[u];
    int du = (int)((int64_t)off[u + 1] - us);
    const int32_t *row = idx + us;
    if (du <= rowcap) {
      for (int ib = 0; ib < du; ib += 4 * PMC_WAVE) {
        int t[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
          int i = ib + q * PMC_WAVE + l;
          t[q] = i < du ? row[i] : 0;
        }
#pragma unroll
        for (int q = 0; q < 4; q++) {
          int i = ib + q * PMC_WAVE + l;
          if (i < du) rowc[i] = t[q];
        }
      }
      wave_sync();
      row = rowc;
    }
    int ncnt = 0;
    for (int ib = 0; ib < cnt; ib += PMC_WAVE) {
      int i = ib + l;
      bool ok = i < cnt;
      int x = ok ? cid[i] : 0;
      int r = ok ? crk[i] : 0;
      bool keep = false;
      if (ok && x != u) {
        int p = lower_bound(row, du, x);
        keep = p < du && row[p] == x;
      }
      uint64_t m = ballot(keep);
      if (keep) {
        int pos = ncnt + __popcll(m & lanemask_lt());
        cid[pos] = x;
        crk[pos] = r;
      }
      ncnt += __popcll(m);
    }
    cnt = ncnt;
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  return csize;
}

template <typename OffT>
__global__ void __launch_bounds__(HEU_T)
    k_heuristic(int n, const OffT *__restrict__ off, const int32_t *__restrict__ idx,
                const int *__restrict__ core, const int *__restrict__ rank,
                const int *__restrict__ order, const int *__restrict__ seed_order,
                int frozen_tau, Bounds B, CliqueState *st, int *candbuf, int dmax,
                int *cliquebuf, int kcap, int chunk, int rowcap, int lcap, HubMaps hubs) {
  extern __shared__ int heu_lds[];
  // per-wave LDS slice: candidate ids and ranks (lcap each), then the row cache
  int *lcand = heu_lds + (threadIdx.x / PMC_WAVE) * (2 * lcap + rowcap);
  int *rowc = lcand + 2 * lcap;
  const int wg = (blockIdx.x * blockDim.x + threadIdx.x) / PMC_WAVE;
  const int l = lane();
  int *cid = candbuf + (size_t)wg * 2 * dmax;
  int *crk = cid + dmax;
  int *cl = cliquebuf + (size_t)wg * kcap;
  const bool frozen = frozen_tau >= 0;
  // with one graph and seeds in decreasing rank, a seed below the running
  // maximum ends the wave: every later seed has no larger core
  const bool monotone = !seed_order && !B.gid;
  // seeds processed by this wave, added to the shared counter once at the end
  // (one atomic per seed on one address throttled large batches)
  unsigned long long done = 0;
  bool fin = false;
  while (!fin) {
    const int c0 = atomic_add_wave(&st->seed_next, chunk);
    if (c0 >= n) break;
    const int si = c0 + l;
    const bool in = l < chunk && si < n;
    const int v = in ? (seed_order ? seed_order[si] : order[n - 1 - si]) : 0;
    const int g = in ? graph_of(B.gid, v) : 0;
    const bool live = in && (frozen || core[v] >= ld_relaxed(&B.bound[g]));
    uint64_t todo = ballot(live);
    if (monotone) {
      // seeds of a chunk have nonincreasing core: everything from the first
      // failing seed on fails too, and so does every later chunk
      uint64_t fail = ballot(in && !live);
      if (fail) {
        todo &= (1ull << (__ffsll((unsigned long long)fail) - 1)) - 1ull;
        fin = true;
      }
    }
    while (todo) {
      const int src = __ffsll((unsigned long long)todo) - 1;
      todo &= todo - 1;
      const int sv = shfl(v, src), sg = shfl(g, src);
      const int tau = frozen ? frozen_tau : ld_relaxed(&B.bound[sg]);
      if (!frozen && core[sv] < tau) {
        if (monotone) {
          fin = true;
          break;
        }
        continue;
      }
      int csize =
          seed_clique<OffT>(sv, tau, off, idx, core, rank, cid, crk, cl, rowc, rowcap, hubs, lcand,
                            lcap, frozen ? -1 : tau);
      done++;
      if (frozen) {
        if (l == 0)
          atomic_max_u64(&B.packed[sg], ((unsigned long long)csize << 32) | (unsigned)rank[sv]);
      } else if (csize > tau) {
        // a clique no larger than the maximum read before the seed cannot
        // raise it (the maximum only grows)
        int old = 0;
        if (l == 0) old = atomic_max(&B.bound[sg], csize);
        old = shfl(old, 0);
        if (old < csize) {
          int *dst = slot_ptr(B, sg, csize);
          for (int i = l; i < csize; i += PMC_WAVE) dst[i] = cl[i];
        }
      }
    }
  }
  if (l == 0 && done) atomic_add_u64(&st->seeds_done, done);
}

// Frozen-threshold winners, one wave per graph: rebuild the winning seed's
// clique into the slot of its size.
template <typename OffT>
__global__ void __launch_bounds__(PMC_WAVE)
    k_heuristic_winner(const OffT *__restrict__ off, const int32_t *__restrict__ idx,
                       const int *__restrict__ core, const int *__restrict__ rank,
                       const int *__restrict__ order, int frozen_tau, Bounds B, int *cid,
                       int *crk, int *cl, int dmax, int kcap, int rowcap, int lcap,
                       HubMaps hubs) {
  extern __shared__ int heu_lds[];
  const int g = blockIdx.x;
  cid += (size_t)g * 2 * dmax;
  crk = cid + dmax;
  cl += (size_t)g * kcap;
  unsigned long long p = B.packed[g];
  int size = (int)(p >> 32);
  if (size == 0) return;
  int v = order[(int)(p & 0xffffffffu)];
  int csize =
      seed_clique<OffT>(v, frozen_tau, off, idx, core, rank, cid, crk, cl, heu_lds + 2 * lcap,
                        rowcap, hubs, heu_lds, lcap);
  int *dst = slot_ptr(B, g, csize);
  for (int i = lane(); i < csize; i += PMC_WAVE) dst[i] = cl[i];
  if (lane() == 0) atomic_max(&B.bound[g], csize);
}

// ---- clique-peeling order (Sec. 6.2): passes over the remaining vertices.
// Pass 0: every remaining seed grows H(v) (remaining neighbours, decreasing
// rank, first fit) and raises owner[x] to key(v) = (|H(v)|, rank(v)) for its
// members.  Pass 1: a seed that owns all its members is taken: its key and
// members go to the taken list.  The host then sorts the taken cliques by
// decreasing key and k_co_place writes them out.
template <typename OffT>
__global__ void __launch_bounds__(HEU_T)
    k_co_pass(int pass, int n, const OffT *__restrict__ off, const int32_t *__restrict__ idx,
              const int *__restrict__ alive, const int *__restrict__ rank,
              unsigned long long *owner, int *head, int *ntaken, unsigned long long *tkey,
              long long *toff, unsigned long long *mcount, int *members, int *candbuf, int dmax,
              int *cliquebuf, int kcap, int rowcap, int lcap) {
  extern __shared__ int heu_lds[];
  int *lcand = heu_lds + (threadIdx.x / PMC_WAVE) * (2 * lcap + rowcap);
  int *rowc = lcand + 2 * lcap;
  const int wg = (blockIdx.x * blockDim.x + threadIdx.x) / PMC_WAVE;
  const int l = lane();
  int *cid = candbuf + (size_t)wg * 2 * dmax;
  int *crk = cid + dmax;
  int *cl = cliquebuf + (size_t)wg * kcap;
  const HubMaps nohubs{nullptr, 0, 1, n};
  while (true) {
    const int c0 = atomic_add_wave(head, PMC_WAVE);
    if (c0 >= n) return;
    const int v = c0 + l;
    uint64_t todo = ballot(v < n && alive[v]);
    while (todo) {
      const int src = __ffsll((unsigned long long)todo) - 1;
      todo &= todo - 1;
      const int sv = c0 + src;
      const int csize = seed_clique<OffT>(sv, 1, off, idx, alive, rank, cid, crk, cl, rowc, rowcap,
                                          nohubs, lcand, lcap);
      const unsigned long long key = ((unsigned long long)csize << 32) | (unsigned)rank[sv];
      if (pass == 0) {
        for (int i = l; i < csize; i += PMC_WAVE)
          atomicMax((unsigned long long *)&owner[cl[i]], key);
      } else {
        bool mine = true;
        for (int i = l; i < csize; i += PMC_WAVE) mine = mine && owner[cl[i]] == key;
        if (ballot(!mine) == 0ull) {
          long long m0 = 0;
          if (l == 0) {
            const int j = atomic_add(ntaken, 1);
            m0 = (long long)atomic_add_u64(mcount, (unsigned long long)csize);
            tkey[j] = key;
            toff[j] = m0;
          }
          m0 = (long long)shfl64((uint64_t)m0, 0);
          for (int i = l; i < csize; i += PMC_WAVE) members[m0 + i] = cl[i];
        }
      }
    }
  }
}

// Sort keys of the taken cliques: low word ~rank (pass 1), high word ~size
// (pass 2, stable), so ascending keys are decreasing (size, rank).
__global__ void k_co_keys(int m, const unsigned long long *tkey, const int32_t *perm, int hi,
                          uint32_t *keys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const unsigned long long k = tkey[perm ? perm[i] : i];
  keys[i] = hi ? ~(uint32_t)(k >> 32) : ~(uint32_t)(k & 0xffffffffu);
}

__global__ void k_co_sizes(int m, const unsigned long long *tkey, const int32_t *perm, int32_t *sz) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) sz[i] = (int32_t)(tkey[perm[i]] >> 32);
}

// One wave per taken clique j (in placing order): members by decreasing degree
// (ties by id) at positions base + pos[j] ...; removes them.
template <typename OffT>
__global__ void __launch_bounds__(PMC_WAVE)
    k_co_place(int m, const OffT *__restrict__ off, const int32_t *perm,
               const unsigned long long *tkey, const long long *toff, const int *members,
               const int64_t *pos, int64_t base, int64_t nb0, int *alive, int32_t *order,
               int64_t *block) {
  const int j = blockIdx.x;
  if (j >= m) return;
  const int e = perm[j];
  const int size = (int)(tkey[e] >> 32);
  const int *mem = members + toff[e];
  const int64_t at = base + pos[j];
  if (lane() == 0) block[nb0 + j] = at;
  for (int i = lane(); i < size; i += PMC_WAVE) {
    const int x = mem[i];
    const int64_t dx = (int64_t)off[x + 1] - (int64_t)off[x];
    int p = 0;
    for (int q = 0; q < size; q++) {
      const int y = mem[q];
      const int64_t dy = (int64_t)off[y + 1] - (int64_t)off[y];
      p += dy > dx || (dy == dx && y < x);
    }
    order[at + p] = x;
    alive[x] = 0;
  }
}

__global__ void k_co_alive(int n, int *alive) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) alive[i] = 1;
}

}  // namespace

int64_t run_clique_order(const GraphView &g, const int32_t *rank, int32_t kmax, int32_t *order,
                         int64_t *block, Scratch &sc) {
  hipStream_t s = sc.stream();
  const int n = (int)g.n;
  if (n == 0) return 0;
  int dmax = 0;
  {
    int32_t *dtmp = sc.get<int32_t>(1);
    PMC_HIP(hipMemsetAsync(dtmp, 0, sizeof(int32_t), s));
    max_degree(g, dtmp, s);
    PMC_HIP(hipMemcpyAsync(&dmax, dtmp, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PMC_HIP(hipStreamSynchronize(s));
  }
  if (dmax < 1) dmax = 1;
  const int kcap = kmax + 1;
  const DevInfo &di = dev_info();
  int64_t nw = (int64_t)di.cus * 8;
  const int64_t cap_w = ((int64_t)1 << 31) / ((int64_t)dmax * 8 + 1);
  if (nw > cap_w) nw = cap_w < 4 ? 4 : cap_w;
  nw = (nw + 3) / 4 * 4;
  if ((int64_t)n + nw * PMC_WAVE >= INT32_MAX) throw Error{1, "graph too large for the clique order"};
  int *candbuf = sc.get<int>((size_t)nw * 2 * dmax);
  int *cliquebuf = sc.get<int>((size_t)nw * kcap);
  int share = di.lds_per_cu / 4 / 8;
  if ((int64_t)share * (HEU_T / PMC_WAVE) * 4 > di.max_lds) share = di.max_lds / 4 / (HEU_T / PMC_WAVE);
  const int lcap = share * 3 / 10 / PMC_WAVE * PMC_WAVE;
  const int rowcap = std::min(4096, (share - 2 * lcap) / PMC_WAVE * PMC_WAVE);
  const size_t lds_bytes = (size_t)(2 * lcap + rowcap) * 4 * (HEU_T / PMC_WAVE);
  int *alive = sc.get<int>(n);
  unsigned long long *owner = sc.get<unsigned long long>(n);
  int *head = sc.get<int>(2);  // claim counter, taken count
  unsigned long long *mcount = sc.get<unsigned long long>(1);
  unsigned long long *tkey = sc.get<unsigned long long>(n);
  long long *toff = sc.get<long long>(n);
  int *members = sc.get<int>(n);
  uint32_t *k0 = sc.get<uint32_t>(n), *k1 = sc.get<uint32_t>(n);
  int32_t *p0 = sc.get<int32_t>(n), *p1 = sc.get<int32_t>(n);
  int32_t *sz = sc.get<int32_t>(n);
  int64_t *pos = sc.get<int64_t>((size_t)n + 1);
  k_co_alive<<<(n + 255) / 256, 256, 0, s>>>(n, alive);
  PMC_HIP(hipGetLastError());
  int64_t placed = 0, nb = 0;
  PMC_DISPATCH_OFF(g, OffT, {
    const OffT *off = (const OffT *)g.off;
    while (placed < n) {
      PMC_HIP(hipMemsetAsync(owner, 0, sizeof(unsigned long long) * n, s));
      PMC_HIP(hipMemsetAsync(mcount, 0, sizeof(unsigned long long), s));
      for (int pass = 0; pass < 2; pass++) {
        PMC_HIP(hipMemsetAsync(head, 0, sizeof(int) * 2, s));
        k_co_pass<OffT><<<(int)(nw / 4), HEU_T, lds_bytes, s>>>(
            pass, n, off, g.idx, alive, rank, owner, head, head + 1, tkey, toff, mcount, members,
            candbuf, dmax, cliquebuf, kcap, rowcap, lcap);
        PMC_HIP(hipGetLastError());
      }
      int m = 0;
      PMC_HIP(hipMemcpyAsync(&m, head + 1, sizeof(int), hipMemcpyDeviceToHost, s));
      PMC_HIP(hipStreamSynchronize(s));
      if (m <= 0) throw Error{5, "clique order made no progress"};
      const int nbk = (m + 255) / 256;
      k_co_keys<<<nbk, 256, 0, s>>>(m, tkey, nullptr, 0, k0);
      radix_sort_pairs(k0, nullptr, k1, p0, m, 32, sc);
      k_co_keys<<<nbk, 256, 0, s>>>(m, tkey, p0, 1, k0);
      radix_sort_pairs(k0, p0, k1, p1, m, 32, sc);
      k_co_sizes<<<nbk, 256, 0, s>>>(m, tkey, p1, sz);
      PMC_HIP(hipGetLastError());
      scan_counts(sz, pos, m, sc);
      int64_t total = 0;
      PMC_HIP(hipMemcpyAsync(&total, pos + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      PMC_HIP(hipStreamSynchronize(s));
      k_co_place<OffT><<<m, PMC_WAVE, 0, s>>>(m, off, p1, tkey, toff, members, pos, placed, nb,
                                              alive, order, block);
      PMC_HIP(hipGetLastError());
      placed += total;
      nb += m;
    }
  });
  PMC_HIP(hipMemcpyAsync(block + nb, &placed, sizeof(int64_t), hipMemcpyHostToDevice, s));
  PMC_HIP(hipStreamSynchronize(s));
  return nb;
}

KTimer::KTimer(hipStream_t st) : s(st) {
  PMC_HIP(hipEventCreate(&a));
  PMC_HIP(hipEventCreate(&b));
}
KTimer::~KTimer() {
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
}
void KTimer::start() { PMC_HIP(hipEventRecord(a, s)); }
float KTimer::stop() {
  PMC_HIP(hipEventRecord(b, s));
  PMC_HIP(hipEventSynchronize(b));
  float ms = 0;
  PMC_HIP(hipEventElapsedTime(&ms, a, b));
  return ms;
}

float run_heuristic(const GraphView &g, const int32_t *core, const int32_t *rank,
                    const int32_t *order, const int32_t *seed_order, int32_t kmax,
                    int32_t frozen_tau, const Bounds &B, CliqueState *st, Scratch &sc) {
  hipStream_t s = sc.stream();
  int n = (int)g.n;
  if (n == 0) return 0.f;
  // the largest degree bounds every candidate list
  int dmax = 0;
  {
    int32_t *dtmp = sc.get<int32_t>(1);
    PMC_HIP(hipMemsetAsync(dtmp, 0, sizeof(int32_t), s));
    max_degree(g, dtmp, s);
    PMC_HIP(hipMemcpyAsync(&dmax, dtmp, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PMC_HIP(hipStreamSynchronize(s));
  }
  if (dmax < 1) dmax = 1;
  int kcap = kmax + 1;
  const DevInfo &di = dev_info();
  int64_t nw = (int64_t)di.cus * tuning().heuristic_waves_per_cu[B.gid ? 1 : 0];
  // keep the candidate buffers to about 2 GiB
  int64_t cap_w = ((int64_t)1 << 31) / ((int64_t)dmax * 8 + 1);
  if (nw > cap_w) nw = cap_w < 4 ? 4 : cap_w;
  nw = (nw + 3) / 4 * 4;
  // one graph in decreasing rank ends each wave at its first seed below the
  // bound, so a small chunk wastes few seeds; any other seed order claims and
  // tests every seed, which a larger chunk makes cheap (the batch setting)
  int chunk = tuning().heuristic_chunk[B.gid || seed_order ? 1 : 0];
  // one graph: a claim of several seeds runs them on one wave, so it pays only
  // when every wave gets many claims (on a graph of a few thousand vertices
  // whose seeds are all heavy, claims of 4 left three waves in four idle and
  // tripled the heuristic)
  if (!B.gid && !seed_order)
    chunk = (int)std::min<int64_t>(chunk, std::max<int64_t>(1, (int64_t)n / (nw * 64)));
  chunk = std::min(std::max(chunk, 1), PMC_WAVE);
  // the claim counter ends below n + (waves * chunk)
  if ((int64_t)n + nw * chunk >= INT32_MAX) chunk = 1;
  if ((int64_t)n + nw >= INT32_MAX) throw Error{1, "graph too large for the heuristic seed counter"};
  int64_t nbuf = std::max<int64_t>(nw, frozen_tau >= 0 ? B.G : 0);
  int *candbuf = sc.get<int>((size_t)nbuf * 2 * dmax);
  int *cliquebuf = sc.get<int>((size_t)nbuf * kcap);
  // LDS row cache per wave: what the waves of a CU can share, at most 4096
  // entries (a row longer than the cache is searched in global memory)
  const int waves_cu = std::max<int>(1, (int)(nw / std::max(di.cus, 1)));
  // per wave: 3/10 of its share for candidate ids, 3/10 for ranks, the rest
  // for the row cache (all multiples of 64 entries)
  int share = di.lds_per_cu / 4 / std::max(waves_cu, 4);
  if ((int64_t)share * (HEU_T / PMC_WAVE) * 4 > di.max_lds) share = di.max_lds / 4 / (HEU_T / PMC_WAVE);
  const int lcap = share * 3 / 10 / PMC_WAVE * PMC_WAVE;
  const int rowcap = std::min(4096, (share - 2 * lcap) / PMC_WAVE * PMC_WAVE);
  const size_t wave_bytes = (size_t)(2 * lcap + rowcap) * 4;
  const size_t lds_bytes = wave_bytes * (HEU_T / PMC_WAVE);
  // hub bitmaps: up to 1,024 of them, at most 256 MiB together
  HubMaps hubs{nullptr, 0, (n + 63) / 64, n};
  hubs.count = (int)std::min<int64_t>(std::min<int64_t>(1024, n),
                                      ((int64_t)256 << 20) / 8 / std::max<int64_t>(hubs.words, 1));
  uint64_t *hubbits = nullptr;
  if (hubs.count > 0) {
    hubbits = sc.get<uint64_t>((size_t)hubs.count * hubs.words);
    PMC_HIP(hipMemsetAsync(hubbits, 0, sizeof(uint64_t) * hubs.count * hubs.words, s));
    hubs.bits = hubbits;
  }
  KTimer kt(s);
  float ms = 0.f;
  PMC_DISPATCH_OFF(g, OffT, {
    kt.start();
    if (hubs.count > 0) {
      k_hub_bits<OffT><<<hubs.count, 256, 0, s>>>((const OffT *)g.off, g.idx, order, n, hubs.words,
                                                 hubbits);
      PMC_HIP(hipGetLastError());
    }
    k_heuristic<OffT><<<nw / 4, HEU_T, lds_bytes, s>>>(n, (const OffT *)g.off, g.idx, core, rank, order,
                                               seed_order, frozen_tau, B, st, candbuf, dmax,
                                               cliquebuf, kcap, chunk, rowcap, lcap, hubs);
    PMC_HIP(hipGetLastError());
    ms = kt.stop();
    if (frozen_tau >= 0) {
      k_heuristic_winner<OffT><<<B.G, PMC_WAVE, wave_bytes, s>>>((const OffT *)g.off, g.idx, core, rank,
                                                        order, frozen_tau, B, candbuf,
                                                        candbuf + dmax, cliquebuf, dmax, kcap,
                                                        rowcap, lcap, hubs);
      PMC_HIP(hipGetLastError());
    }
  });
  return ms;
}

}  // namespace pmc
