// prune.hip -- explicit pruning and orientation (Sec. 4.2 and the reduced
// neighbourhoods N_R of Sec. 4.3), and the root queue of the search loop.
//
// Pruning removes every vertex whose core is below the bound of its graph (a
// single graph is a batch of one).  Survivors are labelled 0..n'-1 in rank
// order; since the rank is nondecreasing in core within a graph, a single
// graph's survivors are a suffix of the ranks and label = rank - r0.  The
// graph becomes an oriented graph on labels: the row of a survivor keeps its
// neighbours of higher rank (searched vertices of lower rank are excluded
// from later neighbourhoods, and every kept neighbour has core >= K(v) >=
// bound, so it survived too).  Rows are sorted, so the local index of a
// subproblem follows the degeneracy rank.
//
// GPU design: keep flags in rank order, the project's scan for labels, then a
// count pass and a fill pass with one wavefront per survivor streaming its
// CSR row coalesced and gathering its neighbours' ranks and labels; kept
// labels are compacted with ballot/prefix counts, sorted in LDS by a bitonic
// network and written contiguously.  Rows longer than the wave's LDS tile go
// to a workgroup kernel with a larger tile.
#include <climits>

#include "common.h"
#include "graph.h"
#include "search.h"

namespace pmc {
namespace {

constexpr int OR_T = 256;            // 4 waves per block
constexpr int OR_WAVE_CAP = 1024;    // row tile of one wave (4 KB LDS)
constexpr int OR_BIG_T = 1024;
constexpr int OR_BIG_CAP = 16384;    // row tile of the workgroup kernel (64 KB LDS)
constexpr int DEG_SLOTS = 64;        // partial counters of the survivors' row entries

// Survivors: position >= min_rank in the search order (the roots already
// searched are a prefix of it and are dropped by a re-prune) and core >= the
// bound of the vertex's graph.  The search order is the degeneracy order
// (order = rank^-1) or, with order NULL, the vertex ids (native order).
__global__ void k_keep_flags(int n, const int32_t *__restrict__ order,
                             const int32_t *__restrict__ core, const int32_t *__restrict__ gid,
                             const int32_t *__restrict__ bound, int min_rank, int32_t *flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int v = order ? order[i] : i;
  flag[i] = i >= min_rank && core[v] >= bound[graph_of(gid, v)] ? 1 : 0;
}

__global__ void k_label_scatter(int n, const int32_t *__restrict__ order,
                                const int32_t *__restrict__ core, const int32_t *__restrict__ gid,
                                const int32_t *__restrict__ flag, const int64_t *__restrict__ pos,
                                int32_t *vlabel, int32_t *lab_vertex, int32_t *lab_core,
                                int32_t *lab_gid) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int v = order ? order[i] : i;
  if (flag[i]) {
    int L = (int)pos[i];
    vlabel[v] = L;
    lab_vertex[L] = v;
    lab_core[L] = core[v];
    if (lab_gid) lab_gid[L] = gid[v];
  } else {
    vlabel[v] = -1;
  }
}

// A neighbour u of the survivor v (label i) stays in v's oriented row when it
// comes later in the search order: in degeneracy order a higher rank, which
// is a label above i (lu = vlabel[u]: the survivors' labels follow their
// ranks, and a neighbour ranked above v has core >= K(v), so it survived
// too; one gather, the one the fill needs anyway, instead of the rank and
// then the label); in native order a larger id and a survivor itself.
__device__ __forceinline__ bool later(bool by_rank, int lu, int u, int v, int i) {
  return by_rank ? lu > i : (u > v && lu >= 0);
}

template <typename OffT>
__global__ void __launch_bounds__(OR_T)
    k_orient_count(int nn, const OffT *__restrict__ off, const int32_t *__restrict__ idx,
                   const int *__restrict__ rank, const int *__restrict__ vlabel,
                   const int *__restrict__ lab_vertex, int *cnt, int *big_list, int *big_n,
                   unsigned long long *deg_sum) {
  int w = (blockIdx.x * blockDim.x + threadIdx.x) / PMC_WAVE;
  int nw = gridDim.x * blockDim.x / PMC_WAVE;
  int l = lane();
  unsigned long long rows = 0;  // entries of the survivors' rows this wave streams
  const bool by_rank = rank != nullptr;
  for (int i = w; i < nn; i += nw) {
    int v = lab_vertex[i];
    int64_t s = (int64_t)off[v], e = (int64_t)off[v + 1];
    rows += (unsigned long long)(e - s);
    int c = 0;
    for (int64_t jb = s; jb < e; jb += PMC_WAVE) {
      int64_t j = jb + l;
      const int u = j < e ? idx[j] : -1;
      const int lu = u >= 0 ? vlabel[u] : -1;
      bool keep = u >= 0 && later(by_rank, lu, u, v, i);
      c += __popcll(ballot(keep));
    }
    if (l == 0) {
      cnt[i] = c;
      if (c > OR_WAVE_CAP) big_list[atomic_add(big_n, 1)] = i;
    }
  }
  // spread over DEG_SLOTS counters so that no address takes more than a few
  // hundred of the waves' atomics
  if (l == 0 && rows) atomic_add_u64(&deg_sum[blockIdx.x % DEG_SLOTS], rows);
}

// Bitonic sort of buf[0..p) (p a power of two) by one wave.
__device__ void wave_bitonic(int *buf, int p) {
  for (int k = 2; k <= p; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane(); i < p; i += PMC_WAVE) {
        int x = i ^ j;
        if (x > i) {
          int a = buf[i], b = buf[x];
          bool up = (i & k) == 0;
          if ((a > b) == up) {
            buf[i] = b;
            buf[x] = a;
          }
        }
      }
      wave_sync();
    }
  }
}

template <typename OffT>
__global__ void __launch_bounds__(OR_T)
    k_orient_fill(int nn, const OffT *__restrict__ off, const int32_t *__restrict__ idx,
                  const int *__restrict__ rank, const int *__restrict__ lab_vertex,
                  const int *__restrict__ vlabel, const int64_t *__restrict__ poff,
                  int32_t *padj) {
  __shared__ int tile[OR_T / PMC_WAVE][OR_WAVE_CAP];
  int wl = threadIdx.x / PMC_WAVE;
  int *buf = tile[wl];
  int w = (blockIdx.x * blockDim.x + threadIdx.x) / PMC_WAVE;
  int nw = gridDim.x * blockDim.x / PMC_WAVE;
  int l = lane();
  for (int i = w; i < nn; i += nw) {
    int64_t o = poff[i];
    int c = (int)(poff[i + 1] - o);
    if (c > OR_WAVE_CAP || c == 0) continue;
    int v = lab_vertex[i];
    int64_t s = (int64_t)off[v], e = (int64_t)off[v + 1];
    int w0 = 0;
    for (int64_t jb = s; jb < e; jb += PMC_WAVE) {
      int64_t j = jb + l;
      int u = j < e ? idx[j] : -1;
      const int lu = u >= 0 ? vlabel[u] : -1;
      bool keep = u >= 0 && later(rank != nullptr, lu, u, v, i);
      uint64_t m = ballot(keep);
      if (keep) buf[w0 + __popcll(m & lanemask_lt())] = lu;
      w0 += __popcll(m);
    }
    int p = 1;
    while (p < c) p <<= 1;
    for (int t = c + l; t < p; t += PMC_WAVE) buf[t] = INT_MAX;
    wave_sync();
    wave_bitonic(buf, p);
    for (int t = l; t < c; t += PMC_WAVE) padj[o + t] = buf[t];
    wave_sync();
  }
}

template <typename OffT>
__global__ void __launch_bounds__(OR_BIG_T)
    k_orient_fill_big(const OffT *__restrict__ off, const int32_t *__restrict__ idx,
                      const int *__restrict__ rank, const int *__restrict__ lab_vertex,
                      const int *__restrict__ vlabel, const int64_t *__restrict__ poff,
                      int32_t *padj, const int *big_list, const int *big_n, int *err) {
  __shared__ int buf[OR_BIG_CAP];
  __shared__ int wcnt[OR_BIG_T / PMC_WAVE + 1];
  int nbig = *big_n;
  for (int b = blockIdx.x; b < nbig; b += gridDim.x) {
    int i = big_list[b];
    int64_t o = poff[i];
    int c = (int)(poff[i + 1] - o);
    if (c > OR_BIG_CAP) {
      if (threadIdx.x == 0) atomicExch(err, 2);
      continue;
    }
    int v = lab_vertex[i];
    int64_t s = (int64_t)off[v], e = (int64_t)off[v + 1];
    // block-wide compaction in row order
    int wid = threadIdx.x / PMC_WAVE;
    int base = 0;
    for (int64_t jb = s; jb < e; jb += OR_BIG_T) {
      int64_t j = jb + threadIdx.x;
      int u = j < e ? idx[j] : -1;
      const int lu = u >= 0 ? vlabel[u] : -1;
      bool keep = u >= 0 && later(rank != nullptr, lu, u, v, i);
      uint64_t m = ballot(keep);
      if (lane() == 0) wcnt[wid] = __popcll(m);
      __syncthreads();
      int pre = 0, tot = 0;
      for (int q = 0; q < OR_BIG_T / PMC_WAVE; q++) {
        if (q < wid) pre += wcnt[q];
        tot += wcnt[q];
      }
      if (keep) buf[base + pre + __popcll(m & lanemask_lt())] = lu;
      base += tot;
      __syncthreads();
    }
    int p = 1;
    while (p < c) p <<= 1;
    for (int t = c + threadIdx.x; t < p; t += OR_BIG_T) buf[t] = INT_MAX;
    __syncthreads();
    for (int k = 2; k <= p; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int t = threadIdx.x; t < p; t += OR_BIG_T) {
          int x = t ^ j;
          if (x > t) {
            int a = buf[t], bb = buf[x];
            bool up = (t & k) == 0;
            if ((a > bb) == up) {
              buf[t] = bb;
              buf[x] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int t = threadIdx.x; t < c; t += OR_BIG_T) padj[o + t] = buf[t];
    __syncthreads();
  }
}

// ---------------------------------------------------------------- queue
// Class of a root by its oriented degree d: bitset words W = ceil(d/64)
// rounded up to a power of two; class c holds W = 2^c.  Non-roots get
// QCLASS_NONE.
__device__ __forceinline__ int root_class(int d) {
  int w = (d + 63) / 64;
  if (w <= 1) return 0;
  int c = 0;
  while ((1 << c) < w) c++;
  return c < SEARCH_CLASSES ? c : SEARCH_CLASSES;  // SEARCH_CLASSES = too large
}

__global__ void k_queue_keys(int nn, const int64_t *__restrict__ poff,
                             const int32_t *__restrict__ lab_gid, const int32_t *__restrict__ bound,
                             int all, const int32_t *__restrict__ disp, int lab_lo, int lab_hi,
                             const int32_t *__restrict__ lab_vertex, int32_t *vdone,
                             int pos_hi, uint32_t *keys, int *hist) {
  __shared__ int h[QCLASS_NONE + 1];
  if (threadIdx.x <= QCLASS_NONE) h[threadIdx.x] = 0;
  __syncthreads();
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nn) {
    int i = disp ? disp[t] : t;
    int d = (int)(poff[i + 1] - poff[i]);
    int need = all ? 0 : bound[graph_of(lab_gid, i)];
    const bool taken = i >= lab_lo && i < lab_hi && t < pos_hi;
    int c = d >= need && taken ? root_class(d) : QCLASS_NONE;
    if (vdone) {
      // a label too small to be a root stays so (the bound only grows): it
      // is done, so a later wave's dispatch order starts past it
      if (vdone[lab_vertex[i]]) c = QCLASS_NONE;
      else if (taken && d < need) vdone[lab_vertex[i]] = 1;
    }
    keys[t] = (uint32_t)c;
    atomicAdd(&h[c], 1);
  }
  __syncthreads();
  if (threadIdx.x <= QCLASS_NONE && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Labels in decreasing order (the dispatch order within each class of a
// single graph's queue).
__global__ void k_rev_iota(int nn, int32_t *v) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nn) v[t] = nn - 1 - t;
}

// Score keys for dispatch by decreasing score (ties by label): a float maps
// to an unsigned key whose ascending order is descending score; NaN and Inf
// get the largest key but one (dispatched last), vertices already searched
// (vdone) the largest.
__global__ void k_score_keys(int nn, const int32_t *__restrict__ lab_vertex,
                             const float *__restrict__ score, const int32_t *__restrict__ vdone,
                             uint32_t *keys) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const int v = lab_vertex[i];
  float f = score[v];
  uint32_t k;
  if (vdone && vdone[v]) {
    k = 0xffffffffu;
  } else if (!isfinite(f)) {
    k = 0xfffffffeu;
  } else {
    uint32_t b = __float_as_uint(f);
    uint32_t asc = (b & 0x80000000u) ? ~b : (b | 0x80000000u);  // ascending order of f
    k = ~asc;                                                    // descending
    if (k >= 0xfffffffeu) k = 0xfffffffdu;
  }
  keys[i] = k;
}

}  // namespace

Labels run_prune_orient(const GraphView &g, const int32_t *core, const int32_t *rank,
                        const int32_t *order, const int32_t *gid, const int32_t *bound,
                        int32_t kmax, Scratch &sc, float *ms_kernels, int64_t *poff_out,
                        int32_t *padj_out, int64_t capacity, int32_t min_rank, bool native) {
  if (native) {  // the search order is the vertex ids
    rank = nullptr;
    order = nullptr;
  }
  hipStream_t s = sc.stream();
  Labels L;
  int n = (int)g.n;
  if (ms_kernels) *ms_kernels = 0.f;
  if (n == 0) {
    L.poff = poff_out ? poff_out : sc.get<int64_t>(1);
    PMC_HIP(hipMemsetAsync(L.poff, 0, sizeof(int64_t), s));
    L.padj = padj_out ? padj_out : sc.get<int32_t>(1);
    return L;
  }
  int nb1 = (n + 255) / 256;
  int32_t *flag = sc.get<int32_t>(n);
  int64_t *pos = sc.get<int64_t>((size_t)n + 1);
  int32_t *vlabel = sc.get<int32_t>(n);
  k_keep_flags<<<nb1, 256, 0, s>>>(n, order, core, gid, bound, min_rank, flag);
  PMC_HIP(hipGetLastError());
  scan_counts(flag, pos, n, sc);
  int64_t nn64 = 0;
  PMC_HIP(hipMemcpyAsync(&nn64, pos + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  PMC_HIP(hipStreamSynchronize(s));
  int nn = (int)nn64;
  L.nn = nn;
  L.vertex = sc.get<int32_t>(std::max(nn, 1));
  L.core = sc.get<int32_t>(std::max(nn, 1));
  L.gid = gid ? sc.get<int32_t>(std::max(nn, 1)) : nullptr;
  k_label_scatter<<<nb1, 256, 0, s>>>(n, order, core, gid, flag, pos, vlabel, L.vertex, L.core,
                                      L.gid);
  PMC_HIP(hipGetLastError());
  L.poff = poff_out ? poff_out : sc.get<int64_t>((size_t)nn + 1);
  if (nn == 0) {
    PMC_HIP(hipMemsetAsync(L.poff, 0, sizeof(int64_t), s));
    L.padj = padj_out ? padj_out : sc.get<int32_t>(1);
    return L;
  }
  int *cnt = sc.get<int>(nn);
  int *big_list = sc.get<int>(nn);
  int *big_n = sc.get<int>(2);
  PMC_HIP(hipMemsetAsync(big_n, 0, 2 * sizeof(int), s));
  unsigned long long *deg_sum = sc.get<unsigned long long>(DEG_SLOTS);
  PMC_HIP(hipMemsetAsync(deg_sum, 0, sizeof(unsigned long long) * DEG_SLOTS, s));
  unsigned long long deg_part[DEG_SLOTS];
  const DevInfo &di = dev_info();
  int nb = (int)std::min<int64_t>((nn + 3) / 4, (int64_t)di.cus * 16);
  KTimer kt(s);
  float kms = 0.f;
  PMC_DISPATCH_OFF(g, OffT, {
    const OffT *off = (const OffT *)g.off;
    kt.start();
    k_orient_count<OffT><<<nb, OR_T, 0, s>>>(nn, off, g.idx, rank, vlabel, L.vertex, cnt,
                                             big_list, big_n, deg_sum);
    PMC_HIP(hipGetLastError());
    kms += kt.stop();
    scan_counts(cnt, L.poff, nn, sc);
    PMC_HIP(hipMemcpyAsync(&L.nnz, L.poff + nn, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PMC_HIP(hipMemcpyAsync(deg_part, deg_sum, sizeof(deg_part), hipMemcpyDeviceToHost, s));
    PMC_HIP(hipStreamSynchronize(s));
    L.deg_sum = 0;
    for (int q = 0; q < DEG_SLOTS; q++) L.deg_sum += (int64_t)deg_part[q];
    if (capacity >= 0 && L.nnz > capacity)
      throw Error{3, "oriented graph needs " + std::to_string(L.nnz) + " entries, capacity " +
                         std::to_string(capacity)};
    L.padj = padj_out ? padj_out : sc.get<int32_t>((size_t)std::max<int64_t>(L.nnz, 1));
    kt.start();
    k_orient_fill<OffT><<<nb, OR_T, 0, s>>>(nn, off, g.idx, rank, L.vertex, vlabel, L.poff,
                                            L.padj);
    PMC_HIP(hipGetLastError());
    kms += kt.stop();
    if (ms_kernels) *ms_kernels = kms;
    if (kmax > OR_WAVE_CAP || native) {  // rows longer than a wave's tile
      k_orient_fill_big<OffT><<<di.cus, OR_BIG_T, 0, s>>>(off, g.idx, rank, L.vertex, vlabel,
                                                          L.poff, L.padj, big_list, big_n,
                                                          big_n + 1);
      PMC_HIP(hipGetLastError());
      int err = 0;
      PMC_HIP(hipMemcpyAsync(&err, big_n + 1, sizeof(int), hipMemcpyDeviceToHost, s));
      PMC_HIP(hipStreamSynchronize(s));
      if (err) throw Error{3, "an oriented row exceeds the 16384-entry sort tile"};
    }
  });
  return L;
}

QueueResult run_queue(const Labels &L, const int32_t *bound, bool all, const float *score,
                      int32_t *queue, Scratch &sc, int lab_lo, int lab_hi, int32_t *vdone,
                      int pos_hi, bool desc) {
  hipStream_t s = sc.stream();
  QueueResult q;
  int nn = L.nn;
  if (nn <= 0) return q;
  int32_t *disp = nullptr;
  if (score) {
    // labels by decreasing score, ties by label (stable sort over label order)
    uint32_t *sk = sc.get<uint32_t>(nn);
    uint32_t *sk2 = sc.get<uint32_t>(nn);
    disp = sc.get<int32_t>(nn);
    k_score_keys<<<(nn + 255) / 256, 256, 0, s>>>(nn, L.vertex, score, vdone, sk);
    PMC_HIP(hipGetLastError());
    radix_sort_pairs(sk, nullptr, sk2, disp, nn, 32, sc);
  } else if (desc) {
    if (pos_hi != INT_MAX) throw Error{1, "a position limit needs a score order"};
    disp = sc.get<int32_t>(nn);
    k_rev_iota<<<(nn + 255) / 256, 256, 0, s>>>(nn, disp);
    PMC_HIP(hipGetLastError());
  }
  uint32_t *keys = sc.get<uint32_t>(nn);
  uint32_t *kout = sc.get<uint32_t>(nn);
  int *hist = sc.get<int>(QCLASS_NONE + 1);
  PMC_HIP(hipMemsetAsync(hist, 0, sizeof(int) * (QCLASS_NONE + 1), s));
  k_queue_keys<<<(nn + 255) / 256, 256, 0, s>>>(nn, L.poff, L.gid, bound, all ? 1 : 0, disp,
                                               lab_lo, lab_hi, L.vertex, vdone, pos_hi, keys,
                                               hist);
  PMC_HIP(hipGetLastError());
  radix_sort_pairs(keys, disp, kout, queue, nn, 8, sc);
  int h[QCLASS_NONE + 1];
  PMC_HIP(hipMemcpyAsync(h, hist, sizeof(h), hipMemcpyDeviceToHost, s));
  PMC_HIP(hipStreamSynchronize(s));
  int acc = 0;
  for (int c = 0; c <= SEARCH_CLASSES; c++) {
    q.start[c] = acc;
    q.count[c] = h[c];
    acc += h[c];
  }
  q.total = acc;
  return q;
}

}  // namespace pmc
