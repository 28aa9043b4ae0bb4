// prune.hip -- explicit pruning and orientation (Sec. 4.2 and the reduced
// neighbourhoods N_R of Sec. 4.3), and the root queue of the search loop.
//
// Pruning removes every vertex with K(v) < bound.  Because the degeneracy rank
// is nondecreasing in core, the survivors are exactly the ranks >= r0(bound),
// so they are relabelled rank - r0 and the graph becomes an oriented graph on
// labels 0..n'-1: the row of label i keeps the neighbours of higher rank
// (searched vertices of lower rank are excluded from later neighbourhoods, and
// every kept neighbour has core >= K(v) >= bound).  Rows are sorted, so the
// local index of a subproblem follows the degeneracy rank.
//
// GPU design: a count pass and a fill pass, one wavefront per surviving
// vertex streaming its CSR row coalesced and gathering the neighbours' ranks;
// kept labels are compacted with ballot/prefix counts, sorted in LDS by a
// bitonic network and written contiguously; row offsets come from the
// project's scan.  Rows longer than the wave's LDS tile go to a workgroup
// kernel with a larger tile.
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

template <typename OffT>
__global__ void __launch_bounds__(OR_T)
    k_orient_count(int nn, int r0, const OffT *__restrict__ off, const int32_t *__restrict__ idx,
                   const int *__restrict__ rank, const int *__restrict__ order, int *cnt,
                   int *big_list, int *big_n) {
  int w = (blockIdx.x * blockDim.x + threadIdx.x) / PMC_WAVE;
  int nw = gridDim.x * blockDim.x / PMC_WAVE;
  int l = lane();
  for (int i = w; i < nn; i += nw) {
    int v = order[r0 + i];
    int rv = r0 + i;
    int64_t s = (int64_t)off[v], e = (int64_t)off[v + 1];
    int c = 0;
    for (int64_t jb = s; jb < e; jb += PMC_WAVE) {
      int64_t j = jb + l;
      bool keep = j < e && rank[idx[j]] > rv;
      c += __popcll(ballot(keep));
    }
    if (l == 0) {
      cnt[i] = c;
      if (c > OR_WAVE_CAP) big_list[atomic_add(big_n, 1)] = i;
    }
  }
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
    k_orient_fill(int nn, int r0, const OffT *__restrict__ off, const int32_t *__restrict__ idx,
                  const int *__restrict__ rank, const int *__restrict__ order,
                  const int64_t *__restrict__ poff, int32_t *padj) {
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
    int v = order[r0 + i];
    int rv = r0 + i;
    int64_t s = (int64_t)off[v], e = (int64_t)off[v + 1];
    int w0 = 0;
    for (int64_t jb = s; jb < e; jb += PMC_WAVE) {
      int64_t j = jb + l;
      int ru = j < e ? rank[idx[j]] : -1;
      bool keep = ru > rv;
      uint64_t m = ballot(keep);
      if (keep) buf[w0 + __popcll(m & lanemask_lt())] = ru - r0;
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
    k_orient_fill_big(int r0, const OffT *__restrict__ off, const int32_t *__restrict__ idx,
                      const int *__restrict__ rank, const int *__restrict__ order,
                      const int64_t *__restrict__ poff, int32_t *padj, const int *big_list,
                      const int *big_n, CliqueState *st) {
  __shared__ int buf[OR_BIG_CAP];
  __shared__ int wcnt[OR_BIG_T / PMC_WAVE + 1];
  int nbig = *big_n;
  for (int b = blockIdx.x; b < nbig; b += gridDim.x) {
    int i = big_list[b];
    int64_t o = poff[i];
    int c = (int)(poff[i + 1] - o);
    if (c > OR_BIG_CAP) {
      if (threadIdx.x == 0) atomicExch(&st->err, 2);
      continue;
    }
    int v = order[r0 + i];
    int rv = r0 + i;
    int64_t s = (int64_t)off[v], e = (int64_t)off[v + 1];
    // block-wide compaction in row order
    int wid = threadIdx.x / PMC_WAVE;
    int base = 0;
    for (int64_t jb = s; jb < e; jb += OR_BIG_T) {
      int64_t j = jb + threadIdx.x;
      int ru = j < e ? rank[idx[j]] : -1;
      bool keep = ru > rv;
      uint64_t m = ballot(keep);
      if (lane() == 0) wcnt[wid] = __popcll(m);
      __syncthreads();
      int pre = 0, tot = 0;
      for (int q = 0; q < OR_BIG_T / PMC_WAVE; q++) {
        if (q < wid) pre += wcnt[q];
        tot += wcnt[q];
      }
      if (keep) buf[base + pre + __popcll(m & lanemask_lt())] = ru - r0;
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

__global__ void k_queue_keys(int nn, const int64_t *__restrict__ poff, int min_deg,
                             const int32_t *__restrict__ disp, uint32_t *keys, int *hist) {
  __shared__ int h[QCLASS_NONE + 1];
  if (threadIdx.x <= QCLASS_NONE) h[threadIdx.x] = 0;
  __syncthreads();
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nn) {
    int i = disp ? disp[t] : t;
    int d = (int)(poff[i + 1] - poff[i]);
    int c = d >= min_deg ? root_class(d) : QCLASS_NONE;
    keys[t] = (uint32_t)c;
    atomicAdd(&h[c], 1);
  }
  __syncthreads();
  if (threadIdx.x <= QCLASS_NONE && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Score keys for dispatch by decreasing score (ties by label): a float maps
// to an unsigned key whose ascending order is descending score; NaN and Inf
// get the largest key (dispatched last).
__global__ void k_score_keys(int nn, int r0, const int32_t *__restrict__ order,
                             const float *__restrict__ score, uint32_t *keys) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  float f = score[order[r0 + i]];
  uint32_t k;
  if (!isfinite(f)) {
    k = 0xffffffffu;
  } else {
    uint32_t b = __float_as_uint(f);
    uint32_t asc = (b & 0x80000000u) ? ~b : (b | 0x80000000u);  // ascending order of f
    k = ~asc;                                                    // descending
    if (k == 0xffffffffu) k = 0xfffffffeu;
  }
  keys[i] = k;
}

}  // namespace

int64_t run_prune_orient(const GraphView &g, const int32_t *rank, const int32_t *order, int32_t r0,
                         int64_t *poff, int32_t *padj, int64_t capacity, int32_t kmax,
                         Scratch &sc, float *ms_kernels) {
  hipStream_t s = sc.stream();
  int nn = (int)(g.n - r0);
  if (nn <= 0) {
    PMC_HIP(hipMemsetAsync(poff, 0, sizeof(int64_t), s));
    return 0;
  }
  int *cnt = sc.get<int>(nn);
  int *big_list = sc.get<int>(nn);
  int *big_n = sc.get<int>(1);
  CliqueState *st = sc.get<CliqueState>(1);
  PMC_HIP(hipMemsetAsync(big_n, 0, sizeof(int), s));
  PMC_HIP(hipMemsetAsync(st, 0, sizeof(CliqueState), s));
  const DevInfo &di = dev_info();
  int nb = (int)std::min<int64_t>((nn + 3) / 4, (int64_t)di.cus * 16);
  KTimer kt(s);
  float kms = 0.f;
  PMC_DISPATCH_OFF(g, OffT, {
    const OffT *off = (const OffT *)g.off;
    kt.start();
    k_orient_count<OffT><<<nb, OR_T, 0, s>>>(nn, r0, off, g.idx, rank, order, cnt, big_list,
                                             big_n);
    PMC_HIP(hipGetLastError());
    kms += kt.stop();
    scan_counts(cnt, poff, nn, sc);
    int64_t total = 0;
    PMC_HIP(hipMemcpyAsync(&total, poff + nn, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PMC_HIP(hipStreamSynchronize(s));
    if (total > capacity)
      throw Error{3, "oriented graph needs " + std::to_string(total) + " entries, capacity " +
                         std::to_string(capacity)};
    kt.start();
    k_orient_fill<OffT><<<nb, OR_T, 0, s>>>(nn, r0, off, g.idx, rank, order, poff, padj);
    PMC_HIP(hipGetLastError());
    kms += kt.stop();
    if (ms_kernels) *ms_kernels = kms;
    if (kmax > OR_WAVE_CAP) {
      k_orient_fill_big<OffT><<<di.cus, OR_BIG_T, 0, s>>>(r0, off, g.idx, rank, order, poff,
                                                          padj, big_list, big_n, st);
      PMC_HIP(hipGetLastError());
      int err = 0;
      PMC_HIP(hipMemcpyAsync(&err, &st->err, sizeof(int), hipMemcpyDeviceToHost, s));
      PMC_HIP(hipStreamSynchronize(s));
      if (err) throw Error{3, "an oriented row exceeds the 16384-entry sort tile"};
    }
    return total;
  });
  return 0;
}

QueueResult run_queue(int nn, int r0, const int64_t *poff, const int32_t *order, int min_deg,
                      const float *score, int32_t *queue, Scratch &sc) {
  hipStream_t s = sc.stream();
  QueueResult q;
  if (nn <= 0) return q;
  int32_t *disp = nullptr;
  if (score) {
    // labels by decreasing score, ties by label (stable sort over label order)
    uint32_t *sk = sc.get<uint32_t>(nn);
    uint32_t *sk2 = sc.get<uint32_t>(nn);
    disp = sc.get<int32_t>(nn);
    k_score_keys<<<(nn + 255) / 256, 256, 0, s>>>(nn, r0, order, score, sk);
    PMC_HIP(hipGetLastError());
    radix_sort_pairs(sk, nullptr, sk2, disp, nn, 32, sc);
  }
  uint32_t *keys = sc.get<uint32_t>(nn);
  uint32_t *kout = sc.get<uint32_t>(nn);
  int *hist = sc.get<int>(QCLASS_NONE + 1);
  PMC_HIP(hipMemsetAsync(hist, 0, sizeof(int) * (QCLASS_NONE + 1), s));
  k_queue_keys<<<(nn + 255) / 256, 256, 0, s>>>(nn, poff, min_deg, disp, keys, hist);
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
