// temporal.hip -- strong-reachability graph of a temporal network (Sec. 7.1
// of the paper: the largest temporal strong component is the maximum clique
// of the graph that joins two vertices when each has a time-respecting path
// to the other).
//
// Definition computed: temporal edges src[e] -> dst[e] come in time order; a
// temporal path uses edges in increasing position of that order.  R[x] is the
// set of vertices with a temporal path to x (x included), built by sweeping
// the edges in order (R[dst] |= R[src]); {a, b} is an edge of the result when
// a is in R[b] and b in R[a].
//
// GPU design: R is an n x n bit matrix (row x = R[x]).  The sweep is cut on
// the host into runs of consecutive edges in which no vertex read by one edge
// is written by another (so the run's ORs commute and see exactly the state
// the sequential sweep would); one cooperative launch processes the runs with
// a grid barrier between them, every (edge, word) pair of a run by its own
// thread with a device-scope 64-bit atomic OR.  The matrix is then transposed
// (64 x 64 bit tiles by wave ballots), rows of R AND R^T give the mutual
// pairs, and a counting pass, a scan and a filling pass write the CSR.
#include <algorithm>
#include <vector>

#include "common.h"
#include "graph.h"

namespace pmc {
namespace {

constexpr int REACH_T = 1024;

__device__ __forceinline__ uint64_t ld_dev64(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_reach_init(int64_t n, int64_t W, uint64_t *R) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * W) return;
  const int64_t x = i / W, w = i % W;
  R[i] = w == x / 64 ? 1ull << (x % 64) : 0ull;
}

struct ReachBar {
  GridBar bar;
};

__global__ void __launch_bounds__(REACH_T)
    k_reach(const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
            const int64_t *__restrict__ runs, int nruns, int64_t W, uint64_t *R, ReachBar *rb) {
  unsigned long long gen = 0;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
  for (int r = 0; r < nruns; r++) {
    const int64_t e0 = runs[r], e1 = runs[r + 1];
    const int64_t items = (e1 - e0) * W;
    for (int64_t i = gtid; i < items; i += gsz) {
      const int64_t e = e0 + i / W, w = i % W;
      const int64_t u = src[e], v = dst[e];
      const uint64_t val = ld_dev64(&R[u * W + w]);
      if (val) atomicOr((unsigned long long *)&R[v * W + w], (unsigned long long)val);
    }
    grid_sync(&rb->bar, gridDim.x, gen);
  }
}

__global__ void k_reach_bar_init(ReachBar *rb) {
  for (int g = 0; g < GRID_GROUPS; g++) rb->bar.group[g][0] = 0;
  rb->bar.top = 0;
}

// T = R^T, one wave per 64 x 64 tile (tile row block i, column word c).
__global__ void k_bit_transpose(int64_t n, int64_t W, const uint64_t *R, uint64_t *T) {
  const int64_t tile = (int64_t)blockIdx.x * (blockDim.x / PMC_WAVE) + threadIdx.x / PMC_WAVE;
  if (tile >= W * W) return;
  const int64_t ib = tile / W, c = tile % W;
  const int l = lane();
  const int64_t row = ib * 64 + l;
  const uint64_t word = row < n ? R[row * W + c] : 0ull;
  uint64_t mine = 0;
  for (int j = 0; j < 64; j++) {
    const uint64_t m = ballot((word >> j) & 1ull);
    if (l == j) mine = m;
  }
  const int64_t orow = c * 64 + l;
  if (orow < n) T[orow * W + ib] = mine;
}

// Mutual pairs per row: popcount(R[x] & T[x]) minus the diagonal.
__global__ void k_strong_count(int64_t n, int64_t W, const uint64_t *R, const uint64_t *T,
                               int32_t *cnt) {
  const int64_t x = (int64_t)blockIdx.x * (blockDim.x / PMC_WAVE) + threadIdx.x / PMC_WAVE;
  if (x >= n) return;
  int c = 0;
  for (int64_t w = lane(); w < W; w += PMC_WAVE) c += __popcll(R[x * W + w] & T[x * W + w]);
  c = wave_sum(c);
  if (lane() == 0) cnt[x] = c - 1;
}

__global__ void k_strong_fill(int64_t n, int64_t W, const uint64_t *R, const uint64_t *T,
                              const int64_t *off, int32_t *adj) {
  const int64_t x = (int64_t)blockIdx.x * (blockDim.x / PMC_WAVE) + threadIdx.x / PMC_WAVE;
  if (x >= n) return;
  const int l = lane();
  int64_t pos = off[x];
  for (int64_t wb = 0; wb < W; wb += PMC_WAVE) {
    const int64_t w = wb + l;
    uint64_t m = w < W ? (R[x * W + w] & T[x * W + w]) : 0ull;
    if (w == x / 64) m &= ~(1ull << (x % 64));
    const int c = __popcll(m);
    const int inc = wave_incl_scan(c);
    int64_t p = pos + inc - c;
    while (m) {
      const int b = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      adj[p++] = (int32_t)(w * 64 + b);
    }
    pos += __builtin_amdgcn_readlane(inc, PMC_WAVE - 1);
  }
}

}  // namespace

int64_t run_strong_reach(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                         int64_t *off, int32_t *adj, int64_t capacity, Scratch &sc) {
  hipStream_t s = sc.stream();
  if (n == 0) {
    PMC_HIP(hipMemsetAsync(off, 0, sizeof(int64_t), s));
    PMC_HIP(hipStreamSynchronize(s));
    return 0;
  }
  const int64_t W = (n + 63) / 64;
  // runs of consecutive edges with no vertex both read and written (host)
  std::vector<int32_t> hs(m), hd(m);
  if (m) {
    PMC_HIP(hipMemcpyAsync(hs.data(), src, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s));
    PMC_HIP(hipMemcpyAsync(hd.data(), dst, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s));
    PMC_HIP(hipStreamSynchronize(s));
  }
  std::vector<int64_t> runs{0};
  std::vector<int32_t> rd(n, -1), wr(n, -1);
  int32_t cur = 0;
  for (int64_t e = 0; e < m; e++) {
    const int32_t u = hs[e], v = hd[e];
    if (u < 0 || u >= n || v < 0 || v >= n)
      throw Error{1, "temporal edge endpoint out of range"};
    if (wr[u] == cur || rd[v] == cur) {
      runs.push_back(e);
      cur++;
    }
    rd[u] = cur;
    wr[v] = cur;
  }
  if (runs.back() != m) runs.push_back(m);
  const int nruns = (int)runs.size() - 1;
  uint64_t *R = sc.get<uint64_t>((size_t)(n * W));
  uint64_t *T = sc.get<uint64_t>((size_t)(n * W));
  int64_t *druns = sc.get<int64_t>(runs.size());
  PMC_HIP(hipMemcpyAsync(druns, runs.data(), sizeof(int64_t) * runs.size(), hipMemcpyHostToDevice, s));
  const int64_t nw = n * W;
  k_reach_init<<<(int)((nw + 255) / 256), 256, 0, s>>>(n, W, R);
  PMC_HIP(hipGetLastError());
  if (nruns > 0) {
    ReachBar *rb = sc.get<ReachBar>(1);
    k_reach_bar_init<<<1, 1, 0, s>>>(rb);
    PMC_HIP(hipGetLastError());
    int per_cu = 0;
    PMC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_reach, REACH_T, 0));
    if (per_cu < 1) throw Error{5, "reachability kernel cannot be made resident"};
    int nblocks = dev_info().cus;
    int32_t *src_ = const_cast<int32_t *>(src);
    int32_t *dst_ = const_cast<int32_t *>(dst);
    int64_t Wv = W;
    int nr = nruns;
    void *args[] = {&src_, &dst_, &druns, &nr, &Wv, &R, &rb};
    PMC_HIP(hipLaunchCooperativeKernel((const void *)k_reach, dim3(nblocks), dim3(REACH_T), args,
                                       0, s));
  }
  const int64_t tiles = W * W;
  k_bit_transpose<<<(int)((tiles + 3) / 4), 256, 0, s>>>(n, W, R, T);
  PMC_HIP(hipGetLastError());
  int32_t *cnt = sc.get<int32_t>((size_t)n);
  k_strong_count<<<(int)((n + 3) / 4), 256, 0, s>>>(n, W, R, T, cnt);
  PMC_HIP(hipGetLastError());
  scan_counts(cnt, off, n, sc);
  int64_t total = 0;
  PMC_HIP(hipMemcpyAsync(&total, off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  PMC_HIP(hipStreamSynchronize(s));
  if (total <= capacity && total > 0) {
    k_strong_fill<<<(int)((n + 3) / 4), 256, 0, s>>>(n, W, R, T, off, adj);
    PMC_HIP(hipGetLastError());
  }
  PMC_HIP(hipStreamSynchronize(s));
  return total;
}

}  // namespace pmc
