// temporal.hip -- strong-reachability graph of a temporal network (Sec. 6.1
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
// GPU design: R is an n x n bit matrix (row x = R[x]).  The OR of one edge
// acts on every bit column of R independently, so the sweep runs once per
// column slice of C source vertices (C = 64, 32, 16 or 8 bits, the widest for
// which the slice of all n rows fits in 128 KB of LDS): one wave per slice
// keeps its n fields in LDS and replays the whole edge sequence there.  The
// host schedules the edges as early as their dependencies allow (an edge
// reading R[u] comes after every earlier edge writing u; an edge writing R[v]
// comes after every earlier edge reading v; ORs into one row commute), so the
// edges of one level touch no row that another edge of the level writes and
// run as one wave instruction; the wave takes the level-sorted sequence 64
// edges at a time, a level at a time inside each group, with no barrier (a
// wave's LDS operations complete in order).  The slice is written back to R,
// which is then transposed (64 x 64 bit tiles by wave ballots); rows of
// R AND R^T give the mutual pairs, and a counting pass, a scan and a filling
// pass write the CSR.

#include <algorithm>
#include <vector>

#include "common.h"
#include "graph.h"

namespace pmc {
namespace {

// Level-sorted edge record: bit 63 marks the first edge of a level, bits
// 34..50 hold u (the row read), bits 0..16 v (the row ORed into).
constexpr int REACH_LDS_WORDS = 16384;  // 128 KB
constexpr uint64_t REC_FIRST = 1ull << 63;

__global__ void k_zero_u64(int64_t cnt, uint64_t *p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) p[i] = 0ull;
}

// Field of vertex x in the slice held in LDS: C bits at bit offset x * C.
template <int C>
__device__ __forceinline__ uint64_t field_get(const uint64_t *col, int x) {
  if constexpr (C == 64) {
    return col[x];
  } else {
    const uint32_t *c32 = (const uint32_t *)col;
    const int b = x * C;
    constexpr uint32_t MASK = C == 32 ? 0xffffffffu : (1u << (C & 31)) - 1u;
    return (c32[b >> 5] >> (b & 31)) & MASK;
  }
}

template <int C>
__device__ __forceinline__ void field_or(uint64_t *col, int x, uint64_t v) {
  if constexpr (C == 64) {
    atomicOr((unsigned long long *)&col[x], (unsigned long long)v);
  } else {
    uint32_t *c32 = (uint32_t *)col;
    const int b = x * C;
    atomicOr(&c32[b >> 5], (uint32_t)v << (b & 31));
  }
}

// One wave per slice k (source vertices [k*C, k*C + C)): sweep the
// level-sorted records rec[0, mr) over the slice in LDS, then OR it into R
// (R zeroed beforehand unless C == 64, where each word has one writer).
template <int C>
__global__ void __launch_bounds__(PMC_WAVE)
    k_reach_slice(const uint64_t *__restrict__ rec, int64_t mr, int n, int64_t W, uint64_t *R) {
  __shared__ uint64_t col[REACH_LDS_WORDS];
  const int l = threadIdx.x;
  const int lo = blockIdx.x * C;
  if constexpr (C == 64) {
    for (int x = l; x < n; x += PMC_WAVE) col[x] = (x >= lo && x < lo + 64) ? 1ull << (x - lo) : 0ull;
  } else {
    uint32_t *c32 = (uint32_t *)col;
    constexpr int PER = 32 / C;
    const int nw = (n + PER - 1) / PER;
    for (int i = l; i < nw; i += PMC_WAVE) {
      uint32_t v = 0;
      for (int j = 0; j < PER; j++) {
        const int x = i * PER + j;
        if (x >= lo && x < lo + C && x < n) v |= 1u << (j * C + (x - lo));
      }
      c32[i] = v;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  wave_sync();
  // groups of 64 records, eight groups loaded ahead of their use
  constexpr int D = 8;
  const int64_t ngroups = (mr + PMC_WAVE - 1) / PMC_WAVE;
  uint64_t buf[D];
#pragma unroll
  for (int j = 0; j < D; j++) {
    const int64_t i = (int64_t)j * PMC_WAVE + l;
    buf[j] = i < mr ? rec[i] : 0ull;
  }
  for (int64_t g0 = 0; g0 < ngroups; g0 += D) {
    uint64_t nxt[D];
#pragma unroll
    for (int j = 0; j < D; j++) {
      const int64_t i = (g0 + D + j) * PMC_WAVE + l;
      nxt[j] = i < mr ? rec[i] : 0ull;
    }
#pragma unroll
    for (int j = 0; j < D; j++) {
      if (g0 + j >= ngroups) break;
      const uint64_t r = buf[j];
      const bool valid = (g0 + j) * PMC_WAVE + l < mr;
      const uint64_t fm = ballot(valid && (r & REC_FIRST));
      const int seg = __popcll(fm & (lanemask_lt() | (1ull << l)));
      const int nseg = __popcll(fm);
      const int u = (int)((r >> 34) & 0x1ffffu), v = (int)(r & 0x1ffffu);
      for (int sg = (fm & 1ull) ? 1 : 0; sg <= nseg; sg++) {
        if (valid && seg == sg) {
          const uint64_t f = field_get<C>(col, u);
          if (f) field_or<C>(col, v, f);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
      }
    }
#pragma unroll
    for (int j = 0; j < D; j++) buf[j] = nxt[j];
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  wave_sync();
  const int64_t w = lo / 64;
  if constexpr (C == 64) {
    for (int x = l; x < n; x += PMC_WAVE) R[(int64_t)x * W + w] = col[x];
  } else {
    for (int x = l; x < n; x += PMC_WAVE) {
      const uint64_t f = field_get<C>(col, x);
      if (f) atomicOr((unsigned long long *)&R[(int64_t)x * W + w], (unsigned long long)(f << (lo % 64)));
    }
  }
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
  // as-early-as-possible levels: after the last write of u, after the last
  // read of v (self-loops change nothing and are dropped)
  std::vector<int32_t> lev(m), lastw(n, -1), lastr(n, -1);
  int32_t nlev = 0;
  int64_t mr = 0;
  for (int64_t e = 0; e < m; e++) {
    const int32_t u = hs[e], v = hd[e];
    if (u < 0 || u >= n || v < 0 || v >= n)
      throw Error{1, "temporal edge endpoint out of range"};
    if (u == v) {
      lev[e] = -1;
      continue;
    }
    const int32_t L = std::max(lastw[u], lastr[v]) + 1;
    lev[e] = L;
    lastr[u] = std::max(lastr[u], L);
    lastw[v] = std::max(lastw[v], L);
    nlev = std::max(nlev, L + 1);
    mr++;
  }
  std::vector<int64_t> lstart(nlev + 1, 0);
  for (int64_t e = 0; e < m; e++)
    if (lev[e] >= 0) lstart[lev[e] + 1]++;
  for (int32_t L = 0; L < nlev; L++) lstart[L + 1] += lstart[L];
  std::vector<uint64_t> rec(std::max<int64_t>(mr, 1));
  {
    std::vector<int64_t> pos(lstart.begin(), lstart.end() - 1);
    for (int64_t e = 0; e < m; e++) {
      const int32_t L = lev[e];
      if (L < 0) continue;
      const int64_t p = pos[L]++;
      rec[p] = ((uint64_t)hs[e] << 34) | (uint64_t)hd[e] | (p == lstart[L] ? REC_FIRST : 0ull);
    }
  }
  uint64_t *R = sc.get<uint64_t>((size_t)(n * W));
  uint64_t *T = sc.get<uint64_t>((size_t)(n * W));
  uint64_t *drec = sc.get<uint64_t>((size_t)std::max<int64_t>(mr, 1));
  if (mr) PMC_HIP(hipMemcpyAsync(drec, rec.data(), sizeof(uint64_t) * mr, hipMemcpyHostToDevice, s));
  const int64_t nw = n * W;
  const int C = n <= REACH_LDS_WORDS ? 64 : n <= 2 * REACH_LDS_WORDS ? 32 : n <= 4 * REACH_LDS_WORDS ? 16 : 8;
  if (C < 64) {
    k_zero_u64<<<(int)((nw + 255) / 256), 256, 0, s>>>(nw, R);
    PMC_HIP(hipGetLastError());
  }
  const int slices = (int)((n + C - 1) / C);
  const int nn = (int)n;
  switch (C) {
    case 64: k_reach_slice<64><<<slices, PMC_WAVE, 0, s>>>(drec, mr, nn, W, R); break;
    case 32: k_reach_slice<32><<<slices, PMC_WAVE, 0, s>>>(drec, mr, nn, W, R); break;
    case 16: k_reach_slice<16><<<slices, PMC_WAVE, 0, s>>>(drec, mr, nn, W, R); break;
    default: k_reach_slice<8><<<slices, PMC_WAVE, 0, s>>>(drec, mr, nn, W, R); break;
  }
  PMC_HIP(hipGetLastError());
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
