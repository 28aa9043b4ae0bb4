// graph_util.hip -- largest degree and the graph-contract check.
#include "common.h"
#include "graph.h"

namespace pmc {
namespace {

// Largest degree: grid-stride per thread, block reduction, one atomic per block.
template <typename OffT>
__global__ void __launch_bounds__(256) k_max_degree(int64_t n, const OffT *off, int32_t *out) {
  __shared__ int wm[4];
  int d = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    d = max(d, (int)((int64_t)off[v + 1] - (int64_t)off[v]));
  d = wave_max(d);
  if (lane() == 0) wm[threadIdx.x / PMC_WAVE] = d;
  __syncthreads();
  if (threadIdx.x == 0) atomic_max(out, max(max(wm[0], wm[1]), max(wm[2], wm[3])));
}

// Violation flags: bit 0 offsets, 1 id range, 2 self-loop, 3 order/duplicate,
// 4 asymmetry, 5 an edge between two graphs of a batch.  One wave per vertex.
template <typename OffT>
__global__ void k_validate(int64_t n, int64_t nnz, const OffT *off, const int32_t *idx,
                           const int32_t *gid, int *flags) {
  int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / PMC_WAVE;
  int64_t nw = (int64_t)gridDim.x * blockDim.x / PMC_WAVE;
  int l = lane();
  for (int64_t v = w; v < n; v += nw) {
    int64_t s = (int64_t)off[v], e = (int64_t)off[v + 1];
    int f = 0;
    if (e < s || s < 0 || e > nnz) {
      f |= 1;
    } else {
      for (int64_t j = s + l; j < e; j += PMC_WAVE) {
        int u = idx[j];
        if (u < 0 || u >= n) { f |= 2; continue; }
        if (u == v) f |= 4;
        if (j > s && idx[j - 1] >= u) f |= 8;
        if (gid && gid[u] != gid[v]) f |= 32;
        int64_t us = (int64_t)off[u], ue = (int64_t)off[u + 1];
        if (ue < us || us < 0 || ue > nnz) { f |= 1; continue; }
        int p = lower_bound(idx + us, (int)(ue - us), (int32_t)v);
        if (!(p < ue - us && idx[us + p] == v)) f |= 16;
      }
    }
    for (int o = 32; o > 0; o >>= 1) f |= __shfl_xor(f, o, PMC_WAVE);
    if (l == 0 && f) atomicOr(flags, f);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if ((int64_t)off[0] != 0 || (int64_t)off[n] != nnz) atomicOr(flags, 1);
  }
}

}  // namespace

void max_degree(const GraphView &g, int32_t *out, hipStream_t s) {
  if (g.n == 0) return;
  int nb = (int)std::min<int64_t>((g.n + 255) / 256, (int64_t)dev_info().cus * 4);
  PMC_DISPATCH_OFF(g, OffT, {
    k_max_degree<OffT><<<nb, 256, 0, s>>>(g.n, (const OffT *)g.off, out);
  });
  PMC_HIP(hipGetLastError());
}

int validate_graph(const GraphView &g, Scratch &sc, const int32_t *gid) {
  hipStream_t s = sc.stream();
  int *flags = sc.get<int>(1);
  PMC_HIP(hipMemsetAsync(flags, 0, sizeof(int), s));
  int nb = (int)std::min<int64_t>((g.n + 3) / 4 + 1, (int64_t)dev_info().cus * 16);
  PMC_DISPATCH_OFF(g, OffT, {
    k_validate<OffT><<<nb, 256, 0, s>>>(g.n, g.nnz, (const OffT *)g.off, g.idx, gid, flags);
  });
  PMC_HIP(hipGetLastError());
  int h = 0;
  PMC_HIP(hipMemcpyAsync(&h, flags, sizeof(int), hipMemcpyDeviceToHost, s));
  PMC_HIP(hipStreamSynchronize(s));
  for (int b = 0; b < 6; b++)
    if (h & (1 << b)) return b + 1;
  return 0;
}

}  // namespace pmc
