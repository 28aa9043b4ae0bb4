// peel_graphs.hip -- k-core decomposition (Sec. 3 of the paper) of every
// graph of a batch on its own: one workgroup per graph, the level-synchronous
// peel of peel.hip (same definition: levels from 0, every remaining vertex of
// remaining degree <= k removed at once per round, a level with nothing to
// remove jumps k to the minimum remaining degree) applied to the graph alone.
#include <algorithm>
#include <climits>
#include <vector>

#include "common.h"
#include "graph.h"

namespace pmc {
namespace {

constexpr int PG_MARK = 1 << 15;  // added to a local degree when the vertex is queued

// Local degree i: the 16-bit half of an LDS word (a degree is below 2^15, the
// mark is bit 15).
__device__ __forceinline__ int pg_deg(const uint32_t *deg2, int i) {
  return (int)((deg2[i >> 1] >> ((i & 1) * 16)) & 0xffffu);
}

// One workgroup per graph (its own levels, level jumps and rounds), with the
// graph's remaining
// degrees (16-bit halves of LDS words, PG_MARK added once queued) and its
// peel queue (16-bit local ids) in LDS; the rows are read from the union's
// CSR, and a removed vertex's row decrements every neighbour, queued or not
// (a queued vertex's half is >= PG_MARK, so it never crosses from k+1 to k
// again, and a half never drops below the mark since each neighbour
// decrements it once).  Round numbers are per graph: within a graph the
// (round, id) order is exactly the order of the graph's own peel, so the
// rank built from them is a degeneracy order of every graph of the batch.
constexpr int PG_EPT = 4;  // consecutive row entries per thread per pass

template <int NT, typename OffT>
__global__ void __launch_bounds__(NT) k_peel_graphs(const int32_t *__restrict__ glist,
                                                    const int64_t *__restrict__ vbase,
                                                    const OffT *__restrict__ off,
                                                    const int32_t *__restrict__ idx, int nmax,
                                                    int *core, int *rnd, int *gstat) {
  extern __shared__ uint32_t pg_lds[];
  __shared__ int pre[NT + 1];
  __shared__ OffT rs[NT];
  __shared__ int red[NT / PMC_WAVE + 1];
  __shared__ int qend, flag;
  constexpr int NW = NT / PMC_WAVE;
  const int g = glist[blockIdx.x];
  const int64_t base = vbase[g];
  const int n = (int)(vbase[g + 1] - base);
  uint32_t *deg2 = pg_lds;
  uint16_t *queue = (uint16_t *)(pg_lds + (nmax + 1) / 2);
  const int t = threadIdx.x, l = lane(), w = t / PMC_WAVE;
  if (t == 0) {
    qend = 0;
    flag = 0;
  }
  __syncthreads();
  for (int i2 = t; i2 < (n + 1) / 2; i2 += NT) {
    uint32_t h = 0;
    for (int q = 0; q < 2; q++) {
      const int i = 2 * i2 + q;
      if (i < n) {
        const int64_t d = (int64_t)off[base + i + 1] - (int64_t)off[base + i];
        if (d >= PG_MARK) flag = 1;  // only a graph with repeated edges gets here
        h |= (uint32_t)(d & (PG_MARK - 1)) << (16 * q);
      }
    }
    deg2[i2] = h;
  }
  __syncthreads();
  if (flag) {
    if (t == 0) gstat[2 * g] = -1;
    return;
  }
  int qh = 0, qe = 0, k = 0, r = 0;
  while (qh < qe || qe < n) {
    if (qh == qe) {  // level jump: k = max(k, minimum remaining degree)
      int m = INT_MAX;
      for (int i = t; i < n; i += NT) {
        const int d = pg_deg(deg2, i);
        if (d < PG_MARK) m = min(m, d);
      }
      m = block_min(m, red);
      k = max(k, m);
      for (int i = t; i < n; i += NT) {
        const int d = pg_deg(deg2, i);
        if (d < PG_MARK && d <= k) {
          atomicAdd(&deg2[i >> 1], (uint32_t)PG_MARK << ((i & 1) * 16));
          queue[atomicAdd(&qend, 1)] = (uint16_t)i;
        }
      }
      __syncthreads();
      qe = qend;
      if (qe == qh) {  // nothing queued: cannot happen with a consistent state
        if (t == 0) gstat[2 * g] = -2;
        return;
      }
    }
    // round r: remove queue[qh, qe); the rows of a chunk of up to NT items
    // are laid end to end and every thread takes PG_EPT consecutive entries
    for (int cb = qh; cb < qe; cb += NT) {
      const int C = min(NT, qe - cb);
      int len = 0;
      OffT st = 0;
      if (t < C) {
        const int64_t v = base + queue[cb + t];
        st = off[v];
        len = (int)(off[v + 1] - st);
        rnd[v] = r;
        core[v] = k;
      }
      const int inc = wave_incl_scan(len);
      if (l == PMC_WAVE - 1) red[w] = inc;
      __syncthreads();
      int before = 0, all = 0;
      for (int i = 0; i < NW; i++) {
        const int c = red[i];
        before += i < w ? c : 0;
        all += c;
      }
      if (t < C) {
        pre[t] = before + inc - len;
        rs[t] = st;
      }
      if (t == 0) pre[C] = all;
      __syncthreads();
      for (int eb = 0; eb < all; eb += NT * PG_EPT) {
        const int e0 = eb + t * PG_EPT;
        int it = 0;
        if (e0 < all) {  // last item whose first entry is <= e0
          int lo = 0, hi = C - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pre[mid] <= e0) lo = mid; else hi = mid - 1;
          }
          it = lo;
        }
        int u[PG_EPT];
#pragma unroll
        for (int q = 0; q < PG_EPT; q++) {
          const int e = e0 + q;
          u[q] = -1;
          if (e < all) {
            while (pre[it + 1] <= e) it++;
            u[q] = (int)(idx[rs[it] + (e - pre[it])] - base);
            if ((unsigned)u[q] >= (unsigned)n) u[q] = -1;  // an edge leaving the graph: skipped
          }
        }
        unsigned cross = 0;
#pragma unroll
        for (int q = 0; q < PG_EPT; q++) {
          if (u[q] < 0) continue;
          const unsigned sh = (unsigned)(u[q] & 1) * 16u;
          const unsigned old = atomicSub(&deg2[u[q] >> 1], 1u << sh);
          if ((int)((old >> sh) & 0xffffu) == k + 1) cross |= 1u << q;
        }
        const int c = __popc(cross);
        const int ci = wave_incl_scan(c);
        const int total = __builtin_amdgcn_readlane(ci, PMC_WAVE - 1);
        if (total) {
          int qb = 0;
          if (l == 0) qb = atomicAdd(&qend, total);
          int pos = __builtin_amdgcn_readfirstlane(qb) + ci - c;
#pragma unroll
          for (int q = 0; q < PG_EPT; q++) {
            if (cross >> q & 1u) {
              atomicAdd(&deg2[u[q] >> 1], (uint32_t)PG_MARK << ((u[q] & 1) * 16));
              queue[pos++] = (uint16_t)u[q];
            }
          }
        }
      }
      __syncthreads();  // pre / rs are rewritten by the next chunk
    }
    qh = qe;
    qe = qend;
    r++;
  }
  if (t == 0) {
    gstat[2 * g] = k;
    gstat[2 * g + 1] = r;
  }
}

}  // namespace

bool peel_graphs_fits(const std::vector<int64_t> &vbase) {
  for (size_t g = 0; g + 1 < vbase.size(); g++)
    if (vbase[g + 1] - vbase[g] > PEEL_GRAPH_MAX_N) return false;
  return true;
}

PeelResult run_peel_graphs(const GraphView &g, const std::vector<int64_t> &vbase, int32_t *core,
                           int32_t *rnd, Scratch &sc, bool timed, std::vector<int32_t> *gkmax,
                           std::vector<int32_t> *grounds) {
  PeelResult res;
  hipStream_t s = sc.stream();
  const int G = (int)vbase.size() - 1;
  if (G <= 0 || g.n == 0) return res;
  if (!peel_graphs_fits(vbase)) throw Error{3, "a graph of the batch exceeds the per-graph peel"};
  // graphs of more than PG_SMALL vertices get 1024 threads, the others 256;
  // each class largest first, so the longest peels start first
  constexpr int PG_SMALL = 4096;
  std::vector<int32_t> order(G);
  for (int i = 0; i < G; i++) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return vbase[a + 1] - vbase[a] > vbase[b + 1] - vbase[b];
  });
  int nbig = 0;
  while (nbig < G && vbase[order[nbig] + 1] - vbase[order[nbig]] > PG_SMALL) nbig++;
  int32_t *glist = sc.get<int32_t>(G);
  int64_t *dvb = sc.get<int64_t>(G + 1);
  int *gstat = sc.get<int>(2 * (size_t)G);
  PMC_HIP(hipMemcpyAsync(glist, order.data(), sizeof(int32_t) * G, hipMemcpyHostToDevice, s));
  PMC_HIP(hipMemcpyAsync(dvb, vbase.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timed) {
    PMC_HIP(hipEventCreate(&e0));
    PMC_HIP(hipEventCreate(&e1));
    PMC_HIP(hipEventRecord(e0, s));
  }
  PMC_DISPATCH_OFF(g, OffT, {
    const OffT *off = (const OffT *)g.off;
    const int32_t *idx = g.idx;
    auto launch = [&](const void *kern, int nt, int first, int count) {
      if (count <= 0) return;
      int nmax = (int)(vbase[order[first] + 1] - vbase[order[first]]);
      const size_t lds = (size_t)8 * ((nmax + 1) / 2);
      if (lds > 65536)
        PMC_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      const int32_t *gl = glist + first;
      void *args[] = {(void *)&gl, (void *)&dvb, (void *)&off, (void *)&idx, &nmax, &core, &rnd,
                      &gstat};
      PMC_HIP(hipLaunchKernel(kern, dim3(count), dim3(nt), args, lds, s));
    };
    launch((const void *)k_peel_graphs<1024, OffT>, 1024, 0, nbig);
    launch((const void *)k_peel_graphs<256, OffT>, 256, nbig, G - nbig);
  });
  if (timed) PMC_HIP(hipEventRecord(e1, s));
  std::vector<int> h(2 * (size_t)G);
  PMC_HIP(hipMemcpyAsync(h.data(), gstat, sizeof(int) * 2 * G, hipMemcpyDeviceToHost, s));
  PMC_HIP(hipStreamSynchronize(s));
  if (timed) {
    PMC_HIP(hipEventElapsedTime(&res.ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  if (gkmax) gkmax->assign(G, 0);
  if (grounds) grounds->assign(G, 0);
  for (int i = 0; i < G; i++) {
    if (h[2 * i] == -1) throw Error{2, "a graph of the batch has a vertex of degree >= 32768 "
                                       "with fewer vertices: repeated edges"};
    if (h[2 * i] < 0) throw Error{5, "per-graph k-core peel reached an inconsistent state"};
    res.kmax = std::max(res.kmax, h[2 * i]);
    res.nrounds = std::max(res.nrounds, h[2 * i + 1]);
    if (gkmax) (*gkmax)[i] = h[2 * i];
    if (grounds) (*grounds)[i] = h[2 * i + 1];
  }
  return res;
}

}  // namespace pmc
