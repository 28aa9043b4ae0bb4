// learn.hip -- the learned vertex ordering: per-vertex features and an
// 8 -> 64 -> 64 -> 1 MLP whose score reorders the heuristic seeds and the
// search roots (it never changes omega).
//
// Features (per vertex v, K = largest core number, at least 1):
//   log1p(deg), log1p(core), core / K, log1p(triangles through v),
//   mean / max / min core of the neighbours over K, and the fraction of
//   neighbours whose core is >= core(v); 0 for the neighbour terms of an
//   isolated vertex.  Triangles are counted on the degeneracy-oriented graph:
//   each triangle a < b < w (rank order) is found once, at a, by searching
//   N+(b) in N+(a).
// MLP: Z1 = X W1 + b1, H1 = relu(Z1), Z2 = H1 W2 + b2, H2 = relu(Z2),
//   s = H2 w3 + b3; training minimises mean((s - y)^2) with Adam.
//
// GPU design: one wavefront per tile of 16 vertices.  The two GEMM layers and
// the three gradient GEMMs run on v_mfma_f32_16x16x16_bf16 (bf16 operands,
// fp32 accumulation).  Operand layout of that instruction (lane l, j = 0..3):
// A[l % 16][4 (l / 16) + j], B[4 (l / 16) + j][l % 16]; the result D holds
// D[4 (l / 16) + j][l % 16].  So the result of one layer is already the A
// operand of the transposed products (H1^T dZ2, X^T dZ1) and the B operand of
// the gradient GEMMs; only the forward layer-2 input and dH1's input go
// through a 16x64 LDS tile.  Weights are staged in LDS as bf16 once per
// workgroup.  Gradients: each wave accumulates its tiles in registers and
// writes one row of partial sums; a second kernel reduces the rows in a fixed
// order (deterministic), and Adam updates the fp32 master weights.
#include <climits>

#include "common.h"
#include "graph.h"
#include "learn.h"

namespace pmc {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int FIN = 8, HID = 64;
constexpr int OFF_W1 = 0, OFF_B1 = 512, OFF_W2 = 576, OFF_B2 = 4672, OFF_W3 = 4736,
              OFF_B3 = 4800;
constexpr int NPART = MLP_PARAMS + 1;  // gradient partials + squared-residual sum
constexpr int MLP_T = 256;             // 4 waves per workgroup

__device__ __forceinline__ short to_bf16(float f) {
  __bf16 h = (__bf16)f;
  return __builtin_bit_cast(short, h);
}

__device__ __forceinline__ f4 mfma(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- features

// Triangles through each vertex, on the oriented graph of all vertices
// (labels = ranks).  One wave per label a: N+(a) is copied into the wave's LDS
// slice when it fits (else searched in place), the row bounds of 64 of its
// members b are fetched at once, and every x in N+(b) is looked up among the
// members of N+(a) after b (x > b, and N+(a) is sorted), so each triangle
// a < b < x is found once, at a.
constexpr int TRI_T = 256;
constexpr int TRI_CAP = 1024;  // LDS entries per wave
__global__ void __launch_bounds__(TRI_T)
    k_triangles(int nn, const int64_t *__restrict__ poff, const int32_t *__restrict__ padj,
                const int32_t *__restrict__ lab_vertex, int *tri) {
  __shared__ int32_t tri_lds[TRI_T / PMC_WAVE][TRI_CAP];
  int32_t *sa = tri_lds[threadIdx.x / PMC_WAVE];
  int w = (blockIdx.x * blockDim.x + threadIdx.x) / PMC_WAVE;
  int nw = gridDim.x * blockDim.x / PMC_WAVE;
  int l = lane();
  for (int a = w; a < nn; a += nw) {
    const int64_t as = poff[a], ae = poff[a + 1];
    const int la = (int)(ae - as);
    const bool in_lds = la <= TRI_CAP;
    if (in_lds)
      for (int i = l; i < la; i += PMC_WAVE) sa[i] = padj[as + i];
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    wave_sync();
    const int32_t *A = in_lds ? sa : padj + as;
    int cnt_a = 0;
    for (int i0 = 0; i0 < la; i0 += PMC_WAVE) {
      const int nb = min(PMC_WAVE, la - i0);
      const int bl = l < nb ? A[i0 + l] : 0;
      const int64_t bsl = l < nb ? poff[bl] : 0, bel = l < nb ? poff[bl + 1] : 0;
      for (int k = 0; k < nb; k++) {
        const int b = __builtin_amdgcn_readlane(bl, k);
        const int64_t bs = (int64_t)shfl64((uint64_t)bsl, k), be = (int64_t)shfl64((uint64_t)bel, k);
        const int lo = i0 + k + 1;  // members of N+(a) after b
        int cnt_b = 0;
        for (int64_t jb = bs; jb < be; jb += PMC_WAVE) {
          const int64_t j = jb + l;
          const int x = j < be ? padj[j] : -1;
          bool found = false;
          if (x >= 0 && lo < la) {
            const int p = lo + lower_bound(A + lo, la - lo, x);
            found = p < la && A[p] == x;
          }
          if (found) atomicAdd(&tri[lab_vertex[x]], 1);
          cnt_b += found ? 1 : 0;
        }
        cnt_b = wave_sum(cnt_b);
        if (l == 0 && cnt_b) atomicAdd(&tri[lab_vertex[b]], cnt_b);
        cnt_a += cnt_b;
      }
    }
    if (l == 0 && cnt_a) atomicAdd(&tri[lab_vertex[a]], cnt_a);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    wave_sync();  // the slice is rewritten for the next label
  }
}

template <typename OffT>
__global__ void __launch_bounds__(256)
    k_features(int n, const OffT *__restrict__ off, const int32_t *__restrict__ idx,
               const int32_t *__restrict__ core, const int *__restrict__ tri, int kmax,
               float *feat) {
  int w = (blockIdx.x * blockDim.x + threadIdx.x) / PMC_WAVE;
  int nw = gridDim.x * blockDim.x / PMC_WAVE;
  int l = lane();
  const float K = (float)max(kmax, 1);
  for (int v = w; v < n; v += nw) {
    int64_t s = (int64_t)off[v], e = (int64_t)off[v + 1];
    int cv = core[v];
    long long sum = 0;
    int mx = INT_MIN, mn = INT_MAX, ge = 0;
    for (int64_t j = s + l; j < e; j += PMC_WAVE) {
      int c = core[idx[j]];
      sum += c;
      mx = max(mx, c);
      mn = min(mn, c);
      ge += c >= cv ? 1 : 0;
    }
    sum = wave_sum64(sum);
    mx = wave_max(mx);
    mn = wave_min(mn);
    ge = wave_sum(ge);
    if (l == 0) {
      int d = (int)(e - s);
      float *f = feat + (size_t)v * FIN;
      f[0] = log1pf((float)d);
      f[1] = log1pf((float)cv);
      f[2] = (float)cv / K;
      f[3] = log1pf((float)tri[v]);
      f[4] = d ? (float)((double)sum / d) / K : 0.f;
      f[5] = d ? (float)mx / K : 0.f;
      f[6] = d ? (float)mn / K : 0.f;
      f[7] = d ? (float)ge / (float)d : 0.f;
    }
  }
}

// --------------------------------------------------------------------- MLP

struct WeightsLds {
  short w1[FIN * HID];  // bf16, W1[k][j]
  short w2[HID * HID];  // bf16, W2[k][j]
  float b1[HID], b2[HID], w3[HID];
  float b3;
};

__device__ void stage_weights(const float *__restrict__ P, WeightsLds &W) {
  for (int i = threadIdx.x; i < FIN * HID; i += blockDim.x) W.w1[i] = to_bf16(P[OFF_W1 + i]);
  for (int i = threadIdx.x; i < HID * HID; i += blockDim.x) W.w2[i] = to_bf16(P[OFF_W2 + i]);
  for (int i = threadIdx.x; i < HID; i += blockDim.x) {
    W.b1[i] = P[OFF_B1 + i];
    W.b2[i] = P[OFF_B2 + i];
    W.w3[i] = P[OFF_W3 + i];
  }
  if (threadIdx.x == 0) W.b3 = P[OFF_B3];
  __syncthreads();
}

// Forward (and, with TRAIN, backward) over tiles of 16 vertices.  partial:
// one row of NPART floats per wave (TRAIN only).
template <bool TRAIN>
__global__ void __launch_bounds__(MLP_T)
    k_mlp(const float *__restrict__ P, const float *__restrict__ feat,
          const float *__restrict__ label, int n, float inv_batch, float *score, float *partial) {
  __shared__ WeightsLds W;
  __shared__ short xt[MLP_T / PMC_WAVE][16 * 16];   // X tile, bf16, [row][feature]
  __shared__ short ht[MLP_T / PMC_WAVE][16 * HID];  // H1 tile, then dZ2 tile, bf16
  stage_weights(P, W);
  const int l = lane(), q16 = l >> 4, c16 = l & 15;
  const int wl = threadIdx.x / PMC_WAVE;
  const int wg = (blockIdx.x * blockDim.x + threadIdx.x) / PMC_WAVE;
  const int nw = gridDim.x * blockDim.x / PMC_WAVE;
  short *X = xt[wl], *T = ht[wl];
  const int ntiles = (n + 15) / 16;
  // gradient accumulators (D layout)
  f4 gW1[4], gW2[4][4];
  float gb1[4] = {0, 0, 0, 0}, gb2[4] = {0, 0, 0, 0}, gw3[4] = {0, 0, 0, 0};
  float gb3 = 0.f, sq = 0.f;
  for (int t = 0; t < 4; t++) {
    gW1[t] = f4{0, 0, 0, 0};
    for (int m = 0; m < 4; m++) gW2[m][t] = f4{0, 0, 0, 0};
  }
  for (int tile = wg; tile < ntiles; tile += nw) {
    const int r0 = tile * 16;
    // ---- X tile: A operand straight from global, and a copy in LDS
    s4 xa;
    {
      int row = r0 + c16;
      for (int j = 0; j < 4; j++) {
        int k = 4 * q16 + j;
        float x = (k < FIN && row < n) ? feat[(size_t)row * FIN + k] : 0.f;
        xa[j] = to_bf16(x);
        X[c16 * 16 + k] = xa[j];
      }
    }
    // ---- layer 1
    s4 h1d[4];  // H1 in D layout (bf16): rows 4 q16 + j, column 16 t + c16
    for (int t = 0; t < 4; t++) {
      s4 b;
      for (int j = 0; j < 4; j++) {
        int k = 4 * q16 + j;
        b[j] = k < FIN ? W.w1[k * HID + 16 * t + c16] : (short)0;
      }
      f4 z = mfma(xa, b, f4{0, 0, 0, 0});
      for (int j = 0; j < 4; j++) {
        float h = fmaxf(z[j] + W.b1[16 * t + c16], 0.f);
        h1d[t][j] = to_bf16(h);
        T[(4 * q16 + j) * HID + 16 * t + c16] = h1d[t][j];
      }
    }
    wave_sync();
    // ---- layer 2
    f4 z2[4];
    for (int t = 0; t < 4; t++) {
      f4 acc = f4{0, 0, 0, 0};
      for (int q = 0; q < 4; q++) {
        s4 a, b;
        for (int j = 0; j < 4; j++) {
          a[j] = T[c16 * HID + 16 * q + 4 * q16 + j];
          b[j] = W.w2[(16 * q + 4 * q16 + j) * HID + 16 * t + c16];
        }
        acc = mfma(a, b, acc);
      }
      for (int j = 0; j < 4; j++) acc[j] += W.b2[16 * t + c16];
      z2[t] = acc;
    }
    // ---- output: s for rows 4 q16 + j, reduced over the 16 lanes of a group
    float s[4];
    for (int j = 0; j < 4; j++) {
      float p = 0.f;
      for (int t = 0; t < 4; t++) p += fmaxf(z2[t][j], 0.f) * W.w3[16 * t + c16];
      for (int o = 1; o < 16; o <<= 1) p += __shfl_xor(p, o, PMC_WAVE);
      s[j] = p + W.b3;
    }
    if (!TRAIN) {
      if (c16 == 0)
        for (int j = 0; j < 4; j++) {
          int row = r0 + 4 * q16 + j;
          if (row < n) score[row] = s[j];
        }
      wave_sync();
      continue;
    }
    // ---- backward
    float dS[4];
    for (int j = 0; j < 4; j++) {
      int row = r0 + 4 * q16 + j;
      float r = row < n ? s[j] - label[row] : 0.f;
      dS[j] = 2.f * r * inv_batch;
      if (c16 == 0) {
        sq += r * r;
        gb3 += dS[j];
      }
    }
    s4 dz2b[4];
    for (int t = 0; t < 4; t++) {
      for (int j = 0; j < 4; j++) {
        float h2 = fmaxf(z2[t][j], 0.f);
        gw3[t] += h2 * dS[j];
        float dz = z2[t][j] > 0.f ? dS[j] * W.w3[16 * t + c16] : 0.f;
        gb2[t] += dz;
        dz2b[t][j] = to_bf16(dz);
      }
    }
    wave_sync();  // every lane has read the H1 tile
    for (int t = 0; t < 4; t++)
      for (int j = 0; j < 4; j++) T[(4 * q16 + j) * HID + 16 * t + c16] = dz2b[t][j];
    // dW2 += H1^T dZ2
    for (int m = 0; m < 4; m++)
      for (int t = 0; t < 4; t++) gW2[m][t] = mfma(h1d[m], dz2b[t], gW2[m][t]);
    wave_sync();
    // dH1 = dZ2 W2^T, dZ1 = dH1 (H1 > 0), dW1 += X^T dZ1
    s4 xta;
    for (int j = 0; j < 4; j++) xta[j] = X[(4 * q16 + j) * 16 + c16];
    for (int t = 0; t < 4; t++) {
      f4 acc = f4{0, 0, 0, 0};
      for (int q = 0; q < 4; q++) {
        s4 a, b;
        for (int j = 0; j < 4; j++) {
          a[j] = T[c16 * HID + 16 * q + 4 * q16 + j];
          b[j] = W.w2[(16 * t + c16) * HID + 16 * q + 4 * q16 + j];
        }
        acc = mfma(a, b, acc);
      }
      s4 dz1b;
      for (int j = 0; j < 4; j++) {
        float dz = h1d[t][j] > 0 ? acc[j] : 0.f;  // bf16 bits > 0 <=> value > 0
        gb1[t] += dz;
        dz1b[j] = to_bf16(dz);
      }
      gW1[t] = mfma(xta, dz1b, gW1[t]);
    }
    wave_sync();
  }
  if (!TRAIN) return;
  // ---- one row of partial sums per wave
  float *row = partial + (size_t)wg * NPART;
  for (int t = 0; t < 4; t++) {
    for (int j = 0; j < 4; j++) {
      int k = 4 * q16 + j;
      if (k < FIN) row[OFF_W1 + k * HID + 16 * t + c16] = gW1[t][j];
      for (int m = 0; m < 4; m++) row[OFF_W2 + (16 * m + k) * HID + 16 * t + c16] = gW2[m][t][j];
    }
    float b1v = gb1[t], b2v = gb2[t], w3v = gw3[t];
    b1v += __shfl_xor(b1v, 16, PMC_WAVE);
    b1v += __shfl_xor(b1v, 32, PMC_WAVE);
    b2v += __shfl_xor(b2v, 16, PMC_WAVE);
    b2v += __shfl_xor(b2v, 32, PMC_WAVE);
    w3v += __shfl_xor(w3v, 16, PMC_WAVE);
    w3v += __shfl_xor(w3v, 32, PMC_WAVE);
    if (q16 == 0) {
      row[OFF_B1 + 16 * t + c16] = b1v;
      row[OFF_B2 + 16 * t + c16] = b2v;
      row[OFF_W3 + 16 * t + c16] = w3v;
    }
  }
  float g3 = gb3, sq2 = sq;
  for (int o = 32; o > 0; o >>= 1) {
    g3 += __shfl_xor(g3, o, PMC_WAVE);
    sq2 += __shfl_xor(sq2, o, PMC_WAVE);
  }
  if (l == 0) {
    row[OFF_B3] = g3;
    row[MLP_PARAMS] = sq2;
  }
}

// Sum of the partial rows, in row order (deterministic).
__global__ void k_reduce_partials(const float *partial, int rows, float *grad) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPART) return;
  float s = 0.f;
  for (int r = 0; r < rows; r++) s += partial[(size_t)r * NPART + p];
  grad[p] = s;
}

__global__ void k_adam(float *P, float *m, float *v, const float *grad, float lr, float c1,
                       float c2) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= MLP_PARAMS) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float g = grad[p];
  float mm = b1 * m[p] + (1.f - b1) * g;
  float vv = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  P[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

int mlp_grid(int n) {
  int tiles = (n + 15) / 16;
  int waves = std::min(tiles, dev_info().cus * 8);
  return std::max(1, (waves + 3) / 4);
}

}  // namespace

void run_features(const GraphView &g, const int32_t *core, const int32_t *rank,
                  const int32_t *order, int32_t kmax, float *feat, Scratch &sc) {
  hipStream_t s = sc.stream();
  int n = (int)g.n;
  if (n == 0) return;
  // oriented graph of all vertices (bound 0): labels are the ranks
  int32_t *zero = sc.get<int32_t>(1);
  PMC_HIP(hipMemsetAsync(zero, 0, sizeof(int32_t), s));
  Labels L = run_prune_orient(g, core, rank, order, nullptr, zero, kmax, sc);
  int *tri = sc.get<int>(n);
  PMC_HIP(hipMemsetAsync(tri, 0, sizeof(int) * n, s));
  int nb = (int)std::min<int64_t>((L.nn + 3) / 4 + 1, (int64_t)dev_info().cus * 16);
  if (L.nn > 0) {
    k_triangles<<<nb, TRI_T, 0, s>>>(L.nn, L.poff, L.padj, L.vertex, tri);
    PMC_HIP(hipGetLastError());
  }
  int nb2 = (int)std::min<int64_t>((n + 3) / 4 + 1, (int64_t)dev_info().cus * 16);
  PMC_DISPATCH_OFF(g, OffT, {
    k_features<OffT><<<nb2, 256, 0, s>>>(n, (const OffT *)g.off, g.idx, core, tri, kmax, feat);
  });
  PMC_HIP(hipGetLastError());
}

void run_mlp_forward(const float *params, const float *feat, int64_t n, float *score,
                     Scratch &sc) {
  if (n <= 0) return;
  k_mlp<false><<<mlp_grid((int)n), MLP_T, 0, sc.stream()>>>(params, feat, nullptr, (int)n, 0.f,
                                                             score, nullptr);
  PMC_HIP(hipGetLastError());
}

float run_mlp_train_step(float *params, float *m, float *v, int64_t step, float lr,
                         const float *feat, const float *label, int64_t n, float *grad_out,
                         Scratch &sc) {
  hipStream_t s = sc.stream();
  if (n <= 0) return 0.f;
  int blocks = mlp_grid((int)n);
  int rows = blocks * (MLP_T / PMC_WAVE);
  float *partial = sc.get<float>((size_t)rows * NPART);
  float *grad = sc.get<float>(NPART);
  k_mlp<true><<<blocks, MLP_T, 0, s>>>(params, feat, label, (int)n, 1.f / (float)n, nullptr,
                                       partial);
  PMC_HIP(hipGetLastError());
  k_reduce_partials<<<(NPART + 255) / 256, 256, 0, s>>>(partial, rows, grad);
  PMC_HIP(hipGetLastError());
  if (grad_out)
    PMC_HIP(hipMemcpyAsync(grad_out, grad, sizeof(float) * MLP_PARAMS, hipMemcpyDeviceToDevice, s));
  if (lr > 0.f) {
    double c1 = 1.0 - std::pow(0.9, (double)step), c2 = 1.0 - std::pow(0.999, (double)step);
    k_adam<<<(MLP_PARAMS + 255) / 256, 256, 0, s>>>(params, m, v, grad, lr, (float)c1, (float)c2);
    PMC_HIP(hipGetLastError());
  }
  float sq = 0.f;
  PMC_HIP(hipMemcpyAsync(&sq, grad + MLP_PARAMS, sizeof(float), hipMemcpyDeviceToHost, s));
  PMC_HIP(hipStreamSynchronize(s));
  return sq / (float)n;
}

}  // namespace pmc
