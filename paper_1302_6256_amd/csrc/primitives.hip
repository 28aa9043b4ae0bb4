// primitives.hip -- project-written device-wide scan and stable radix sort
// (their counters are attributable in profiles; no library sort is used).
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include "common.h"
#include "runtime.h"

namespace pmc {

const DevInfo &dev_info() {
  static thread_local int dev = -1;
  static thread_local DevInfo info;
  int d = 0;
  PMC_HIP(hipGetDevice(&d));
  if (d != dev) {
    PMC_HIP(hipDeviceGetAttribute(&info.cus, hipDeviceAttributeMultiprocessorCount, d));
    PMC_HIP(hipDeviceGetAttribute(&info.max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, d));
    PMC_HIP(hipDeviceGetAttribute(&info.lds_per_cu,
                                  hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, d));
    dev = d;
  }
  return info;
}

size_t &scratch_hint() {
  static thread_local size_t hint = 0;
  return hint;
}

namespace {
std::mutex pool_mu;
std::map<int, hipMemPool_t> &pool_map() {
  static std::map<int, hipMemPool_t> *pools = new std::map<int, hipMemPool_t>();
  return *pools;
}

// Destroys the library's pools at process exit.  Registered with atexit
// after the HIP runtime has initialised (the first pool is created after the
// first HIP call), so it runs before the runtime's own teardown and before
// tools loaded into the process finalise, rather than leaving live pools to
// an unspecified teardown order.
void release_pools() {
  std::lock_guard<std::mutex> lock(pool_mu);
  for (auto &kv : pool_map()) {
    if (hipSetDevice(kv.first) != hipSuccess) continue;
    (void)hipDeviceSynchronize();
    (void)hipMemPoolTrimTo(kv.second, 0);
    (void)hipMemPoolDestroy(kv.second);
  }
  pool_map().clear();
  (void)hipGetLastError();
}
}  // namespace

hipMemPool_t scratch_pool() {
  int d = 0;
  PMC_HIP(hipGetDevice(&d));
  std::lock_guard<std::mutex> lock(pool_mu);
  auto &pools = pool_map();
  auto it = pools.find(d);
  if (it != pools.end()) return it->second;
  static bool registered = (std::atexit(release_pools) == 0);
  (void)registered;
  hipMemPoolProps props;
  std::memset(&props, 0, sizeof(props));
  props.allocType = hipMemAllocationTypePinned;
  props.handleTypes = hipMemHandleTypeNone;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = d;
  hipMemPool_t pool;
  PMC_HIP(hipMemPoolCreate(&pool, &props));
  uint64_t keep = UINT64_MAX;
  PMC_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
  pools[d] = pool;
  return pool;
}

namespace {

constexpr int SCAN_T = 256;
constexpr int SCAN_I = 8;
constexpr int SCAN_TILE = SCAN_T * SCAN_I;

// Inclusive block scan of one value per thread (256 threads, 4 waves).
template <typename T>
__device__ T block_incl_scan(T v, T *lds_w, T &total) {
  int l = lane(), w = threadIdx.x / PMC_WAVE;
  for (int o = 1; o < PMC_WAVE; o <<= 1) {
    T u = __shfl_up(v, o, PMC_WAVE);
    if (l >= o) v += u;
  }
  if (l == PMC_WAVE - 1) lds_w[w] = v;
  __syncthreads();
  T pre = 0;
  total = 0;
  for (int i = 0; i < SCAN_T / PMC_WAVE; i++) {
    T x = lds_w[i];
    if (i < w) pre += x;
    total += x;
  }
  __syncthreads();
  return v + pre;
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(SCAN_T) k_tile_sums(const TI *in, TO *part, int64_t n) {
  __shared__ TO lw[SCAN_T / PMC_WAVE];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  TO s = 0;
  for (int i = 0; i < SCAN_I; i++) {
    int64_t j = base + (int64_t)i * SCAN_T + threadIdx.x;
    if (j < n) s += (TO)in[j];
  }
  TO tot;
  block_incl_scan<TO>(s, lw, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Single block: exclusive scan of the tile partials in place.
template <typename TO>
__global__ void __launch_bounds__(SCAN_T) k_scan_partials(TO *part, int64_t nt) {
  __shared__ TO lw[SCAN_T / PMC_WAVE];
  TO carry = 0;
  for (int64_t b = 0; b < nt; b += SCAN_T) {
    int64_t j = b + threadIdx.x;
    TO v = j < nt ? part[j] : 0;
    TO tot;
    TO inc = block_incl_scan<TO>(v, lw, tot);
    if (j < nt) part[j] = carry + inc - v;
    carry += tot;
  }
}

// Exclusive scan of each tile using blocked items per thread (coalesced by
// striding through LDS), plus the tile's offset.
template <typename TI, typename TO>
__global__ void __launch_bounds__(SCAN_T) k_tile_scan(const TI *in, TO *out, const TO *part,
                                                      int64_t n, int write_total) {
  __shared__ TO buf[SCAN_TILE];
  __shared__ TO lw[SCAN_T / PMC_WAVE];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  for (int i = 0; i < SCAN_I; i++) {
    int64_t j = base + (int64_t)i * SCAN_T + threadIdx.x;
    buf[i * SCAN_T + threadIdx.x] = j < n ? (TO)in[j] : 0;
  }
  __syncthreads();
  TO loc[SCAN_I];
  TO s = 0;
  for (int i = 0; i < SCAN_I; i++) {
    loc[i] = buf[threadIdx.x * SCAN_I + i];
    s += loc[i];
  }
  TO tot;
  TO inc = block_incl_scan<TO>(s, lw, tot);
  TO run = part[blockIdx.x] + inc - s;
  for (int i = 0; i < SCAN_I; i++) {
    buf[threadIdx.x * SCAN_I + i] = run;
    run += loc[i];
  }
  __syncthreads();
  for (int i = 0; i < SCAN_I; i++) {
    int64_t j = base + (int64_t)i * SCAN_T + threadIdx.x;
    if (j < n) out[j] = buf[i * SCAN_T + threadIdx.x];
  }
  if (write_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_T - 1)
    out[n] = part[blockIdx.x] + tot;
}

template <typename TI, typename TO>
void scan_impl(const TI *in, TO *out, int64_t n, Scratch &sc, int write_total) {
  hipStream_t s = sc.stream();
  if (n == 0) {
    if (write_total) PMC_HIP(hipMemsetAsync(out, 0, sizeof(TO), s));
    return;
  }
  int64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
  TO *part = sc.get<TO>(nt);
  k_tile_sums<TI, TO><<<nt, SCAN_T, 0, s>>>(in, part, n);
  k_scan_partials<TO><<<1, SCAN_T, 0, s>>>(part, nt);
  k_tile_scan<TI, TO><<<nt, SCAN_T, 0, s>>>(in, out, part, n, write_total);
  PMC_HIP(hipGetLastError());
}

// ------------------------------------------------------------ radix sort
constexpr int RX_T = 256;
constexpr int RX_SUB = 16;
constexpr int RX_TILE = RX_T * RX_SUB;
constexpr int RX_W = RX_T / PMC_WAVE;

__global__ void __launch_bounds__(RX_T) k_radix_hist(const uint32_t *keys, int64_t n, int shift,
                                                     int32_t *hist, int ntiles) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RX_TILE;
  for (int i = 0; i < RX_SUB; i++) {
    int64_t j = base + (int64_t)i * RX_T + threadIdx.x;
    if (j < n) atomicAdd(&h[(keys[j] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: items of a tile keep their relative order within a digit.
__global__ void __launch_bounds__(RX_T) k_radix_scatter(const uint32_t *kin, const int32_t *vin,
                                                        uint32_t *kout, int32_t *vout, int64_t n,
                                                        int shift, const int32_t *gofs,
                                                        int ntiles) {
  __shared__ int run[256];
  __shared__ int cnt[RX_W][256];
  __shared__ int tbase[256];
  int t = threadIdx.x, w = t / PMC_WAVE;
  run[t] = 0;
  for (int i = 0; i < RX_W; i++) cnt[i][t] = 0;
  tbase[t] = gofs[(int64_t)t * ntiles + blockIdx.x];
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RX_TILE;
  for (int sub = 0; sub < RX_SUB; sub++) {
    int64_t j = base + (int64_t)sub * RX_T + t;
    bool valid = j < n;
    uint32_t k = valid ? kin[j] : 0u;
    int32_t v = valid ? (vin ? vin[j] : (int32_t)j) : 0;
    uint32_t d = (k >> shift) & 255u;
    uint64_t m = ballot(valid);
    for (int b = 0; b < 8; b++) {
      uint64_t bb = ballot((d >> b) & 1u);
      m &= ((d >> b) & 1u) ? bb : ~bb;
    }
    int r = __popcll(m & lanemask_lt());
    if (valid && r == 0) cnt[w][d] = __popcll(m);
    __syncthreads();
    if (valid) {
      int off = run[d] + r;
      for (int i = 0; i < w; i++) off += cnt[i][d];
      int64_t dst = (int64_t)tbase[d] + off;
      kout[dst] = k;
      vout[dst] = v;
    }
    __syncthreads();
    int add = 0;
    for (int i = 0; i < RX_W; i++) {
      add += cnt[i][t];
      cnt[i][t] = 0;
    }
    run[t] += add;
    __syncthreads();
  }
}

}  // namespace

void scan_counts(const int32_t *in, int64_t *out, int64_t n, Scratch &sc) {
  scan_impl<int32_t, int64_t>(in, out, n, sc, 1);
}
void scan_i32(const int32_t *in, int32_t *out, int64_t n, Scratch &sc) {
  scan_impl<int32_t, int32_t>(in, out, n, sc, 0);
}

void radix_sort_pairs(const uint32_t *keys_in, const int32_t *vals_in, uint32_t *keys_out,
                      int32_t *vals_out, int64_t n, int bits, Scratch &sc) {
  hipStream_t s = sc.stream();
  if (n == 0) return;
  int passes = std::max(1, (bits + 7) / 8);
  int ntiles = (int)((n + RX_TILE - 1) / RX_TILE);
  int32_t *hist = sc.get<int32_t>((size_t)256 * ntiles);
  int32_t *gofs = sc.get<int32_t>((size_t)256 * ntiles);
  uint32_t *kt = nullptr;
  int32_t *vt = nullptr;
  if (passes > 1) {
    kt = sc.get<uint32_t>(n);
    vt = sc.get<int32_t>(n);
  }
  // ping-pong so that the last pass lands in the outputs
  const uint32_t *ki = keys_in;
  const int32_t *vi = vals_in;
  for (int p = 0; p < passes; p++) {
    bool last = p == passes - 1;
    uint32_t *ko = ((passes - 1 - p) % 2 == 0) ? keys_out : kt;
    int32_t *vo = ((passes - 1 - p) % 2 == 0) ? vals_out : vt;
    (void)last;
    k_radix_hist<<<ntiles, RX_T, 0, s>>>(ki, n, 8 * p, hist, ntiles);
    scan_i32(hist, gofs, (int64_t)256 * ntiles, sc);
    k_radix_scatter<<<ntiles, RX_T, 0, s>>>(ki, vi, ko, vo, n, 8 * p, gofs, ntiles);
    PMC_HIP(hipGetLastError());
    ki = ko;
    vi = vo;
  }
}

}  // namespace pmc
