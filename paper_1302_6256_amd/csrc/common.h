// common.h -- device helpers of the gfx950 library (wave64 primitives, grid
// barrier, memory-scope atomics).  Used only inside csrc/.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PMC_WAVE 64

namespace pmc {

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

// Full-wave ballot (wave64).
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Lanes below the calling lane.
__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = lane();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Keeps the compiler from moving memory operations across this point and
// makes earlier LDS writes of this wave visible to its later LDS reads (LDS
// operations of one wave execute in order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <typename T>
__device__ __forceinline__ T shfl(T v, int src) {
  return __shfl(v, src, PMC_WAVE);
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = __shfl(lo, src, PMC_WAVE);
  hi = __shfl(hi, src, PMC_WAVE);
  return ((uint64_t)hi << 32) | lo;
}

// Wave reductions (every lane receives the result).
__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, PMC_WAVE));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, PMC_WAVE));
  return v;
}
__device__ __forceinline__ int wave_sum(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, PMC_WAVE);
  return v;
}
__device__ __forceinline__ long long wave_sum64(long long v) {
  for (int o = 32; o > 0; o >>= 1) {
    long long w = ((long long)__shfl_xor((int)(v >> 32), o, PMC_WAVE) << 32) |
                  (unsigned)__shfl_xor((int)(v & 0xffffffff), o, PMC_WAVE);
    v += w;
  }
  return v;
}

// Device-scope (agent) atomics.
__device__ __forceinline__ int ld_relaxed(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_acquire(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int atomic_add(int *p, int v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-uniform atomic add by a wave: every lane issues it (lane 0 with v,
// the others with 0; the compiler folds the lanes into one atomic), so no
// lane-0 branch surrounds it, and the result (the value before the wave's
// add) is read from lane 0 into a scalar.  A claim made under a lane-0
// branch and broadcast by a shuffle can be restructured by the compiler so
// that the other lanes loop back without lane 0.
__device__ __forceinline__ int atomic_add_wave(int *p, int v) {
  return __builtin_amdgcn_readfirstlane(atomic_add(p, lane() == 0 ? v : 0));
}
__device__ __forceinline__ unsigned long long atomic_add_u64(unsigned long long *p,
                                                             unsigned long long v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int atomic_sub(int *p, int v) {
  return __hip_atomic_fetch_sub(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int atomic_max(int *p, int v) {
  return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int atomic_min(int *p, int v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long atomic_max_u64(unsigned long long *p,
                                                             unsigned long long v) {
  return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-aggregated append: every lane with `pred` gets a distinct slot of
// *counter; one atomic per wave.  Must be called by the whole wave.
__device__ __forceinline__ int wave_append(int *counter, bool pred) {
  uint64_t m = ballot(pred);
  int base = 0;
  if (m) {
    int leader = __ffsll((unsigned long long)m) - 1;
    if (lane() == leader) base = atomic_add(counter, __popcll(m));
    base = __shfl(base, leader, PMC_WAVE);
  }
  return base + __popcll(m & lanemask_lt());
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP moves (row shifts
// by 1, 2, 4, 8 within each row of 16 lanes, then the row-15 and row-31
// broadcasts across rows): register-level, no LDS traffic.  Lanes must all be
// active.
__device__ __forceinline__ int wave_incl_scan(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// Wave-aggregated append of `cnt` items per lane: lane l gets the first of
// its cnt consecutive slots of *counter; one atomic per wave, none if the
// wave appends nothing.  Must be called by the whole wave.
__device__ __forceinline__ int wave_append_n(int *counter, int cnt) {
  const int inc = wave_incl_scan(cnt);
  const int total = __builtin_amdgcn_readlane(inc, PMC_WAVE - 1);
  int base = 0;
  if (total) {
    if (lane() == 0) base = atomic_add(counter, total);
    base = __builtin_amdgcn_readfirstlane(base);
  }
  return base + inc - cnt;
}

// Workgroup-aggregated append: one atomic per workgroup.  Must be called by
// every thread of the workgroup in uniform control flow; `lds` holds
// blockDim.x / 64 + 1 ints.
__device__ __forceinline__ int block_append(int *counter, bool pred, int *lds) {
  const int w = threadIdx.x / PMC_WAVE, nw = blockDim.x / PMC_WAVE;
  uint64_t m = ballot(pred);
  if (lane() == 0) lds[w] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int i = 0; i < nw; i++) {
      int c = lds[i];
      lds[i] = tot;
      tot += c;
    }
    lds[nw] = tot ? atomic_add(counter, tot) : 0;
  }
  __syncthreads();
  int pos = lds[nw] + lds[w] + __popcll(m & lanemask_lt());
  __syncthreads();
  return pos;
}

// Workgroup minimum, returned to every thread (uniform control flow; `lds`
// holds blockDim.x / 64 ints).
__device__ __forceinline__ int block_min(int v, int *lds) {
  const int w = threadIdx.x / PMC_WAVE, nw = blockDim.x / PMC_WAVE;
  v = wave_min(v);
  if (lane() == 0) lds[w] = v;
  __syncthreads();
  int r = lds[0];
  for (int i = 1; i < nw; i++) r = min(r, lds[i]);
  __syncthreads();
  return r;
}

// Device-coherent plain accesses: relaxed atomics at device (agent) scope.
// They are performed at the device's coherence point, so data that one
// workgroup stores this way is seen by another workgroup's device-scope load
// without any cache writeback.
__device__ __forceinline__ void st_dev(int *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_dev(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_dev_u32(const unsigned *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier for a cooperative launch (all blocks co-resident).
// Two-level arrival on monotonic counters: blocks are grouped by
// blockIdx % GRID_GROUPS (the round-robin placement of workgroups over the 8
// XCDs) and each group counts arrivals on its own cache line, so no counter
// sees more than ~nblocks/8 atomics at once.  At barrier number g (from 0)
// the arrival that takes a group's count to (g+1) * group size is that
// group's last; it bumps the top counter without waiting for the result, and
// every block waits until the top counter reaches (g+1) * groups.  Counters
// only grow (a block cannot arrive at barrier g+1 before every block arrived
// at g), so nothing is reset and the release costs one returning atomic plus
// the poll.
// Memory contract: data exchanged across the barrier is written AND read with
// device-scope accesses (st_dev / ld_dev / atomics), which are performed at
// the device's coherence point; every wave drains its outstanding memory
// operations before the workgroup arrives, so everything stored before the
// barrier is visible to every device-scope load after it.  Plain loads are
// used only for data that no workgroup of the launch writes (the CSR), so no
// cache writeback or invalidation is needed.
constexpr int GRID_GROUPS = 8;
struct GridBar {
  unsigned long long group[GRID_GROUPS][16];  // one 128-byte line per group
  unsigned long long top;
  unsigned long long pad0[15];
};

__device__ __forceinline__ void grid_sync(GridBar *bar, unsigned nblocks,
                                          unsigned long long &gen_local) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long g1 = (unsigned long long)gen_local + 1;
    const unsigned grp = blockIdx.x % GRID_GROUPS;
    const unsigned gsize = nblocks / GRID_GROUPS + (grp < nblocks % GRID_GROUPS ? 1u : 0u);
    const unsigned ngroups = nblocks < GRID_GROUPS ? nblocks : GRID_GROUPS;
    unsigned long long prev = __hip_atomic_fetch_add(&bar->group[grp][0], 1ull, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
    if (prev == g1 * gsize - 1)
      __hip_atomic_fetch_add(&bar->top, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (__hip_atomic_load(&bar->top, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
           g1 * ngroups)
      __builtin_amdgcn_s_sleep(1);
  }
  gen_local++;
  __syncthreads();
}

template <typename OffT>
__device__ __forceinline__ int64_t ld_off(const OffT *off, int64_t v) {
  return (int64_t)off[v];
}

// Lower bound of x in the sorted array a[0..len).
template <typename T>
__device__ __forceinline__ int lower_bound(const T *a, int len, T x) {
  int lo = 0, hi = len;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

}  // namespace pmc
