// runtime.h -- host-side plumbing of the library: error propagation, stream-
// ordered scratch allocation, and launchers of the project-written
// primitives.  Used only inside csrc/.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

namespace pmc {

// Thrown inside the library only; converted to a status at the C boundary.
struct Error {
  int status;
  std::string msg;
};

#define PMC_HIP(call)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      throw ::pmc::Error{e_ == hipErrorOutOfMemory ? 4 : 5,                                  \
                         std::string(#call) + ": " + hipGetErrorString(e_)};                 \
  } while (0)

// The library's stream-ordered memory pool of the current device.  Freed
// scratch stays in the pool (release threshold = unlimited), so a repeated
// call reuses the previous call's pages instead of mapping new ones.
hipMemPool_t scratch_pool();

// Bytes of scratch the previous call used (a size hint for the first chunk).
size_t &scratch_hint();

// Scratch memory of one call: 256-byte aligned pieces carved from a few large
// chunks allocated on the stream from the library's pool, all released
// (stream-ordered) when the object goes out of scope.  Stream-ordered
// allocation calls cost tens of microseconds each, so a call makes one or two
// of them rather than one per buffer; the first chunk is sized from the
// previous call's total.
//
// A Scratch built over a fixed device buffer (base, bytes) instead carves
// every piece from that buffer, allocates and frees nothing, and throws a
// capacity error when the buffer is exhausted.
class Scratch {
 public:
  explicit Scratch(hipStream_t s) : s_(s) {}
  Scratch(hipStream_t s, void *fixed, size_t fixed_bytes) : s_(s), fixed_(true) {
    chunks_.push_back({(char *)fixed, fixed_bytes, 0});
  }
  ~Scratch() {
    if (fixed_) return;
    if (total_) scratch_hint() = total_;
    for (auto &c : chunks_) (void)hipFreeAsync(c.base, s_);
  }
  template <typename T>
  T *get(size_t count) {
    size_t bytes = count * sizeof(T);
    bytes = bytes == 0 ? 256 : (bytes + 255) / 256 * 256;
    if (fixed_ && chunks_.back().used + bytes > chunks_.back().size)
      throw Error{3, "the fixed scratch buffer (" + std::to_string(chunks_.back().size) +
                         " bytes) is too small for this call"};
    if (chunks_.empty() || chunks_.back().used + bytes > chunks_.back().size) {
      size_t want = chunks_.empty() ? scratch_hint() : 2 * chunks_.back().size;
      want = std::max(want, std::max(bytes, (size_t)64 << 20));
      void *p = nullptr;
      hipError_t e = hipMallocFromPoolAsync(&p, want, scratch_pool(), s_);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        want = bytes;  // retry with exactly what is needed
        e = hipMallocFromPoolAsync(&p, want, scratch_pool(), s_);
      }
      if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{4, "scratch allocation of " + std::to_string(bytes) + " bytes failed"};
      }
      chunks_.push_back({(char *)p, want, 0});
    }
    Chunk &c = chunks_.back();
    T *r = (T *)(c.base + c.used);
    c.used += bytes;
    total_ += bytes;
    return r;
  }
  hipStream_t stream() const { return s_; }

 private:
  struct Chunk {
    char *base;
    size_t size, used;
  };
  hipStream_t s_;
  bool fixed_ = false;
  std::vector<Chunk> chunks_;
  size_t total_ = 0;
};

// Device properties cached per device.
struct DevInfo {
  int cus = 256;
  int max_lds = 65536;      // LDS bytes per workgroup
  int lds_per_cu = 65536;   // LDS bytes per CU
};
const DevInfo &dev_info();

// Exclusive scan of n int32 counts into n+1 int64 offsets (out[n] = total).
void scan_counts(const int32_t *in, int64_t *out, int64_t n, Scratch &sc);
// Exclusive scan of n int32 values into n int32 (the caller knows the total fits).
void scan_i32(const int32_t *in, int32_t *out, int64_t n, Scratch &sc);

// Stable LSD radix sort of (key, value) pairs on key bits [0, bits).
// vals_in NULL means values 0..n-1.  Outputs may not alias inputs.
void radix_sort_pairs(const uint32_t *keys_in, const int32_t *vals_in, uint32_t *keys_out,
                      int32_t *vals_out, int64_t n, int bits, Scratch &sc);

}  // namespace pmc
