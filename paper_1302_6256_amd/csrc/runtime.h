// runtime.h -- host-side plumbing of the library: error propagation, stream-
// ordered scratch allocation, and launchers of the project-written
// primitives.  Used only inside csrc/.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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

// Scratch memory allocated on the stream, released (stream-ordered) when the
// object goes out of scope.
class Scratch {
 public:
  explicit Scratch(hipStream_t s) : s_(s) {}
  ~Scratch() {
    for (void *p : ptrs_) (void)hipFreeAsync(p, s_);
  }
  template <typename T>
  T *get(size_t count) {
    void *p = nullptr;
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMallocAsync(&p, bytes, s_);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error{4, "scratch allocation of " + std::to_string(bytes) + " bytes failed"};
    }
    ptrs_.push_back(p);
    return (T *)p;
  }
  hipStream_t stream() const { return s_; }

 private:
  hipStream_t s_;
  std::vector<void *> ptrs_;
};

// Device properties cached per device.
struct DevInfo {
  int cus = 256;
  int max_lds = 65536;
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
