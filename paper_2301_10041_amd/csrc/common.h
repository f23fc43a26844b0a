// Shared helpers of libfsi: device buffers, error propagation, launch shapes and
// wavefront reductions for gfx950 (64-lane wavefronts).
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fsi.h"

namespace fsi {

// Error carried through the C++ layers and turned into an fsi_status at the ABI.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define FSI_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::fsi::Error(e_ == hipErrorOutOfMemory ? FSI_E_NOMEM : FSI_E_HIP,          \
                         std::string(#call) + ": " + hipGetErrorString(e_));           \
  } while (0)

#define FSI_CHECK_LAUNCH() FSI_HIP(hipGetLastError())

#define FSI_REQUIRE(cond, code, msg) \
  do {                               \
    if (!(cond)) throw ::fsi::Error((code), (msg)); \
  } while (0)

// Owning device allocation of n elements of T.
template <typename T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    if (count == 0) count = 1;   // keep a valid pointer for empty arrays
    FSI_HIP(hipMalloc(&p, count * sizeof(T)));
    n = count;
  }
  // grow-only reallocation (contents are not preserved)
  void reserve(size_t count) { if (count > n || p == nullptr) alloc(count); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  size_t bytes() const { return n * sizeof(T); }
  T *get() const { return p; }
};

constexpr int kWave = 64;

// A per-lane view of a device array for kernels over K independent systems (lane = blockIdx.y):
// lane k uses p + k s; s = 0 for data shared by every lane.  A plain pointer converts to a
// view with s = 0, so one-system call sites are unchanged.
template <typename T>
struct LP {
  T *p = nullptr;
  int64_t s = 0;
  LP() = default;
  __host__ __device__ LP(T *ptr, int64_t stride = 0) : p(ptr), s(stride) {}
  template <typename U, typename = typename std::enable_if<std::is_convertible<U *, T *>::value>::type>
  __host__ __device__ LP(const LP<U> &o) : p(o.p), s(o.s) {}
  __host__ __device__ T *at(int k) const { return p + (int64_t)k * s; }
  __host__ __device__ LP operator+(int64_t o) const { return LP(p + o, s); }
};

inline unsigned grid_for(int64_t items, int block) {
  int64_t g = (items + block - 1) / block;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// Sum over the 64 lanes of a wavefront (every lane gets the result).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sum over aligned groups of G lanes (G a power of two <= 64).
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}


}  // namespace fsi
