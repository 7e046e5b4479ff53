// Internal helpers shared by the HIP sources of libagc (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <unordered_map>

#include "agc.h"

namespace agc {

constexpr int kWG = 256;    // threads per workgroup: four wave64s
constexpr int kWave = 64;
constexpr int kWaves = kWG / kWave;

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define AGC_HIP(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::agc::Error(e_ == hipErrorOutOfMemory ? AGC_ERR_OUT_OF_MEMORY : AGC_ERR_DEVICE, \
                         std::string(#call) + ": " + hipGetErrorString(e_));              \
  } while (0)

#define AGC_LAUNCH_CHECK() AGC_HIP(hipGetLastError())

#define AGC_REQUIRE(cond, msg)                                        \
  do {                                                                \
    if (!(cond)) throw ::agc::Error(AGC_ERR_INVALID_ARG, (msg));      \
  } while (0)

inline unsigned blocks_for(int64_t n, int64_t per) {
  int64_t b = (n + per - 1) / per;
  return (unsigned)(b < 1 ? 1 : b);
}

inline int bits_for(uint64_t maxval) {  // bits needed to represent values in [0, maxval]
  int b = 0;
  while (b < 64 && (maxval >> b) != 0) ++b;
  return b;
}

// ----------------------------------------------------------------- workspace

// Grow-only device buffer.  Reallocation calls hipFree, which waits for the
// device, so a buffer is never released while a kernel still reads it.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  void* ensure(size_t bytes) {
    if (bytes <= cap && p) return p;
    if (p) AGC_HIP(hipFree(p));
    p = nullptr;
    cap = 0;
    size_t want = bytes < 256 ? 256 : bytes;
    AGC_HIP(hipMalloc(&p, want));
    cap = want;
    return p;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

class Workspace {
 public:
  template <class T>
  T* get(const std::string& name, int64_t count) {
    return static_cast<T*>(bufs_[name].ensure(sizeof(T) * (size_t)(count < 1 ? 1 : count)));
  }
  void release() {
    for (auto& kv : bufs_) kv.second.release();
    bufs_.clear();
  }

 private:
  std::unordered_map<std::string, DevBuf> bufs_;
};

// ------------------------------------------------------------------ device

// Bits of the per-call device error word.
enum : unsigned { kErrRange = 1u, kErrTag = 2u, kErrElem = 4u, kErrMap = 8u, kErrNoDiag = 16u,
                  kErrNotSPD = 32u };

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  return (lane_id() == 0) ? 0ull : (~0ull >> (64 - lane_id()));
}

// Device-scope load that bypasses a possibly stale per-CU cache line.
template <class T>
__device__ __forceinline__ T load_agent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive/inclusive scan of one uint32 per thread over a workgroup of kWG
// threads.  `lds` holds kWaves entries.  Returns the exclusive prefix; *total
// receives the workgroup total.
__device__ __forceinline__ uint32_t wg_exclusive_scan(uint32_t v, uint32_t* lds, uint32_t* total) {
  const unsigned lane = lane_id();
  const unsigned wave = threadIdx.x / kWave;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint32_t y = __shfl_up(x, d);
    if (lane >= (unsigned)d) x += y;
  }
  if (lane == kWave - 1) lds[wave] = x;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    uint32_t s = lds[w];
    if (w < (int)wave) off += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

// Fixed-order workgroup sum of one double per thread (tree over lanes, then waves).
__device__ __forceinline__ double wg_sum(double v, double* lds) {
  const unsigned lane = lane_id();
  const unsigned wave = threadIdx.x / kWave;
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_down(v, d);
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < kWaves; ++w) t += lds[w];
  }
  __syncthreads();
  return t;  // valid in thread 0
}

}  // namespace agc
