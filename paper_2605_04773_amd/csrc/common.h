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

// Where device memory comes from: hipMalloc / hipFree, or a caller's pair
// of functions (agc_set_allocator).  tl_alloc is the allocator of the
// context whose entry point runs on this thread (set for the duration of
// the call by API_BEGIN); null means hipMalloc.
struct Allocator {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free)(void*, void*) = nullptr;
  void* user = nullptr;
};
inline thread_local const Allocator* tl_alloc = nullptr;
struct AllocScope {
  const Allocator* prev;
  explicit AllocScope(const Allocator* a) : prev(tl_alloc) { tl_alloc = (a && a->alloc) ? a : nullptr; }
  ~AllocScope() { tl_alloc = prev; }
};

// Grow-only device buffer, released through the allocator it came from.
// With hipMalloc, reallocation calls hipFree, which waits for the device,
// so a buffer is never released while a kernel still reads it; a caller's
// allocator receives its blocks back in the order of the context's stream
// (a stream-ordered caching allocator on that stream keeps the same
// guarantee).
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  Allocator al;   // the source of p
  void* ensure(size_t bytes) {
    if (bytes <= cap && p) return p;
    release_or_throw();
    const size_t want = bytes < 256 ? 256 : bytes;
    if (tl_alloc) {
      al = *tl_alloc;
      p = al.alloc(want, al.user);
      if (!p) throw Error(AGC_ERR_OUT_OF_MEMORY, "the caller's allocator returned no memory");
    } else {
      al = Allocator{};
      AGC_HIP(hipMalloc(&p, want));
    }
    cap = want;
    return p;
  }
  void release() {
    if (p) {
      if (al.free) al.free(p, al.user);
      else (void)hipFree(p);
    }
    p = nullptr;
    cap = 0;
    al = Allocator{};
  }

 private:
  void release_or_throw() {
    if (p && !al.free) AGC_HIP(hipFree(p));
    else if (p) al.free(p, al.user);
    p = nullptr;
    cap = 0;
    al = Allocator{};
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
                  kErrNotSPD = 32u, kErrDegenerate = 64u, kErrUnused = 128u,
                  kErrDiagLb = 256u };

inline unsigned grid_blocks(int64_t n) {   // grid for a grid-stride loop over n items
  int64_t b = (n + kWG - 1) / kWG;
  if (b > 65536) b = 65536;
  return (unsigned)(b < 1 ? 1 : b);
}

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// Workgroups are dispatched round-robin over the eight XCDs (each with its
// own L2).  This renumbering gives XCD x the contiguous range of blocks
// [x*q + min(x, rem), ...) so that neighbouring tiles, and the vector
// entries they gather, share one L2.  A bijection for any grid size.
constexpr unsigned kXcds = 8;
#ifndef AGC_XCD_MAP
#define AGC_XCD_MAP 1
#endif
__device__ __forceinline__ int64_t xcd_block() {
#if AGC_XCD_MAP
  const unsigned b = blockIdx.x, G = gridDim.x;
  const unsigned x = b % kXcds, i = b / kXcds;
  const unsigned q = G / kXcds, rem = G % kXcds;
  return (int64_t)x * q + (x < rem ? x : rem) + i;
#else
  return blockIdx.x;
#endif
}

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

// ------------------------------------------------------ wave64 DPP moves
// GFX9 data-parallel-primitive lane moves (VALU, no LDS traffic).  A lane
// whose source lies outside the pattern, or whose 16-lane row is masked off,
// keeps `old`.  Every lane of the wave must be active.
enum : int {
  kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118,
  kDppRowBcast15 = 0x142,   // lane 15 of each row -> the next row
  kDppRowBcast31 = 0x143,   // lane 31 -> rows 2 and 3
  kDppWaveShr1 = 0x138      // lane i-1 -> lane i
};

template <int CTRL, int ROWS>
__device__ __forceinline__ int32_t dpp_move(int32_t old, int32_t x) {
  return __builtin_amdgcn_update_dpp(old, x, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_move(float old, float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), CTRL, ROWS, 0xf, false));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double old, double x) {
  const int32_t lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(x), CTRL, ROWS, 0xf, false);
  const int32_t hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(x), CTRL, ROWS, 0xf, false);
  return __hiloint2double(hi, lo);
}

// One Hillis-Steele step of a segmented inclusive scan: add the value of the
// source lane when it carries the same key.  Keys never equal INT32_MIN.
template <int CTRL, int ROWS, int N, class T>
__device__ __forceinline__ void seg_scan_step(int32_t key, T (&v)[N]) {
  const int32_t ku = dpp_move<CTRL, ROWS>((int32_t)INT32_MIN, key);
  T vu[N];
#pragma unroll
  for (int i = 0; i < N; ++i) vu[i] = dpp_move<CTRL, ROWS>((T)0, v[i]);
  if (ku == key) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += vu[i];
  }
}

// Segmented inclusive scan over the wave of N doubles per lane, segments
// being runs of equal, non-decreasing keys: shifts 1, 2, 4, 8 inside each
// row of 16 lanes, then row 0 -> 1 and 2 -> 3, then lane 31 -> rows 2, 3.
// The order of additions is fixed.
template <int N, class T>
__device__ __forceinline__ void wave_seg_scan(int32_t key, T (&v)[N]) {
  seg_scan_step<kDppRowShr1, 0xf>(key, v);
  seg_scan_step<kDppRowShr2, 0xf>(key, v);
  seg_scan_step<kDppRowShr4, 0xf>(key, v);
  seg_scan_step<kDppRowShr8, 0xf>(key, v);
  seg_scan_step<kDppRowBcast15, 0xa>(key, v);
  seg_scan_step<kDppRowBcast31, 0xc>(key, v);
}

// Fixed-order sums of K doubles per thread over the workgroup with one
// barrier; every thread receives the totals.  lds holds K * kWaves doubles
// and must not be reused before another barrier.
template <int K>
__device__ __forceinline__ void wg_sum_all(double (&v)[K], double* lds) {
  wave_seg_scan<K>(0, v);
  const unsigned wave = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[k * kWaves + wave] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) t += lds[k * kWaves + w];
    v[k] = t;
  }
}

// Fixed-order workgroup sum of one double per thread.  Valid in every
// thread; lds (kWaves doubles) may be reused after return.
__device__ __forceinline__ double wg_sum(double v, double* lds) {
  double a[1] = {v};
  wg_sum_all<1>(a, lds);
  __syncthreads();
  return a[0];
}

}  // namespace agc
