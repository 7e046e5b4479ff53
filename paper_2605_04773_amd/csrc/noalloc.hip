// Aggregation that allocates nothing: its scratch (parent forest, root
// flags and ranks, tile sums, block bounds) is a fixed device array of this file,
// one copy per GPU, whose device address is looked up once per device when a
// context is created there.  For callers that cannot allocate device memory
// during the call (graph capture, tight serving loops).
#include <mutex>

#include "internal.h"

namespace agc {
namespace {

// A parent word per vertex plus root bits and in-tile ranks (3 words per 64
// vertices), root counts per tile of 4096 vertices, block bounds and
// alignment slack:
// agg_scratch_words(kNoallocMaxVerts) fits (checked at set-up).  4,194,304
// vertices: 18.1 MB per GPU, held until the process ends.
constexpr int32_t kNoallocMaxVerts = 1 << 22;
constexpr int64_t kScratchWords = (int64_t)kNoallocMaxVerts + kNoallocMaxVerts / 16 + (1 << 16);

static __device__ __align__(256) uint32_t scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint32_t* g_ptr[kMaxDevices] = {};   // device address of scratch, per device

}  // namespace

// With `device` current: finds the address of this device's copy of the
// array (once per device).  The array's name is a host-side stand-in, never
// passed to a kernel; only this address is.
void noalloc_setup(int device) {
  AGC_REQUIRE(device >= 0 && device < kMaxDevices, "device index beyond the scratch table");
  AGC_REQUIRE(agg_scratch_words(kNoallocMaxVerts) <= kScratchWords, "no-allocation scratch too small");
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[device]) return;
  void* p = nullptr;
  AGC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  AGC_REQUIRE(p != nullptr && ((uintptr_t)p & 255u) == 0, "no-allocation scratch: bad symbol address");
  g_ptr[device] = (uint32_t*)p;
}

static uint32_t* noalloc_ptr(int device) {
  std::lock_guard<std::mutex> lock(g_mu);
  return (device >= 0 && device < kMaxDevices) ? g_ptr[device] : nullptr;
}

}  // namespace agc

extern "C" agc_status agc_aggregate_noalloc(agc_context* c, int32_t n_verts, int64_t n_edges, const int32_t* edges,
                                            const uint8_t* tags, int32_t* map, int32_t* n_coarse) {
  API_BEGIN(c)
  AGC_REQUIRE(n_verts >= 0 && n_edges >= 0, "negative size");
  AGC_REQUIRE(n_verts <= agc::kNoallocMaxVerts,
              "agc_aggregate_noalloc: n_verts exceeds 4194304, the size of its fixed scratch");
  AGC_REQUIRE(n_coarse, "n_coarse is null");
  AGC_REQUIRE(n_verts == 0 || map, "map is null");
  AGC_REQUIRE(n_edges == 0 || (edges && tags), "edges/tags null");
  AGC_REQUIRE(((uintptr_t)edges & 7) == 0, "edges must be 8-byte aligned");
  uint32_t* base = agc::noalloc_ptr(c->device);
  AGC_REQUIRE(base != nullptr, "no-allocation scratch not set up on this device");
  *n_coarse = agc::aggregate_into(c, n_verts, n_edges, edges, tags, map, agc::agg_scratch_carve(base, n_verts));
  API_END(c)
}
