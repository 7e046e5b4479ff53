// Device-wide primitives: exclusive scan, stable LSD radix sort, error word.
//
// All of them are deterministic: no floating point is involved, and every
// output position is a function of the input alone (integer atomics are used
// only for counts, whose result does not depend on their order).
#include "internal.h"

namespace agc {

// ------------------------------------------------------------------ scan

constexpr int kScanItems = 8;
constexpr int kScanTile = kWG * kScanItems;

__global__ __launch_bounds__(kWG) void k_scan_tile(const uint32_t* __restrict__ in,
                                                   uint32_t* __restrict__ out,
                                                   uint32_t* __restrict__ tile_sums, int64_t n) {
  __shared__ uint32_t lds[kWaves];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t k = base + i;
    v[i] = (k < n) ? in[k] : 0u;
    s += v[i];
  }
  uint32_t total;
  uint32_t off = wg_exclusive_scan(s, lds, &total);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t k = base + i;
    if (k < n) out[k] = off;
    off += v[i];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kWG) void k_scan_add(uint32_t* __restrict__ out,
                                                  const uint32_t* __restrict__ tile_off, int64_t n) {
  const uint32_t add = tile_off[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  for (int i = threadIdx.x; i < kScanTile; i += kWG) {
    int64_t k = base + i;
    if (k < n) out[k] += add;
  }
}

__global__ void k_scan_total(uint32_t* out, const uint32_t* tile_off, int64_t n_tiles, int64_t n) {
  out[n] = tile_off[n_tiles];
}

void scan_u32(agc_context* c, const uint32_t* in, uint32_t* out, int64_t n, const std::string& tag) {
  if (n <= 0) {
    AGC_HIP(hipMemsetAsync(out, 0, sizeof(uint32_t), c->stream));
    return;
  }
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  uint32_t* sums = c->ws.get<uint32_t>(tag + ".sums", tiles + 1);
  k_scan_tile<<<(unsigned)tiles, kWG, 0, c->stream>>>(in, out, sums, n);
  AGC_LAUNCH_CHECK();
  if (tiles == 1) {
    // single tile: its total is the grand total, its offset is 0
    k_scan_total<<<1, 1, 0, c->stream>>>(out, sums, 0, n);
    AGC_LAUNCH_CHECK();
    return;
  }
  // sums[0..tiles] becomes the exclusive scan of the tile totals
  scan_u32(c, sums, sums, tiles, tag + "+");
  k_scan_add<<<(unsigned)tiles, kWG, 0, c->stream>>>(out, sums, n);
  AGC_LAUNCH_CHECK();
  k_scan_total<<<1, 1, 0, c->stream>>>(out, sums, tiles, n);
  AGC_LAUNCH_CHECK();
}

// ------------------------------------------------------------ radix sort

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;   // == kWG: thread t owns digit t
constexpr int kSortItems = 8;
constexpr int kSortTile = kWG * kSortItems;
static_assert(kRadix == kWG, "one digit per thread");

template <class K>
__global__ __launch_bounds__(kWG) void k_radix_hist(const K* __restrict__ keys, int64_t n, int shift,
                                                    uint32_t* __restrict__ hist, int64_t n_tiles) {
  __shared__ uint32_t h[kRadix];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    int64_t k = base + r * kWG + threadIdx.x;
    if (k < n) atomicAdd(&h[(unsigned)((keys[k] >> shift) & (kRadix - 1))], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter.  Items of a tile are taken in rounds of kWG consecutive
// keys; inside a round the rank of a key among equal digits is (earlier
// waves' counts) + (lower lanes with the same digit, from 8 ballots).
template <class K>
__global__ __launch_bounds__(kWG) void k_radix_scatter(const K* __restrict__ keys_in,
                                                       const uint32_t* __restrict__ vals_in,
                                                       K* __restrict__ keys_out,
                                                       uint32_t* __restrict__ vals_out, int64_t n,
                                                       int shift, const uint32_t* __restrict__ offs,
                                                       int64_t n_tiles) {
  __shared__ uint32_t base[kRadix];
  __shared__ uint32_t wcnt[kWaves][kRadix];
  const unsigned t = threadIdx.x;
  const unsigned wave = t / kWave;
  base[t] = offs[(int64_t)t * n_tiles + blockIdx.x];
  const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
  const uint64_t lt = lanemask_lt();
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t k = tile0 + r * kWG + t;
    if (tile0 + r * kWG >= n) break;            // uniform across the workgroup
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wcnt[w][t] = 0;
    __syncthreads();
    const bool valid = k < n;
    K key = valid ? keys_in[k] : (K)0;
    uint32_t val = valid ? vals_in[k] : 0u;
    const unsigned digit = (unsigned)((key >> shift) & (kRadix - 1));
    uint64_t match = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (digit >> b) & 1u;
      const uint64_t m = __ballot(bit);
      match &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(match & lt);
    if (valid && rank == 0) wcnt[wave][digit] = (uint32_t)__popcll(match);
    __syncthreads();
    if (valid) {
      uint32_t pos = base[digit] + rank;
      for (unsigned w = 0; w < wave; ++w) pos += wcnt[w][digit];
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) add += wcnt[w][t];
    base[t] += add;
    __syncthreads();
  }
}

template <class K>
static bool radix_sort(agc_context* c, K* keys, uint32_t* vals, K* keys_alt, uint32_t* vals_alt,
                       int64_t n, int nbits, const std::string& tag) {
  if (n <= 1 || nbits <= 0) return false;
  const int64_t tiles = (n + kSortTile - 1) / kSortTile;
  uint32_t* hist = c->ws.get<uint32_t>(tag + ".hist", (int64_t)kRadix * tiles + 1);
  K* src_k = keys;
  uint32_t* src_v = vals;
  K* dst_k = keys_alt;
  uint32_t* dst_v = vals_alt;
  bool in_alt = false;
  for (int shift = 0; shift < nbits; shift += kRadixBits) {
    k_radix_hist<K><<<(unsigned)tiles, kWG, 0, c->stream>>>(src_k, n, shift, hist, tiles);
    AGC_LAUNCH_CHECK();
    scan_u32(c, hist, hist, (int64_t)kRadix * tiles, tag + ".scan");
    k_radix_scatter<K><<<(unsigned)tiles, kWG, 0, c->stream>>>(src_k, src_v, dst_k, dst_v, n, shift,
                                                               hist, tiles);
    AGC_LAUNCH_CHECK();
    std::swap(src_k, dst_k);
    std::swap(src_v, dst_v);
    in_alt = !in_alt;
  }
  return in_alt;
}

bool radix_sort_u64(agc_context* c, uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                    uint32_t* vals_alt, int64_t n, int nbits, const std::string& tag) {
  return radix_sort<uint64_t>(c, keys, vals, keys_alt, vals_alt, n, nbits, tag);
}

bool radix_sort_u32(agc_context* c, uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                    uint32_t* vals_alt, int64_t n, int nbits, const std::string& tag) {
  return radix_sort<uint32_t>(c, keys, vals, keys_alt, vals_alt, n, nbits, tag);
}

// ------------------------------------------------------------ error word

void err_reset(agc_context* c) { AGC_HIP(hipMemsetAsync(c->d_err, 0, sizeof(unsigned), c->stream)); }

unsigned err_fetch(agc_context* c) {
  AGC_HIP(hipMemcpyAsync(c->h_err, c->d_err, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
  AGC_HIP(hipStreamSynchronize(c->stream));
  return *c->h_err;
}

void err_throw(unsigned bits) {
  if (!bits) return;
  std::string m = "bad input:";
  if (bits & kErrRange) m += " vertex id out of range;";
  if (bits & kErrTag) m += " tag not 0 or 1;";
  if (bits & kErrElem) m += " element with a repeated or out-of-range vertex;";
  if (bits & kErrMap) m += " map value out of range;";
  if (bits & kErrNoDiag) m += " row without a diagonal block;";
  int code = AGC_ERR_BAD_INPUT;
  if (bits & kErrNotSPD) {
    m += " diagonal 3x3 block not positive definite;";
    code = AGC_ERR_NOT_SPD;
  }
  if (bits & kErrNoDiag) code = AGC_ERR_NOT_SPD;
  throw Error(code, m);
}

}  // namespace agc
