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
// Up to this many tiles every workgroup sums the totals of the tiles before
// it itself (two launches); beyond, one workgroup scans the tile totals
// first (three launches).
constexpr int64_t kScanDirectTiles = 2048;

__device__ __forceinline__ void scan_load(const uint32_t* __restrict__ in, int64_t n, uint32_t v[kScanItems],
                                          uint32_t* s) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  *s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t k = base + i;
    v[i] = (k < n) ? in[k] : 0u;
    *s += v[i];
  }
}

// tile_sums[w] = sum of tile w
__global__ __launch_bounds__(kWG) void k_scan_sums(const uint32_t* __restrict__ in, int64_t n,
                                                   uint32_t* __restrict__ tile_sums) {
  __shared__ uint32_t lds[kWaves];
  uint32_t v[kScanItems], s;
  scan_load(in, n, v, &s);
  uint32_t total;
  (void)wg_exclusive_scan(s, lds, &total);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// One workgroup: tile_sums[0..tiles] becomes the exclusive scan of the
// tile totals (in place), tile_sums[tiles] the grand total.
__global__ __launch_bounds__(kWG) void k_scan_sums_scan(uint32_t* __restrict__ tile_sums, int64_t tiles) {
  __shared__ uint32_t lds[kWaves];
  uint32_t carry = 0;
  for (int64_t base = 0; base < tiles; base += kWG) {
    const int64_t k = base + threadIdx.x;
    const uint32_t v = (k < tiles) ? tile_sums[k] : 0u;
    uint32_t total;
    const uint32_t off = wg_exclusive_scan(v, lds, &total);
    if (k < tiles) tile_sums[k] = carry + off;
    carry += total;
  }
  if (threadIdx.x == 0) tile_sums[tiles] = carry;
}

// Exclusive scan of tile w from its offset.  offs == nullptr: the offset is
// the sum of tile_sums[0..w), formed here (and the grand total by the last
// tile); otherwise offs[w] is the offset and offs[tiles] the total.
__global__ __launch_bounds__(kWG) void k_scan_apply(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                    int64_t n, const uint32_t* __restrict__ tile_sums,
                                                    const uint32_t* __restrict__ offs) {
  __shared__ uint32_t lds[kWaves];
  __shared__ uint32_t lds2[kWaves];
  uint32_t v[kScanItems], s;
  scan_load(in, n, v, &s);
  const int64_t w = blockIdx.x, tiles = gridDim.x;
  uint32_t base_off;
  if (offs) {
    base_off = offs[w];
  } else {
    uint32_t part = 0;
    const int64_t upto = (w == tiles - 1) ? tiles : w;   // the last tile also forms the total
    for (int64_t k = threadIdx.x; k < upto; k += kWG) part += (k < w) ? tile_sums[k] : 0u;
    uint32_t last = 0;
    if (w == tiles - 1 && threadIdx.x == 0) last = tile_sums[w];
    uint32_t before;
    (void)wg_exclusive_scan(part, lds2, &before);
    base_off = before;
    if (w == tiles - 1 && threadIdx.x == 0) out[n] = before + last;
  }
  uint32_t total;
  uint32_t off = base_off + wg_exclusive_scan(s, lds, &total);
  const int64_t base = w * kScanTile + (int64_t)threadIdx.x * kScanItems;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t k = base + i;
    if (k < n) out[k] = off;
    off += v[i];
  }
  if (offs && w == tiles - 1 && threadIdx.x == 0) out[n] = offs[tiles];
}

int64_t scan_sums_words(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

void scan_u32(agc_context* c, const uint32_t* in, uint32_t* out, int64_t n, const std::string& tag) {
  if (n <= 0) {
    AGC_HIP(hipMemsetAsync(out, 0, sizeof(uint32_t), c->stream));
    return;
  }
  scan_u32_into(c, in, out, n, c->ws.get<uint32_t>(tag + ".sums", scan_sums_words(n)));
}

__global__ void k_zero_first(uint32_t* __restrict__ out) { *out = 0u; }

void scan_u32_into(agc_context* c, const uint32_t* in, uint32_t* out, int64_t n, uint32_t* sums) {
  if (n <= 0) {
    k_zero_first<<<1, 1, 0, c->stream>>>(out);
    AGC_LAUNCH_CHECK();
    return;
  }
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  k_scan_sums<<<(unsigned)tiles, kWG, 0, c->stream>>>(in, n, sums);
  AGC_LAUNCH_CHECK();
  if (tiles <= kScanDirectTiles) {
    k_scan_apply<<<(unsigned)tiles, kWG, 0, c->stream>>>(in, out, n, sums, nullptr);
  } else {
    k_scan_sums_scan<<<1, kWG, 0, c->stream>>>(sums, tiles);
    AGC_LAUNCH_CHECK();
    k_scan_apply<<<(unsigned)tiles, kWG, 0, c->stream>>>(in, out, n, sums, sums);
  }
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

// Stable scatter of one tile.  Its keys and values are all loaded first.
// The tile's count of each digit comes from the scanned histogram (the
// difference of two neighbouring offsets), and their exclusive scan gives
// the digit's first position in the tile.  The items are then ranked in
// rounds of kWG consecutive keys (rank among equal digits: earlier rounds'
// and earlier waves' counts plus the lower lanes with the same digit, from
// eight ballots) and placed in LDS in digit order; finally the tile is
// written out in that order, so that consecutive threads store consecutive
// positions of one digit.
template <class K>
__global__ __launch_bounds__(kWG) void k_radix_scatter(const K* __restrict__ keys_in,
                                                       const uint32_t* __restrict__ vals_in,
                                                       K* __restrict__ keys_out,
                                                       uint32_t* __restrict__ vals_out, int64_t n,
                                                       int shift, const uint32_t* __restrict__ offs,
                                                       int64_t n_tiles) {
  __shared__ K lk[kSortTile];
  __shared__ uint32_t lv[kSortTile];
  __shared__ uint32_t gbase[kRadix];   // global position of the digit's first item, less its tile position
  __shared__ uint32_t run[kRadix];     // next tile position of the digit
  __shared__ uint32_t wcnt[kWaves][kRadix];
  __shared__ uint32_t red[kWaves];
  const unsigned t = threadIdx.x;
  const unsigned wave = t / kWave;
  const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
  const int len = (n - tile0 < kSortTile) ? (int)(n - tile0) : kSortTile;
  K key[kSortItems];
  uint32_t val[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {   // past the end: the last item again, never placed
    const int64_t k = tile0 + r * kWG + t;
    const int64_t kc = k < n ? k : n - 1;
    key[r] = keys_in[kc];
    val[r] = vals_in[kc];
  }
  const int64_t h = (int64_t)t * n_tiles + blockIdx.x;   // thread t owns digit t
  const uint32_t g0 = offs[h];
  uint32_t tile_total;
  const uint32_t ls = wg_exclusive_scan(offs[h + 1] - g0, red, &tile_total);
  gbase[t] = g0 - ls;
  run[t] = ls;
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    if (r * kWG >= len) break;   // uniform across the workgroup
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wcnt[w][t] = 0;
    __syncthreads();
    const bool valid = r * kWG + (int)t < len;
    const unsigned digit = (unsigned)((key[r] >> shift) & (kRadix - 1));
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
      uint32_t pos = run[digit] + rank;
      for (unsigned w = 0; w < wave; ++w) pos += wcnt[w][digit];
      lk[pos] = key[r];
      lv[pos] = val[r];
    }
    __syncthreads();
    // column t of wcnt is read and cleared by thread t alone from here on
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) add += wcnt[w][t];
    run[t] += add;
  }
  __syncthreads();
  for (int p = (int)t; p < len; p += kWG) {
    const K kk = lk[p];
    const uint32_t gp = gbase[(unsigned)((kk >> shift) & (kRadix - 1))] + (uint32_t)p;
    keys_out[gp] = kk;
    vals_out[gp] = lv[p];
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
  if (bits & kErrUnused) m += " a coarse label in [0, n_coarse) has no member;";
  if (bits & kErrDiagLb) m += " diag_lb not positive and finite;";
  if (bits & kErrNoDiag) m += " row without a diagonal block;";
  if (bits & kErrDegenerate) m += " rest element with zero volume;";
  int code = AGC_ERR_BAD_INPUT;
  if (bits & kErrNotSPD) {
    m += " diagonal 3x3 block not positive definite;";
    code = AGC_ERR_NOT_SPD;
  }
  if (bits & kErrNoDiag) code = AGC_ERR_NOT_SPD;
  throw Error(code, m);
}

}  // namespace agc
