// Deterministic segmented sum over sorted keys (internal).
//
// Items are processed in tiles of kWG (one per thread).  Inside a tile a
// wave64 segmented scan (DPP lane moves) and a carry across the four waves (LDS)
// give every run its partial sum.  A run whose segment starts inside the tile
// writes its partial to the output; a run that continues a segment started in
// an earlier tile writes its partial to carry[tile].  A second kernel adds,
// for every segment that crosses tiles, the carries of its continuation tiles
// in a fixed tree order.  Nothing depends on scheduling, so results are
// bitwise reproducible.
#pragma once

#include "internal.h"

namespace agc {

template <class K>
__global__ __launch_bounds__(kWG) void k_seg_heads(const K* __restrict__ keys, int64_t n,
                                                   uint32_t* __restrict__ tile_heads) {
  __shared__ uint32_t lds[kWaves];
  const int64_t k = (int64_t)blockIdx.x * kWG + threadIdx.x;
  uint32_t h = 0;
  if (k < n) h = (k == 0 || keys[k - 1] != keys[k]) ? 1u : 0u;
  uint32_t total;
  (void)wg_exclusive_scan(h, lds, &total);
  if (threadIdx.x == 0) tile_heads[blockIdx.x] = total;
}

// Op: Acc type, W values per item;
//   load(item, Acc v[W]); store(seg, const Acc v[W]); add(seg, const Acc v[W])
template <int W, class Acc, class K, class Op>
__global__ __launch_bounds__(kWG) void k_seg_reduce(const K* __restrict__ keys, int64_t n,
                                                    const uint32_t* __restrict__ seg_base, Op op,
                                                    Acc* __restrict__ carry, K* __restrict__ ukeys) {
  __shared__ uint32_t lds_u[kWaves];
  __shared__ int64_t tail_seg[kWaves];
  __shared__ int tail_single[kWaves];
  __shared__ Acc tail_v[kWaves][W];
  const unsigned t = threadIdx.x, lane = lane_id(), wave = t / kWave;
  const int64_t k = (int64_t)blockIdx.x * kWG + t;
  const bool valid = k < n;
  K key = valid ? keys[k] : (K)0;
  const bool head = valid && (k == 0 || keys[k - 1] != key);
  uint32_t tot;
  const uint32_t excl = wg_exclusive_scan(head ? 1u : 0u, lds_u, &tot);
  const int64_t base = (int64_t)seg_base[blockIdx.x];
  int64_t seg = valid ? base + (int64_t)(excl + (head ? 1u : 0u)) - 1 : INT64_MAX;
  Acc v[W];
  if (valid) {
    op.load(k, v);
  } else {
#pragma unroll
    for (int i = 0; i < W; ++i) v[i] = (Acc)0;
  }
  // wave-level segmented inclusive scan (DPP lane moves; every lane is active
  // here).  Within a tile a segment's index minus the tile's base fits in 32 bits.
  wave_seg_scan<W>(valid ? (int32_t)(seg - base) : INT32_MAX, v);
  const int64_t seg0 = __shfl(seg, 0);
  if (lane == kWave - 1) {
    tail_seg[wave] = seg;
    tail_single[wave] = (seg0 == seg) ? 1 : 0;
#pragma unroll
    for (int i = 0; i < W; ++i) tail_v[wave][i] = v[i];
  }
  __syncthreads();
  if (wave > 0 && valid && tail_seg[wave - 1] == seg) {
    Acc cin[W];
#pragma unroll
    for (int i = 0; i < W; ++i) cin[i] = (Acc)0;
    for (int u = (int)wave - 1; u >= 0; --u) {
      if (tail_seg[u] != seg) break;
#pragma unroll
      for (int i = 0; i < W; ++i) cin[i] += tail_v[u][i];
      if (!tail_single[u]) break;
    }
#pragma unroll
    for (int i = 0; i < W; ++i) v[i] += cin[i];
  }
  if (!valid) return;
  if (head && ukeys) ukeys[seg] = key;
  const bool last = (k == n - 1) || (t == kWG - 1) || (keys[k + 1] != key);
  if (!last) return;
  if (seg >= base) {
    op.store(seg, v);
  } else {
#pragma unroll
    for (int i = 0; i < W; ++i) carry[(int64_t)blockIdx.x * W + i] = v[i];
  }
}

template <int W, class Acc, class K, class Op>
__global__ __launch_bounds__(kWG) void k_seg_fix(const K* __restrict__ keys, int64_t n, int64_t n_tiles,
                                                 const uint32_t* __restrict__ seg_base, Op op,
                                                 const Acc* __restrict__ carry) {
  __shared__ int64_t first_head;
  __shared__ Acc red[kWaves][W];
  const int64_t t = blockIdx.x;
  if (t + 1 >= n_tiles) return;
  const bool owner = seg_base[t + 1] > seg_base[t];
  const int64_t nxt = (t + 1) * kWG;          // first item of tile t+1 (< n)
  const bool continues = keys[nxt] == keys[nxt - 1];
  if (!owner || !continues) return;
  const int64_t s = (int64_t)seg_base[t + 1] - 1;
  // first tile after t that holds a head
  if (threadIdx.x == 0) first_head = n_tiles;
  __syncthreads();
  for (int64_t u0 = t + 1; u0 < n_tiles; u0 += kWG) {
    const int64_t u = u0 + threadIdx.x;
    if (u < n_tiles && seg_base[u + 1] > seg_base[u]) atomicMin((unsigned long long*)&first_head,
                                                                 (unsigned long long)u);
    __syncthreads();
    const bool found = first_head < n_tiles;
    __syncthreads();
    if (found) break;
  }
  int64_t t_end = n_tiles - 1;
  if (first_head < n_tiles) {
    const int64_t u = first_head;
    t_end = (keys[u * kWG] == keys[u * kWG - 1]) ? u : u - 1;
  }
  Acc acc[W];
#pragma unroll
  for (int i = 0; i < W; ++i) acc[i] = (Acc)0;
  for (int64_t u = t + 1 + threadIdx.x; u <= t_end; u += kWG) {
#pragma unroll
    for (int i = 0; i < W; ++i) acc[i] += carry[u * W + i];
  }
  const unsigned lane = lane_id(), wave = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < W; ++i) {
    Acc x = acc[i];
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_down(x, d);
    if (lane == 0) red[wave][i] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Acc tot[W];
#pragma unroll
    for (int i = 0; i < W; ++i) {
      Acc x = (Acc)0;
      for (int w = 0; w < kWaves; ++w) x += red[w][i];
      tot[i] = x;
    }
    op.add(s, tot);
  }
}

// Runs the three kernels.  Returns the number of segments (synchronises when
// want_count is true; otherwise returns -1).
template <int W, class Acc, class K, class Op>
int64_t seg_reduce(agc_context* c, const K* keys, int64_t n, const Op& op, K* ukeys, bool want_count,
                   const std::string& tag) {
  if (n <= 0) return 0;
  const int64_t tiles = (n + kWG - 1) / kWG;
  uint32_t* sb = c->ws.get<uint32_t>(tag + ".segbase", tiles + 1);
  Acc* carry = c->ws.get<Acc>(tag + ".carry", tiles * W);
  k_seg_heads<K><<<(unsigned)tiles, kWG, 0, c->stream>>>(keys, n, sb);
  AGC_LAUNCH_CHECK();
  scan_u32(c, sb, sb, tiles, tag + ".scan");
  k_seg_reduce<W, Acc, K, Op><<<(unsigned)tiles, kWG, 0, c->stream>>>(keys, n, sb, op, carry, ukeys);
  AGC_LAUNCH_CHECK();
  if (tiles > 1) {
    k_seg_fix<W, Acc, K, Op><<<(unsigned)tiles, kWG, 0, c->stream>>>(keys, n, tiles, sb, op, carry);
    AGC_LAUNCH_CHECK();
  }
  if (!want_count) return -1;
  uint32_t cnt = 0;
  AGC_HIP(hipMemcpyAsync(&cnt, sb + tiles, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  AGC_HIP(hipStreamSynchronize(c->stream));
  return (int64_t)cnt;
}

}  // namespace agc
