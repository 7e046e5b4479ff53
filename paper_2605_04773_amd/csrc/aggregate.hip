// Fine-to-coarse aggregation, restriction and prolongation.
//
// Sec. 4.1 and supplement Sec. 1: super-nodes are the connected components of
// the graph of collapsible edges, and the supplement's elected-lane popcount
// plus group prefix sum (Alg. 2, Sec. 1.3) orders them by their smallest fine
// id.  The paper finds components with 32-bit in-warp hash masks applied
// level by level.  On gfx950 a parent forest does the same job for any
// component size, in two passes: each block of consecutive vertex ids is
// resolved by union-find in one workgroup's LDS (the paper's in-group
// merge, with groups of 4096 instead of 32 vertices), then the edges between
// blocks are joined by lock-free union-find on the global forest.  A pointer
// only ever moves to a smaller vertex of the same component, so the
// surviving root of every component is its smallest vertex whatever the
// order of the races.  Flagging the roots and an exclusive scan then give
// exactly the canonical labels.
#include "segreduce.h"

namespace agc {

// Plain (cached) loads: a stale value read from this XCD's cache is still an
// ancestor of the node (parents only ever move towards smaller ids), so a
// walk that starts from it still ends at a root, and the compare-and-swap
// that hooks a root works on the device-coherent value and reports the
// current one when it fails.
__device__ __forceinline__ int32_t ld_parent(const int32_t* p, int32_t v) { return p[v]; }

__device__ __forceinline__ void st_parent(int32_t* p, int32_t v, int32_t x) {
  __hip_atomic_store(p + v, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of v with path shortening.  Invariant: parent[x] <= x, roots satisfy
// parent[x] == x, and a value written is always an ancestor of the node.
__device__ int32_t find_root(int32_t* parent, int32_t v) {
  int32_t cur = ld_parent(parent, v);
  if (cur != v) {
    int32_t prev = v, nxt;
    while (cur > (nxt = ld_parent(parent, cur))) {
      st_parent(parent, prev, nxt);
      prev = cur;
      cur = nxt;
    }
  }
  return cur;
}

// find_root whose answer is a root at the time of the call: the walk uses
// plain loads, but a node that looks like a root in this XCD's cache is
// confirmed with a device-coherent load (a hook made on another XCD leaves
// the cached line stale until it is evicted; hooking a stale root would only
// fail its compare-and-swap, at the cost of a device-scope round trip).
__device__ int32_t find_root_coherent(int32_t* parent, int32_t v) {
  int32_t x = v;
  for (;;) {
    int32_t r = find_root(parent, x);
    const int32_t q = __hip_atomic_load(parent + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (q == r) return r;
    x = q;
  }
}

__global__ void k_cc_init(int32_t* __restrict__ parent, int32_t n) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    parent[v] = (int32_t)v;
}

// ---------------------------------------------------------------- blocks
//
// The vertices are cut into blocks of kCcBlock consecutive ids.  Pass one
// gives each block to one workgroup, which joins the collapsible edges with
// both ends in its block by union-find in LDS and writes every vertex's
// local root (the smallest id of its local component) as its parent: no
// global atomics, and the global forest starts with depth one.  Pass two
// reads every edge and hooks, with global compare-and-swap, only those the
// first pass did not join.  With a mesh's edge list ordered by smaller end
// (as a sorted, deduplicated list is) the first pass takes each block's
// edges as one contiguous range and the second pass joins few trees: the
// local components of a block are mostly whole cross-sections of the
// collapsible regions.  Any order is still correct: the ranges cover every
// edge, and an edge the first pass cannot join locally is joined by the
// second.

#ifndef AGC_CC_LOG
#define AGC_CC_LOG 12
#endif
constexpr int kCcLog = AGC_CC_LOG;
constexpr int kCcBlock = 1 << kCcLog;   // vertices per block (4096: 16 KB of LDS)
#ifndef AGC_CC_THREADS
#define AGC_CC_THREADS 1024
#endif
constexpr int kCcThreads = AGC_CC_THREADS;   // threads of a block's workgroup
constexpr int kCcBatch = 8;             // edges a thread loads at once

__device__ __forceinline__ int32_t edge_key(const int32_t* edges, int64_t e) {
  const int2 uv = reinterpret_cast<const int2*>(edges)[e];
  return uv.x < uv.y ? uv.x : uv.y;
}

// First edge index whose smaller end is >= target, for edges ordered by
// smaller end; one wave probes 64 positions per step (four steps for 16 M
// edges).  For an unordered list it returns some index in [0, m].
__device__ int64_t wave_lower_bound(const int32_t* edges, int64_t m, int32_t target) {
  const unsigned lane = lane_id();
  int64_t lo = 0, hi = m;                 // the answer lies in [lo, hi]
  while (hi - lo > kWave) {
    const int64_t span = hi - lo;
    const int64_t p = lo + span * (lane + 1) / (kWave + 1);
    const bool less = edge_key(edges, p) < target;
    const int c = __popcll(__ballot(less));
    const int64_t nlo = (c > 0) ? lo + span * c / (kWave + 1) + 1 : lo;
    const int64_t nhi = (c < kWave) ? lo + span * (c + 1) / (kWave + 1) : hi;
    lo = nlo;
    hi = nhi;
  }
  const int64_t p = lo + lane;
  const bool less = p < hi && edge_key(edges, p) < target;
  return lo + __popcll(__ballot(less));
}

__device__ __forceinline__ int32_t lds_ld(int32_t* a) {
  return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(int32_t* a, int32_t x) {
  __hip_atomic_store(a, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Root of x in the block's LDS forest with path halving (x points at its
// grandparent as the walk passes).  Invariant: lp[x] <= x, roots lp[x] == x,
// and a stored value is always an ancestor of its node.
__device__ int32_t lds_find(int32_t* lp, int32_t x) {
  for (;;) {
    const int32_t p = lds_ld(lp + x);
    if (p == x) return x;
    const int32_t gp = lds_ld(lp + p);
    if (gp == p) return p;
    lds_st(lp + x, gp);
    x = gp;
  }
}

// Union of a and b: the larger root is hooked below the smaller, so every
// local root is the smallest slot of its tree.
__device__ void lds_union(int32_t* lp, int32_t a, int32_t b) {
  for (;;) {
    a = lds_find(lp, a);
    b = lds_find(lp, b);
    if (a == b) return;
    const int32_t lo = a < b ? a : b, hi = a < b ? b : a;
    int32_t expect = hi;
    if (__hip_atomic_compare_exchange_strong(lp + hi, &expect, lo, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WORKGROUP))
      return;
    a = lo;           // hi was hooked meanwhile: continue from its new parent
    b = expect;
  }
}

// Pass one.  Workgroup b: vertices [b W, b W + W), edges
// [min(a_b, a_b+1), max(a_b, a_b+1)) with a_b the first edge whose smaller
// end is >= b W.  Writes parent[] of its vertices and bounds[b] (and
// bounds[nb] = m from the last block).  Malformed edges are skipped here and
// reported by pass two.
__global__ __launch_bounds__(kCcThreads) void k_cc_local(const int32_t* __restrict__ edges,
                                                         const uint8_t* __restrict__ tags, int64_t m, int32_t n,
                                                         int32_t* __restrict__ parent, int64_t* __restrict__ bounds,
                                                         unsigned* __restrict__ err) {
  __shared__ int32_t lp[kCcBlock];
  __shared__ int64_t rng[2];
  const int32_t nb = (int32_t)(((int64_t)n + kCcBlock - 1) >> kCcLog);
  const int32_t b = blockIdx.x;
  const int32_t v0 = b << kCcLog;
  const unsigned wave = threadIdx.x / kWave;
  if (wave < 2) {
    const int32_t blk = b + (int32_t)wave;
    int64_t a;
    if (blk == 0) a = 0;
    else if (blk >= nb) a = m;
    else a = wave_lower_bound(edges, m, blk << kCcLog);
    if (lane_id() == 0) rng[wave] = a;
  }
  for (int i = threadIdx.x; i < kCcBlock; i += kCcThreads) lp[i] = i;
  __syncthreads();
  const int64_t a0 = rng[0], a1 = rng[1];
  if (threadIdx.x == 0) {
    bounds[b] = a0;
    if (b == nb - 1) bounds[nb] = m;
    if (b == 0) *err = 0u;   // the call's error word, set by pass two only
  }
  const int64_t e0 = a0 < a1 ? a0 : a1, e1 = a0 < a1 ? a1 : a0;
  // kCcBatch edges per thread are loaded together (indices past the range
  // repeat its last edge and are masked), then joined
  for (int64_t eb = e0 + threadIdx.x; eb < e1; eb += (int64_t)kCcThreads * kCcBatch) {
    int2 uv[kCcBatch];
    uint8_t tg[kCcBatch];
#pragma unroll
    for (int j = 0; j < kCcBatch; ++j) {
      const int64_t e = eb + (int64_t)j * kCcThreads;
      const int64_t ec = e < e1 ? e : e1 - 1;
      uv[j] = reinterpret_cast<const int2*>(edges)[ec];
      tg[j] = tags[ec];
    }
#pragma unroll
    for (int j = 0; j < kCcBatch; ++j) {
      const uint32_t lu = (uint32_t)(uv[j].x - v0), lv = (uint32_t)(uv[j].y - v0);
      if (eb + (int64_t)j * kCcThreads < e1 && tg[j] == 1 && lu != lv && lu < (uint32_t)kCcBlock &&
          lv < (uint32_t)kCcBlock && uv[j].x < n && uv[j].y < n)
        lds_union(lp, (int32_t)lu, (int32_t)lv);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kCcBlock; i += kCcThreads) {
    const int32_t v = v0 + i;
    if (v >= n) break;
    int32_t x = i, p;
    while ((p = lp[x]) != x) x = p;       // no unions run any more: a plain walk
    parent[v] = v0 + x;
  }
}

// Pass two: validates every edge and hooks the collapsible ones that pass
// one did not join (lock-free union-find on the global forest; larger root
// below smaller, so every root stays the smallest id of its tree).  The ends
// of such an edge lie in two blocks, so their parents (the local roots of
// pass one) differ, and along a block boundary long runs of edges join the
// same two local trees.  Each workgroup takes a contiguous range of edges;
// the lanes of a wave with the same pair of parents leave the union to one
// of them, and a workgroup remembers in LDS the pairs it has joined (a pair
// joined once stays joined; a stale or overwritten entry only repeats a
// union, which changes nothing).  Loop bounds are uniform per workgroup, so
// all lanes of a wave take part in the ballots.
constexpr int kCrossCache = 512;   // remembered pairs per workgroup (direct-mapped)

constexpr int kCrossBatch = 4;     // edges per lane loaded together

__global__ __launch_bounds__(kWG) void k_cc_cross(const int32_t* __restrict__ edges, const uint8_t* __restrict__ tags,
                                                  int64_t m, int32_t* parent, int32_t n,
                                                  const int64_t* __restrict__ bounds, unsigned* err) {
  __shared__ uint64_t seen[kCrossCache];
  for (int i = threadIdx.x; i < kCrossCache; i += kWG) seen[i] = ~0ull;
  __syncthreads();
  const int64_t per = (m + gridDim.x - 1) / gridDim.x;
  const int64_t e_lo = (int64_t)blockIdx.x * per, e_hi = e_lo + per < m ? e_lo + per : m;
  const unsigned lane = lane_id();
  for (int64_t base = e_lo; base < e_hi; base += (int64_t)kWG * kCrossBatch) {
    // kCrossBatch edges per lane: their ids and tags, then the parents of
    // their ends, each group of loads issued together (indices past the
    // range repeat its last edge and are masked)
    int2 uv[kCrossBatch];
    uint8_t tg[kCrossBatch];
#pragma unroll
    for (int j = 0; j < kCrossBatch; ++j) {
      const int64_t e = base + (int64_t)j * kWG + threadIdx.x;
      const int64_t ec = e < e_hi ? e : e_hi - 1;
      uv[j] = reinterpret_cast<const int2*>(edges)[ec];
      tg[j] = tags[ec];
    }
    bool want[kCrossBatch];
    int32_t pu[kCrossBatch], pv[kCrossBatch];
#pragma unroll
    for (int j = 0; j < kCrossBatch; ++j) {
      const int64_t e = base + (int64_t)j * kWG + threadIdx.x;
      const int32_t u = uv[j].x, v = uv[j].y;
      want[j] = false;
      if (e < e_hi) {
        if (u < 0 || u >= n || v < 0 || v >= n) {
          atomicOr(err, kErrRange);
        } else if (tg[j] > 1) {
          atomicOr(err, kErrTag);
        } else if (tg[j] == 1 && u != v) {
          want[j] = true;
          const int32_t bu = u >> kCcLog;
          if (bu == (v >> kCcLog)) {            // joined by pass one if e lies in its block's range
            const int64_t s0 = bounds[bu], s1 = bounds[bu + 1];
            want[j] = !(e >= (s0 < s1 ? s0 : s1) && e < (s0 < s1 ? s1 : s0));
          }
        }
      }
      // the ends' parents: their local roots from pass one, or ancestors of them
      pu[j] = want[j] ? ld_parent(parent, u) : 0;
      pv[j] = want[j] ? ld_parent(parent, v) : 0;
    }
#pragma unroll
    for (int j = 0; j < kCrossBatch; ++j) {
      const int32_t lo = pu[j] < pv[j] ? pu[j] : pv[j], hi = pu[j] < pv[j] ? pv[j] : pu[j];
      const bool w = want[j] && pu[j] != pv[j];
      uint64_t pend = __ballot(w);
      while (pend) {
        const int leader = __ffsll((unsigned long long)pend) - 1;
        const int32_t h = __shfl(hi, leader), l = __shfl(lo, leader);
        pend &= ~__ballot(w && hi == h && lo == l);
        if ((int)lane == leader) {
          const uint64_t key = ((uint64_t)(uint32_t)h << 32) | (uint32_t)l;
          const uint32_t slot = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 55) & (kCrossCache - 1);
          if (seen[slot] != key) {
            int32_t ru = find_root_coherent(parent, l), rv = find_root_coherent(parent, h);
            while (ru != rv) {
              const int32_t a = ru < rv ? ru : rv, b = ru < rv ? rv : ru;
              const int32_t old = atomicCAS(parent + b, b, a);
              if (old == b) break;                    // hooked b below a
              // b stopped being a root meanwhile: continue from its new root
              const int32_t r = find_root_coherent(parent, old);
              if (ru == b) ru = r; else rv = r;
            }
            seen[slot] = key;
          }
        }
      }
    }
  }
}

// Root words and their ranks within tiles of kWave words (4096 vertices),
// one tile per workgroup: word w holds, in bit i, whether vertex 64 w + i is
// a root (parent[v] == v: the smallest id of a component); lrank[w] = the
// roots of the tile's words before w; tsum[t] = the roots of tile t.
constexpr int kRootTileWords = kWave;
constexpr int kRootWordsPerWave = kRootTileWords / kWaves;
__global__ __launch_bounds__(kWG) void k_cc_rootrank(const int32_t* __restrict__ parent, int32_t n,
                                                     uint64_t* __restrict__ bits, uint32_t* __restrict__ lrank,
                                                     uint32_t* __restrict__ tsum) {
  __shared__ uint32_t cnt[kRootTileWords];
  const unsigned wave = threadIdx.x / kWave, lane = lane_id();
  const int64_t nw = ((int64_t)n + kWave - 1) / kWave;
  const int64_t w0 = (int64_t)blockIdx.x * kRootTileWords + wave * kRootWordsPerWave;
  int32_t pv[kRootWordsPerWave];
#pragma unroll
  for (int i = 0; i < kRootWordsPerWave; ++i) {   // all loads in flight before the ballots
    const int64_t v = (w0 + i) * kWave + lane;
    pv[i] = v < n ? parent[v] : -1;
  }
#pragma unroll
  for (int i = 0; i < kRootWordsPerWave; ++i) {
    const int64_t v = (w0 + i) * kWave + lane;
    const uint64_t word = __ballot(v < n && pv[i] == (int32_t)v);
    if (lane == 0) {
      cnt[wave * kRootWordsPerWave + i] = (uint32_t)__popcll(word);
      if (w0 + i < nw) bits[w0 + i] = word;
    }
  }
  __syncthreads();
  if (wave == 0) {
    const uint32_t c = cnt[lane];
    uint32_t x = c;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const uint32_t y = __shfl_up(x, d);
      if (lane >= (unsigned)d) x += y;
    }
    const int64_t w = (int64_t)blockIdx.x * kRootTileWords + lane;
    if (w < nw) lrank[w] = x - c;
    if (lane == kWave - 1) tsum[blockIdx.x] = x;
  }
}

// Tiles whose prefix every label workgroup sums itself, in LDS: up to
// 4096 x 4096 vertices.  Beyond, the prefix is scanned once beforehand
// (tp: exclusive, the total at tp[tiles]).
constexpr int64_t kLabelLdsTiles = 4096;

// map[v] = number of roots below v's root r: those of the tiles before r's
// (the exclusive prefix of tsum), of the words before r's in its tile
// (lrank) and of the bits under r in its word.  *count = all roots.
template <bool kLdsPrefix>
__global__ __launch_bounds__(kWG) void k_cc_label(const int32_t* __restrict__ parent,
                                                  const uint64_t* __restrict__ bits,
                                                  const uint32_t* __restrict__ lrank,
                                                  const uint32_t* __restrict__ tsum, const uint32_t* __restrict__ tp,
                                                  int64_t tiles, int32_t n, int32_t* __restrict__ map,
                                                  uint32_t* __restrict__ count) {
  __shared__ uint32_t pre[kLdsPrefix ? kLabelLdsTiles : 1];
  __shared__ uint32_t red[kWaves];
  if constexpr (kLdsPrefix) {
    // thread t sums tiles [t per, (t + 1) per), then the workgroup scans those sums
    const int64_t per = (tiles + kWG - 1) / kWG;
    const int64_t lo = (int64_t)threadIdx.x * per;
    uint32_t sum = 0;
    for (int64_t k = lo; k < lo + per && k < tiles; ++k) sum += tsum[k];
    uint32_t total;
    uint32_t off = wg_exclusive_scan(sum, red, &total);
    for (int64_t k = lo; k < lo + per && k < tiles; ++k) {
      pre[k] = off;
      off += tsum[k];
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = total;
  } else {
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = tp[tiles];
  }
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t x = (int32_t)v, p;
    while ((p = parent[x]) != x) x = p;       // read-only walk to the root
    const int32_t w = x >> 6;
    const int32_t t = w / kRootTileWords;
    const uint64_t below = (x & 63) ? (bits[w] << (64 - (x & 63))) : 0ull;   // bits of the word under x
    const uint32_t tile_pre = kLdsPrefix ? pre[t] : tp[t];
    map[v] = (int32_t)(tile_pre + lrank[w] + (uint32_t)__popcll(below));
  }
}

static unsigned gs_blocks(int64_t n) {
  int64_t b = (n + kWG - 1) / kWG;
  if (b > 65536) b = 65536;
  return (unsigned)(b < 1 ? 1 : b);
}

__global__ void k_clear_u32(unsigned* __restrict__ w) { *w = 0u; }

int32_t aggregate_into(agc_context* c, int32_t n, int64_t m, const int32_t* edges, const uint8_t* tags, int32_t* map,
                       const AggScratch& s) {
  if (n == 0) return 0;
  int32_t* parent = s.parent;
  const unsigned nb = (unsigned)(((int64_t)n + kCcBlock - 1) >> kCcLog);
  k_cc_local<<<nb, kCcThreads, 0, c->stream>>>(edges, tags, m, n, parent, s.bounds, c->d_err);
  AGC_LAUNCH_CHECK();
  if (m > 0) {
    // contiguous ranges of at least 2048 edges, up to eight workgroups per CU
    int64_t g = (m + 2047) / 2048;
    if (g > 2048) g = 2048;
    k_cc_cross<<<(unsigned)g, kWG, 0, c->stream>>>(edges, tags, m, parent, n, s.bounds, c->d_err);
    AGC_LAUNCH_CHECK();
  }
  const int64_t tiles = agg_root_tiles(n);
  k_cc_rootrank<<<(unsigned)tiles, kWG, 0, c->stream>>>(parent, n, s.bits, s.lrank, s.tsum);
  AGC_LAUNCH_CHECK();
  // up to eight workgroups per CU walk the vertices (each sums the tile prefix once)
  int64_t lb = ((int64_t)n + kWG - 1) / kWG;
  if (lb > 2048) lb = 2048;
  uint32_t* count = c->d_err + 1;   // beside the error word: one copy brings both back
  if (tiles <= kLabelLdsTiles) {
    k_cc_label<true><<<(unsigned)lb, kWG, 0, c->stream>>>(parent, s.bits, s.lrank, s.tsum, nullptr, tiles, n, map,
                                                          count);
  } else {
    scan_u32_into(c, s.tsum, s.tp, tiles, s.scan_sums);
    k_cc_label<false><<<(unsigned)lb, kWG, 0, c->stream>>>(parent, s.bits, s.lrank, s.tsum, s.tp, tiles, n, map,
                                                           count);
  }
  AGC_LAUNCH_CHECK();
  AGC_HIP(hipMemcpyAsync(c->h_err, c->d_err, 2 * sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
  AGC_HIP(hipStreamSynchronize(c->stream));
  err_throw(c->h_err[0]);
  return (int32_t)c->h_err[1];
}

// parent [n], root bits [nw] (64-bit), in-tile word ranks [nw], tile sums
// and their scanned prefix [tiles + 1] each, scan sums, bounds [nb + 1]
// (64-bit), each from a 256-byte boundary; nw = words of 64 vertices, tiles
// = root tiles of 64 words, nb = vertex blocks
static int64_t round64(int64_t w) { return (w + 63) & ~(int64_t)63; }

int64_t agg_root_tiles(int32_t n) {
  const int64_t nw = ((int64_t)n + kWave - 1) / kWave;
  return (nw + kRootTileWords - 1) / kRootTileWords;
}

int64_t agg_scratch_words(int32_t n) {
  const int64_t nw = ((int64_t)n + kWave - 1) / kWave;
  const int64_t tiles = agg_root_tiles(n);
  const int64_t nb = ((int64_t)n + kCcBlock - 1) >> kCcLog;
  return round64(n) + round64(2 * nw) + round64(nw) + 2 * round64(tiles + 1) + round64(scan_sums_words(tiles)) +
         round64(2 * (nb + 1));
}

AggScratch agg_scratch_carve(uint32_t* base, int32_t n) {
  const int64_t nw = ((int64_t)n + kWave - 1) / kWave;
  const int64_t tiles = agg_root_tiles(n);
  AggScratch s;
  int64_t off = 0;
  s.parent = reinterpret_cast<int32_t*>(base);
  off = round64((int64_t)n);
  s.bits = reinterpret_cast<uint64_t*>(base + off);
  off += round64(2 * nw);
  s.lrank = base + off;
  off += round64(nw);
  s.tsum = base + off;
  off += round64(tiles + 1);
  s.tp = base + off;
  off += round64(tiles + 1);
  s.scan_sums = base + off;
  off += round64(scan_sums_words(tiles));
  s.bounds = reinterpret_cast<int64_t*>(base + off);
  return s;
}

int32_t aggregate(agc_context* c, int32_t n, int64_t m, const int32_t* edges, const uint8_t* tags, int32_t* map) {
  if (n == 0) return 0;
  uint32_t* base = c->ws.get<uint32_t>("agg.scratch", agg_scratch_words(n));
  return aggregate_into(c, n, m, edges, tags, map, agg_scratch_carve(base, n));
}

// ------------------------------------------------------------- members

__global__ void k_members_init(const int32_t* __restrict__ map, int32_t n, int32_t n_c, uint32_t* __restrict__ k,
                               uint32_t* __restrict__ v, unsigned* err) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = map[i];
    if (c < 0 || c >= n_c) atomicOr(err, kErrMap);
    k[i] = (uint32_t)(c < 0 ? 0 : (c >= n_c ? n_c - 1 : c));
    v[i] = (uint32_t)i;
  }
}

// Over the sorted labels: every label in [0, n_c) must occur (the first is 0,
// the last n_c - 1, and neighbours differ by at most one), or the segment
// index of a label would not be the label itself.
__global__ void k_members_check(const uint32_t* __restrict__ k, int32_t n, int32_t n_c, unsigned* err) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t c = k[i];
    bool bad = (i == 0) ? c != 0u : c - k[i - 1] > 1u;
    if (i == n - 1) bad = bad || c != (uint32_t)(n_c - 1);
    if (bad) atomicOr(err, kErrUnused);
  }
}

void group_members(agc_context* c, int32_t n, const int32_t* map, int32_t n_c, uint32_t* members,
                   uint32_t* mkeys) {
  uint32_t* k2 = c->ws.get<uint32_t>("mem.k2", n);
  uint32_t* v2 = c->ws.get<uint32_t>("mem.v2", n);
  err_reset(c);
  k_members_init<<<gs_blocks(n), kWG, 0, c->stream>>>(map, n, n_c, mkeys, members, c->d_err);
  AGC_LAUNCH_CHECK();
  const bool alt = radix_sort_u32(c, mkeys, members, k2, v2, n, bits_for((uint64_t)(n_c > 0 ? n_c - 1 : 0)),
                                  "mem.sort");
  if (alt) {
    AGC_HIP(hipMemcpyAsync(mkeys, k2, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, c->stream));
    AGC_HIP(hipMemcpyAsync(members, v2, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, c->stream));
  }
  k_members_check<<<gs_blocks(n), kWG, 0, c->stream>>>(mkeys, n, n_c, c->d_err);
  AGC_LAUNCH_CHECK();
}

struct RestrictOp {
  const uint32_t* members;
  const double* v;
  double* out;
  __device__ void load(int64_t k, double x[3]) const {
    const int64_t i = members[k];
#pragma unroll
    for (int r = 0; r < 3; ++r) x[r] = v[3 * i + r];
  }
  __device__ void store(int64_t s, const double x[3]) const {
#pragma unroll
    for (int r = 0; r < 3; ++r) out[3 * s + r] = x[r];
  }
  __device__ void add(int64_t s, const double x[3]) const {
#pragma unroll
    for (int r = 0; r < 3; ++r) out[3 * s + r] += x[r];
  }
};

// members/mkeys from group_members, which flags a label without members
// (the caller fetches the error word); with every label used, segment s is
// coarse node s.
void restrict_sorted(agc_context* c, int32_t n, int32_t n_c, const uint32_t* members, const uint32_t* mkeys,
                     const double* v, double* v_c) {
  (void)n_c;
  RestrictOp op{members, v, v_c};
  seg_reduce<3, double, uint32_t, RestrictOp>(c, mkeys, n, op, (uint32_t*)nullptr, false, "rst.seg");
}

// ------------------------------------------------------- error bound

struct MassOp {   // D_c = sum of d over the members of c, in member order
  const uint32_t* members;
  const double* d;
  double* out;
  __device__ void load(int64_t k, double x[1]) const { x[0] = d[members[k]]; }
  __device__ void store(int64_t s, const double x[1]) const { out[s] = x[0]; }
  __device__ void add(int64_t s, const double x[1]) const { out[s] += x[0]; }
};

// Per workgroup: sum over coarse nodes of |r_c|^2 / D_c, min over vertices
// of d_v, sum over vertices of |x_c[map v]|^2 (map null: identity).
constexpr unsigned kCertGrid = 512;
__global__ __launch_bounds__(kWG) void k_cert_part(const double* __restrict__ dc, const double* __restrict__ r_c,
                                                   int32_t n_c, const double* __restrict__ d,
                                                   const int32_t* __restrict__ map, const double* __restrict__ x_c,
                                                   int32_t n, double* __restrict__ part, unsigned* err) {
  __shared__ double lds[2 * kWaves];
  __shared__ double lmin[kWaves];
  double t[2] = {0.0, 0.0};
  double mn = INFINITY;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n_c; i += (int64_t)gridDim.x * kWG) {
    const double D = dc[i];
    bad |= !(D > 0.0 && D < INFINITY);
    const double a = r_c[3 * i], b = r_c[3 * i + 1], e = r_c[3 * i + 2];
    t[0] += (a * a + b * b + e * e) / D;
  }
  for (int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x; v < n; v += (int64_t)gridDim.x * kWG) {
    const double dv = d[v];
    bad |= !(dv > 0.0 && dv < INFINITY);
    mn = dv < mn ? dv : mn;
    const int64_t c = map ? map[v] : v;
    const double a = x_c[3 * c], b = x_c[3 * c + 1], e = x_c[3 * c + 2];
    t[1] += a * a + b * b + e * e;
  }
  if (bad) atomicOr(err, kErrDiagLb);
  wg_sum_all<2>(t, lds);
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const double q = __shfl_xor(mn, o);
    mn = q < mn ? q : mn;
  }
  if (lane_id() == 0) lmin[threadIdx.x / kWave] = mn;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = lmin[0];
    for (int w = 1; w < kWaves; ++w) m = lmin[w] < m ? lmin[w] : m;
    part[blockIdx.x] = t[0];
    part[kCertGrid + blockIdx.x] = m;
    part[2 * kCertGrid + blockIdx.x] = t[1];
  }
}

__global__ __launch_bounds__(kWG) void k_cert_final(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double lds[2 * kWaves];
  __shared__ double lmin[kWaves];
  double t[2] = {0.0, 0.0};
  double mn = INFINITY;
  for (unsigned i = threadIdx.x; i < kCertGrid; i += kWG) {
    t[0] += part[i];
    t[1] += part[2 * kCertGrid + i];
    mn = part[kCertGrid + i] < mn ? part[kCertGrid + i] : mn;
  }
  wg_sum_all<2>(t, lds);
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const double q = __shfl_xor(mn, o);
    mn = q < mn ? q : mn;
  }
  if (lane_id() == 0) lmin[threadIdx.x / kWave] = mn;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = lmin[0];
    for (int w = 1; w < kWaves; ++w) m = lmin[w] < m ? lmin[w] : m;
    out[0] = t[0];
    out[1] = m;
    out[2] = t[1];
  }
}

Certificate certify(agc_context* c, int32_t n, int32_t n_c, const int32_t* map, const uint32_t* members,
                    const uint32_t* mkeys, const double* d, const double* x_c, const double* r_c) {
  const double* dc = d;
  if (map) {
    double* D = c->ws.get<double>("cert.dc", n_c);
    MassOp op{members, d, D};
    seg_reduce<1, double, uint32_t, MassOp>(c, mkeys, n, op, (uint32_t*)nullptr, false, "cert.seg");
    dc = D;
  }
  double* part = c->ws.get<double>("cert.part", 3 * kCertGrid + 3);
  k_clear_u32<<<1, 1, 0, c->stream>>>(c->d_err);
  k_cert_part<<<kCertGrid, kWG, 0, c->stream>>>(dc, r_c, n_c, d, map, x_c, n, part, c->d_err);
  k_cert_final<<<1, kWG, 0, c->stream>>>(part, part + 3 * kCertGrid);
  AGC_LAUNCH_CHECK();
  double* h = (double*)c->h_pcg;   // pinned scratch; no PCG is in flight here
  AGC_HIP(hipMemcpyAsync(h, part + 3 * kCertGrid, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  err_throw(err_fetch(c));   // synchronises
  Certificate out;
  out.bound = sqrt(h[0] / h[1]);
  out.x_norm = sqrt(h[2]);
  return out;
}

__global__ void k_prolong(const int32_t* __restrict__ map, int32_t n, int32_t n_c, const double* __restrict__ xc,
                          double* __restrict__ x, unsigned* err) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cc = map[v];
    if (cc < 0 || cc >= n_c) {
      atomicOr(err, kErrMap);
      x[3 * v] = x[3 * v + 1] = x[3 * v + 2] = 0.0;
      continue;
    }
    x[3 * v] = xc[3 * cc];
    x[3 * v + 1] = xc[3 * cc + 1];
    x[3 * v + 2] = xc[3 * cc + 2];
  }
}

void prolongate(agc_context* c, int32_t n, const int32_t* map, int32_t n_c, const double* xc, double* x) {
  if (n == 0) return;
  k_prolong<<<gs_blocks(n), kWG, 0, c->stream>>>(map, n, n_c, xc, x, c->d_err);
  AGC_LAUNCH_CHECK();
}

// ------------------------------------------------------- affine embedding

// From the members sorted by (node, id): the first member of each node (its
// smallest id) and the member counts, without atomics.
__global__ void k_aff_segments(const uint32_t* __restrict__ members, const uint32_t* __restrict__ mkeys, int32_t n,
                               int32_t n_c, uint32_t* __restrict__ start, int32_t* __restrict__ rep) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t c = mkeys[k];
    if (k == 0 || mkeys[k - 1] != c) {
      start[c] = (uint32_t)k;
      rep[c] = (int32_t)members[k];
    }
    if (k == n - 1) start[n_c] = (uint32_t)n;
  }
}

// homogeneous rest coordinate of vertex v in the frame of its node c
__device__ __forceinline__ double aff_coord(const double* __restrict__ rest, const int32_t* __restrict__ rep,
                                            int64_t v, int32_t c, int q) {
  return q < 3 ? rest[3 * v + q] - rest[3 * (int64_t)rep[c] + q] : 1.0;
}

// flag12[c] = (members > threshold); flag3[c] = the complement
__global__ void k_aff_flags(const uint32_t* __restrict__ start, int32_t n_c, int32_t threshold,
                            uint32_t* __restrict__ f3, uint32_t* __restrict__ f12) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_c; c += (int64_t)gridDim.x * blockDim.x) {
    const bool big = start[c + 1] - start[c] > (uint32_t)threshold;
    f3[c] = big ? 0u : 1u;
    f12[c] = big ? 1u : 0u;
  }
}

__global__ void k_aff_labels(const uint32_t* __restrict__ r3, const uint32_t* __restrict__ r12,
                             const uint32_t* __restrict__ f12, int32_t n_c, int32_t* __restrict__ newlab,
                             int32_t* __restrict__ offset) {
  const int32_t n3 = (int32_t)r3[n_c];
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_c; c += (int64_t)gridDim.x * blockDim.x) {
    if (f12[c]) {
      newlab[c] = n3 + (int32_t)r12[c];
      offset[c] = n3 + 4 * (int32_t)r12[c];
    } else {
      newlab[c] = (int32_t)r3[c];
      offset[c] = (int32_t)r3[c];
    }
  }
}

void affine_classify(agc_context* c, int32_t n, const int32_t* map, const uint32_t* members, const uint32_t* mkeys,
                     int32_t n_c, int32_t threshold, const double* rest, AffineMap& am) {
  AGC_REQUIRE(threshold >= 0, "affine threshold < 0");
  AGC_REQUIRE(rest, "rest positions are required for the affine embedding");
  am.n_c = n_c;
  am.map = map;
  am.rest = rest;
  am.newlab = c->ws.get<int32_t>("aff.newlab", n_c);
  am.offset = c->ws.get<int32_t>("aff.offset", n_c);
  am.rep = c->ws.get<int32_t>("aff.rep", n_c);
  uint32_t* start = c->ws.get<uint32_t>("aff.start", n_c + 1);
  uint32_t* f3 = c->ws.get<uint32_t>("aff.f3", n_c + 1);
  uint32_t* f12 = c->ws.get<uint32_t>("aff.f12", n_c + 1);
  uint32_t* r3 = c->ws.get<uint32_t>("aff.r3", n_c + 1);
  uint32_t* r12 = c->ws.get<uint32_t>("aff.r12", n_c + 1);
  err_reset(c);
  // every label in [0, n_c) has members (a canonical map), so every start is written
  k_aff_segments<<<gs_blocks(n), kWG, 0, c->stream>>>(members, mkeys, n, n_c, start, am.rep);
  k_aff_flags<<<gs_blocks(n_c), kWG, 0, c->stream>>>(start, n_c, threshold, f3, f12);
  AGC_LAUNCH_CHECK();
  scan_u32(c, f3, r3, n_c, "aff.s3");
  scan_u32(c, f12, r12, n_c, "aff.s12");
  k_aff_labels<<<gs_blocks(n_c), kWG, 0, c->stream>>>(r3, r12, f12, n_c, am.newlab, am.offset);
  AGC_LAUNCH_CHECK();
  uint32_t tot[2] = {0, 0};
  AGC_HIP(hipMemcpyAsync(&tot[0], r3 + n_c, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  AGC_HIP(hipMemcpyAsync(&tot[1], r12 + n_c, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  err_throw(err_fetch(c));   // synchronises
  am.n3 = (int32_t)tot[0];
  am.n12 = (int32_t)tot[1];
  const int64_t flat = (int64_t)am.n3 + 4 * (int64_t)am.n12;
  AGC_REQUIRE(flat < INT32_MAX / 3, "too many coarse DoF");
  am.n_flat = (int32_t)flat;
}

// Per member f of a node: its value weighted by the four homogeneous rest
// coordinates (12 values); a 12-DoF node keeps all four sums, a 3-DoF node
// the last (the plain sum).
struct AffineRestrictOp {
  const uint32_t* members;
  const uint32_t* mkeys;
  const double* v;
  const double* rest;
  const int32_t* rep;
  const int32_t* newlab;
  const int32_t* offset;
  int32_t n3;
  double* out;
  __device__ void load(int64_t k, double x[12]) const {
    const int64_t f = members[k];
    const int32_t c = (int32_t)mkeys[k];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double w = aff_coord(rest, rep, f, c, q);
#pragma unroll
      for (int i = 0; i < 3; ++i) x[3 * q + i] = w * v[3 * f + i];
    }
  }
  __device__ void put(int64_t s, const double x[12], bool add) const {
    const int64_t o = offset[s];
    if (newlab[s] >= n3) {
#pragma unroll
      for (int q = 0; q < 12; ++q) out[3 * o + q] = add ? out[3 * o + q] + x[q] : x[q];
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i) out[3 * o + i] = add ? out[3 * o + i] + x[9 + i] : x[9 + i];
    }
  }
  __device__ void store(int64_t s, const double x[12]) const { put(s, x, false); }
  __device__ void add(int64_t s, const double x[12]) const { put(s, x, true); }
};

void affine_restrict(agc_context* c, int32_t n, const AffineMap& am, const uint32_t* members, const uint32_t* mkeys,
                     const double* v, double* v_flat) {
  AffineRestrictOp op{members, mkeys, v, am.rest, am.rep, am.newlab, am.offset, am.n3, v_flat};
  seg_reduce<12, double, uint32_t, AffineRestrictOp>(c, mkeys, n, op, (uint32_t*)nullptr, false, "arst.seg");
}

__global__ void k_aff_prolong(const int32_t* __restrict__ map, int32_t n, int32_t n_c,
                              const int32_t* __restrict__ newlab, const int32_t* __restrict__ offset, int32_t n3,
                              const double* __restrict__ rest, const int32_t* __restrict__ rep,
                              const double* __restrict__ xf,
                              double* __restrict__ x, unsigned* err) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = map[v];
    double o[3] = {0.0, 0.0, 0.0};
    if (c < 0 || c >= n_c) {
      atomicOr(err, kErrMap);
    } else {
      const int64_t b = offset[c];
      if (newlab[c] >= n3) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double w = aff_coord(rest, rep, v, c, q);
#pragma unroll
          for (int i = 0; i < 3; ++i) o[i] += w * xf[3 * (b + q) + i];
        }
      } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) o[i] = xf[3 * b + i];
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) x[3 * v + i] = o[i];
  }
}

void affine_prolongate(agc_context* c, int32_t n, const AffineMap& am, const double* x_flat, double* x) {
  k_aff_prolong<<<gs_blocks(n), kWG, 0, c->stream>>>(am.map, n, am.n_c, am.newlab, am.offset, am.n3, am.rest,
                                                     am.rep, x_flat, x, c->d_err);
  AGC_LAUNCH_CHECK();
}

}  // namespace agc
