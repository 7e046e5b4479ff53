// Fine-to-coarse aggregation, restriction and prolongation.
//
// Sec. 4.1 and supplement Sec. 1: super-nodes are the connected components of
// the graph of collapsible edges, and the supplement's elected-lane popcount
// plus group prefix sum (Alg. 2, Sec. 1.3) orders them by their smallest fine
// id.  The paper finds components with 32-bit in-warp hash masks applied
// level by level.  On gfx950 a parent forest does the same job for any
// component size: every vertex first points at its smallest collapsible
// neighbour, a few rounds of minimum-label hooking of roots with path
// flattening merge the trees, and a final edge-parallel pass of lock-free
// union-find guarantees that every edge ends inside one tree.  A pointer
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

__global__ void k_cc_init(int32_t* __restrict__ parent, int32_t n) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    parent[v] = (int32_t)v;
}

// Pre-linking: every vertex points at its smallest neighbour over a
// collapsible edge (if smaller than itself).  The atomics of one vertex
// number its lower neighbours only, so they barely contend, and afterwards
// most edges of a component already lead to one root.  Also validates.
__global__ void k_cc_link_min(const int32_t* __restrict__ edges, const uint8_t* __restrict__ tags, int64_t m,
                              int32_t* parent, int32_t n, unsigned* err) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    const int2 uv = reinterpret_cast<const int2*>(edges)[e];
    const int32_t u = uv.x, v = uv.y;
    const uint8_t t = tags[e];
    if (u < 0 || u >= n || v < 0 || v >= n) {
      atomicOr(err, kErrRange);
      continue;
    }
    if (t > 1) {
      atomicOr(err, kErrTag);
      continue;
    }
    if (t == 0 || u == v) continue;
    const int32_t lo = u < v ? u : v, hi = u < v ? v : u;
    atomicMin(parent + hi, lo);
  }
}

// Root-level linking round (minimum-label hooking in the manner of
// Shiloach-Vishkin): for a collapsible edge whose ends have different
// parents pu, pv, the larger of the two is pointed at the smaller.  Both lie
// in the edge's component and the value only decreases, so the forest stays
// valid; a pointer it replaces may drop a link, which the final lock-free
// pass over every edge restores.
// Lanes of a wave that hook the same vertex first take the minimum of their
// targets, so each distinct vertex costs one atomic per wave (the trees of a
// large component meet along long boundaries, whose edges sit side by side
// in the edge list).  The loop bound is uniform per workgroup, so every lane
// of a wave takes part in the lane exchanges.
__global__ void k_cc_link_roots(const int32_t* __restrict__ edges, const uint8_t* __restrict__ tags, int64_t m,
                                int32_t* parent, int32_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < m; base += stride) {
    const int64_t e = base + threadIdx.x;
    bool want = false;
    int32_t lo = 0, hi = 0;
    if (e < m && tags[e] == 1) {
      const int2 uv = reinterpret_cast<const int2*>(edges)[e];
      const int32_t u = uv.x, v = uv.y;
      if (u != v && u >= 0 && u < n && v >= 0 && v < n) {
        const int32_t pu = parent[u], pv = parent[v];
        lo = pu < pv ? pu : pv;
        hi = pu < pv ? pv : pu;
        want = pu != pv && parent[hi] > lo;
      }
    }
    uint64_t pend = __ballot(want);
    while (pend) {
      const int leader = __ffsll((unsigned long long)pend) - 1;
      const int32_t h = __shfl(hi, leader);
      const bool mine = want && hi == h;
      int32_t mn = mine ? lo : INT32_MAX;
#pragma unroll
      for (int d = kWave / 2; d > 0; d >>= 1) {
        const int32_t o = __shfl_xor(mn, d);
        mn = o < mn ? o : mn;
      }
      if ((int)lane_id() == leader) atomicMin(parent + h, mn);
      pend &= ~__ballot(mine);
      want = want && !mine;
    }
  }
}

// parent[v] = root of v by a read-only walk.  Entries other threads update
// meanwhile only move to ancestors, so every walk still ends at a root.
__global__ void k_cc_flatten(int32_t* parent, int32_t n) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t x = parent[v], p;
    while ((p = parent[x]) != x) x = p;
    parent[v] = x;
  }
}

// Lock-free union of the remaining edges whose ends sit in different trees
// (input already validated by k_cc_link_min).
__global__ void k_cc_hook(const int32_t* __restrict__ edges, const uint8_t* __restrict__ tags, int64_t m,
                          int32_t* parent, int32_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    const int2 uv = reinterpret_cast<const int2*>(edges)[e];
    const int32_t u = uv.x, v = uv.y;
    if (tags[e] != 1 || u == v || u < 0 || u >= n || v < 0 || v >= n) continue;
    int32_t ru = find_root(parent, u), rv = find_root(parent, v);
    while (ru != rv) {
      const int32_t lo = ru < rv ? ru : rv, hi = ru < rv ? rv : ru;
      const int32_t old = atomicCAS(parent + hi, hi, lo);
      if (old == hi) break;                       // hooked hi below lo
      // hi stopped being a root meanwhile: continue from its new root
      const int32_t r = find_root(parent, old);
      if (ru == hi) ru = r; else rv = r;
    }
  }
}

__global__ void k_cc_compress(int32_t* parent, int32_t n, uint32_t* __restrict__ flag) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = find_root(parent, (int32_t)v);
    flag[v] = (r == (int32_t)v) ? 1u : 0u;
  }
}

__global__ void k_cc_label(const int32_t* __restrict__ parent, const uint32_t* __restrict__ rank, int32_t n,
                           int32_t* __restrict__ map) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t x = (int32_t)v, p;
    while ((p = parent[x]) != x) x = p;       // read-only walk to the root
    map[v] = (int32_t)rank[x];
  }
}

// Root-linking rounds before the lock-free pass.  On the tet grids two
// rounds leave (almost) no edge between different trees; the lock-free pass
// merges whatever remains, so the count only affects speed.
constexpr int kRootRounds = 2;

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
  uint32_t* flag = s.flag;
  k_clear_u32<<<1, 1, 0, c->stream>>>(c->d_err);
  k_cc_init<<<gs_blocks(n), kWG, 0, c->stream>>>(parent, n);
  AGC_LAUNCH_CHECK();
  if (m > 0) {
    k_cc_link_min<<<gs_blocks(m), kWG, 0, c->stream>>>(edges, tags, m, parent, n, c->d_err);
    k_cc_flatten<<<gs_blocks(n), kWG, 0, c->stream>>>(parent, n);
    for (int r = 0; r < kRootRounds; ++r) {
      k_cc_link_roots<<<gs_blocks(m), kWG, 0, c->stream>>>(edges, tags, m, parent, n);
      k_cc_flatten<<<gs_blocks(n), kWG, 0, c->stream>>>(parent, n);
    }
    k_cc_hook<<<gs_blocks(m), kWG, 0, c->stream>>>(edges, tags, m, parent, n);
    AGC_LAUNCH_CHECK();
  }
  k_cc_compress<<<gs_blocks(n), kWG, 0, c->stream>>>(parent, n, flag);
  AGC_LAUNCH_CHECK();
  scan_u32_into(c, flag, flag, n, s.scan_sums);
  k_cc_label<<<gs_blocks(n), kWG, 0, c->stream>>>(parent, flag, n, map);
  AGC_LAUNCH_CHECK();
  uint32_t* h = (uint32_t*)c->h_pcg;   // pinned scratch of the context; no PCG is in flight here
  AGC_HIP(hipMemcpyAsync(h, flag + n, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  err_throw(err_fetch(c));   // synchronises
  return (int32_t)h[0];
}

int64_t agg_scratch_words(int32_t n) { return 2 * ((int64_t)n + 64) + scan_sums_words(n) + 64; }

AggScratch agg_scratch_carve(uint32_t* base, int32_t n) {
  AggScratch s;
  s.parent = reinterpret_cast<int32_t*>(base);
  s.flag = base + ((int64_t)n + 64);
  s.scan_sums = base + 2 * ((int64_t)n + 64);
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
