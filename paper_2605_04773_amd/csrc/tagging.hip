// Green-strain-increment edge tags (Sec. 4.2 "Adaptive Coarsening
// Criterion", Eq. 3): per tetrahedron F = Ds Dm^{-1}, G = (F^T F - I) / 2,
// and dG = G(x_cur) - G(x_prev); an edge is protected (tag 0) when any
// tetrahedron containing it has ||dG||_F above the threshold, collapsible
// (tag 1) otherwise.
//
// The mesh is static, so the tagger precomputes once (the paper precomputes
// the edge-element adjacency for the same reason): every tetrahedron's
// Dm^{-1} (nine planes) and, for each of its six edges, the index of that
// pair among the distinct pairs of the caller's edge list (-1 when absent).
// A call is then one pass over the tetrahedra, which marks hot pairs with
// byte stores of the same value (no read-modify-write, so the result does not
// depend on their order), and one pass over the edge list.
#include <memory>

#include "internal.h"

namespace agc {

constexpr int kPairA[6] = {0, 0, 0, 1, 1, 2};
constexpr int kPairB[6] = {1, 2, 3, 2, 3, 3};

// Validates a tetrahedron and stores Dm^{-1} (planes i*ne + e, row-major i).
__global__ void k_tag_rest(const int32_t* __restrict__ tets, int64_t ne, const double* __restrict__ rest, int32_t n,
                           double* __restrict__ dminv, unsigned* err) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
    int32_t v[4];
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      v[a] = tets[4 * e + a];
      ok = ok && v[a] >= 0 && v[a] < n;
    }
    ok = ok && v[0] != v[1] && v[0] != v[2] && v[0] != v[3] && v[1] != v[2] && v[1] != v[3] && v[2] != v[3];
    double inv[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (!ok) {
      atomicOr(err, kErrElem);
    } else {
      double m[9];   // columns: X_1 - X_0, X_2 - X_0, X_3 - X_0
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) m[3 * i + k] = rest[3 * (int64_t)v[k + 1] + i] - rest[3 * (int64_t)v[0] + i];
      const double c00 = m[4] * m[8] - m[5] * m[7], c01 = m[5] * m[6] - m[3] * m[8], c02 = m[3] * m[7] - m[4] * m[6];
      const double det = m[0] * c00 + m[1] * c01 + m[2] * c02;
      if (!(det != 0.0) || !isfinite(det)) {
        atomicOr(err, kErrDegenerate);
      } else {
        const double r = 1.0 / det;
        inv[0] = c00 * r;
        inv[1] = (m[2] * m[7] - m[1] * m[8]) * r;
        inv[2] = (m[1] * m[5] - m[2] * m[4]) * r;
        inv[3] = c01 * r;
        inv[4] = (m[0] * m[8] - m[2] * m[6]) * r;
        inv[5] = (m[2] * m[3] - m[0] * m[5]) * r;
        inv[6] = c02 * r;
        inv[7] = (m[1] * m[6] - m[0] * m[7]) * r;
        inv[8] = (m[0] * m[4] - m[1] * m[3]) * r;
      }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) dminv[(int64_t)i * ne + e] = inv[i];
  }
}

// key of an edge: lo * n + hi (self-loops keep lo == hi and match no element)
__global__ void k_tag_edge_keys(const int32_t* __restrict__ edges, int64_t m, int32_t n, uint64_t* __restrict__ keys,
                                uint32_t* __restrict__ ids, unsigned* err) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
    const int2 uv = reinterpret_cast<const int2*>(edges)[k];
    int32_t u = uv.x, v = uv.y;
    if (u < 0 || u >= n || v < 0 || v >= n) {
      atomicOr(err, kErrRange);
      u = v = 0;
    }
    const uint64_t lo = (uint64_t)(u < v ? u : v), hi = (uint64_t)(u < v ? v : u);
    keys[k] = lo * (uint64_t)n + hi;
    ids[k] = (uint32_t)k;
  }
}

__global__ void k_tag_heads(const uint64_t* __restrict__ sk, int64_t m, uint32_t* __restrict__ flag) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x)
    flag[k] = (k == 0 || sk[k] != sk[k - 1]) ? 1u : 0u;
}

// unique keys and, for each caller edge, the index of its key
__global__ void k_tag_unique(const uint64_t* __restrict__ sk, const uint32_t* __restrict__ sid,
                             const uint32_t* __restrict__ pos, int64_t m, uint64_t* __restrict__ ukey,
                             uint32_t* __restrict__ ekey) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t u = pos[k + 1] - 1;   // heads in [0, k] minus one
    if (k == 0 || sk[k] != sk[k - 1]) ukey[u] = sk[k];
    ekey[sid[k]] = u;
  }
}

// for each tetrahedron edge, the index of its pair among the unique keys, or -1
__global__ void k_tag_tet_edges(const int32_t* __restrict__ tets, int64_t ne, int32_t n,
                                const uint64_t* __restrict__ ukey, int64_t nu, int32_t* __restrict__ tedge) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const int32_t a = tets[4 * e + kPairA[p]], b = tets[4 * e + kPairB[p]];
      int32_t found = -1;
      if (a >= 0 && a < n && b >= 0 && b < n && a != b) {
        const uint64_t key = (uint64_t)(a < b ? a : b) * (uint64_t)n + (uint64_t)(a < b ? b : a);
        int64_t lo = 0, hi = nu;   // first index with ukey >= key
        while (lo < hi) {
          const int64_t mid = (lo + hi) >> 1;
          if (ukey[mid] < key) lo = mid + 1;
          else hi = mid;
        }
        if (lo < nu && ukey[lo] == key) found = (int32_t)lo;
      }
      tedge[(int64_t)p * ne + e] = found;
    }
  }
}

__global__ void k_tag_clear(uint8_t* __restrict__ hot, int64_t nu) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nu; k += (int64_t)gridDim.x * blockDim.x)
    hot[k] = 0;
}

// G = (F^T F - I) / 2 of F = Ds Dm^{-1} for the positions x of a tetrahedron
__device__ __forceinline__ void green(const double* __restrict__ x, const int32_t v[4], const double mi[9],
                                      double g[6]) {
  double ds[9];   // columns: x_1 - x_0, x_2 - x_0, x_3 - x_0
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i) ds[3 * i + k] = x[3 * (int64_t)v[k + 1] + i] - x[3 * (int64_t)v[0] + i];
  double f[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) f[3 * i + j] = ds[3 * i] * mi[j] + ds[3 * i + 1] * mi[3 + j] + ds[3 * i + 2] * mi[6 + j];
  // symmetric G: 00, 01, 02, 11, 12, 22
  const int pi[6] = {0, 0, 0, 1, 1, 2}, pj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int i = pi[q], j = pj[q];
    const double c = f[i] * f[j] + f[3 + i] * f[3 + j] + f[6 + i] * f[6 + j];
    g[q] = 0.5 * (c - (i == j ? 1.0 : 0.0));
  }
}

__global__ void k_tag_green(const int32_t* __restrict__ tets, int64_t ne, const double* __restrict__ dminv,
                            const int32_t* __restrict__ tedge, const double* __restrict__ xc,
                            const double* __restrict__ xp, double thr, uint8_t* __restrict__ hot) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
    int32_t v[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) v[a] = tets[4 * e + a];
    double mi[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) mi[i] = dminv[(int64_t)i * ne + e];
    double gc[6], gp[6];
    green(xc, v, mi, gc);
    green(xp, v, mi, gp);
    // ||dG||_F^2: diagonal entries once, off-diagonal ones twice
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double d = gc[q] - gp[q];
      s += (q == 0 || q == 3 || q == 5) ? d * d : 2.0 * d * d;
    }
    if (sqrt(s) > thr) {
#pragma unroll
      for (int p = 0; p < 6; ++p) {
        const int32_t u = tedge[(int64_t)p * ne + e];
        if (u >= 0) hot[u] = 1;
      }
    }
  }
}

__global__ void k_tag_out(const uint32_t* __restrict__ ekey, const uint8_t* __restrict__ hot, int64_t m,
                          uint8_t* __restrict__ tags, unsigned long long* n_hot) {
  unsigned long long cnt = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
    const uint8_t h = hot[ekey[k]];
    tags[k] = h ? 0 : 1;
    cnt += h;
  }
  // integer count: the total does not depend on the order of the additions
  for (int d = kWave / 2; d > 0; d >>= 1) cnt += __shfl_down(cnt, d);
  if (lane_id() == 0 && cnt) atomicAdd(n_hot, cnt);
}

}  // namespace agc

// ------------------------------------------------------------------- ABI


extern "C" {

agc_status agc_tagger_create(agc_context* c, int32_t n_verts, int64_t n_tets, const int32_t* tets,
                             const double* rest, int64_t n_edges, const int32_t* edges, agc_tagger** out) {
  using namespace agc;
  API_BEGIN(c)
  AGC_REQUIRE(out, "out is null");
  *out = nullptr;
  AGC_REQUIRE(n_verts >= 1 && n_tets >= 0 && n_edges >= 0, "bad sizes");
  AGC_REQUIRE(n_tets == 0 || (tets && rest), "tets/rest null");
  AGC_REQUIRE(n_edges == 0 || edges, "edges null");
  AGC_REQUIRE(((uintptr_t)edges & 7) == 0, "edges must be 8-byte aligned");
  AGC_REQUIRE(n_edges < (int64_t)UINT32_MAX, "too many edges");
  std::unique_ptr<agc_tagger> t(new agc_tagger());
  t->n = n_verts;
  t->ne = n_tets;
  t->m = n_edges;
  err_reset(c);
  int32_t* tt = (int32_t*)t->tets.ensure(sizeof(int32_t) * 4 * (size_t)(n_tets > 0 ? n_tets : 1));
  double* dminv = (double*)t->dminv.ensure(sizeof(double) * 9 * (size_t)(n_tets > 0 ? n_tets : 1));
  if (n_tets > 0) {
    AGC_HIP(hipMemcpyAsync(tt, tets, sizeof(int32_t) * 4 * (size_t)n_tets, hipMemcpyDeviceToDevice, c->stream));
    k_tag_rest<<<grid_blocks(n_tets), kWG, 0, c->stream>>>(tt, n_tets, rest, n_verts, dminv, c->d_err);
    AGC_LAUNCH_CHECK();
  }
  // distinct pairs of the edge list, sorted
  const int64_t m = n_edges;
  uint32_t* ekey = (uint32_t*)t->ekey.ensure(sizeof(uint32_t) * (size_t)(m > 0 ? m : 1));
  uint64_t* ukey = nullptr;
  if (m > 0) {
    uint64_t* k1 = c->ws.get<uint64_t>("tag.k1", m);
    uint64_t* k2 = c->ws.get<uint64_t>("tag.k2", m);
    uint32_t* v1 = c->ws.get<uint32_t>("tag.v1", m);
    uint32_t* v2 = c->ws.get<uint32_t>("tag.v2", m);
    k_tag_edge_keys<<<grid_blocks(m), kWG, 0, c->stream>>>(edges, m, n_verts, k1, v1, c->d_err);
    AGC_LAUNCH_CHECK();
    const bool alt = radix_sort_u64(c, k1, v1, k2, v2, m, bits_for((uint64_t)n_verts * (uint64_t)n_verts - 1),
                                    "tag.sort");
    uint64_t* sk = alt ? k2 : k1;
    uint32_t* sv = alt ? v2 : v1;
    // pos[0..m] = exclusive scan of the head flags; the distinct index of
    // sorted position k is pos[k + 1] - 1, and pos[m] the number of distinct pairs
    uint32_t* pos = c->ws.get<uint32_t>("tag.pos", m + 1);
    k_tag_heads<<<grid_blocks(m), kWG, 0, c->stream>>>(sk, m, pos);
    AGC_LAUNCH_CHECK();
    scan_u32(c, pos, pos, m, "tag.scan");
    uint32_t nu32 = 0;
    AGC_HIP(hipMemcpyAsync(&nu32, pos + m, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    AGC_HIP(hipStreamSynchronize(c->stream));
    t->nu = nu32;
    ukey = c->ws.get<uint64_t>("tag.ukey", t->nu);
    k_tag_unique<<<grid_blocks(m), kWG, 0, c->stream>>>(sk, sv, pos, m, ukey, ekey);
    AGC_LAUNCH_CHECK();
  }
  int32_t* tedge = (int32_t*)t->tedge.ensure(sizeof(int32_t) * 6 * (size_t)(n_tets > 0 ? n_tets : 1));
  if (n_tets > 0) {
    k_tag_tet_edges<<<grid_blocks(n_tets), kWG, 0, c->stream>>>(tt, n_tets, n_verts, ukey, t->nu, tedge);
    AGC_LAUNCH_CHECK();
  }
  t->hot.ensure((size_t)(t->nu > 0 ? t->nu : 1));
  t->count.ensure(sizeof(unsigned long long));
  err_throw(err_fetch(c));
  *out = t.release();
  API_END(c)
}

agc_status agc_tagger_destroy(agc_context* c, agc_tagger* t) {
  if (!c || !t) return AGC_ERR_INVALID_ARG;
  delete t;   // releases its buffers
  return AGC_OK;
}

agc_status agc_tag_edges(agc_context* c, const agc_tagger* t, const double* x_cur, const double* x_prev,
                         double threshold, uint8_t* tags, int64_t* n_protected) {
  using namespace agc;
  API_BEGIN(c)
  AGC_REQUIRE(t, "tagger is null");
  AGC_REQUIRE(t->ne == 0 || (x_cur && x_prev), "positions null");
  AGC_REQUIRE(t->m == 0 || tags, "tags null");
  AGC_REQUIRE(threshold >= 0.0, "threshold < 0");
  uint8_t* hot = (uint8_t*)t->hot.p;
  unsigned long long* cnt = (unsigned long long*)t->count.p;
  k_tag_clear<<<grid_blocks(t->nu), kWG, 0, c->stream>>>(hot, t->nu);
  AGC_LAUNCH_CHECK();
  if (t->ne > 0) {
    k_tag_green<<<grid_blocks(t->ne), kWG, 0, c->stream>>>((const int32_t*)t->tets.p, t->ne, (const double*)t->dminv.p,
                                                          (const int32_t*)t->tedge.p, x_cur, x_prev, threshold, hot);
    AGC_LAUNCH_CHECK();
  }
  if (n_protected) AGC_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), c->stream));
  if (t->m > 0) {
    k_tag_out<<<grid_blocks(t->m), kWG, 0, c->stream>>>((const uint32_t*)t->ekey.p, hot, t->m, tags, cnt);
    AGC_LAUNCH_CHECK();
  }
  if (n_protected) {
    unsigned long long h = 0;
    if (t->m > 0) {
      AGC_HIP(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, c->stream));
      AGC_HIP(hipStreamSynchronize(c->stream));
    }
    *n_protected = (int64_t)h;
  }
  API_END(c)
}

}  // extern "C"
