// Galerkin assembly of the coarse system from per-element 12x12 blocks.
//
// Sec. 4.1 ("Algebraic Coarsening and System Assembly") and supplement Sec. 2:
// every fine 3x3 block (i, j) is moved to (map i, map j) and equal keys are
// summed, which is the Galerkin product A_c = P^T H P.  The paper reduces an
// unordered fine triplet list with a hash and a second hash reduction after
// the remap.  Here the work is split into
//   (static, once per mesh)  the fine upper-triangle pattern and, for every
//                            fine block, the fixed list of element sub-blocks
//                            that sum into it;
//   (per Newton iteration)   a gather-sum of element sub-blocks into fine
//                            upper blocks; coarse upper keys
//                            (min(map i, map j), max(..)) sorted by a stable
//                            radix sort; a segmented reduction in sorted
//                            order; a mirror into full symmetric BSR storage.
// Only the upper triangle is reduced (the paper also accumulates only the
// diagonal and upper blocks, Sec. 5.2 "Overall Performance"); the lower
// triangle is the transpose of the same sums, so A_c is exactly symmetric.
#include <string>
#include <vector>

#include "segreduce.h"

namespace agc {

// ------------------------------------------------------------ small kernels

__global__ void k_iota_u32(uint32_t* __restrict__ v, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    v[k] = (uint32_t)k;
}

__global__ void k_zero_u32(uint32_t* __restrict__ v, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    v[k] = 0u;
}

__global__ void k_fill_i32(int32_t* __restrict__ v, int64_t n, int32_t x) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    v[k] = x;
}

static unsigned grid_stride_blocks(int64_t n) {
  int64_t b = (n + kWG - 1) / kWG;
  if (b > 65536) b = 65536;
  return (unsigned)(b < 1 ? 1 : b);
}

// --------------------------------------------------------------- mesh plan

__global__ void k_elem_check(const int32_t* __restrict__ ev, int64_t ne, int32_t n, unsigned* err) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
    int v[4];
    bool bad = false;
    for (int a = 0; a < 4; ++a) {
      v[a] = ev[4 * e + a];
      bad |= (v[a] < 0 || v[a] >= n);
    }
    for (int a = 0; a < 4; ++a)
      for (int b = a + 1; b < 4; ++b) bad |= (v[a] == v[b]);
    if (bad) atomicOr(err, kErrElem);
  }
}

// 10 upper pairs per element: (a,a) and (a,b) a<b, oriented so the block is
// (min vertex, max vertex); payload e*16 + a'*4 + b' names sub-block (a', b').
__global__ void k_elem_pairs(const int32_t* __restrict__ ev, int64_t ne, int32_t n,
                             uint64_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
    int v[4];
    for (int a = 0; a < 4; ++a) v[a] = ev[4 * e + a];
    int q = 0;
    for (int a = 0; a < 4; ++a) {
      for (int b = a; b < 4; ++b, ++q) {
        int aa = a, bb = b;
        if (v[aa] > v[bb]) { aa = b; bb = a; }
        keys[10 * e + q] = (uint64_t)v[aa] * (uint64_t)n + (uint64_t)v[bb];
        vals[10 * e + q] = (uint32_t)(e * 16 + aa * 4 + bb);
      }
    }
  }
}

template <class K>
__global__ void k_head_flags(const K* __restrict__ keys, int64_t n, uint32_t* __restrict__ f) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    f[k] = (k == 0 || keys[k - 1] != keys[k]) ? 1u : 0u;
}

// heads -> segment starts (ptr) and unique keys split into (row, col) = (key / n, key % n)
__global__ void k_compact_heads(const uint64_t* __restrict__ keys, int64_t n, const uint32_t* __restrict__ pos,
                                uint64_t ncol, uint32_t* __restrict__ ptr, int32_t* __restrict__ row,
                                int32_t* __restrict__ col) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = keys[k];
    if (k == 0 || keys[k - 1] != key) {
      const uint32_t s = pos[k];
      ptr[s] = (uint32_t)k;
      row[s] = (int32_t)(key / ncol);
      col[s] = (int32_t)(key % ncol);
    }
    if (k == n - 1) ptr[pos[n]] = (uint32_t)n;
  }
}

__global__ void k_split_keys(const uint64_t* __restrict__ ukeys, int64_t nu, uint64_t ncol,
                             int32_t* __restrict__ row, int32_t* __restrict__ col) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nu; k += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = ukeys[k];
    row[k] = (int32_t)(key / ncol);
    col[k] = (int32_t)(key % ncol);
  }
}

// ------------------------------------------------ full symmetric pattern

// start[k] = first position whose key is >= k, for k in [0, n_keys], over
// ascending keys; empty keys get empty ranges.  One coalesced pass, no atomics.
template <class K>
__global__ void k_key_starts(const K* __restrict__ keys, int64_t m, int64_t n_keys, uint32_t* __restrict__ start) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = (int64_t)keys[i];
    const int64_t prev = (i == 0) ? -1 : (int64_t)keys[i - 1];
    for (int64_t j = prev + 1; j <= k; ++j) start[j] = (uint32_t)i;
    if (i == m - 1)
      for (int64_t j = k + 1; j <= n_keys; ++j) start[j] = (uint32_t)m;
  }
}

// per row r: upper count (row r), lower count (column r above the diagonal),
// full row length.  The diagonal entry of column r is the last in CSC order.
__global__ void k_full_counts(const uint32_t* __restrict__ up_start, const uint32_t* __restrict__ col_start,
                              const uint32_t* __restrict__ csc_u, const int32_t* __restrict__ ur, int32_t n,
                              uint32_t* __restrict__ cnt_low, uint32_t* __restrict__ len) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t cup = up_start[r + 1] - up_start[r];
    const uint32_t c0 = col_start[r], c1 = col_start[r + 1];
    const uint32_t has_diag = (c1 > c0 && ur[csc_u[c1 - 1]] == (int32_t)r) ? 1u : 0u;
    cnt_low[r] = c1 - c0 - has_diag;
    len[r] = cup + (c1 - c0 - has_diag);
  }
}

// upper entries: position after the row's lower part
__global__ void k_place_upper(const int32_t* __restrict__ ur, const int32_t* __restrict__ uc, int64_t nu,
                              const uint32_t* __restrict__ row_ptr, const uint32_t* __restrict__ cnt_low,
                              const uint32_t* __restrict__ up_start, int32_t* __restrict__ col,
                              int32_t* __restrict__ rowidx, uint32_t* __restrict__ src,
                              int32_t* __restrict__ diag) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < nu; u += (int64_t)gridDim.x * blockDim.x) {
    const int r = ur[u], c = uc[u];
    const int64_t p = (int64_t)row_ptr[r] + cnt_low[r] + (u - (int64_t)up_start[r]);
    col[p] = c;
    rowidx[p] = r;
    src[p] = (uint32_t)(2 * u);
    if (r == c) diag[r] = (int32_t)p;
  }
}

// mirrored entries: upper entries sorted by column (stable, so by row inside a
// column); the rank inside the column is the position in the lower part.
__global__ void k_place_lower(const uint32_t* __restrict__ csc_u, int64_t nu, const int32_t* __restrict__ ur,
                              const int32_t* __restrict__ uc, const uint32_t* __restrict__ col_start,
                              const uint32_t* __restrict__ row_ptr, int32_t* __restrict__ col,
                              int32_t* __restrict__ rowidx, uint32_t* __restrict__ src) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nu; q += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t u = csc_u[q];
    const int r = ur[u], c = uc[u];
    if (r == c) continue;
    const int64_t p = (int64_t)row_ptr[c] + (q - (int64_t)col_start[c]);
    col[p] = r;
    rowidx[p] = c;
    src[p] = 2u * u + 1u;
  }
}

__global__ void k_check_diag(const int32_t* __restrict__ diag, int32_t n, unsigned* err) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    if (diag[r] < 0) atomicOr(err, kErrNoDiag);
}

__global__ void k_u32_to_i32(const uint32_t* __restrict__ a, int32_t* __restrict__ b, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    b[k] = (int32_t)a[k];
}

// Builds the full symmetric pattern from upper entries (ur, uc) sorted by
// (row, col).  src[p] = 2*u (+1 when block p is the transpose of upper u).
struct FullPattern {
  int32_t* row_ptr;  // [n+1]
  int32_t* col;      // [nnz]
  int32_t* rowidx;   // [nnz]
  uint32_t* src;     // [nnz]
  int32_t* diag;     // [n]
};

static int64_t build_full(agc_context* c, int32_t n, int64_t nu, const int32_t* ur, const int32_t* uc,
                          FullPattern out, const std::string& tag) {
  AGC_REQUIRE(nu >= 1, "empty pattern");
  uint32_t* cnt_low = c->ws.get<uint32_t>(tag + ".clow", n + 1);
  uint32_t* up_start = c->ws.get<uint32_t>(tag + ".ups", n + 1);
  uint32_t* col_start = c->ws.get<uint32_t>(tag + ".cols", n + 1);
  uint32_t* rp = c->ws.get<uint32_t>(tag + ".rp", n + 1);
  const unsigned gn = grid_stride_blocks(n + 1), gu = grid_stride_blocks(nu);
  // stable sort of the upper entries by column: CSC order, by row inside a column
  uint32_t* kc = c->ws.get<uint32_t>(tag + ".kc", nu);
  uint32_t* kc2 = c->ws.get<uint32_t>(tag + ".kc2", nu);
  uint32_t* vu = c->ws.get<uint32_t>(tag + ".vu", nu);
  uint32_t* vu2 = c->ws.get<uint32_t>(tag + ".vu2", nu);
  AGC_HIP(hipMemcpyAsync(kc, uc, sizeof(uint32_t) * nu, hipMemcpyDeviceToDevice, c->stream));
  k_iota_u32<<<gu, kWG, 0, c->stream>>>(vu, nu);
  AGC_LAUNCH_CHECK();
  const bool alt = radix_sort_u32(c, kc, vu, kc2, vu2, nu, bits_for((uint64_t)(n > 0 ? n - 1 : 0)), tag + ".sort");
  const uint32_t* csc_u = alt ? vu2 : vu;
  const uint32_t* csc_key = alt ? kc2 : kc;
  // row starts of the upper entries and column starts of the CSC order
  k_key_starts<int32_t><<<gu, kWG, 0, c->stream>>>(ur, nu, n, up_start);
  k_key_starts<uint32_t><<<gu, kWG, 0, c->stream>>>(csc_key, nu, n, col_start);
  k_full_counts<<<gn, kWG, 0, c->stream>>>(up_start, col_start, csc_u, ur, n, cnt_low, rp);
  AGC_LAUNCH_CHECK();
  scan_u32(c, rp, rp, n, tag + ".s1");
  k_fill_i32<<<gn, kWG, 0, c->stream>>>(out.diag, n, -1);
  AGC_LAUNCH_CHECK();
  k_place_upper<<<gu, kWG, 0, c->stream>>>(ur, uc, nu, rp, cnt_low, up_start, out.col, out.rowidx, out.src,
                                           out.diag);
  AGC_LAUNCH_CHECK();
  k_place_lower<<<gu, kWG, 0, c->stream>>>(csc_u, nu, ur, uc, col_start, rp, out.col, out.rowidx, out.src);
  AGC_LAUNCH_CHECK();
  k_u32_to_i32<<<gn, kWG, 0, c->stream>>>(rp, out.row_ptr, n + 1);
  AGC_LAUNCH_CHECK();
  k_check_diag<<<gn, kWG, 0, c->stream>>>(out.diag, n, c->d_err);
  AGC_LAUNCH_CHECK();
  return 2 * nu;  // upper bound; exact count = 2 nu - n_diag, read by the caller
}

// ------------------------------------------------- fine gather tables

// Pieces per gather workgroup: 96 pieces of 36 float64 values are 27 KB of
// LDS, which leaves room for five workgroups per CU.
#ifndef AGC_GATHER_PIECES
#define AGC_GATHER_PIECES 96
#endif
constexpr int kGatherPieces = AGC_GATHER_PIECES;
// Plan entries and blocks of a workgroup: a piece of row v serves at most the
// four blocks of row v that its element touches.
constexpr int kGatherEntries = 4 * kGatherPieces;

// deg[v] = number of elements around v: the plan length of the diagonal
// block (v, v), the first upper block of row v (rows without elements: 0)
__global__ void k_row_degree(const uint32_t* __restrict__ row_f0, const uint32_t* __restrict__ pptr, int32_t n,
                             uint32_t* __restrict__ deg) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t f = row_f0[v];
    deg[v] = f < row_f0[v + 1] ? pptr[f + 1] - pptr[f] : 0u;
  }
}

// piece_src[piece_base[v] + s] = e*4 + a of the s-th element around v (the
// diagonal block's plan, in element order)
__global__ void k_piece_src(const uint32_t* __restrict__ row_f0, const uint32_t* __restrict__ pptr,
                            const uint32_t* __restrict__ plan, const uint32_t* __restrict__ piece_base, int32_t n,
                            uint32_t* __restrict__ src) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t g0 = piece_base[v], d = piece_base[v + 1] - g0;
    if (d == 0) continue;
    const uint32_t k0 = pptr[row_f0[v]];
    for (uint32_t s = 0; s < d; ++s) src[g0 + s] = plan[k0 + s] >> 2;
  }
}

// pentry[k] = (row_off[v] + s) * 4 + b for plan entry k = (e, a, b) of a
// block of row v, where s is the position of e among the elements around v.
// The plan of a block lists its elements in increasing order, a subsequence
// of those around v, so one forward walk per block finds them; s is kept
// below the row's degree, so every use indexes a piece of the row.
__global__ void k_piece_entries(const int32_t* __restrict__ fu_row, const uint32_t* __restrict__ row_f0,
                                const uint32_t* __restrict__ pptr, const uint32_t* __restrict__ plan,
                                const uint16_t* __restrict__ row_off, int64_t nf, uint16_t* __restrict__ pentry) {
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < nf; f += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = fu_row[f];
    const uint32_t fd = row_f0[v];
    const uint32_t d0 = pptr[fd], dl = pptr[fd + 1] - d0;
    const uint32_t off = row_off[v];
    uint32_t s = 0;
    for (uint32_t k = pptr[f]; k < pptr[f + 1]; ++k) {
      const uint32_t code = plan[k];
      while (s + 1 < dl && (plan[d0 + s] >> 4) < (code >> 4)) ++s;
      const uint32_t piece = off + s;
      pentry[k] = (uint16_t)(((piece < 16383u ? piece : 16383u) << 2) | (code & 3u));
    }
  }
}

// wg_info[g] = {first piece, pieces, f0, f1, k0, k1, 0, 0} of the rows [v0, v1);
// pieces = all ones for a run whose pieces or plan entries exceed the LDS arrays
__global__ void k_wg_info(const int32_t* __restrict__ wg_row, int64_t n_wg, const uint32_t* __restrict__ piece_base,
                          const uint32_t* __restrict__ row_f0, const uint32_t* __restrict__ pptr,
                          uint32_t* __restrict__ info) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_wg; g += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v0 = wg_row[g], v1 = wg_row[g + 1];
    const uint32_t f0 = row_f0[v0], f1 = row_f0[v1];
    uint32_t* o = info + 8 * g;
    const uint32_t np = piece_base[v1] - piece_base[v0];
    const bool fits = np <= (uint32_t)kGatherPieces && pptr[f1] - pptr[f0] <= (uint32_t)kGatherEntries;
    o[0] = piece_base[v0];
    o[1] = fits ? np : 0xffffffffu;   // a run that does not fit reads from global memory
    o[2] = f0;
    o[3] = f1;
    o[4] = pptr[f0];
    o[5] = pptr[f1];
    o[6] = 0;
    o[7] = 0;
  }
}

// Rows to gather workgroups: runs of consecutive rows whose pieces fit in
// kGatherPieces; a row with more pieces than that has a workgroup of its own
// (which reads from global memory instead).
static void gather_tables(agc_context* c, Mesh& m) {
  const int32_t n = m.n_verts;
  uint32_t* rf = c->ws.get<uint32_t>("mesh.rowf0", n + 1);
  uint32_t* pb = c->ws.get<uint32_t>("mesh.pbase", n + 1);
  const uint32_t* pptr = (const uint32_t*)m.plan_ptr.p;
  const uint32_t* plan = (const uint32_t*)m.plan.p;
  k_key_starts<int32_t><<<grid_stride_blocks(m.nf), kWG, 0, c->stream>>>((const int32_t*)m.fu_row.p, m.nf, n, rf);
  AGC_LAUNCH_CHECK();
  k_row_degree<<<grid_stride_blocks(n), kWG, 0, c->stream>>>(rf, pptr, n, pb);
  AGC_LAUNCH_CHECK();
  scan_u32(c, pb, pb, n, "mesh.pscan");
  uint32_t* src = (uint32_t*)m.piece_src.ensure(sizeof(uint32_t) * 4 * m.n_elems);
  k_piece_src<<<grid_stride_blocks(n), kWG, 0, c->stream>>>(rf, pptr, plan, pb, n, src);
  AGC_LAUNCH_CHECK();
  std::vector<uint32_t> h(n + 1);
  AGC_HIP(hipMemcpyAsync(h.data(), pb, sizeof(uint32_t) * (n + 1), hipMemcpyDeviceToHost, c->stream));
  AGC_HIP(hipStreamSynchronize(c->stream));
  AGC_REQUIRE(h[n] == 4 * (uint64_t)m.n_elems, "gather tables: piece count");
  std::vector<int32_t> wr{0};
  std::vector<uint16_t> off(n);
  for (int32_t v = 0; v < n;) {
    int32_t u = v + 1;
    while (u < n && h[u + 1] - h[v] <= (uint32_t)kGatherPieces) ++u;
    for (int32_t x = v; x < u; ++x) {
      const uint32_t o = h[x] - h[v];
      off[x] = (uint16_t)(o < 16383u ? o : 16383u);
    }
    wr.push_back(u);
    v = u;
  }
  m.n_wg = (int64_t)wr.size() - 1;
  int32_t* wg = c->ws.get<int32_t>("mesh.wgrow", wr.size());
  uint16_t* offd = c->ws.get<uint16_t>("mesh.rowoff", n);
  AGC_HIP(hipMemcpyAsync(wg, wr.data(), sizeof(int32_t) * wr.size(), hipMemcpyHostToDevice, c->stream));
  AGC_HIP(hipMemcpyAsync(offd, off.data(), sizeof(uint16_t) * n, hipMemcpyHostToDevice, c->stream));
  uint32_t* info = (uint32_t*)m.wg_info.ensure(sizeof(uint32_t) * 8 * m.n_wg);
  k_wg_info<<<grid_stride_blocks(m.n_wg), kWG, 0, c->stream>>>(wg, m.n_wg, pb, rf, pptr, info);
  AGC_LAUNCH_CHECK();
  uint16_t* pe = (uint16_t*)m.pentry.ensure(sizeof(uint16_t) * 10 * m.n_elems);
  k_piece_entries<<<grid_stride_blocks(m.nf), kWG, 0, c->stream>>>((const int32_t*)m.fu_row.p, rf, pptr, plan, offd,
                                                                    m.nf, pe);
  AGC_LAUNCH_CHECK();
  // the host vectors above must outlive the copies
  AGC_HIP(hipStreamSynchronize(c->stream));
}

// ------------------------------------------------------------ mesh build

void mesh_build(agc_context* c, Mesh& m, int32_t n, int64_t ne, const int32_t* ev) {
  m.n_verts = n;
  m.n_elems = ne;
  AGC_REQUIRE(ne >= 1, "mesh needs at least one element");
  AGC_REQUIRE(10 * ne < (int64_t)UINT32_MAX && 16 * ne < (int64_t)UINT32_MAX, "too many elements");
  int32_t* evd = (int32_t*)m.elem_verts.ensure(sizeof(int32_t) * 4 * ne);
  AGC_HIP(hipMemcpyAsync(evd, ev, sizeof(int32_t) * 4 * ne, hipMemcpyDeviceToDevice, c->stream));
  err_reset(c);
  k_elem_check<<<grid_stride_blocks(ne), kWG, 0, c->stream>>>(evd, ne, n, c->d_err);
  AGC_LAUNCH_CHECK();
  err_throw(err_fetch(c));

  // fine upper pattern and the summation plan
  const int64_t np = 10 * ne;
  uint64_t* k1 = c->ws.get<uint64_t>("mesh.k1", np);
  uint64_t* k2 = c->ws.get<uint64_t>("mesh.k2", np);
  uint32_t* v1 = c->ws.get<uint32_t>("mesh.v1", np);
  uint32_t* v2 = c->ws.get<uint32_t>("mesh.v2", np);
  k_elem_pairs<<<grid_stride_blocks(ne), kWG, 0, c->stream>>>(evd, ne, n, k1, v1);
  AGC_LAUNCH_CHECK();
  const int nb = bits_for((uint64_t)n * (uint64_t)n - 1);
  const bool alt = radix_sort_u64(c, k1, v1, k2, v2, np, nb, "mesh.sort");
  uint64_t* sk = alt ? k2 : k1;
  uint32_t* sv = alt ? v2 : v1;
  uint32_t* pos = c->ws.get<uint32_t>("mesh.pos", np + 1);
  k_head_flags<uint64_t><<<grid_stride_blocks(np), kWG, 0, c->stream>>>(sk, np, pos);
  AGC_LAUNCH_CHECK();
  scan_u32(c, pos, pos, np, "mesh.scan");
  uint32_t nf32 = 0;
  AGC_HIP(hipMemcpyAsync(&nf32, pos + np, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
  AGC_HIP(hipStreamSynchronize(c->stream));
  m.nf = nf32;
  uint32_t* pptr = (uint32_t*)m.plan_ptr.ensure(sizeof(uint32_t) * (m.nf + 1));
  int32_t* fr = (int32_t*)m.fu_row.ensure(sizeof(int32_t) * m.nf);
  int32_t* fc = (int32_t*)m.fu_col.ensure(sizeof(int32_t) * m.nf);
  k_compact_heads<<<grid_stride_blocks(np), kWG, 0, c->stream>>>(sk, np, pos, (uint64_t)n, pptr, fr, fc);
  AGC_LAUNCH_CHECK();
  uint32_t* plan = (uint32_t*)m.plan.ensure(sizeof(uint32_t) * np);
  AGC_HIP(hipMemcpyAsync(plan, sv, sizeof(uint32_t) * np, hipMemcpyDeviceToDevice, c->stream));

  // full fine pattern (static)
  m.ff_row_ptr.ensure(sizeof(int32_t) * (n + 1));
  // padded as Matrix::reserve pads its pattern: the SpMV loads four blocks whole
  m.ff_col.ensure(sizeof(int32_t) * (size_t)(plane_stride(2 * m.nf) + 4));
  m.ff_rowidx.ensure(sizeof(int32_t) * (size_t)(plane_stride(2 * m.nf) + 4));
  m.ff_src.ensure(sizeof(uint32_t) * 2 * m.nf);
  m.ff_diag.ensure(sizeof(int32_t) * (n + 1));
  FullPattern fp{(int32_t*)m.ff_row_ptr.p, (int32_t*)m.ff_col.p, (int32_t*)m.ff_rowidx.p,
                 (uint32_t*)m.ff_src.p, (int32_t*)m.ff_diag.p};
  err_reset(c);
  build_full(c, n, m.nf, fr, fc, fp, "mesh.full");
  int32_t nnz = 0;
  AGC_HIP(hipMemcpyAsync(&nnz, fp.row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  err_throw(err_fetch(c));
  m.ff_nnzb = nnz;
  gather_tables(c, m);
}

// ------------------------------------------------------- per-step assembly

// F[3r+s][f] = sum over the plan of f of entry (r, s) of element sub-block
// (a, b), in plan order.  Three threads per fine block, one per row r: each
// reads three contiguous values per plan entry, and the loop is unrolled so
// that the loads of several entries are in flight together (the sums keep
// plan order).
constexpr int kGatherUnroll = 4;
template <class In, class Acc>
__device__ __forceinline__ void fine_gather_one(const In* __restrict__ eh, const uint32_t* __restrict__ pptr,
                                                const uint32_t* __restrict__ plan, int64_t nf, Acc* __restrict__ F,
                                                int64_t t) {
  const int64_t f = t / 3;
  const int r = (int)(t - 3 * f);
  Acc acc[3] = {(Acc)0, (Acc)0, (Acc)0};
  const uint32_t k0 = pptr[f], k1 = pptr[f + 1];
  uint32_t k = k0;
  for (; k + kGatherUnroll <= k1; k += kGatherUnroll) {
    In v[kGatherUnroll][3];
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) {
      const uint32_t code = plan[k + u];
      const In* p = eh + (int64_t)(code >> 4) * 144 + (3 * ((code >> 2) & 3) + r) * 12 + 3 * (code & 3);
#pragma unroll
      for (int s = 0; s < 3; ++s) v[u][s] = p[s];
    }
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u)
#pragma unroll
      for (int s = 0; s < 3; ++s) acc[s] += (Acc)v[u][s];
  }
  for (; k < k1; ++k) {
    const uint32_t code = plan[k];
    const In* p = eh + (int64_t)(code >> 4) * 144 + (3 * ((code >> 2) & 3) + r) * 12 + 3 * (code & 3);
#pragma unroll
    for (int s = 0; s < 3; ++s) acc[s] += (Acc)p[s];
  }
#pragma unroll
  for (int s = 0; s < 3; ++s) F[(int64_t)(3 * r + s) * nf + f] = acc[s];
}

// The gather by runs of rows (one run per workgroup, described by wg_info):
// the workgroup copies the pieces of its rows into LDS, whole and with
// 16-byte loads, together with its plan entries (pentry) and block offsets,
// then forms the sums of its blocks from LDS exactly as fine_gather_one does
// (same entries, same order, so the same bits).  A run of one row with more
// than kGatherPieces pieces reads from global memory.  Grid-stride over the
// runs: one pass with the full grid, or a capped grid when it runs beside
// other work.  staged = 0 (element blocks not 16-byte aligned): every run
// reads from global memory.
template <class In, class Acc>
__global__ __launch_bounds__(kWG) void k_fine_gather(const In* __restrict__ eh, const uint32_t* __restrict__ pptr,
                                                     const uint32_t* __restrict__ plan,
                                                     const uint16_t* __restrict__ pentry,
                                                     const uint32_t* __restrict__ piece_src,
                                                     const uint4* __restrict__ wg_info, int64_t n_wg, int64_t nf,
                                                     Acc* __restrict__ F, int staged) {
  constexpr int kPieceVals = 36;
  constexpr int kChunks = kPieceVals * (int)sizeof(In) / 16;   // 16-byte chunks per piece
  constexpr int kFill = (kGatherPieces * kChunks + kWG - 1) / kWG;
  __shared__ __align__(16) In lds[kGatherPieces * kPieceVals];
  __shared__ uint16_t le[kGatherEntries];       // plan entries of the run, from k0
  __shared__ uint16_t lp[kGatherEntries + 1];   // plan offsets of its blocks, from f0
  for (int64_t g = blockIdx.x; g < n_wg; g += gridDim.x) {
    const uint4 wa = wg_info[2 * g], wb = wg_info[2 * g + 1];
    const uint32_t p0 = wa.x, np = wa.y, f0 = wa.z, f1 = wa.w, k0 = wb.x, k1 = wb.y;
    if (!staged || np > (uint32_t)kGatherPieces) {   // the same for the whole workgroup
      for (int64_t t = 3 * (int64_t)f0 + threadIdx.x; t < 3 * (int64_t)f1; t += kWG)
        fine_gather_one<In, Acc>(eh, pptr, plan, nf, F, t);
      continue;
    }
    if (np == 0) continue;   // rows without elements: no blocks
    const uint32_t nc = np * kChunks, ne = k1 - k0, nb = f1 - f0;
    // Branch-free loads (indices past the end repeat the last one), all
    // issued before the first store: the piece sources, then the pieces,
    // the entries and the block offsets.
    constexpr int kE = (kGatherEntries + kWG - 1) / kWG, kB = (kGatherEntries + 1 + kWG - 1) / kWG;
    uint32_t srcs[kFill];
#pragma unroll
    for (int u = 0; u < kFill; ++u) {
      const uint32_t cidx = min(threadIdx.x + u * kWG, nc - 1);
      srcs[u] = piece_src[p0 + cidx / kChunks];
    }
    uint16_t ev[kE];
    uint32_t bv[kB];
#pragma unroll
    for (int u = 0; u < kE; ++u) ev[u] = pentry[k0 + min(threadIdx.x + u * kWG, ne - 1)];
#pragma unroll
    for (int u = 0; u < kB; ++u) bv[u] = pptr[f0 + min(threadIdx.x + u * kWG, nb)];
    uint4 buf[kFill];
#pragma unroll
    for (int u = 0; u < kFill; ++u) {
      const uint32_t cidx = min(threadIdx.x + u * kWG, nc - 1);
      const uint32_t q = cidx - (cidx / kChunks) * kChunks;
      buf[u] = reinterpret_cast<const uint4*>(eh + (int64_t)(srcs[u] >> 2) * 144 + kPieceVals * (srcs[u] & 3))[q];
    }
    // the stores use the same clamped indices (a repeated index stores the
    // value its owner stores), so no store is conditional and the loads
    // above stay in flight together
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kE; ++u) le[min(threadIdx.x + u * kWG, ne - 1)] = ev[u];
#pragma unroll
    for (int u = 0; u < kB; ++u) lp[min(threadIdx.x + u * kWG, nb)] = (uint16_t)(bv[u] - k0);
#pragma unroll
    for (int u = 0; u < kFill; ++u) reinterpret_cast<uint4*>(lds)[min(threadIdx.x + u * kWG, nc - 1)] = buf[u];
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < 3 * nb; t += kWG) {
      const uint32_t fl = t / 3;
      const int r = (int)(t - 3 * fl);
      Acc acc[3] = {(Acc)0, (Acc)0, (Acc)0};
      const uint32_t e1 = lp[fl + 1];
      for (uint32_t e = lp[fl]; e < e1; ++e) {
        const uint32_t pe = le[e];
        const In* pv = lds + (pe >> 2) * kPieceVals + 12 * r + 3 * (pe & 3u);
#pragma unroll
        for (int sx = 0; sx < 3; ++sx) acc[sx] += (Acc)pv[sx];
      }
      const int64_t f = (int64_t)f0 + fl;
#pragma unroll
      for (int sx = 0; sx < 3; ++sx) F[(int64_t)(3 * r + sx) * nf + f] = acc[sx];
    }
    __syncthreads();   // the next run refills the shared arrays
  }
}

// Full matrix values (planes of stride vs) from upper blocks U (planes of
// stride us) and src; vals32 != nullptr also receives the values rounded to
// float32 (same pattern and stride).
template <class Acc>
__global__ __launch_bounds__(kWG) void k_fill_vals(const uint32_t* __restrict__ src, int64_t nnz,
                                                   const Acc* __restrict__ U, int64_t us,
                                                   Acc* __restrict__ vals, int64_t vs, float* __restrict__ vals32) {
  const int64_t p = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (p >= nnz) return;
  const uint32_t s = src[p];
  const int64_t u = s >> 1;
  Acc v[9];
  if (s & 1u) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int q = 0; q < 3; ++q) v[3 * r + q] = U[(int64_t)(3 * q + r) * us + u];
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) v[i] = U[(int64_t)i * us + u];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) vals[(int64_t)i * vs + p] = v[i];
  if (vals32) {
#pragma unroll
    for (int i = 0; i < 9; ++i) vals32[(int64_t)i * vs + p] = (float)v[i];
  }
}

// A float32 companion of a float64 matrix: same (borrowed) pattern and stride.
static float* companion32(const Matrix& a, Matrix* out32) {
  if (!out32) return nullptr;
  out32->reserve_values(a.n, a.nnzb, AGC_F32);
  out32->borrow_pattern(a.rp(), a.ci(), a.ri(), a.dg());
  return (float*)out32->vals.p;
}

template <class In, class Acc>
static void launch_gather(agc_context* c, const Mesh& m, const In* eh, Acc* F, hipStream_t st, unsigned grid) {
  // the pieces are copied with 16-byte loads
  const int staged = ((uintptr_t)eh & 15u) == 0 ? 1 : 0;
  k_fine_gather<In, Acc><<<grid, kWG, 0, st>>>(
      eh, (const uint32_t*)m.plan_ptr.p, (const uint32_t*)m.plan.p, (const uint16_t*)m.pentry.p,
      (const uint32_t*)m.piece_src.p, (const uint4*)m.wg_info.p, m.n_wg, m.nf, F, staged);
  AGC_LAUNCH_CHECK();
}

template <class In, class Acc>
static void gather_fine(agc_context* c, const Mesh& m, const void* eh, Acc* F) {
  launch_gather<In, Acc>(c, m, (const In*)eh, F, c->stream, (unsigned)m.n_wg);
}

template <class Acc>
static Acc* fine_upper(agc_context* c, const Mesh& m, const void* eh, int32_t h_dtype) {
  Acc* F = c->ws.get<Acc>(sizeof(Acc) == 8 ? "asm.F64" : "asm.F32", 9 * m.nf);
  if (h_dtype == AGC_F64) gather_fine<double, Acc>(c, m, eh, F);
  else gather_fine<float, Acc>(c, m, eh, F);
  return F;
}

// the float64 fine upper blocks left in the workspace by an earlier gather
static double* upper_ready(agc_context* c, const Mesh& m) { return c->ws.get<double>("asm.F64", 9 * m.nf); }

// The fine matrix borrows the mesh's static pattern (no copy per assembly).
void assemble_fine(agc_context* c, const Mesh& m, const void* eh, int32_t h_dtype, int32_t out_dtype,
                   Matrix& out, Matrix* out32, bool reuse_upper) {
  AGC_REQUIRE(!reuse_upper || out_dtype == AGC_F64, "reused fine blocks are float64");
  AGC_REQUIRE(!out32 || out_dtype == AGC_F64, "a float32 companion needs a float64 matrix");
  const int32_t n = m.n_verts;
  const int64_t nnz = m.ff_nnzb;
  out.reserve_values(n, nnz, out_dtype);
  out.borrow_pattern((const int32_t*)m.ff_row_ptr.p, (const int32_t*)m.ff_col.p, (const int32_t*)m.ff_rowidx.p,
                     (const int32_t*)m.ff_diag.p);
  if (out_dtype == AGC_F64) {
    double* F = reuse_upper ? upper_ready(c, m) : fine_upper<double>(c, m, eh, h_dtype);
    float* v32 = companion32(out, out32);
    k_fill_vals<double><<<blocks_for(nnz, kWG), kWG, 0, c->stream>>>((const uint32_t*)m.ff_src.p, nnz, F, m.nf,
                                                                    (double*)out.vals.p, out.stride, v32);
  } else {
    float* F = fine_upper<float>(c, m, eh, h_dtype);
    k_fill_vals<float><<<blocks_for(nnz, kWG), kWG, 0, c->stream>>>((const uint32_t*)m.ff_src.p, nnz, F, m.nf,
                                                                   (float*)out.vals.p, out.stride, nullptr);
  }
  AGC_LAUNCH_CHECK();
}

// Coarse upper key of every fine upper block; payload f*4 + orient with
// orient 0: B, 1: B^T (the pair lands below the diagonal), 2: B + B^T (an
// off-diagonal fine block inside one aggregate folds onto the diagonal).
__global__ void k_coarse_keys(const int32_t* __restrict__ fr, const int32_t* __restrict__ fc, int64_t nf,
                              const int32_t* __restrict__ map, int32_t n_c, uint64_t* __restrict__ keys,
                              uint32_t* __restrict__ vals, unsigned* err) {
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < nf; f += (int64_t)gridDim.x * blockDim.x) {
    const int i = fr[f], j = fc[f];
    const int ci = map[i], cj = map[j];
    if (ci < 0 || ci >= n_c || cj < 0 || cj >= n_c) {
      atomicOr(err, kErrMap);
      keys[f] = 0;
      vals[f] = (uint32_t)(f * 4);
      continue;
    }
    uint32_t o;
    uint64_t key;
    if (ci < cj) { key = (uint64_t)ci * n_c + cj; o = 0; }
    else if (ci > cj) { key = (uint64_t)cj * n_c + ci; o = 1; }
    else { key = (uint64_t)ci * n_c + ci; o = (i == j) ? 0u : 2u; }
    keys[f] = key;
    vals[f] = (uint32_t)(f * 4) | o;
  }
}

// Upper pair q (0..9) of an element: (0,0) (0,1) (0,2) (0,3) (1,1) (1,2)
// (1,3) (2,2) (2,3) (3,3).
__device__ __forceinline__ void upper_pair(int q, int& a, int& b) {
  a = q < 4 ? 0 : (q < 7 ? 1 : (q < 9 ? 2 : 3));
  b = a + (q < 4 ? q : (q < 7 ? q - 4 : (q < 9 ? q - 7 : 0)));
}

// Coarse upper keys of the per-call elements (contact stencils found anew
// every Newton iteration), item nf + 10 e + q for upper pair q = (a, b) of
// element e: its fine block (v_a, v_b) is sub-block (a, b) of the element
// block, oriented and folded as in k_coarse_keys.  Flags element ids out of
// range or repeated (kErrElem) and map values out of range (kErrMap).
__global__ void k_contact_keys(const int32_t* __restrict__ xv, int64_t nx, int32_t n, const int32_t* __restrict__ map,
                               int32_t n_c, int64_t nf, uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                               unsigned* err) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < 10 * nx; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = t / 10;
    int a, b;
    upper_pair((int)(t - 10 * e), a, b);
    const int32_t va = xv[4 * e + a], vb = xv[4 * e + b];
    const int64_t item = nf + t;
    if (va < 0 || va >= n || vb < 0 || vb >= n || (a != b && va == vb)) {
      atomicOr(err, kErrElem);
      keys[item] = 0;
      vals[item] = (uint32_t)(item * 4);
      continue;
    }
    const int32_t ca = map[va], cb = map[vb];
    if (ca < 0 || ca >= n_c || cb < 0 || cb >= n_c) {
      atomicOr(err, kErrMap);
      keys[item] = 0;
      vals[item] = (uint32_t)(item * 4);
      continue;
    }
    uint32_t o;
    uint64_t key;
    if (ca < cb) { key = (uint64_t)ca * n_c + cb; o = 0; }
    else if (ca > cb) { key = (uint64_t)cb * n_c + ca; o = 1; }
    else { key = (uint64_t)ca * n_c + ca; o = (a == b) ? 0u : 2u; }
    keys[item] = key;
    vals[item] = (uint32_t)(item * 4) | o;
  }
}

template <class Acc>
struct CoarseOp {
  const uint32_t* payload;
  const Acc* F;
  int64_t nf;
  Acc* U;   // planes of stride us
  int64_t us;
  const double* xH;   // per-call element blocks (items nf + 10 e + q), or null
  // every field named at each use: the affine assembly reduces the fine items
  // only, into planes of stride nf
  CoarseOp(const uint32_t* payload_, const Acc* F_, int64_t nf_, Acc* U_, int64_t us_, const double* xH_)
      : payload(payload_), F(F_), nf(nf_), U(U_), us(us_), xH(xH_) {}
  __device__ void load(int64_t k, Acc v[9]) const {
    const uint32_t code = payload[k];
    const int64_t f = code >> 2;
    const uint32_t o = code & 3u;
    Acc b[9];
    if (f < nf) {
#pragma unroll
      for (int i = 0; i < 9; ++i) b[i] = F[(int64_t)i * nf + f];
    } else {
      const int64_t t = f - nf, e = t / 10;
      int pa, pb;
      upper_pair((int)(t - 10 * e), pa, pb);
      const double* h = xH + e * 144 + 36 * pa + 3 * pb;   // rows 3 pa.., columns 3 pb..
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) b[3 * r + q] = (Acc)h[12 * r + q];
    }
    if (o == 0) {
#pragma unroll
      for (int i = 0; i < 9; ++i) v[i] = b[i];
    } else if (o == 1) {
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int s = 0; s < 3; ++s) v[3 * r + s] = b[3 * s + r];
    } else {
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int s = 0; s < 3; ++s) v[3 * r + s] = b[3 * r + s] + b[3 * s + r];
    }
  }
  __device__ void store(int64_t s, const Acc v[9]) const {
#pragma unroll
    for (int i = 0; i < 9; ++i) U[(int64_t)i * us + s] = v[i];
  }
  __device__ void add(int64_t s, const Acc v[9]) const {
#pragma unroll
    for (int i = 0; i < 9; ++i) U[(int64_t)i * us + s] += v[i];
  }
};

template <class Acc>
static void coarse_impl(agc_context* c, const Mesh& m, const void* eh, int32_t h_dtype, const int32_t* map,
                        int32_t n_c, Matrix& out, Matrix* out32, bool reuse_upper, const Contacts& x) {
  const int64_t nf = m.nf;
  const int64_t ni = nf + 10 * x.n;   // items: the fine upper blocks, then the per-call elements' upper pairs
  AGC_REQUIRE(ni < (int64_t(1) << 30), "too many fine blocks and contact pairs");
  Acc* F;
  if constexpr (sizeof(Acc) == 8) F = reuse_upper ? upper_ready(c, m) : fine_upper<Acc>(c, m, eh, h_dtype);
  else F = fine_upper<Acc>(c, m, eh, h_dtype);
  uint64_t* k1 = c->ws.get<uint64_t>("asm.k1", ni);
  uint64_t* k2 = c->ws.get<uint64_t>("asm.k2", ni);
  uint32_t* v1 = c->ws.get<uint32_t>("asm.v1", ni);
  uint32_t* v2 = c->ws.get<uint32_t>("asm.v2", ni);
  err_reset(c);
  k_coarse_keys<<<grid_stride_blocks(nf), kWG, 0, c->stream>>>((const int32_t*)m.fu_row.p, (const int32_t*)m.fu_col.p,
                                                              nf, map, n_c, k1, v1, c->d_err);
  AGC_LAUNCH_CHECK();
  if (x.n > 0) {
    k_contact_keys<<<grid_stride_blocks(10 * x.n), kWG, 0, c->stream>>>(x.verts, x.n, m.n_verts, map, n_c, nf, k1, v1,
                                                                        c->d_err);
    AGC_LAUNCH_CHECK();
  }
  const int nb = bits_for((uint64_t)n_c * (uint64_t)n_c - 1);
  const bool alt = radix_sort_u64(c, k1, v1, k2, v2, ni, nb, "asm.sort");
  uint64_t* sk = alt ? k2 : k1;
  uint32_t* sv = alt ? v2 : v1;
  uint64_t* uk = alt ? k1 : k2;   // free buffer for the unique keys
  Acc* U = c->ws.get<Acc>(sizeof(Acc) == 8 ? "asm.U64" : "asm.U32", 9 * ni);
  CoarseOp<Acc> op(sv, F, nf, U, ni, x.H);
  const int64_t nu = seg_reduce<9, Acc, uint64_t, CoarseOp<Acc>>(c, sk, ni, op, uk, true, "asm.seg");
  int32_t* ur = c->ws.get<int32_t>("asm.ur", nu);
  int32_t* uc = c->ws.get<int32_t>("asm.uc", nu);
  k_split_keys<<<grid_stride_blocks(nu), kWG, 0, c->stream>>>(uk, nu, (uint64_t)n_c, ur, uc);
  AGC_LAUNCH_CHECK();
  // the full pattern has at most 2 nu blocks; the exact count is read back
  out.reserve(n_c, 2 * nu, sizeof(Acc) == 8 ? AGC_F64 : AGC_F32);
  uint32_t* src = c->ws.get<uint32_t>("asm.src", 2 * nu);
  build_full(c, n_c, nu, ur, uc, FullPattern{out.rp(), out.ci(), out.ri(), src, out.dg()}, "asm.full");
  int32_t nnz = 0;
  AGC_HIP(hipMemcpyAsync(&nnz, out.rp() + n_c, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  err_throw(err_fetch(c));
  out.set_nnzb(nnz);
  float* v32 = companion32(out, out32);
  k_fill_vals<Acc><<<blocks_for(nnz, kWG), kWG, 0, c->stream>>>(src, nnz, U, ni, (Acc*)out.vals.p, out.stride, v32);
  AGC_LAUNCH_CHECK();
}

void assemble_coarse(agc_context* c, const Mesh& m, const void* eh, int32_t h_dtype, const int32_t* map,
                     int32_t n_c, int32_t out_dtype, Matrix& out, Matrix* out32, bool reuse_upper,
                     const Contacts& x) {
  AGC_REQUIRE(n_c >= 1 && n_c <= m.n_verts, "n_coarse out of range");
  AGC_REQUIRE(!out32 || out_dtype == AGC_F64, "a float32 companion needs a float64 matrix");
  AGC_REQUIRE(!reuse_upper || (out_dtype == AGC_F64 && h_dtype == AGC_F64), "reused fine blocks are float64");
  AGC_REQUIRE(x.n == 0 || (x.verts && x.H), "contact elements need ids and blocks");
  if (out_dtype == AGC_F64) coarse_impl<double>(c, m, eh, h_dtype, map, n_c, out, out32, reuse_upper, x);
  else coarse_impl<float>(c, m, eh, h_dtype, map, n_c, out, nullptr, false, x);
}

// ------------------------------------------------ affine embedding (Eq. 4)
//
// A fine upper block B of vertices (i, j) adds A_u B' A_w^T to the node pair
// of its vertices, u the vertex in the lower node (new order), w the other,
// B' = B or B^T accordingly (as in the 3-DoF assembly).  With A = Xbar (x) I_3
// the 3x3 sub-block (a, b) of that product is Xbar_u[a] Xbar_w[b] B'; a
// 3-DoF node has the single sub-block a = 3 of weight 1 (supplement Alg. 4
// flattens the same 1 / 4 / 16 sub-blocks).  Fine blocks are sorted by node
// pair with the pairs that touch a 12-DoF node last: the others reduce as in
// the 3-DoF assembly; those in four passes, one per row sub-block a, each
// summing the four column sub-blocks.  The sums are flattened to 3x3 blocks
// at (offset + a, offset + b), the upper blocks sorted, and the full
// symmetric matrix built as before.

// key: bit nb set for a pair with a 12-DoF node; below it lo * n_c + hi (new labels)
__global__ void k_aff_keys(const int32_t* __restrict__ fr, const int32_t* __restrict__ fc, int64_t nf,
                           const int32_t* __restrict__ map, int32_t n_c, const int32_t* __restrict__ newlab,
                           int32_t n3, int nb, uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                           unsigned* err) {
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < nf; f += (int64_t)gridDim.x * blockDim.x) {
    const int32_t i = fr[f], j = fc[f];
    const int32_t mi = map[i], mj = map[j];
    if (mi < 0 || mi >= n_c || mj < 0 || mj >= n_c) {
      atomicOr(err, kErrMap);
      keys[f] = 0;
      vals[f] = (uint32_t)(f * 4);
      continue;
    }
    const int32_t ci = newlab[mi], cj = newlab[mj];
    uint32_t o;
    int32_t lo, hi;
    if (ci < cj) { lo = ci; hi = cj; o = 0; }
    else if (ci > cj) { lo = cj; hi = ci; o = 1; }
    else { lo = hi = ci; o = (i == j) ? 0u : 2u; }
    const uint64_t aff = hi >= n3 ? 1ull : 0ull;
    keys[f] = (aff << nb) | ((uint64_t)lo * (uint64_t)n_c + (uint64_t)hi);
    vals[f] = (uint32_t)(f * 4) | o;
  }
}

// The same keys for the per-call elements' upper pairs (items nf + 10 e + q,
// as in k_contact_keys; vertex pair (v_a, v_b) of upper pair q = (a, b)).
__global__ void k_aff_contact_keys(const int32_t* __restrict__ xv, int64_t nx, int32_t n,
                                   const int32_t* __restrict__ map, int32_t n_c, const int32_t* __restrict__ newlab,
                                   int32_t n3, int nb, int64_t nf, uint64_t* __restrict__ keys,
                                   uint32_t* __restrict__ vals, unsigned* err) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < 10 * nx; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = t / 10;
    int a, b;
    upper_pair((int)(t - 10 * e), a, b);
    const int32_t va = xv[4 * e + a], vb = xv[4 * e + b];
    const int64_t item = nf + t;
    if (va < 0 || va >= n || vb < 0 || vb >= n || (a != b && va == vb)) {
      atomicOr(err, kErrElem);
      keys[item] = 0;
      vals[item] = (uint32_t)(item * 4);
      continue;
    }
    const int32_t mi = map[va], mj = map[vb];
    if (mi < 0 || mi >= n_c || mj < 0 || mj >= n_c) {
      atomicOr(err, kErrMap);
      keys[item] = 0;
      vals[item] = (uint32_t)(item * 4);
      continue;
    }
    const int32_t ci = newlab[mi], cj = newlab[mj];
    uint32_t o;
    int32_t lo, hi;
    if (ci < cj) { lo = ci; hi = cj; o = 0; }
    else if (ci > cj) { lo = cj; hi = ci; o = 1; }
    else { lo = hi = ci; o = (a == b) ? 0u : 2u; }
    const uint64_t aff = hi >= n3 ? 1ull : 0ull;
    keys[item] = (aff << nb) | ((uint64_t)lo * (uint64_t)n_c + (uint64_t)hi);
    vals[item] = (uint32_t)(item * 4) | o;
  }
}

// first position whose key has bit nb set (the caller presets *split = n)
__global__ void k_aff_split(const uint64_t* __restrict__ keys, int64_t n, int nb, int64_t* split) {
  const uint64_t t = 1ull << nb;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    if (keys[k] >= t && (k == 0 || keys[k - 1] < t)) *split = k;
}

__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }

// The sub-blocks (a, 0..3) of one fine block's contribution.
struct AffineOp {
  const uint32_t* payload;   // the affine part of the sorted payloads
  const double* F;           // fine upper blocks, planes [9][nf]
  int64_t nf;
  const int32_t* fr;
  const int32_t* fc;
  const int32_t* map;
  const int32_t* newlab;
  int32_t n3;
  const double* rest;
  const int32_t* rep;        // smallest member of each (canonical) node
  int a;                     // row sub-block of this pass
  double* U;                 // planes [36][us]: 9 b + (3 r + s)
  int64_t us;
  const int32_t* xv;         // per-call elements (items nf + 10 e + q): ids and blocks, or null
  const double* xH;
  // homogeneous rest coordinate in the node's frame (a 3-DoF node: (0, 0, 0, 1))
  __device__ void xbar(int32_t v, bool big, double x[4]) const {
    if (big) {
      const int64_t r = rep[map[v]];
#pragma unroll
      for (int q = 0; q < 3; ++q) x[q] = rest[3 * (int64_t)v + q] - rest[3 * r + q];
    } else {
      x[0] = x[1] = x[2] = 0.0;
    }
    x[3] = 1.0;
  }
  __device__ void load(int64_t k, double v[36]) const {
    const uint32_t code = payload[k];
    const int64_t f = code >> 2;
    const uint32_t o = code & 3u;
    int32_t i, j;
    double b[9], bt[9];
    if (f < nf) {
      i = fr[f];
      j = fc[f];
#pragma unroll
      for (int q = 0; q < 9; ++q) b[q] = F[(int64_t)q * nf + f];
    } else {
      const int64_t t = f - nf, e = t / 10;
      int pa, pb;
      upper_pair((int)(t - 10 * e), pa, pb);
      i = xv[4 * e + pa];
      j = xv[4 * e + pb];
      const double* h = xH + e * 144 + 36 * pa + 3 * pb;
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) b[3 * r + q] = h[12 * r + q];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) bt[3 * r + c] = b[3 * c + r];
    const int32_t ci = newlab[map[i]], cj = newlab[map[j]];
    const int32_t u = (o == 1) ? j : i, w = (o == 1) ? i : j;
    const int32_t cu = (o == 1) ? cj : ci, cw = (o == 1) ? ci : cj;
    double xu[4], xw[4];
    xbar(u, cu >= n3, xu);
    xbar(w, cw >= n3, xw);
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      if (o == 2) {
        // i != j inside one node: (a, b) gets T(a, b) and T(b, a)^T of T = A_i B A_j^T.
        // On the diagonal (b = a) both weights agree: w (B + B^T), formed so that the
        // block is bitwise symmetric (a fused w1 B + w2 B^T would round its two
        // triangles differently).
        const double w1 = xu[a] * xw[bb], w2 = xu[bb] * xw[a];
        if (bb == a) {
#pragma unroll
          for (int q = 0; q < 9; ++q) v[9 * bb + q] = w1 * (b[q] + bt[q]);
        } else {
#pragma unroll
          for (int q = 0; q < 9; ++q) v[9 * bb + q] = w1 * b[q] + w2 * bt[q];
        }
      } else {
        const double w1 = xu[a] * xw[bb];
#pragma unroll
        for (int q = 0; q < 9; ++q) v[9 * bb + q] = w1 * (o == 1 ? bt[q] : b[q]);
      }
    }
  }
  __device__ void store(int64_t s, const double v[36]) const {
#pragma unroll
    for (int q = 0; q < 36; ++q) U[(int64_t)q * us + s] = v[q];
  }
  __device__ void add(int64_t s, const double v[36]) const {
#pragma unroll
    for (int q = 0; q < 36; ++q) U[(int64_t)q * us + s] += v[q];
  }
};

__device__ __forceinline__ int aff_outputs(int32_t lo, int32_t hi, int32_t n3) {
  if (lo < n3) return 4;        // a 3-DoF row node against a 12-DoF node
  return lo == hi ? 10 : 16;    // one 12-DoF node (upper sub-blocks), or two
}

__global__ void k_aff_count_out(const uint64_t* __restrict__ ukeys, int64_t nua, int nb, int32_t n_c, int32_t n3,
                                uint32_t* __restrict__ cnt) {
  const uint64_t mask = (1ull << nb) - 1;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nua; s += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = ukeys[s] & mask;
    cnt[s] = (uint32_t)aff_outputs((int32_t)(key / (uint64_t)n_c), (int32_t)(key % (uint64_t)n_c), n3);
  }
}

// flat upper blocks of the affine pairs, appended after `base` entries
__global__ void k_aff_flatten(const uint64_t* __restrict__ ukeys, int64_t nua, int nb, int32_t n_c, int32_t n3,
                              const uint32_t* __restrict__ pos, const double* __restrict__ U0,
                              const double* __restrict__ U1, const double* __restrict__ U2,
                              const double* __restrict__ U3, int64_t ua_stride, int64_t base, int32_t n_flat,
                              uint64_t* __restrict__ fkeys, double* __restrict__ UC, int64_t uc_stride) {
  const uint64_t mask = (1ull << nb) - 1;
  const int da[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3}, db[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nua; s += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = ukeys[s] & mask;
    const int32_t lo = (int32_t)(key / (uint64_t)n_c), hi = (int32_t)(key % (uint64_t)n_c);
    const int cnt = aff_outputs(lo, hi, n3);
    const int64_t off_lo = lo < n3 ? lo : n3 + 4 * (int64_t)(lo - n3);
    const int64_t off_hi = n3 + 4 * (int64_t)(hi - n3);
    for (int t = 0; t < cnt; ++t) {
      int a, b;
      if (cnt == 4) { a = 3; b = t; }
      else if (cnt == 10) { a = da[t]; b = db[t]; }
      else { a = t >> 2; b = t & 3; }
      const int64_t r = lo < n3 ? off_lo : off_lo + a;
      const int64_t c = off_hi + b;
      const double* U = a == 0 ? U0 : (a == 1 ? U1 : (a == 2 ? U2 : U3));
      const int64_t p = base + pos[s] + t;
      fkeys[p] = (uint64_t)r * (uint64_t)n_flat + (uint64_t)c;
#pragma unroll
      for (int q = 0; q < 9; ++q) UC[(int64_t)q * uc_stride + p] = U[(int64_t)(9 * b + q) * ua_stride + s];
    }
  }
}

// the 3-DoF pairs: flat key (labels are flat) and their sums
__global__ void k_aff_plain(const uint64_t* __restrict__ ukeys, int64_t nu9, int32_t n_c, int32_t n_flat,
                            const double* __restrict__ U9, int64_t u9_stride, uint64_t* __restrict__ fkeys,
                            double* __restrict__ UC, int64_t uc_stride) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nu9; s += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = ukeys[s];
    const uint64_t lo = key / (uint64_t)n_c, hi = key % (uint64_t)n_c;
    fkeys[s] = lo * (uint64_t)n_flat + hi;
#pragma unroll
    for (int q = 0; q < 9; ++q) UC[(int64_t)q * uc_stride + s] = U9[(int64_t)q * u9_stride + s];
  }
}

// sorted flat keys -> (row, col) and the values gathered into sorted order
__global__ void k_aff_sorted(const uint64_t* __restrict__ sk, const uint32_t* __restrict__ perm, int64_t nu,
                             int32_t n_flat, const double* __restrict__ UC, int64_t uc_stride,
                             int32_t* __restrict__ ur, int32_t* __restrict__ uc, double* __restrict__ US) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nu; k += (int64_t)gridDim.x * blockDim.x) {
    ur[k] = (int32_t)(sk[k] / (uint64_t)n_flat);
    uc[k] = (int32_t)(sk[k] % (uint64_t)n_flat);
    const int64_t p = perm[k];
#pragma unroll
    for (int q = 0; q < 9; ++q) US[(int64_t)q * nu + k] = UC[(int64_t)q * uc_stride + p];
  }
}

void assemble_coarse_affine(agc_context* c, const Mesh& m, const double* eh, const AffineMap& am, Matrix& out,
                            Matrix* out32, bool reuse_upper, const Contacts& x) {
  AGC_REQUIRE(x.n == 0 || (x.verts && x.H), "contact elements need ids and blocks");
  const int64_t nf = m.nf;
  const int64_t ni = nf + 10 * x.n;   // items: the fine upper blocks, then the per-call elements' upper pairs
  AGC_REQUIRE(ni < (int64_t(1) << 30), "too many fine blocks and contact pairs");
  const int32_t n_c = am.n_c, n3 = am.n3, n_flat = am.n_flat;
  double* F = reuse_upper ? upper_ready(c, m) : fine_upper<double>(c, m, eh, AGC_F64);
  uint64_t* k1 = c->ws.get<uint64_t>("asm.k1", ni);
  uint64_t* k2 = c->ws.get<uint64_t>("asm.k2", ni);
  uint32_t* v1 = c->ws.get<uint32_t>("asm.v1", ni);
  uint32_t* v2 = c->ws.get<uint32_t>("asm.v2", ni);
  const int nb = bits_for((uint64_t)n_c * (uint64_t)n_c - 1);
  err_reset(c);
  k_aff_keys<<<grid_stride_blocks(nf), kWG, 0, c->stream>>>((const int32_t*)m.fu_row.p, (const int32_t*)m.fu_col.p,
                                                           nf, am.map, n_c, am.newlab, n3, nb, k1, v1, c->d_err);
  AGC_LAUNCH_CHECK();
  if (x.n > 0) {
    k_aff_contact_keys<<<grid_stride_blocks(10 * x.n), kWG, 0, c->stream>>>(x.verts, x.n, m.n_verts, am.map, n_c,
                                                                            am.newlab, n3, nb, nf, k1, v1, c->d_err);
    AGC_LAUNCH_CHECK();
  }
  const bool alt = radix_sort_u64(c, k1, v1, k2, v2, ni, nb + 1, "aasm.sort");
  uint64_t* sk = alt ? k2 : k1;
  uint32_t* sv = alt ? v2 : v1;
  uint64_t* uk = alt ? k1 : k2;   // free buffer for the unique keys
  int64_t* dsplit = c->ws.get<int64_t>("aasm.split", 1);
  k_set_i64<<<1, 1, 0, c->stream>>>(dsplit, ni);
  k_aff_split<<<grid_stride_blocks(ni), kWG, 0, c->stream>>>(sk, ni, nb, dsplit);
  AGC_LAUNCH_CHECK();
  int64_t split = 0;
  AGC_HIP(hipMemcpyAsync(&split, dsplit, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  AGC_HIP(hipStreamSynchronize(c->stream));
  // the 3-DoF pairs
  double* U9 = c->ws.get<double>("aasm.U9", 9 * ni);   // CoarseOp writes planes of stride ni
  int64_t nu9 = 0;
  if (split > 0) {
    CoarseOp<double> op(sv, F, nf, U9, ni, x.H);
    nu9 = seg_reduce<9, double, uint64_t, CoarseOp<double>>(c, sk, split, op, uk, true, "aasm.seg9");
  }
  // the pairs with a 12-DoF node: four passes of four sub-blocks
  const int64_t na = ni - split;
  int64_t nua = 0;
  double* UA[4] = {nullptr, nullptr, nullptr, nullptr};
  uint64_t* uka = c->ws.get<uint64_t>("aasm.uka", na > 0 ? na : 1);
  if (na > 0) {
    for (int a = 0; a < 4; ++a) {
      UA[a] = c->ws.get<double>("aasm.UA" + std::to_string(a), 36 * na);
      AffineOp op{sv + split, F, nf, (const int32_t*)m.fu_row.p, (const int32_t*)m.fu_col.p, am.map, am.newlab,
                  n3, am.rest, am.rep, a, UA[a], na, x.verts, x.H};
      const int64_t cnt = seg_reduce<36, double, uint64_t, AffineOp>(c, sk + split, na, op, a == 0 ? uka : nullptr,
                                                                      a == 0, "aasm.seg36");
      if (a == 0) nua = cnt;
    }
  }
  // flat upper blocks: the 3-DoF ones, then the flattened affine ones
  uint32_t* acnt = c->ws.get<uint32_t>("aasm.acnt", nua + 1);
  int64_t n_aff_out = 0;
  if (nua > 0) {
    k_aff_count_out<<<grid_stride_blocks(nua), kWG, 0, c->stream>>>(uka, nua, nb, n_c, n3, acnt);
    AGC_LAUNCH_CHECK();
    scan_u32(c, acnt, acnt, nua, "aasm.scan");
    uint32_t t = 0;
    AGC_HIP(hipMemcpyAsync(&t, acnt + nua, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    AGC_HIP(hipStreamSynchronize(c->stream));
    n_aff_out = t;
  }
  const int64_t nu = nu9 + n_aff_out;
  AGC_REQUIRE(nu >= 1, "empty coarse pattern");
  uint64_t* fk1 = c->ws.get<uint64_t>("aasm.fk1", nu);
  uint64_t* fk2 = c->ws.get<uint64_t>("aasm.fk2", nu);
  uint32_t* fp1 = c->ws.get<uint32_t>("aasm.fp1", nu);
  uint32_t* fp2 = c->ws.get<uint32_t>("aasm.fp2", nu);
  double* UC = c->ws.get<double>("aasm.UC", 9 * nu);
  if (nu9 > 0) {
    k_aff_plain<<<grid_stride_blocks(nu9), kWG, 0, c->stream>>>(uk, nu9, n_c, n_flat, U9, ni, fk1, UC, nu);
    AGC_LAUNCH_CHECK();
  }
  if (nua > 0) {
    k_aff_flatten<<<grid_stride_blocks(nua), kWG, 0, c->stream>>>(uka, nua, nb, n_c, n3, acnt, UA[0], UA[1], UA[2],
                                                                 UA[3], na, nu9, n_flat, fk1, UC, nu);
    AGC_LAUNCH_CHECK();
  }
  k_iota_u32<<<grid_stride_blocks(nu), kWG, 0, c->stream>>>(fp1, nu);
  AGC_LAUNCH_CHECK();
  const bool falt = radix_sort_u64(c, fk1, fp1, fk2, fp2, nu, bits_for((uint64_t)n_flat * (uint64_t)n_flat - 1),
                                   "aasm.fsort");
  int32_t* ur = c->ws.get<int32_t>("aasm.ur", nu);
  int32_t* ucol = c->ws.get<int32_t>("aasm.uc", nu);
  double* US = c->ws.get<double>("aasm.US", 9 * nu);
  k_aff_sorted<<<grid_stride_blocks(nu), kWG, 0, c->stream>>>(falt ? fk2 : fk1, falt ? fp2 : fp1, nu, n_flat, UC, nu,
                                                             ur, ucol, US);
  AGC_LAUNCH_CHECK();
  out.reserve(n_flat, 2 * nu, AGC_F64);
  uint32_t* src = c->ws.get<uint32_t>("aasm.src", 2 * nu);
  build_full(c, n_flat, nu, ur, ucol, FullPattern{out.rp(), out.ci(), out.ri(), src, out.dg()}, "aasm.full");
  int32_t nnz = 0;
  AGC_HIP(hipMemcpyAsync(&nnz, out.rp() + n_flat, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  err_throw(err_fetch(c));
  out.set_nnzb(nnz);
  float* v32 = companion32(out, out32);
  k_fill_vals<double><<<blocks_for(nnz, kWG), kWG, 0, c->stream>>>(src, nnz, US, nu, (double*)out.vals.p, out.stride,
                                                                   v32);
  AGC_LAUNCH_CHECK();
}

// -------------------------------------------------------- adjoint outer product

__global__ __launch_bounds__(kWG) void k_elem_outer(const int32_t* __restrict__ ev, int64_t ne,
                                                    const double* __restrict__ dg, const double* __restrict__ x,
                                                    double* __restrict__ dh) {
  const int64_t total = 144 * ne;
  for (int64_t idx = (int64_t)blockIdx.x * kWG + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kWG) {
    const int64_t e = idx / 144;
    const int k = (int)(idx - e * 144);
    const int row = k / 12, col = k - 12 * (k / 12);
    const int a = row / 3, r = row - 3 * a, b = col / 3, s = col - 3 * b;
    const int va = ev[4 * e + a], vb = ev[4 * e + b];
    dh[idx] = -dg[3 * (int64_t)va + r] * x[3 * (int64_t)vb + s];
  }
}

void elem_outer_list(agc_context* c, const int32_t* ev, int64_t ne, const double* dg, const double* x, double* dh) {
  if (ne <= 0) return;
  const int64_t total = 144 * ne;
  int64_t b = (total + kWG - 1) / kWG;
  if (b > 262144) b = 262144;
  k_elem_outer<<<(unsigned)b, kWG, 0, c->stream>>>(ev, ne, dg, x, dh);
  AGC_LAUNCH_CHECK();
}

void elem_outer(agc_context* c, const Mesh& m, const double* dg, const double* x, double* dh) {
  elem_outer_list(c, (const int32_t*)m.elem_verts.p, m.n_elems, dg, x, dh);
}

}  // namespace agc
