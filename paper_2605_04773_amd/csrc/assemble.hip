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
  m.ff_col.ensure(sizeof(int32_t) * 2 * m.nf);
  m.ff_rowidx.ensure(sizeof(int32_t) * 2 * m.nf);
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

  AGC_HIP(hipStreamSynchronize(c->stream));
}

// ------------------------------------------------------- per-step assembly

// F[3r+s][f] = sum over the plan of f of entry (r, s) of element sub-block
// (a, b), in plan order.  Three threads per fine block, one per row r: each
// reads three contiguous values per plan entry, and the loop is unrolled so
// that the loads of several entries are in flight together (the sums keep
// plan order).
constexpr int kGatherUnroll = 4;
template <class In, class Acc>
__global__ __launch_bounds__(kWG) void k_fine_gather(const In* __restrict__ eh, const uint32_t* __restrict__ pptr,
                                                     const uint32_t* __restrict__ plan, int64_t nf,
                                                     Acc* __restrict__ F) {
  const int64_t t = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (t >= 3 * nf) return;
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
static void gather_fine(agc_context* c, const Mesh& m, const void* eh, Acc* F) {
  k_fine_gather<In, Acc><<<blocks_for(3 * m.nf, kWG), kWG, 0, c->stream>>>(
      (const In*)eh, (const uint32_t*)m.plan_ptr.p, (const uint32_t*)m.plan.p, m.nf, F);
  AGC_LAUNCH_CHECK();
}

template <class Acc>
static Acc* fine_upper(agc_context* c, const Mesh& m, const void* eh, int32_t h_dtype) {
  Acc* F = c->ws.get<Acc>(sizeof(Acc) == 8 ? "asm.F64" : "asm.F32", 9 * m.nf);
  if (h_dtype == AGC_F64) gather_fine<double, Acc>(c, m, eh, F);
  else gather_fine<float, Acc>(c, m, eh, F);
  return F;
}

// The fine matrix borrows the mesh's static pattern (no copy per assembly).
void assemble_fine(agc_context* c, const Mesh& m, const void* eh, int32_t h_dtype, int32_t out_dtype,
                   Matrix& out, Matrix* out32) {
  AGC_REQUIRE(!out32 || out_dtype == AGC_F64, "a float32 companion needs a float64 matrix");
  const int32_t n = m.n_verts;
  const int64_t nnz = m.ff_nnzb;
  out.reserve_values(n, nnz, out_dtype);
  out.borrow_pattern((const int32_t*)m.ff_row_ptr.p, (const int32_t*)m.ff_col.p, (const int32_t*)m.ff_rowidx.p,
                     (const int32_t*)m.ff_diag.p);
  if (out_dtype == AGC_F64) {
    double* F = fine_upper<double>(c, m, eh, h_dtype);
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

template <class Acc>
struct CoarseOp {
  const uint32_t* payload;
  const Acc* F;
  int64_t nf;
  Acc* U;   // planes of stride nf
  __device__ void load(int64_t k, Acc v[9]) const {
    const uint32_t code = payload[k];
    const int64_t f = code >> 2;
    const uint32_t o = code & 3u;
    Acc b[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) b[i] = F[(int64_t)i * nf + f];
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
    for (int i = 0; i < 9; ++i) U[(int64_t)i * nf + s] = v[i];
  }
  __device__ void add(int64_t s, const Acc v[9]) const {
#pragma unroll
    for (int i = 0; i < 9; ++i) U[(int64_t)i * nf + s] += v[i];
  }
};

template <class Acc>
static void coarse_impl(agc_context* c, const Mesh& m, const void* eh, int32_t h_dtype, const int32_t* map,
                        int32_t n_c, Matrix& out, Matrix* out32) {
  const int64_t nf = m.nf;
  Acc* F = fine_upper<Acc>(c, m, eh, h_dtype);
  uint64_t* k1 = c->ws.get<uint64_t>("asm.k1", nf);
  uint64_t* k2 = c->ws.get<uint64_t>("asm.k2", nf);
  uint32_t* v1 = c->ws.get<uint32_t>("asm.v1", nf);
  uint32_t* v2 = c->ws.get<uint32_t>("asm.v2", nf);
  err_reset(c);
  k_coarse_keys<<<grid_stride_blocks(nf), kWG, 0, c->stream>>>((const int32_t*)m.fu_row.p, (const int32_t*)m.fu_col.p,
                                                              nf, map, n_c, k1, v1, c->d_err);
  AGC_LAUNCH_CHECK();
  const int nb = bits_for((uint64_t)n_c * (uint64_t)n_c - 1);
  const bool alt = radix_sort_u64(c, k1, v1, k2, v2, nf, nb, "asm.sort");
  uint64_t* sk = alt ? k2 : k1;
  uint32_t* sv = alt ? v2 : v1;
  uint64_t* uk = alt ? k1 : k2;   // free buffer for the unique keys
  Acc* U = c->ws.get<Acc>(sizeof(Acc) == 8 ? "asm.U64" : "asm.U32", 9 * nf);
  CoarseOp<Acc> op{sv, F, nf, U};
  const int64_t nu = seg_reduce<9, Acc, uint64_t, CoarseOp<Acc>>(c, sk, nf, op, uk, true, "asm.seg");
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
  k_fill_vals<Acc><<<blocks_for(nnz, kWG), kWG, 0, c->stream>>>(src, nnz, U, nf, (Acc*)out.vals.p, out.stride, v32);
  AGC_LAUNCH_CHECK();
}

void assemble_coarse(agc_context* c, const Mesh& m, const void* eh, int32_t h_dtype, const int32_t* map,
                     int32_t n_c, int32_t out_dtype, Matrix& out, Matrix* out32) {
  AGC_REQUIRE(n_c >= 1 && n_c <= m.n_verts, "n_coarse out of range");
  AGC_REQUIRE(!out32 || out_dtype == AGC_F64, "a float32 companion needs a float64 matrix");
  if (out_dtype == AGC_F64) coarse_impl<double>(c, m, eh, h_dtype, map, n_c, out, out32);
  else coarse_impl<float>(c, m, eh, h_dtype, map, n_c, out, nullptr);
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

void elem_outer(agc_context* c, const Mesh& m, const double* dg, const double* x, double* dh) {
  const int64_t total = 144 * m.n_elems;
  int64_t b = (total + kWG - 1) / kWG;
  if (b > 262144) b = 262144;
  k_elem_outer<<<(unsigned)b, kWG, 0, c->stream>>>((const int32_t*)m.elem_verts.p, m.n_elems, dg, x, dh);
  AGC_LAUNCH_CHECK();
}

}  // namespace agc
