// BSR 3x3 SpMV and 3x3 block-Jacobi PCG (Alg. overview, solve step;
// Sec. 5.1 "Preconditioners").
//
// SpMV is nonzero-balanced: workgroup w owns blocks [256 w, 256 w + 256), one
// block per thread, whatever the row lengths.  A coarse matrix has one hub
// row per giant aggregate (tens of thousands of blocks) next to rows of ~13,
// so splitting by rows would leave most of the chip idle behind one wave.
// Values are stored as nine planes, so each of the nine loads of a wave is a
// contiguous 512 B (float64) or 256 B (float32) read.  A row is summed by a
// wave64 segmented scan plus a carry across the four waves; a row that
// crosses workgroups leaves one partial per workgroup in `carry`, and the
// consumer adds them in workgroup order.  All reductions have a fixed order,
// so every run gives bitwise identical iterates.
//
// PCG per iteration, three launches:
//   K_a  q = A p and p^T q            (last workgroup: alpha = r^T z / p^T q)
//   K_b  x += alpha p, r -= alpha q, z = D^{-1} r, r^T z, r^T r
//                                     (last workgroup: beta, convergence)
//   K_c  p = z + beta p
// The scalars live in device memory; the host looks at them only every few
// iterations.  Launches after convergence return at once.
#include "internal.h"

namespace agc {

constexpr int kSpmvTile = kWG;   // blocks per workgroup

// ------------------------------------------------------------- SpMV core

// Segmented (by row) sum of one 3-vector per thread over the workgroup.
// Returns the run-inclusive sum in v for every thread.
__device__ __forceinline__ void wg_row_scan(int32_t row, double v[3], int32_t* t_row, int* t_single,
                                            double (*t_v)[3]) {
  const unsigned lane = lane_id(), wave = threadIdx.x / kWave;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int32_t ru = __shfl_up(row, d);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double vu = __shfl_up(v[i], d);
      if (lane >= (unsigned)d && ru == row) v[i] += vu;
    }
  }
  const int32_t row0 = __shfl(row, 0);
  if (lane == kWave - 1) {
    t_row[wave] = row;
    t_single[wave] = (row0 == row) ? 1 : 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) t_v[wave][i] = v[i];
  }
  __syncthreads();
  if (wave > 0 && t_row[wave - 1] == row) {
    double cin[3] = {0.0, 0.0, 0.0};
    for (int u = (int)wave - 1; u >= 0; --u) {
      if (t_row[u] != row) break;
#pragma unroll
      for (int i = 0; i < 3; ++i) cin[i] += t_v[u][i];
      if (!t_single[u]) break;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) v[i] += cin[i];
  }
}

// One tile of y = A x.  Complete rows go to y; rows crossing the tile edge
// go to carry[(w*2 + slot)*3 + i] (slot 1: the row starts in this tile,
// slot 0: it started earlier).  With pdot != nullptr returns, in thread 0,
// the tile's contribution to pdot^T (A x).
template <class T>
__device__ __forceinline__ double spmv_tile(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                            const int32_t* __restrict__ ri, const T* __restrict__ vals,
                                            int64_t nnzb, const double* __restrict__ x, double* __restrict__ y,
                                            double* __restrict__ carry, const double* __restrict__ pdot,
                                            double* red) {
  __shared__ int32_t t_row[kWaves];
  __shared__ int t_single[kWaves];
  __shared__ double t_v[kWaves][3];
  const int64_t w = blockIdx.x;
  const int64_t k = w * kSpmvTile + threadIdx.x;
  const bool valid = k < nnzb;
  int32_t row = INT32_MAX;
  double v[3] = {0.0, 0.0, 0.0};
  if (valid) {
    row = ri[k];
    const int64_t cx = (int64_t)col[k] * 3;
    const double x0 = x[cx], x1 = x[cx + 1], x2 = x[cx + 2];
    double a[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) a[i] = (double)vals[(int64_t)i * nnzb + k];
    v[0] = a[0] * x0 + a[1] * x1 + a[2] * x2;
    v[1] = a[3] * x0 + a[4] * x1 + a[5] * x2;
    v[2] = a[6] * x0 + a[7] * x1 + a[8] * x2;
  }
  wg_row_scan(row, v, t_row, t_single, t_v);
  double d = 0.0;
  if (valid) {
    const int64_t t0 = w * kSpmvTile;
    const int64_t t1 = (t0 + kSpmvTile < nnzb) ? t0 + kSpmvTile : nnzb;
    const bool last = (k == t1 - 1) || (ri[k + 1] != row);
    if (last) {
      const int64_t rs = rp[row], re = rp[row + 1];
      const bool before = rs < t0, after = re > t1;
      if (!before && !after) {
#pragma unroll
        for (int i = 0; i < 3; ++i) y[3 * (int64_t)row + i] = v[i];
      } else {
        const int slot = before ? 0 : 1;
#pragma unroll
        for (int i = 0; i < 3; ++i) carry[(w * 2 + slot) * 3 + i] = v[i];
      }
      if (pdot) d = pdot[3 * (int64_t)row] * v[0] + pdot[3 * (int64_t)row + 1] * v[1] +
                    pdot[3 * (int64_t)row + 2] * v[2];
    }
  }
  if (!pdot) return 0.0;
  return wg_sum(d, red);
}

// q[r] for a row whose blocks may span several tiles.
__device__ __forceinline__ void row_result(const int32_t* __restrict__ rp, const double* __restrict__ y,
                                           const double* __restrict__ carry, int64_t r, double q[3]) {
  const int64_t rs = rp[r], re = rp[r + 1];
  const int64_t w0 = rs / kSpmvTile, w1 = (re - 1) / kSpmvTile;
  if (re <= rs) {
    q[0] = q[1] = q[2] = 0.0;
  } else if (w0 == w1) {
#pragma unroll
    for (int i = 0; i < 3; ++i) q[i] = y[3 * r + i];
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i) q[i] = carry[(w0 * 2 + 1) * 3 + i];
    for (int64_t w = w0 + 1; w <= w1; ++w) {
#pragma unroll
      for (int i = 0; i < 3; ++i) q[i] += carry[(w * 2 + 0) * 3 + i];
    }
  }
}

template <class T>
__global__ __launch_bounds__(kWG) void k_spmv(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                              const int32_t* __restrict__ ri, const T* __restrict__ vals,
                                              int64_t nnzb, const double* __restrict__ x, double* __restrict__ y,
                                              double* __restrict__ carry) {
  __shared__ double red[kWaves];
  (void)spmv_tile<T>(rp, col, ri, vals, nnzb, x, y, carry, nullptr, red);
}

// rows that cross tiles: y[r] = sum of their partials in tile order
__global__ __launch_bounds__(kWG) void k_spmv_fix(const int32_t* __restrict__ rp, int32_t n,
                                                  const double* __restrict__ carry, double* __restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (r >= n) return;
  const int64_t rs = rp[r], re = rp[r + 1];
  if (re <= rs) {
    y[3 * r] = y[3 * r + 1] = y[3 * r + 2] = 0.0;
    return;
  }
  if (rs / kSpmvTile == (re - 1) / kSpmvTile) return;
  double q[3];
  row_result(rp, y, carry, r, q);
#pragma unroll
  for (int i = 0; i < 3; ++i) y[3 * r + i] = q[i];
}

static double* spmv_carry(agc_context* c, const Matrix& a) {
  const int64_t tiles = (a.nnzb + kSpmvTile - 1) / kSpmvTile;
  return c->ws.get<double>("spmv.carry", tiles * 6 + 6);
}

void spmv(agc_context* c, const Matrix& a, const double* x, double* y) {
  if (a.n == 0) return;
  double* carry = spmv_carry(c, a);
  const unsigned tiles = blocks_for(a.nnzb, kSpmvTile);
  if (a.nnzb > 0) {
    if (a.dtype == AGC_F64)
      k_spmv<double><<<tiles, kWG, 0, c->stream>>>(a.rp(), a.ci(), a.ri(), (const double*)a.vals.p, a.nnzb, x, y,
                                                  carry);
    else
      k_spmv<float><<<tiles, kWG, 0, c->stream>>>(a.rp(), a.ci(), a.ri(), (const float*)a.vals.p, a.nnzb, x, y,
                                                 carry);
    AGC_LAUNCH_CHECK();
  }
  k_spmv_fix<<<blocks_for(a.n, kWG), kWG, 0, c->stream>>>(a.rp(), a.n, carry, y);
  AGC_LAUNCH_CHECK();
}

// ------------------------------------------------------- block Jacobi

template <class T>
__global__ __launch_bounds__(kWG) void k_jacobi(const int32_t* __restrict__ diag, const T* __restrict__ vals,
                                                int64_t nnzb, int32_t n, double* __restrict__ dinv,
                                                unsigned* err) {
  const int64_t r = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (r >= n) return;
  const int64_t d = diag[r];
  double m[9];
  bool ok = d >= 0;
  if (ok) {
#pragma unroll
    for (int i = 0; i < 9; ++i) m[i] = (double)vals[(int64_t)i * nnzb + d];
  }
  // Cholesky of the symmetric block (lower triangle read)
  double l00 = 0, l10 = 0, l20 = 0, l11 = 0, l21 = 0, l22 = 0;
  if (ok) {
    const double s0 = m[0];
    ok = s0 > 0.0;
    l00 = sqrt(s0);
    l10 = m[3] / l00;
    l20 = m[6] / l00;
    const double s1 = m[4] - l10 * l10;
    ok = ok && s1 > 0.0;
    l11 = sqrt(s1);
    l21 = (m[7] - l20 * l10) / l11;
    const double s2 = m[8] - l20 * l20 - l21 * l21;
    ok = ok && s2 > 0.0;
    l22 = sqrt(s2);
  }
  double out[9];
  if (ok) {
    const double m00 = 1.0 / l00, m11 = 1.0 / l11, m22 = 1.0 / l22;
    const double m10 = -l10 * m00 * m11;
    const double m21 = -l21 * m11 * m22;
    const double m20 = -(l20 * m00 + l21 * m10) * m22;
    // D^{-1} = L^{-T} L^{-1}; L^{-1} = [[m00,0,0],[m10,m11,0],[m20,m21,m22]]
    out[0] = m00 * m00 + m10 * m10 + m20 * m20;
    out[1] = m10 * m11 + m20 * m21;
    out[2] = m20 * m22;
    out[4] = m11 * m11 + m21 * m21;
    out[5] = m21 * m22;
    out[8] = m22 * m22;
    out[3] = out[1];
    out[6] = out[2];
    out[7] = out[5];
  } else {
    atomicOr(err, d < 0 ? kErrNoDiag : kErrNotSPD);
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i] = 0.0;
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) dinv[(int64_t)i * n + r] = out[i];
}

// ------------------------------------------------------------------ PCG

// Last-workgroup-done reduction: thread 0 of every workgroup publishes its
// partial(s) with a device-coherent store, waits until the store has
// completed, then takes a ticket; the workgroup that takes the final ticket
// reads all partials with device-coherent loads and sums them in index
// order.  A device-scope fence would do the same job but on gfx950 it writes
// back and invalidates the whole L2 of the XCD, once per workgroup.
__device__ __forceinline__ void publish(double* part, int64_t i, double v) {
  __hip_atomic_store(part + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool take_last(uint32_t* ticket, unsigned n_groups) {
  __shared__ bool is_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_s_waitcnt(0);   // thread 0's published partials have completed
    const uint32_t t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    is_last = (t == n_groups - 1);
  }
  __syncthreads();
  return is_last;
}

__device__ __forceinline__ double sum_partials(const double* part, unsigned n, double* red) {
  double s = 0.0;
  for (unsigned i = threadIdx.x; i < n; i += kWG) s += load_agent(part + i);
  return wg_sum(s, red);
}

// Two-level version for grids of thousands of workgroups: a single ticket
// counter would serialise one device-scope atomic per workgroup.  Workgroups
// are grouped by kTicketGroup; the last of each group sums its group's
// partials and takes a ticket on the top counter; the last of those sums the
// group sums.  All sums run in index order.  K values per workgroup, valid in
// thread 0 on entry; on return true, tot[] is valid in thread 0.
constexpr unsigned kTicketGroup = 128;
// Counters sit 256 bytes apart: atomics that share a cache line are
// serialised at the same cache slice even when their addresses differ.
constexpr unsigned kTicketStride = 64;

struct Tickets {
  uint32_t* group;   // [n_groups * kTicketStride], zero between launches
  uint32_t* top;     // [1], zero between launches, on a line of its own
  double* part;      // [K][G]
  double* gpart;     // [K][n_groups]
};

template <int K>
__device__ bool reduce_last(const double (&v)[K], const Tickets& tk, double* red, double (&tot)[K]) {
  __shared__ bool flag;
  const unsigned G = gridDim.x, b = blockIdx.x, g = b / kTicketGroup;
  const unsigned NG = (G + kTicketGroup - 1) / kTicketGroup;
  const unsigned g0 = g * kTicketGroup;
  const unsigned gsize = (G - g0 < kTicketGroup) ? G - g0 : kTicketGroup;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) publish(tk.part, (int64_t)k * G + b, v[k]);
  }
  if (!take_last(tk.group + g * kTicketStride, gsize)) return false;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = (threadIdx.x < gsize) ? load_agent(tk.part + (int64_t)k * G + g0 + threadIdx.x) : 0.0;
    s = wg_sum(s, red);
    if (threadIdx.x == 0) publish(tk.gpart, (int64_t)k * NG + g, s);
  }
  if (threadIdx.x == 0)
    __hip_atomic_store(tk.group + g * kTicketStride, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!take_last(tk.top, NG)) return false;
#pragma unroll
  for (int k = 0; k < K; ++k) tot[k] = sum_partials(tk.gpart + (int64_t)k * NG, NG, red);
  if (threadIdx.x == 0) __hip_atomic_store(tk.top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  (void)flag;
  return true;
}

__device__ __forceinline__ void dinv_apply(const double* __restrict__ dinv, int64_t n, int64_t r, const double v[3],
                                           double z[3]) {
  double m[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) m[i] = dinv[(int64_t)i * n + r];
  z[0] = m[0] * v[0] + m[1] * v[1] + m[2] * v[2];
  z[1] = m[3] * v[0] + m[4] * v[1] + m[5] * v[2];
  z[2] = m[6] * v[0] + m[7] * v[1] + m[8] * v[2];
}

// r = b - q, z = D^{-1} r, p = z; rz, rr, bb
__global__ __launch_bounds__(kWG) void k_pcg_init(const double* __restrict__ b, const double* __restrict__ q,
                                                  const double* __restrict__ dinv, int32_t n, double* __restrict__ r,
                                                  double* __restrict__ z, double* __restrict__ p,
                                                  Tickets tk, PcgState* st, double rtol, int32_t max_iter) {
  __shared__ double red[kWaves];
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  double rz = 0.0, rr = 0.0, bb = 0.0;
  if (i < n) {
    double rv[3], zv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double bk = b[3 * i + k];
      rv[k] = bk - q[3 * i + k];
      bb += bk * bk;
    }
    dinv_apply(dinv, n, i, rv, zv);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      r[3 * i + k] = rv[k];
      z[3 * i + k] = zv[k];
      p[3 * i + k] = zv[k];
      rz += rv[k] * zv[k];
      rr += rv[k] * rv[k];
    }
  }
  const double v[3] = {wg_sum(rz, red), wg_sum(rr, red), wg_sum(bb, red)};
  double tot[3];
  if (!reduce_last<3>(v, tk, red, tot)) return;
  const double trz = tot[0], trr = tot[1], tbb = tot[2];
  if (threadIdx.x == 0) {
    st->rz = trz;
    st->rr = trr;
    st->bb = tbb;
    st->tol2 = rtol * rtol * tbb;
    st->iter = 0;
    st->max_iter = max_iter;
    st->ticket_a = 0;
    st->ticket_b = 0;
    st->ticket_c = 0;
    int done = 0;
    if (!(trr == trr) || !(trz == trz)) done = 3;
    else if (tbb == 0.0 || trr <= st->tol2) done = 1;
    else if (max_iter <= 0) done = 2;
    st->done = done;
  }
}

template <class T>
__global__ __launch_bounds__(kWG) void k_pcg_a(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                               const int32_t* __restrict__ ri, const T* __restrict__ vals,
                                               int64_t nnzb, const double* __restrict__ p, double* __restrict__ q,
                                               double* __restrict__ carry, Tickets tk, PcgState* st) {
  __shared__ double red[kWaves];
  if (st->done) return;
  const double v[1] = {spmv_tile<T>(rp, col, ri, vals, nnzb, p, q, carry, p, red)};
  double tot[1];
  if (!reduce_last<1>(v, tk, red, tot)) return;
  const double pq = tot[0];
  if (threadIdx.x == 0) {
    st->pq = pq;
    if (pq > 0.0 && pq == pq) st->alpha = st->rz / pq;
    else st->done = 3;
  }
}

__global__ __launch_bounds__(kWG) void k_pcg_b(const int32_t* __restrict__ rp, int32_t n,
                                               const double* __restrict__ qy, const double* __restrict__ carry,
                                               const double* __restrict__ dinv, const double* __restrict__ p,
                                               double* __restrict__ x, double* __restrict__ r,
                                               double* __restrict__ z, Tickets tk, PcgState* st) {
  __shared__ double red[kWaves];
  if (st->done) return;
  const double alpha = st->alpha;
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  double rz = 0.0, rr = 0.0;
  if (i < n) {
    double q[3], rv[3], zv[3];
    row_result(rp, qy, carry, i, q);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      x[3 * i + k] += alpha * p[3 * i + k];
      rv[k] = r[3 * i + k] - alpha * q[k];
      r[3 * i + k] = rv[k];
    }
    dinv_apply(dinv, n, i, rv, zv);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      z[3 * i + k] = zv[k];
      rz += rv[k] * zv[k];
      rr += rv[k] * rv[k];
    }
  }
  const double v[2] = {wg_sum(rz, red), wg_sum(rr, red)};
  double tot[2];
  if (!reduce_last<2>(v, tk, red, tot)) return;
  const double trz = tot[0], trr = tot[1];
  if (threadIdx.x == 0) {
    st->beta = trz / st->rz;
    st->rz = trz;
    st->rr = trr;
    st->iter += 1;
    if (!(trr == trr) || !(trz == trz)) st->done = 3;
    else if (trr <= st->tol2) st->done = 1;
    else if (st->iter >= st->max_iter) st->done = 2;
  }
}

__global__ __launch_bounds__(kWG) void k_pcg_c(int64_t n3, const double* __restrict__ z, double* __restrict__ p,
                                               const PcgState* st) {
  if (st->done) return;
  const double beta = st->beta;
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n3) p[i] = z[i] + beta * p[i];
}

int pcg(agc_context* c, const Matrix& a, const double* b, double* x, double rtol, int32_t max_iter, int32_t* iters,
        double* rel) {
  const int32_t n = a.n;
  const int64_t n3 = 3 * (int64_t)n;
  *iters = 0;
  *rel = 0.0;
  if (n == 0) return AGC_OK;
  double* dinv = c->ws.get<double>("pcg.dinv", 9 * (int64_t)n);
  double* r = c->ws.get<double>("pcg.r", n3);
  double* z = c->ws.get<double>("pcg.z", n3);
  double* p = c->ws.get<double>("pcg.p", n3);
  double* q = c->ws.get<double>("pcg.q", n3);
  const unsigned gr = blocks_for(n, kWG);
  const unsigned gs = blocks_for(a.nnzb, kSpmvTile);
  const unsigned gmax = gr > gs ? gr : gs;
  const unsigned ngmax = (gmax + kTicketGroup - 1) / kTicketGroup;
  // one ticket state serves the three kernels: they run one after another and
  // every counter is back at zero when a kernel ends
  const int64_t ncnt = (int64_t)(ngmax + 1) * kTicketStride;
  uint32_t* cnt = c->ws.get<uint32_t>("pcg.tickets", ncnt);
  Tickets tk{cnt, cnt + (int64_t)ngmax * kTicketStride, c->ws.get<double>("pcg.part", 3 * (int64_t)gmax),
             c->ws.get<double>("pcg.gpart", 3 * (int64_t)ngmax)};
  double* carry = spmv_carry(c, a);
  PcgState* st = (PcgState*)c->d_pcg;
  PcgState* hs = (PcgState*)c->h_pcg;

  err_reset(c);
  AGC_HIP(hipMemsetAsync(st, 0, sizeof(PcgState), c->stream));
  AGC_HIP(hipMemsetAsync(cnt, 0, sizeof(uint32_t) * ncnt, c->stream));
  if (a.dtype == AGC_F64)
    k_jacobi<double><<<gr, kWG, 0, c->stream>>>(a.dg(), (const double*)a.vals.p, a.nnzb, n, dinv, c->d_err);
  else
    k_jacobi<float><<<gr, kWG, 0, c->stream>>>(a.dg(), (const float*)a.vals.p, a.nnzb, n, dinv, c->d_err);
  AGC_LAUNCH_CHECK();
  spmv(c, a, x, q);   // q = A x0
  k_pcg_init<<<gr, kWG, 0, c->stream>>>(b, q, dinv, n, r, z, p, tk, st, rtol, max_iter);
  AGC_LAUNCH_CHECK();
  if (err_fetch(c)) return AGC_ERR_NOT_SPD;

  // The host enqueues iterations in chunks and reads the device scalars in
  // between.  The chunk length is the number of iterations the residual's
  // observed geometric decay still needs, so few launches land after
  // convergence (those return at once).
  const bool kt = c->kernel_timing;
  int chunk = 8;
  int64_t launched = 0, chunk_start = 0;
  int prev_it = -1;
  double prev_rr = 0.0;
  for (;;) {
    AGC_HIP(hipMemcpyAsync(hs, st, sizeof(PcgState), hipMemcpyDeviceToHost, c->stream));
    AGC_HIP(hipStreamSynchronize(c->stream));
    if (kt) {
      // SpMV launches that did work: global index < completed iterations
      for (int64_t j = chunk_start; j < launched && j < hs->iter; ++j) {
        float ms = 0.f;
        const int s = (int)(j - chunk_start);
        AGC_HIP(hipEventElapsedTime(&ms, c->kev[2 * s], c->kev[2 * s + 1]));
        c->spmv_ms += ms;
        c->spmv_n += 1;
      }
    }
    if (hs->done) break;
    // the device stops at max_iter; this only guards the host against a lost state
    if (launched > (int64_t)max_iter + 64) throw Error(AGC_ERR_DEVICE, "PCG state did not advance");
    if (prev_it >= 0 && hs->iter > prev_it && hs->rr > 0.0 && hs->rr < prev_rr) {
      const double rate = log(hs->rr / prev_rr) / (double)(hs->iter - prev_it);
      const double remaining = log(hs->tol2 / hs->rr) / rate;
      chunk = remaining < 2.0 ? 2 : (remaining > 256.0 ? 256 : (int)ceil(remaining));
    } else if (prev_it >= 0) {
      chunk = chunk < 32 ? 2 * chunk : 64;
    }
    if (chunk > kMaxChunk) chunk = kMaxChunk;
    prev_it = hs->iter;
    prev_rr = hs->rr;
    chunk_start = launched;
    launched += chunk;
    for (int it = 0; it < chunk; ++it) {
      if (kt) AGC_HIP(hipEventRecord(c->kev[2 * it], c->stream));
      if (a.dtype == AGC_F64)
        k_pcg_a<double><<<gs, kWG, 0, c->stream>>>(a.rp(), a.ci(), a.ri(), (const double*)a.vals.p, a.nnzb, p, q,
                                                   carry, tk, st);
      else
        k_pcg_a<float><<<gs, kWG, 0, c->stream>>>(a.rp(), a.ci(), a.ri(), (const float*)a.vals.p, a.nnzb, p, q,
                                                  carry, tk, st);
      if (kt) AGC_HIP(hipEventRecord(c->kev[2 * it + 1], c->stream));
      k_pcg_b<<<gr, kWG, 0, c->stream>>>(a.rp(), n, q, carry, dinv, p, x, r, z, tk, st);
      k_pcg_c<<<blocks_for(n3, kWG), kWG, 0, c->stream>>>(n3, z, p, st);
    }
    AGC_LAUNCH_CHECK();
  }
  *iters = hs->iter;
  if (hs->bb == 0.0) {
    AGC_HIP(hipMemsetAsync(x, 0, sizeof(double) * n3, c->stream));
    *rel = 0.0;
    return AGC_OK;
  }
  *rel = sqrt(hs->rr / hs->bb);
  if (hs->done == 1) return AGC_OK;
  if (hs->done == 2) return AGC_ERR_NOT_CONVERGED;
  return AGC_ERR_NOT_SPD;
}

// ------------------------------------------------------ vector helpers

__global__ __launch_bounds__(kWG) void k_sq_part(const double* __restrict__ v, int64_t n, double* __restrict__ part) {
  __shared__ double red[kWaves];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG) s += v[i] * v[i];
  s = wg_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kWG) void k_sum_part(const double* __restrict__ part, unsigned n, double* __restrict__ out) {
  __shared__ double red[kWaves];
  double s = 0.0;
  for (unsigned i = threadIdx.x; i < n; i += kWG) s += part[i];
  s = wg_sum(s, red);
  if (threadIdx.x == 0) *out = s;
}

double norm2(agc_context* c, const double* v, int64_t n3, const std::string& tag) {
  const unsigned G = 1024;
  double* part = c->ws.get<double>(tag + ".part", G + 1);
  k_sq_part<<<G, kWG, 0, c->stream>>>(v, n3, part);
  k_sum_part<<<1, kWG, 0, c->stream>>>(part, G, part + G);
  AGC_LAUNCH_CHECK();
  double h = 0.0;
  AGC_HIP(hipMemcpyAsync(&h, part + G, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  AGC_HIP(hipStreamSynchronize(c->stream));
  return sqrt(h);
}

__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}

void axpy_vec(agc_context* c, double* y, const double* x, double a, int64_t n3) {
  int64_t b = (n3 + kWG - 1) / kWG;
  if (b > 65536) b = 65536;
  k_axpy<<<(unsigned)(b < 1 ? 1 : b), kWG, 0, c->stream>>>(y, x, a, n3);
  AGC_LAUNCH_CHECK();
}

}  // namespace agc
