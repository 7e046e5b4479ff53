// BSR 3x3 SpMV and 3x3 block-Jacobi PCG (Alg. overview, solve step;
// Sec. 5.1 "Preconditioners").
//
// SpMV is nonzero-balanced: workgroup w owns blocks [1024 w, 1024 w + 1024),
// four consecutive blocks per thread, whatever the row lengths.  A coarse
// matrix has one hub row per giant aggregate (tens of thousands of blocks)
// next to rows of ~13, so splitting by rows would leave most of the chip
// idle behind one wave.  Values are stored as nine planes (stride padded to
// 64 blocks), so a thread's four values of one plane are one 16- or 32-byte
// load and a wave's loads are contiguous.  Rows are summed inside a thread in
// order, then across threads by a wave64 segmented scan plus a carry across
// the four waves; a row that crosses workgroups leaves one partial per
// workgroup in `carry`, and the consumer adds them in workgroup order.
//
// PCG, two launches per iteration j (plus one tiny check per chunk):
//   K_a  reduce K_b's partials -> r^T z, r^T r; stop test; beta_j;
//        p_j = z + beta_j p_{j-1} formed on the fly from z and the previous p
//        (ping-pong buffers; the thread holding a row's diagonal block stores
//        p_j for that row); q = A p_j; partial p_j^T q per workgroup.
//   K_b  reduce K_a's partials -> p_j^T q, alpha_j; x += alpha p_j,
//        r -= alpha q, z = D^{-1} r; partial r^T z, r^T r per workgroup.
// No atomics and no fences: every workgroup of a kernel sums all partials
// of the previous kernel in the same fixed order (the kernel boundary makes
// them visible), so every workgroup takes the same decisions and every run
// gives bitwise identical iterates.  The host reads the scalars only
// between chunks of iterations; launches after convergence return at once.
#include "internal.h"

namespace agc {

constexpr int kItems = 4;
constexpr int kTile = kWG * kItems;   // blocks per SpMV workgroup

// ------------------------------------------------------------ loads

__device__ __forceinline__ void load4(const int32_t* p, int32_t o[4]) {
  const int4 v = *reinterpret_cast<const int4*>(p);
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void load4(const float* p, double o[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void load4(const double* p, double o[4]) {
  const double2 a = reinterpret_cast<const double2*>(p)[0];
  const double2 b = reinterpret_cast<const double2*>(p)[1];
  o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}

// The vector the SpMV multiplies: x itself, or p = z + beta p_old.
struct GatherX {
  const double* x;
  __device__ __forceinline__ void get(int64_t c, double o[3]) const {
    o[0] = x[3 * c];
    o[1] = x[3 * c + 1];
    o[2] = x[3 * c + 2];
  }
};
struct GatherP {
  const double* z;
  const double* p;
  double beta;
  __device__ __forceinline__ void get(int64_t c, double o[3]) const {
#pragma unroll
    for (int i = 0; i < 3; ++i) o[i] = z[3 * c + i] + beta * p[3 * c + i];
  }
};

// ------------------------------------------------------------- SpMV core

// Segmented (by key) inclusive sum of one 3-vector per thread over the
// workgroup, keys non-decreasing in thread order.
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

// One tile of y = A g.  Complete rows go to y; rows crossing the tile edge go
// to carry[(w*2 + slot)*3 + i] (slot 1: the row starts in this tile, slot 0:
// it started earlier).  Only the first and the last row of a tile can cross
// its edges, and the two neighbouring row indices tell which do.
// PNEW: the thread holding the diagonal block of a row stores the gathered
// vector of that row to pnew.  DOT: returns, in thread 0, the tile's part of
// g^T (A g), summed block by block.
template <class T, class G, bool DOT, bool PNEW>
__device__ __forceinline__ double spmv_tile(const int32_t* __restrict__ ri, const int32_t* __restrict__ col,
                                            const T* __restrict__ vals, int64_t nnzb, int64_t stride, const G& g,
                                            double* __restrict__ y, double* __restrict__ carry,
                                            double* __restrict__ pnew, double* red) {
  __shared__ int32_t t_row[kWaves];
  __shared__ int t_single[kWaves];
  __shared__ double t_v[kWaves][3];
  __shared__ int32_t w_row[kWaves];
  __shared__ double w_s[kWaves][3];
  __shared__ int32_t edge[2];   // row continuing from the previous tile / into the next one, or -1
  const int64_t w = blockIdx.x;
  const int64_t t0 = w * kTile;
  const int64_t t1 = (t0 + kTile < nnzb) ? t0 + kTile : nnzb;
  const int64_t k0 = t0 + (int64_t)threadIdx.x * kItems;
  if (threadIdx.x == 0) {
    const int32_t first = ri[t0];
    edge[0] = (t0 > 0 && ri[t0 - 1] == first) ? first : -1;
    const int32_t last = ri[t1 - 1];
    edge[1] = (t1 < nnzb && ri[t1] == last) ? last : -1;
  }
  const int64_t kn = k0 + kItems;
  const int32_t next_row = (kn < t1) ? ri[kn] : INT32_MAX;
  int32_t r[kItems], c[kItems];
  double v[kItems][3];
  double dot = 0.0;
  if (t0 + kTile <= nnzb) {
    double a[9][kItems];
    load4(ri + k0, r);
    load4(col + k0, c);
#pragma unroll
    for (int i = 0; i < 9; ++i) load4(vals + (int64_t)i * stride + k0, a[i]);
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      double xv[3];
      g.get(c[j], xv);
      v[j][0] = a[0][j] * xv[0] + a[1][j] * xv[1] + a[2][j] * xv[2];
      v[j][1] = a[3][j] * xv[0] + a[4][j] * xv[1] + a[5][j] * xv[2];
      v[j][2] = a[6][j] * xv[0] + a[7][j] * xv[1] + a[8][j] * xv[2];
      if (PNEW && c[j] == r[j]) {
#pragma unroll
        for (int i = 0; i < 3; ++i) pnew[3 * (int64_t)r[j] + i] = xv[i];
      }
      if (DOT) {
        double pr[3];
        g.get(r[j], pr);
        dot += pr[0] * v[j][0] + pr[1] * v[j][1] + pr[2] * v[j][2];
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int64_t k = k0 + j;
      if (k < nnzb) {
        r[j] = ri[k];
        c[j] = col[k];
        double a[9], xv[3];
#pragma unroll
        for (int i = 0; i < 9; ++i) a[i] = (double)vals[(int64_t)i * stride + k];
        g.get(c[j], xv);
        v[j][0] = a[0] * xv[0] + a[1] * xv[1] + a[2] * xv[2];
        v[j][1] = a[3] * xv[0] + a[4] * xv[1] + a[5] * xv[2];
        v[j][2] = a[6] * xv[0] + a[7] * xv[1] + a[8] * xv[2];
        if (PNEW && c[j] == r[j]) {
#pragma unroll
          for (int i = 0; i < 3; ++i) pnew[3 * (int64_t)r[j] + i] = xv[i];
        }
        if (DOT) {
          double pr[3];
          g.get(r[j], pr);
          dot += pr[0] * v[j][0] + pr[1] * v[j][1] + pr[2] * v[j][2];
        }
      } else {
        r[j] = INT32_MAX;
        c[j] = 0;
        v[j][0] = v[j][1] = v[j][2] = 0.0;
      }
    }
  }
  // the thread's last run, scanned across threads
  const int32_t head = r[0], tail = r[kItems - 1];
  double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < kItems; ++j)
    if (r[j] == tail) {
#pragma unroll
      for (int i = 0; i < 3; ++i) s[i] += v[j][i];
    }
  wg_row_scan(tail, s, t_row, t_single, t_v);
  const unsigned lane = lane_id(), wave = threadIdx.x / kWave;
  int32_t prev_tail = __shfl_up(tail, 1);
  double prev_s[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) prev_s[i] = __shfl_up(s[i], 1);
  if (lane == kWave - 1) {
    w_row[wave] = tail;
#pragma unroll
    for (int i = 0; i < 3; ++i) w_s[wave][i] = s[i];
  }
  __syncthreads();
  if (lane == 0) {
    if (wave > 0) {
      prev_tail = w_row[wave - 1];
#pragma unroll
      for (int i = 0; i < 3; ++i) prev_s[i] = w_s[wave - 1][i];
    } else {
      prev_tail = INT32_MIN;
    }
  }
  const int32_t e_before = edge[0], e_after = edge[1];
  double acc[3] = {0.0, 0.0, 0.0};
  if (prev_tail == head) {
#pragma unroll
    for (int i = 0; i < 3; ++i) acc[i] = prev_s[i];
  }
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
#pragma unroll
    for (int i = 0; i < 3; ++i) acc[i] += v[j][i];
    const int32_t nr = (j + 1 < kItems) ? r[j + 1] : next_row;
    if (nr != r[j]) {
      const int32_t row = r[j];
      if (row != INT32_MAX) {
        const bool before = row == e_before, after = row == e_after;
        if (!before && !after) {
#pragma unroll
          for (int i = 0; i < 3; ++i) y[3 * (int64_t)row + i] = acc[i];
        } else {
          const int slot = before ? 0 : 1;
#pragma unroll
          for (int i = 0; i < 3; ++i) carry[(w * 2 + slot) * 3 + i] = acc[i];
        }
      }
      acc[0] = acc[1] = acc[2] = 0.0;
    }
  }
  if (!DOT) return 0.0;
  return wg_sum(dot, red);
}

// q[r] for a row whose blocks may span several tiles.
__device__ __forceinline__ void row_result(const int32_t* __restrict__ rp, const double* __restrict__ y,
                                           const double* __restrict__ carry, int64_t r, double q[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) q[i] = y[3 * r + i];   // issued with the row pointers; used unless split
  const int64_t rs = rp[r], re = rp[r + 1];
  const int64_t w0 = rs / kTile, w1 = (re - 1) / kTile;
  if (re <= rs) {
    q[0] = q[1] = q[2] = 0.0;
  } else if (w0 != w1) {
#pragma unroll
    for (int i = 0; i < 3; ++i) q[i] = carry[(w0 * 2 + 1) * 3 + i];
    for (int64_t w = w0 + 1; w <= w1; ++w) {
#pragma unroll
      for (int i = 0; i < 3; ++i) q[i] += carry[(w * 2 + 0) * 3 + i];
    }
  }
}

template <class T>
__global__ __launch_bounds__(kWG) void k_spmv(const int32_t* __restrict__ col, const int32_t* __restrict__ ri,
                                              const T* __restrict__ vals, int64_t nnzb, int64_t stride,
                                              const double* __restrict__ x, double* __restrict__ y,
                                              double* __restrict__ carry) {
  __shared__ double red[kWaves];
  (void)spmv_tile<T, GatherX, false, false>(ri, col, vals, nnzb, stride, GatherX{x}, y, carry, nullptr, red);
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
  if (rs / kTile == (re - 1) / kTile) return;
  double q[3];
  row_result(rp, y, carry, r, q);
#pragma unroll
  for (int i = 0; i < 3; ++i) y[3 * r + i] = q[i];
}

static double* spmv_carry(agc_context* c, const Matrix& a) {
  const int64_t tiles = (a.nnzb + kTile - 1) / kTile;
  return c->ws.get<double>("spmv.carry", tiles * 6 + 6);
}

void spmv(agc_context* c, const Matrix& a, const double* x, double* y) {
  if (a.n == 0) return;
  double* carry = spmv_carry(c, a);
  const unsigned tiles = blocks_for(a.nnzb, kTile);
  if (a.nnzb > 0) {
    if (a.dtype == AGC_F64)
      k_spmv<double><<<tiles, kWG, 0, c->stream>>>(a.ci(), a.ri(), (const double*)a.vals.p, a.nnzb, a.stride, x, y,
                                                  carry);
    else
      k_spmv<float><<<tiles, kWG, 0, c->stream>>>(a.ci(), a.ri(), (const float*)a.vals.p, a.nnzb, a.stride, x, y,
                                                 carry);
    AGC_LAUNCH_CHECK();
  }
  k_spmv_fix<<<blocks_for(a.n, kWG), kWG, 0, c->stream>>>(a.rp(), a.n, carry, y);
  AGC_LAUNCH_CHECK();
}

// ------------------------------------------------------- block Jacobi

template <class T>
__global__ __launch_bounds__(kWG) void k_jacobi(const int32_t* __restrict__ diag, const T* __restrict__ vals,
                                                int64_t stride, int32_t n, double* __restrict__ dinv,
                                                unsigned* err) {
  const int64_t r = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (r >= n) return;
  const int64_t d = diag[r];
  double m[9];
  bool ok = d >= 0;
  if (ok) {
#pragma unroll
    for (int i = 0; i < 9; ++i) m[i] = (double)vals[(int64_t)i * stride + d];
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

// Sums K rows of per-workgroup partials part[k][0..G) in a fixed order and
// gives every thread the totals.
template <int K>
__device__ __forceinline__ void all_sum(const double* __restrict__ part, unsigned G, double* red, double* bc,
                                        double (&tot)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (unsigned i = threadIdx.x; i < G; i += kWG) s += part[(int64_t)k * G + i];
    s = wg_sum(s, red);
    if (threadIdx.x == 0) bc[k] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) tot[k] = bc[k];
}

// The stop test on the scalars of iteration j (r^T z, r^T r, and at j = 0
// also b^T b): returns the done code.  Every workgroup computes the same.
__device__ __forceinline__ int stop_code(int64_t j, double rz, double rr, double bb, double tol2, int32_t max_iter) {
  if (!(rr == rr) || !(rz == rz)) return 3;
  if ((j == 0 && bb == 0.0) || rr <= tol2) return 1;
  if (j >= max_iter) return 2;
  return 0;
}

// partials of the update kernels: [3][G_rows] = r^T z, r^T r, b^T b (init only)
__device__ __forceinline__ void iteration_scalars(int64_t j, const double* pb, unsigned gb, PcgState* st, double rtol,
                                                  double* red, double* bc, int* done_out, double* rz_out,
                                                  double* beta_out) {
  double t[3];
  all_sum<3>(pb, gb, red, bc, t);
  const double rz = t[0], rr = t[1];
  double tol2;
  if (j == 0) {
    tol2 = rtol * rtol * t[2];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->bb = t[2];
      st->tol2 = tol2;
    }
  } else {
    tol2 = st->tol2;
  }
  const int done = stop_code(j, rz, rr, t[2], tol2, st->max_iter);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->iter = (int32_t)j;
    st->rr = rr;
    st->rz_hist[j & 1] = rz;
    if (done) st->done = done;
  }
  *done_out = done;
  *rz_out = rz;
  *beta_out = (j == 0) ? 0.0 : rz / st->rz_hist[(j - 1) & 1];
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

// r = b - q, z = D^{-1} r, p_old = 0; partials of r^T z, r^T r, b^T b
__global__ __launch_bounds__(kWG) void k_pcg_init(const double* __restrict__ b, const double* __restrict__ q,
                                                  const double* __restrict__ dinv, int32_t n, double* __restrict__ r,
                                                  double* __restrict__ z, double* __restrict__ p_old,
                                                  double* __restrict__ pb) {
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
      p_old[3 * i + k] = 0.0;
      rz += rv[k] * zv[k];
      rr += rv[k] * rv[k];
    }
  }
  const unsigned G = gridDim.x;
  rz = wg_sum(rz, red);
  rr = wg_sum(rr, red);
  bb = wg_sum(bb, red);
  if (threadIdx.x == 0) {
    pb[blockIdx.x] = rz;
    pb[G + blockIdx.x] = rr;
    pb[2 * G + blockIdx.x] = bb;
  }
}

template <class T>
__global__ __launch_bounds__(kWG) void k_pcg_a(int64_t j, const int32_t* __restrict__ col,
                                               const int32_t* __restrict__ ri, const T* __restrict__ vals,
                                               int64_t nnzb, int64_t stride, const double* __restrict__ z,
                                               const double* __restrict__ p_old, double* __restrict__ p_new,
                                               double* __restrict__ q, double* __restrict__ carry,
                                               const double* __restrict__ pb, unsigned gb, double* __restrict__ pa,
                                               PcgState* st, double rtol) {
  __shared__ double red[kWaves];
  __shared__ double bc[3];
  if (st->done) return;
  int done;
  double rz, beta;
  iteration_scalars(j, pb, gb, st, rtol, red, bc, &done, &rz, &beta);
  if (done) return;
  const GatherP g{z, p_old, beta};
  const double d = spmv_tile<T, GatherP, true, true>(ri, col, vals, nnzb, stride, g, q, carry, p_new, red);
  if (threadIdx.x == 0) pa[blockIdx.x] = d;
}

__global__ __launch_bounds__(kWG) void k_pcg_b(int64_t j, const int32_t* __restrict__ rp, int32_t n,
                                               const double* __restrict__ qy, const double* __restrict__ carry,
                                               const double* __restrict__ dinv, const double* __restrict__ p,
                                               double* __restrict__ x, double* __restrict__ r,
                                               double* __restrict__ z, const double* __restrict__ pa, unsigned ga,
                                               double* __restrict__ pb, PcgState* st) {
  __shared__ double red[kWaves];
  __shared__ double bc[1];
  if (st->done) return;
  double pq[1];
  all_sum<1>(pa, ga, red, bc, pq);
  if (!(pq[0] > 0.0)) {   // p^T A p <= 0 or NaN: not SPD (every workgroup sees the same value)
    if (blockIdx.x == 0 && threadIdx.x == 0) st->done = 3;
    return;
  }
  const double alpha = st->rz_hist[j & 1] / pq[0];
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
  const unsigned G = gridDim.x;
  rz = wg_sum(rz, red);
  rr = wg_sum(rr, red);
  if (threadIdx.x == 0) {
    pb[blockIdx.x] = rz;
    pb[G + blockIdx.x] = rr;
    pb[2 * G + blockIdx.x] = 0.0;
  }
}

// The stop test of iteration j alone (one workgroup), run at the end of a chunk.
__global__ __launch_bounds__(kWG) void k_pcg_check(int64_t j, const double* __restrict__ pb, unsigned gb,
                                                   PcgState* st, double rtol) {
  __shared__ double red[kWaves];
  __shared__ double bc[3];
  if (st->done) return;
  int done;
  double rz, beta;
  iteration_scalars(j, pb, gb, st, rtol, red, bc, &done, &rz, &beta);
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
  double* pp[2] = {c->ws.get<double>("pcg.p0", n3), c->ws.get<double>("pcg.p1", n3)};
  double* q = c->ws.get<double>("pcg.q", n3);
  const unsigned gr = blocks_for(n, kWG);
  const unsigned gs = blocks_for(a.nnzb, kTile);
  double* pb = c->ws.get<double>("pcg.pb", 3 * (int64_t)gr);
  double* pa = c->ws.get<double>("pcg.pa", gs);
  double* carry = spmv_carry(c, a);
  PcgState* st = (PcgState*)c->d_pcg;
  PcgState* hs = (PcgState*)c->h_pcg;
  *hs = PcgState{};
  hs->max_iter = max_iter;
  AGC_HIP(hipMemcpyAsync(st, hs, sizeof(PcgState), hipMemcpyHostToDevice, c->stream));

  err_reset(c);
  if (a.dtype == AGC_F64)
    k_jacobi<double><<<gr, kWG, 0, c->stream>>>(a.dg(), (const double*)a.vals.p, a.stride, n, dinv, c->d_err);
  else
    k_jacobi<float><<<gr, kWG, 0, c->stream>>>(a.dg(), (const float*)a.vals.p, a.stride, n, dinv, c->d_err);
  AGC_LAUNCH_CHECK();
  spmv(c, a, x, q);   // q = A x0
  // iteration j reads p_{j-1} from pp[(j+1)%2] and writes p_j to pp[j%2]
  k_pcg_init<<<gr, kWG, 0, c->stream>>>(b, q, dinv, n, r, z, pp[1], pb);
  AGC_LAUNCH_CHECK();
  k_pcg_check<<<1, kWG, 0, c->stream>>>(0, pb, gr, st, rtol);
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
    for (int it = 0; it < chunk; ++it) {
      const int64_t j = launched + it;
      const double* p_old = pp[(j + 1) & 1];
      double* p_new = pp[j & 1];
      if (kt) AGC_HIP(hipEventRecord(c->kev[2 * it], c->stream));
      if (a.dtype == AGC_F64)
        k_pcg_a<double><<<gs, kWG, 0, c->stream>>>(j, a.ci(), a.ri(), (const double*)a.vals.p, a.nnzb, a.stride, z,
                                                   p_old, p_new, q, carry, pb, gr, pa, st, rtol);
      else
        k_pcg_a<float><<<gs, kWG, 0, c->stream>>>(j, a.ci(), a.ri(), (const float*)a.vals.p, a.nnzb, a.stride, z,
                                                  p_old, p_new, q, carry, pb, gr, pa, st, rtol);
      if (kt) AGC_HIP(hipEventRecord(c->kev[2 * it + 1], c->stream));
      k_pcg_b<<<gr, kWG, 0, c->stream>>>(j, a.rp(), n, q, carry, dinv, p_new, x, r, z, pa, gs, pb, st);
    }
    launched += chunk;
    k_pcg_check<<<1, kWG, 0, c->stream>>>(launched, pb, gr, st, rtol);
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
