// BSR 3x3 SpMV and 3x3 block-Jacobi PCG (Alg. overview, solve step;
// Sec. 5.1 "Preconditioners").
//
// SpMV is nonzero-balanced: workgroup w owns a tile of consecutive blocks
// (two per thread for a float64 matrix, four for float32: 512 or 1024 per
// tile), whatever the row lengths.  A coarse
// matrix has one hub row per giant aggregate (tens of thousands of blocks)
// next to rows of ~13, so splitting by rows would leave most of the chip
// idle behind one wave.  Values are stored as nine planes (stride padded to
// 64 blocks), so a thread's values of one plane are one or two 16-byte loads
// and a wave's loads are contiguous.  Rows are summed inside a thread in
// order, then across the threads of a wave by a DPP segmented scan, then
// across the four waves through LDS (one barrier per tile).  A row that
// crosses workgroups leaves one partial per workgroup in `carry`, and the
// consumer adds them in workgroup order.
//
// PCG in its single-reduction form (Chronopoulos and Gear): besides p it
// carries s = A p, so that both inner products of an iteration, gamma =
// r^T z and delta = z^T A z, are known before any vector changes, and the
// only vector the SpMV gathers is z.  In exact arithmetic the iterates are
// those of standard PCG.  z = D^{-1} r, r, p and s are stored in the
// matrix's value type: with a float32 matrix (the inner solve of the mixed
// path, which only has to reach a loose tolerance before float64
// refinement) the SpMV gathers 12 bytes per column instead of 24 and the
// update moves 72 bytes per row less; each stored vector is rounded once and
// used as stored, while x, A z and every inner product stay float64.  Two
// launches per iteration j (plus one tiny check per chunk):
//   K_1  w = A z_j and a partial z_j^T w per workgroup.
//   K_2  reduce the partials -> gamma_j, r_j^T r_j, delta_j; stop test;
//        beta_j = gamma_j / gamma_{j-1},
//        alpha_j = gamma_j / (delta_j - beta_j gamma_j / alpha_{j-1});
//        p = z + beta p, s = w + beta s, x += alpha p, r -= alpha s,
//        z = D^{-1} r; partial gamma_{j+1}, r^T r per workgroup.
// No atomics and no fences: every workgroup of a kernel sums all partials
// of the previous kernels in the same fixed order (the kernel boundary makes
// them visible), so every workgroup takes the same decisions and every run
// gives bitwise identical iterates.  Both kernels issue their loads of the
// matrix and vectors before that reduction, so its latency overlaps them.
// The host reads the scalars only between chunks of iterations; launches
// after convergence read one flag and return.
#include "internal.h"

namespace agc {

// Consecutive blocks per SpMV thread, by value type (a multiple of 2); a
// workgroup's tile is kWG times that.  Two float64 blocks per thread keep the
// kernel at 76 VGPRs (six waves per SIMD) instead of 120 (four): measured
// 160 instead of 193 us per launch on the 10.4 M-block coarse matrix of the
// 128^3 grid, and 416 instead of 504 us on its fine matrix.
#ifndef AGC_SPMV_ITEMS_F64
#define AGC_SPMV_ITEMS_F64 2
#endif
#ifndef AGC_SPMV_ITEMS_F32
#define AGC_SPMV_ITEMS_F32 4
#endif
#ifndef AGC_SPMV_NT_F64
#define AGC_SPMV_NT_F64 1
#endif
#ifndef AGC_SPMV_NT_F32
#define AGC_SPMV_NT_F32 1
#endif
template <class T>
struct Shape {
  static constexpr int items = sizeof(T) == 8 ? AGC_SPMV_ITEMS_F64 : AGC_SPMV_ITEMS_F32;
  static constexpr bool nt = sizeof(T) == 8 ? AGC_SPMV_NT_F64 : AGC_SPMV_NT_F32;
  static constexpr int64_t tile = (int64_t)kWG * items;
  static_assert(items % 2 == 0, "blocks per thread: a multiple of 2");
};
inline int64_t tile_of(int32_t dtype) { return dtype == AGC_F64 ? Shape<double>::tile : Shape<float>::tile; }

// ------------------------------------------------------------ loads

// Matrix loads stream.  With the non-temporal hint they do not push the
// gathered vectors out of L2; per value type (NT = the Shape's nt), since
// it was measured faster for the float32 matrix and slower for the float64
// one (whose larger stream fills the queues either way).
typedef int32_t vi4 __attribute__((ext_vector_type(4)));
typedef int32_t vi2 __attribute__((ext_vector_type(2)));
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef float vf2 __attribute__((ext_vector_type(2)));
typedef double vd2 __attribute__((ext_vector_type(2)));
template <bool NT, class V>
__device__ __forceinline__ V stream_load(const V* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT>
__device__ __forceinline__ void load4(const int32_t* p, int32_t o[4]) {
  const vi4 v = stream_load<NT>(reinterpret_cast<const vi4*>(p));
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
template <bool NT>
__device__ __forceinline__ void load4(const float* p, float o[4]) {
  const vf4 v = stream_load<NT>(reinterpret_cast<const vf4*>(p));
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
template <bool NT>
__device__ __forceinline__ void load4(const double* p, double o[4]) {
  const vd2 a = stream_load<NT>(reinterpret_cast<const vd2*>(p));
  const vd2 b = stream_load<NT>(reinterpret_cast<const vd2*>(p) + 1);
  o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}
template <bool NT>
__device__ __forceinline__ void load2(const int32_t* p, int32_t o[2]) {
  const vi2 v = stream_load<NT>(reinterpret_cast<const vi2*>(p));
  o[0] = v.x; o[1] = v.y;
}
template <bool NT>
__device__ __forceinline__ void load2(const float* p, float o[2]) {
  const vf2 v = stream_load<NT>(reinterpret_cast<const vf2*>(p));
  o[0] = v.x; o[1] = v.y;
}
template <bool NT>
__device__ __forceinline__ void load2(const double* p, double o[2]) {
  const vd2 a = stream_load<NT>(reinterpret_cast<const vd2*>(p));
  o[0] = a.x; o[1] = a.y;
}

// I consecutive values: I / 4 four-wide loads, then a two-wide one if I % 4 == 2
template <bool NT, class T, int I>
__device__ __forceinline__ void load_items(const T* p, T (&o)[I]) {
#pragma unroll
  for (int h = 0; h < I / 4; ++h) load4<NT>(p + 4 * h, o + 4 * h);
  if constexpr (I % 4 == 2) load2<NT>(p + 4 * (I / 4), o + 4 * (I / 4));
}

// The vector the SpMV multiplies, stored in V (double, or float for the
// preconditioned vector of the float32-matrix PCG).
template <class V>
struct Gather {
  using E = V;   // gathered values stay in the vector's type until used
  const V* x;
  __device__ __forceinline__ void get(int64_t c, V o[3]) const {
    o[0] = x[3 * c];
    o[1] = x[3 * c + 1];
    o[2] = x[3 * c + 2];
  }
};
using GatherX = Gather<double>;

// ------------------------------------------------------------- SpMV core

// A thread's four blocks, loaded before anything that needs a scalar from
// the previous kernel.  Blocks past nnzb carry row INT32_MAX and column 0.
template <class T>
struct Quad {
  static constexpr int kItems = Shape<T>::items;
  int32_t r[kItems], c[kItems];
  T a[9][kItems];
  int32_t next_row;   // row of the block after the thread's last one; INT32_MAX at the tile end
  int32_t edge[4];    // ri[t0 - 1], ri[t0], ri[t1 - 1], ri[t1] (-1 where absent); the same in every thread
};

// A thread's rows and columns (and the tile's edge rows)...  The pattern
// arrays hold at least plane_stride(nnzb) + 4 entries and the values nine
// planes of plane_stride(nnzb) plus 4 spare entries per plane, so the four
// blocks from any k0 < nnzb can be loaded whole; a thread past
// the end loads block 0, and blocks at or past nnzb are masked (row
// INT32_MAX, column 0; their values are whatever the padding holds, and the
// SpMV zeroes their products).  No load sits under a branch, so the wait for
// the indices is the only one before the gathers are issued.
template <class T>
__device__ __forceinline__ void load_quad_index(int64_t w, const int32_t* __restrict__ ri,
                                                const int32_t* __restrict__ col, int64_t nnzb, Quad<T>& q) {
  constexpr int kItems = Shape<T>::items;
  constexpr int64_t kTile = Shape<T>::tile;
  const int64_t t0 = w * kTile;
  const int64_t t1 = (t0 + kTile < nnzb) ? t0 + kTile : nnzb;
  const int64_t k0 = t0 + (int64_t)threadIdx.x * kItems;
  const int64_t kl = k0 < nnzb ? k0 : 0;
  int32_t r4[kItems], c4[kItems];
  load_items<Shape<T>::nt>(ri + kl, r4);
  load_items<Shape<T>::nt>(col + kl, c4);
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const bool in = k0 + j < nnzb;
    q.r[j] = in ? r4[j] : INT32_MAX;
    q.c[j] = in ? c4[j] : 0;
  }
  const int64_t kn = k0 + kItems;
  const int32_t nr = ri[kn < t1 ? kn : t0];
  q.next_row = kn < t1 ? nr : INT32_MAX;
  // uniform across the workgroup
  const int32_t before = ri[t0 > 0 ? t0 - 1 : 0], after = ri[t1 < nnzb ? t1 : t1 - 1];
  q.edge[0] = t0 > 0 ? before : -1;
  q.edge[1] = ri[t0];
  q.edge[2] = ri[t1 - 1];
  q.edge[3] = t1 < nnzb ? after : -1;
}

// ...and its nine value planes.
template <class T>
__device__ __forceinline__ void load_quad_vals(int64_t w, const T* __restrict__ vals, int64_t nnzb, int64_t stride,
                                               Quad<T>& q) {
  constexpr int kItems = Shape<T>::items;
  const int64_t k0 = w * Shape<T>::tile + (int64_t)threadIdx.x * kItems;
  const int64_t kl = k0 < nnzb ? k0 : 0;
#pragma unroll
  for (int i = 0; i < 9; ++i) load_items<Shape<T>::nt>(vals + (int64_t)i * stride + kl, q.a[i]);
  // the loads above are issued before the gathers that follow
  __builtin_amdgcn_sched_barrier(0);
}

template <class T>
__device__ __forceinline__ void load_quad(int64_t w, const int32_t* __restrict__ ri, const int32_t* __restrict__ col,
                                          const T* __restrict__ vals, int64_t nnzb, int64_t stride, Quad<T>& q) {
  load_quad_index(w, ri, col, nnzb, q);
  load_quad_vals(w, vals, nnzb, stride, q);
}

struct TileLds {
  int32_t row[kWaves];      // key of lane 63 of each wave
  int32_t single[kWaves];   // 1 if that key's run reaches back to lane 0 whole
  double v[kWaves][3];      // lane 63's scanned sums
  double dot[kWaves];
  int32_t edge[2];          // row continuing from the previous tile / into the next one, or -1
};

// One tile of y = A g from a loaded quad.  Complete rows go to y; rows
// crossing the tile edge go to carry[(w*2 + slot)*3 + i] (slot 1: the row
// starts in this tile, slot 0: it started earlier).  Only the first and the
// last row of a tile can cross its edges.
// DOT: returns, in every thread, the tile's part of g^T (A g) (each block's
// product dotted with its row's g, in block order per thread, then lanes,
// then waves).
template <class T, class G, bool DOT>
__device__ __forceinline__ double spmv_tile(int64_t w, const Quad<T>& q, const G& g, double* __restrict__ y,
                                            double* __restrict__ carry, TileLds& L) {
  constexpr int kItems = Shape<T>::items;
  const unsigned lane = lane_id(), wave = threadIdx.x / kWave;
  double v[kItems][3];
  double dot = 0.0;
  using E = typename G::E;
  E pr0[3] = {E(0), E(0), E(0)}, pr3[3] = {E(0), E(0), E(0)};
  if (DOT) {   // gathered unconditionally (a masked row reads entry 0), with the columns
    const int32_t r0 = q.r[0] != INT32_MAX ? q.r[0] : 0;
    const int32_t r3 = q.r[kItems - 1] != INT32_MAX ? q.r[kItems - 1] : r0;
    g.get(r0, pr0);
    g.get(r3, pr3);
  }
  E xg[kItems][3];
#pragma unroll
  for (int j = 0; j < kItems; ++j) g.get(q.c[j], xg[j]);
  // all gathers are in flight before any product is formed: left to itself
  // the scheduler interleaves them with the arithmetic, one round trip each
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const double xv[3] = {(double)xg[j][0], (double)xg[j][1], (double)xg[j][2]};
    const bool in = q.r[j] != INT32_MAX;   // a masked block's values may be padding
    const double v0 = (double)q.a[0][j] * xv[0] + (double)q.a[1][j] * xv[1] + (double)q.a[2][j] * xv[2];
    const double v1 = (double)q.a[3][j] * xv[0] + (double)q.a[4][j] * xv[1] + (double)q.a[5][j] * xv[2];
    const double v2 = (double)q.a[6][j] * xv[0] + (double)q.a[7][j] * xv[1] + (double)q.a[8][j] * xv[2];
    v[j][0] = in ? v0 : 0.0;
    v[j][1] = in ? v1 : 0.0;
    v[j][2] = in ? v2 : 0.0;
  }
  if (DOT) {
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int32_t rj = q.r[j];
      if (rj == INT32_MAX) continue;
      E pr[3];
      if (rj == q.r[0]) {
#pragma unroll
        for (int i = 0; i < 3; ++i) pr[i] = pr0[i];
      } else if (rj == q.r[kItems - 1]) {
#pragma unroll
        for (int i = 0; i < 3; ++i) pr[i] = pr3[i];
      } else {
        g.get(rj, pr);
      }
      dot += (double)pr[0] * v[j][0] + (double)pr[1] * v[j][1] + (double)pr[2] * v[j][2];
    }
  }
  // the thread's last run, scanned across the wave, then across waves
  const int32_t head = q.r[0], tail = q.r[kItems - 1];
  double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int j = 0; j < kItems; ++j)
    if (q.r[j] == tail) {
#pragma unroll
      for (int i = 0; i < 3; ++i) s[i] += v[j][i];
    }
  wave_seg_scan<3>(tail, s);
  double d1[1] = {dot};
  if (DOT) wave_seg_scan<1>(0, d1);
  const int32_t tail0 = __builtin_amdgcn_readfirstlane(tail);   // lane 0 is active
  if (lane == kWave - 1) {
    L.row[wave] = tail;
    L.single[wave] = (tail0 == tail) ? 1 : 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) L.v[wave][i] = s[i];
    if (DOT) L.dot[wave] = d1[0];
  }
  if (threadIdx.x == 0) {
    L.edge[0] = (q.edge[0] == q.edge[1]) ? q.edge[1] : -1;
    L.edge[1] = (q.edge[3] == q.edge[2]) ? q.edge[2] : -1;
  }
  __syncthreads();
  // carry into this wave: the previous waves' sums of row R = key of the
  // previous wave's lane 63, walking back while that row fills whole waves
  int32_t R = INT32_MIN;
  double cin[3] = {0.0, 0.0, 0.0};
  if (wave > 0) {
    R = L.row[wave - 1];
    for (int u = (int)wave - 1; u >= 0; --u) {
      if (L.row[u] != R) break;
#pragma unroll
      for (int i = 0; i < 3; ++i) cin[i] += L.v[u][i];
      if (!L.single[u]) break;
    }
  }
  if (tail == R) {
#pragma unroll
    for (int i = 0; i < 3; ++i) s[i] += cin[i];
  }
  // exclusive value for the head row: lane i-1's scanned tail, (R, cin) for lane 0
  const int32_t prev_row = dpp_move<kDppWaveShr1, 0xf>(R, tail);
  double acc[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double ps = dpp_move<kDppWaveShr1, 0xf>(cin[i], s[i]);
    acc[i] = (prev_row == head) ? ps : 0.0;
  }
  const int32_t e_before = L.edge[0], e_after = L.edge[1];
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
#pragma unroll
    for (int i = 0; i < 3; ++i) acc[i] += v[j][i];
    const int32_t nr = (j + 1 < kItems) ? q.r[j + 1] : q.next_row;
    if (nr != q.r[j]) {
      const int32_t row = q.r[j];
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
  double t = 0.0;
#pragma unroll
  for (int u = 0; u < kWaves; ++u) t += L.dot[u];
  return t;
}

constexpr int kCarryBatch = 16;

// q = y[r] corrected for a row whose blocks may span several tiles (rs, re:
// its block range): then q is the last partial of its first tile plus the
// first partials of the later ones, added in tile order.
__device__ __forceinline__ void row_fix(int64_t rs, int64_t re, const double* __restrict__ carry, double q[3],
                                        int64_t kTile) {
  const int64_t w0 = rs / kTile, w1 = (re - 1) / kTile;
  if (re <= rs) {
    q[0] = q[1] = q[2] = 0.0;
  } else if (w0 != w1) {
    // a hub row spans dozens of tiles: the carries are loaded kCarryBatch at a time
#pragma unroll
    for (int i = 0; i < 3; ++i) q[i] = carry[(w0 * 2 + 1) * 3 + i];
    for (int64_t w = w0 + 1; w <= w1; w += kCarryBatch) {
      double h[kCarryBatch][3];
#pragma unroll
      for (int u = 0; u < kCarryBatch; ++u) {
#pragma unroll
        for (int i = 0; i < 3; ++i) h[u][i] = w + u <= w1 ? carry[((w + u) * 2 + 0) * 3 + i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kCarryBatch; ++u) {
        if (w + u <= w1) {
#pragma unroll
          for (int i = 0; i < 3; ++i) q[i] += h[u][i];
        }
      }
    }
  }
}

// row_fix for the 64 rows of a wave at once; every lane of the wave calls it
// (in: the lane has a row).  A row over two tiles adds its one carry on its
// own lane, as row_fix does.  The carries of a longer (hub) row are loaded by
// the whole wave, 64 per round, and summed across the lanes in a fixed
// order: per lane in tile order, then by a butterfly.  Few registers are
// live, so the rare hub row does not lower the occupancy of the caller.
__device__ __forceinline__ void row_fix_wave(bool in, int64_t rs, int64_t re, const double* __restrict__ carry,
                                             double q[3], int64_t kTile) {
  const int32_t w0 = (int32_t)(rs / kTile), w1 = (int32_t)((re - 1) / kTile);
  if (in && re <= rs) q[0] = q[1] = q[2] = 0.0;
  const bool split = in && re > rs && w0 != w1;
  if (split) {
#pragma unroll
    for (int i = 0; i < 3; ++i) q[i] = carry[((int64_t)w0 * 2 + 1) * 3 + i];
    if (w1 == w0 + 1) {
#pragma unroll
      for (int i = 0; i < 3; ++i) q[i] += carry[((int64_t)w1 * 2 + 0) * 3 + i];
    }
  }
  uint64_t hub = __ballot(split && w1 > w0 + 1);
  const int lane = (int)(threadIdx.x & 63);
  while (hub) {
    const int src = __ffsll((unsigned long long)hub) - 1;
    hub &= hub - 1;
    const int32_t a = __shfl(w0, src) + 1, b = __shfl(w1, src);
    double h[3] = {0.0, 0.0, 0.0};
    for (int32_t w = a + lane; w <= b; w += 64) {
#pragma unroll
      for (int i = 0; i < 3; ++i) h[i] += carry[((int64_t)w * 2 + 0) * 3 + i];
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
#pragma unroll
      for (int i = 0; i < 3; ++i) h[i] += __shfl_xor(h[i], d);
    }
    if (lane == src) {
#pragma unroll
      for (int i = 0; i < 3; ++i) q[i] += h[i];
    }
  }
}

// q[r] for a row whose blocks may span several tiles.
__device__ __forceinline__ void row_result(const int32_t* __restrict__ rp, const double* __restrict__ y,
                                           const double* __restrict__ carry, int64_t r, double q[3], int64_t kTile) {
#pragma unroll
  for (int i = 0; i < 3; ++i) q[i] = y[3 * r + i];   // issued with the row pointers; used unless split
  row_fix(rp[r], rp[r + 1], carry, q, kTile);
}

template <class T>
__global__ __launch_bounds__(kWG) void k_spmv(const int32_t* __restrict__ col, const int32_t* __restrict__ ri,
                                              const T* __restrict__ vals, int64_t nnzb, int64_t stride,
                                              const double* __restrict__ x, double* __restrict__ y,
                                              double* __restrict__ carry) {
  __shared__ TileLds L;
  const int64_t w = xcd_block();
  Quad<T> q;
  load_quad(w, ri, col, vals, nnzb, stride, q);
  (void)spmv_tile<T, GatherX, false>(w, q, GatherX{x}, y, carry, L);
}

// rows that cross tiles: y[r] = sum of their partials in tile order
template <class T>
__global__ __launch_bounds__(kWG) void k_spmv_fix(const int32_t* __restrict__ rp, int32_t n,
                                                  const double* __restrict__ carry, double* __restrict__ y) {
  constexpr int64_t kTile = Shape<T>::tile;
  const int64_t r = (int64_t)blockIdx.x * kWG + threadIdx.x;
  if (r >= n) return;
  const int64_t rs = rp[r], re = rp[r + 1];
  if (re <= rs) {
    y[3 * r] = y[3 * r + 1] = y[3 * r + 2] = 0.0;
    return;
  }
  if (rs / kTile == (re - 1) / kTile) return;
  double q[3];
  row_result(rp, y, carry, r, q, kTile);
#pragma unroll
  for (int i = 0; i < 3; ++i) y[3 * r + i] = q[i];
}

static double* spmv_carry(agc_context* c, const Matrix& a) {
  const int64_t tiles = (a.nnzb + tile_of(a.dtype) - 1) / tile_of(a.dtype);
  return c->ws.get<double>("spmv.carry", tiles * 6 + 6);
}

void spmv(agc_context* c, const Matrix& a, const double* x, double* y) {
  if (a.n == 0) return;
  double* carry = spmv_carry(c, a);
  const unsigned tiles = blocks_for(a.nnzb, tile_of(a.dtype));
  if (a.nnzb > 0) {
    if (a.dtype == AGC_F64)
      k_spmv<double><<<tiles, kWG, 0, c->stream>>>(a.ci(), a.ri(), (const double*)a.vals.p, a.nnzb, a.stride, x, y,
                                                  carry);
    else
      k_spmv<float><<<tiles, kWG, 0, c->stream>>>(a.ci(), a.ri(), (const float*)a.vals.p, a.nnzb, a.stride, x, y,
                                                 carry);
    AGC_LAUNCH_CHECK();
  }
  if (a.dtype == AGC_F64) k_spmv_fix<double><<<blocks_for(a.n, kWG), kWG, 0, c->stream>>>(a.rp(), a.n, carry, y);
  else k_spmv_fix<float><<<blocks_for(a.n, kWG), kWG, 0, c->stream>>>(a.rp(), a.n, carry, y);
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
  // D^{-1} is symmetric: six planes 00, 01, 02, 11, 12, 22
  dinv[0 * (int64_t)n + r] = out[0];
  dinv[1 * (int64_t)n + r] = out[1];
  dinv[2 * (int64_t)n + r] = out[2];
  dinv[3 * (int64_t)n + r] = out[4];
  dinv[4 * (int64_t)n + r] = out[5];
  dinv[5 * (int64_t)n + r] = out[8];
}

// ------------------------------------------------------------------ PCG

// Per-workgroup partials are stored in rows of part_stride(G) doubles (G
// rounded up to even), so that a row can be read with 16-byte loads: lane t
// of batch m reads entries 2 (m kWG + t) and the one after.  part_sum is this
// thread's share of the fixed-order sum of a row; part_load issues the first
// kPartBatch loads in one go, so that a kernel can issue them before its
// other loads and add them (part_finish) while those are in flight.  A lane
// past the end reads a valid pair elsewhere in the row (rather than every
// such lane hitting entry 0) and masks it.
constexpr int kPartBatch = 2;
__host__ __device__ inline int64_t part_stride(int64_t G) { return (G + 1) & ~(int64_t)1; }
__device__ __forceinline__ void part_load(const double* __restrict__ part, unsigned G, vd2 (&v)[kPartBatch]) {
#pragma unroll
  for (int m = 0; m < kPartBatch; ++m) {
    const unsigned e = 2 * (m * kWG + threadIdx.x);
    const unsigned ec = e < G ? e : (e % G) & ~1u;
    const vd2 q = *reinterpret_cast<const vd2*>(part + ec);
    v[m].x = e < G ? q.x : 0.0;
    v[m].y = e + 1 < G ? q.y : 0.0;
  }
}
__device__ __forceinline__ double part_finish(const double* __restrict__ part, unsigned G,
                                              const vd2 (&v)[kPartBatch]) {
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < kPartBatch; ++m) {
    s += v[m].x;
    s += v[m].y;
  }
  for (unsigned e = 2 * (kPartBatch * kWG + threadIdx.x); e < G; e += 2 * kWG) {
    s += part[e];
    if (e + 1 < G) s += part[e + 1];
  }
  return s;
}
__device__ __forceinline__ double part_sum(const double* __restrict__ part, unsigned G) {
  vd2 v[kPartBatch];
  part_load(part, G, v);
  return part_finish(part, G, v);
}

// Sums K rows of per-workgroup partials part[k][0..G) (row stride
// part_stride(G)) in a fixed order and gives every thread the totals (one
// barrier; lds holds K * kWaves doubles).
template <int K>
__device__ __forceinline__ void all_sum(const double* __restrict__ part, unsigned G, double* lds, double (&tot)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) tot[k] = part_sum(part + (int64_t)k * part_stride(G), G);
  wg_sum_all<K>(tot, lds);
}

// The stop test on the scalars of iteration j (r^T z, r^T r, and at j = 0
// also b^T b): returns the done code.  Every workgroup computes the same.
__device__ __forceinline__ int stop_code(int64_t j, double rz, double rr, double bb, double tol2, int32_t max_iter) {
  if (!(rr == rr) || !(rz == rz)) return 3;
  if ((j == 0 && bb == 0.0) || rr <= tol2) return 1;
  if (j >= max_iter) return 2;
  return 0;
}

// The scalars an iteration reads from the device state, read together when
// a kernel starts: read after a barrier, they would add a round trip to the
// kernel's critical path.
struct StateIn {
  int32_t done, max_iter;
  double tol2, rz_prev, alpha_prev;   // the last two: of iteration j - 1 (unused at j = 0)
};
__device__ __forceinline__ StateIn read_state(const PcgState* st, int64_t j) {
  StateIn s;
  s.done = st->done;
  s.max_iter = st->max_iter;
  s.tol2 = st->tol2;
  s.rz_prev = st->rz_hist[(j - 1) & 1];
  s.alpha_prev = st->alpha_hist[(j - 1) & 1];
  return s;
}

// The stop test of iteration j on the totals t of the update partials
// (gamma_j, r_j^T r_j, b^T b at j = 0); block 0 records the scalars.  Every
// workgroup computes the same.
__device__ __forceinline__ int stop_scalars(int64_t j, const double* t, PcgState* st, const StateIn& in,
                                            double rtol) {
  double tol2;
  if (j == 0) {
    tol2 = rtol * rtol * t[2];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->bb = t[2];
      st->tol2 = tol2;
    }
  } else {
    tol2 = in.tol2;
  }
  const int done = stop_code(j, t[0], t[1], t[2], tol2, in.max_iter);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->iter = (int32_t)j;
    st->rr = t[1];
    st->rr_ring[j % kRrRing] = t[1];
    if (done) st->done = done;
  }
  return done;
}

// the six distinct entries of a row's D^{-1} block: 00, 01, 02, 11, 12, 22
__device__ __forceinline__ void load_dinv(const double* __restrict__ dinv, int64_t n, int64_t r, double m[6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) m[i] = dinv[(int64_t)i * n + r];
}
__device__ __forceinline__ void apply3(const double m[6], const double v[3], double z[3]) {
  z[0] = m[0] * v[0] + m[1] * v[1] + m[2] * v[2];
  z[1] = m[1] * v[0] + m[3] * v[1] + m[4] * v[2];
  z[2] = m[2] * v[0] + m[4] * v[1] + m[5] * v[2];
}

// r = b - q (q == nullptr: x0 = 0, r = b, and x is zeroed here), z = D^{-1} r
// (stored as Z), p = s = 0; partials of gamma_0, r^T r, b^T b
template <class Z>
__global__ __launch_bounds__(kWG) void k_pcg_init(const double* __restrict__ b, const double* __restrict__ q,
                                                  const double* __restrict__ dinv, int32_t n, double* __restrict__ x,
                                                  Z* __restrict__ r, Z* __restrict__ z,
                                                  Z* __restrict__ p, Z* __restrict__ sv,
                                                  double* __restrict__ pb) {
  __shared__ double lds[3 * kWaves];
  const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
  double t[3] = {0.0, 0.0, 0.0};   // r^T z, r^T r, b^T b
  if (i < n) {
    double rv[3], zv[3], m[6];
    load_dinv(dinv, n, i, m);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double bk = b[3 * i + k];
      rv[k] = (double)(Z)(q ? bk - q[3 * i + k] : bk);   // the stored r, as every later use sees it
      t[2] += bk * bk;
    }
    apply3(m, rv, zv);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      zv[k] = (double)(Z)zv[k];   // the stored z is the one every inner product sees
      r[3 * i + k] = (Z)rv[k];
      z[3 * i + k] = (Z)zv[k];
      p[3 * i + k] = (Z)0;
      sv[3 * i + k] = (Z)0;
      if (!q) x[3 * i + k] = 0.0;
      t[0] += rv[k] * zv[k];
      t[1] += rv[k] * rv[k];
    }
  }
  wg_sum_all<3>(t, lds);
  const unsigned G = gridDim.x;
  if (threadIdx.x == 0) {
    const int64_t gs = part_stride(G);
    pb[blockIdx.x] = t[0];
    pb[gs + blockIdx.x] = t[1];
    pb[2 * gs + blockIdx.x] = t[2];
  }
}

// Occupancy hints (waves per SIMD the register allocation must allow; 0 =
// the compiler's choice) for the two per-iteration kernels.
#ifndef AGC_SPMV_WAVES
#define AGC_SPMV_WAVES 0
#endif
#ifndef AGC_UPDATE_WAVES
#define AGC_UPDATE_WAVES 0
#endif
#if AGC_SPMV_WAVES > 0
#define AGC_SPMV_OCC __attribute__((amdgpu_waves_per_eu(AGC_SPMV_WAVES)))
#else
#define AGC_SPMV_OCC
#endif
#if AGC_UPDATE_WAVES > 0
#define AGC_UPDATE_OCC __attribute__((amdgpu_waves_per_eu(AGC_UPDATE_WAVES)))
#else
#define AGC_UPDATE_OCC
#endif

// K_1: w = A z, partial z^T w per tile
template <class T>
__global__ __launch_bounds__(kWG) AGC_SPMV_OCC void k_pcg_spmv(const int32_t* __restrict__ col, const int32_t* __restrict__ ri,
                                                  const T* __restrict__ vals, int64_t nnzb, int64_t stride,
                                                  const T* __restrict__ z, double* __restrict__ w,
                                                  double* __restrict__ carry, double* __restrict__ pa,
                                                  const PcgState* st) {
  __shared__ TileLds L;
  const int64_t t = xcd_block();
  Quad<T> q;
  // The flag is read with the index loads, before the value planes: a launch
  // after convergence then reads only the indices, and a working one does
  // not wait for the flag before it starts loading.
  load_quad_index(t, ri, col, nnzb, q);
  if (st->done) return;
  load_quad_vals(t, vals, nnzb, stride, q);
  const double d = spmv_tile<T, Gather<T>, true>(t, q, Gather<T>{z}, w, carry, L);
  if (threadIdx.x == 0) pa[t] = d;
}

// Between K_1 and K_2 on large systems: every workgroup of K_2 sums all the
// partials it reads, so their reading grows as (workgroups of K_2) x
// (partials); past kReduceWork that is shrunk to kReduceSlices partials per
// quantity here.  Workgroup q sums slice q of each of the four rows (the
// three of pb, rows of G, and pa, ga long) in a fixed order and writes
// red[k][q] (rows of part_stride(kReduceSlices)).
constexpr int kReduceSlices = 64;
constexpr int64_t kReduceWork = int64_t(1) << 23;   // doubles read per update, summed over its workgroups
__global__ __launch_bounds__(kWG) void k_pcg_reduce(const double* __restrict__ pb, unsigned G,
                                                    const double* __restrict__ pa, unsigned ga,
                                                    double* __restrict__ red) {
  __shared__ double lds[4 * kWaves];
  const unsigned q = blockIdx.x;
  double t[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double* row = k < 3 ? pb + k * part_stride(G) : pa;
    const unsigned len = k < 3 ? G : ga;
    const unsigned lo = (unsigned)((uint64_t)len * q / kReduceSlices);
    const unsigned hi = (unsigned)((uint64_t)len * (q + 1) / kReduceSlices);
    double acc = 0.0;
    for (unsigned e = lo + threadIdx.x; e < hi; e += kWG) acc += row[e];
    t[k] = acc;
  }
  wg_sum_all<4>(t, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) red[k * part_stride(kReduceSlices) + q] = t[k];
  }
}

// K_2: the update of iteration j.  Reads the partials pb_in of gamma_j and
// r_j^T r_j (and b^T b at j = 0), rows of gin, and pa of delta_j; writes
// those of j + 1 to pb_out, rows of G = gridDim.x (a different buffer: every
// workgroup reads all of pb_in).  On large systems pb_in and pa are the
// rows of k_pcg_reduce.
template <class Z>
__global__ __launch_bounds__(kWG) AGC_UPDATE_OCC void k_pcg_update(int64_t j, const int32_t* __restrict__ rp, int32_t n,
                                                    const double* __restrict__ wy, const double* __restrict__ carry,
                                                    const double* __restrict__ dinv, Z* __restrict__ p,
                                                    Z* __restrict__ sv, double* __restrict__ x,
                                                    Z* __restrict__ r, Z* __restrict__ z,
                                                    const double* __restrict__ pa, unsigned ga,
                                                    const double* __restrict__ pb_in, unsigned gin,
                                                    double* __restrict__ pb_out,
                                                    PcgState* st, double rtol) {
  __shared__ double lds_a[4 * kWaves], lds_c[2 * kWaves];
  const int64_t blk = xcd_block();
  const int64_t i = blk * kWG + threadIdx.x;
  const bool in = i < n;
  const int64_t ic = in ? i : (int64_t)n - 1;   // threads past the end load the last row and store nothing
  const unsigned G = gridDim.x;
  const StateIn in_state = read_state(st, j);
  // Issue order: the partials of the scalars (in L2), then the row's vectors
  // (one row per thread, no branch), then the sum of the partials, which
  // waits for the partials alone; the vectors arrive meanwhile.
  const int64_t GS = part_stride(G), GIS = part_stride(gin);
  vd2 part[4][kPartBatch];
#pragma unroll
  for (int k = 0; k < 3; ++k) part_load(pb_in + k * GIS, gin, part[k]);
  part_load(pa, ga, part[3]);
  const int64_t rs = rp[ic], re = rp[ic + 1];
  double wv[3], pv[3], sw[3], xv[3], rv[3], zv[3], m[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    wv[k] = wy[3 * ic + k];
    pv[k] = p[3 * ic + k];
    sw[k] = sv[3 * ic + k];
    xv[k] = x[3 * ic + k];
    rv[k] = r[3 * ic + k];
    zv[k] = (double)z[3 * ic + k];
  }
  load_dinv(dinv, n, ic, m);
  if (in_state.done) return;
  // gamma_j, r_j^T r_j, b^T b (j = 0) and delta_j, in one reduction
  double t[4];
#pragma unroll
  for (int k = 0; k < 3; ++k) t[k] = part_finish(pb_in + k * GIS, gin, part[k]);
  t[3] = part_finish(pa, ga, part[3]);
  wg_sum_all<4>(t, lds_a);
  if (stop_scalars(j, t, st, in_state, rtol)) return;
  row_fix_wave(in, rs, re, carry, wv, Shape<Z>::tile);
  const double gamma = t[0];
  double beta = 0.0, den = t[3];
  if (j > 0) {
    beta = gamma / in_state.rz_prev;
    den = t[3] - beta * gamma / in_state.alpha_prev;
  }
  if (!(den > 0.0)) {   // p^T A p <= 0 or NaN: not SPD (every workgroup sees the same value)
    if (blockIdx.x == 0 && threadIdx.x == 0) st->done = 3;
    return;
  }
  const double alpha = gamma / den;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->rz_hist[j & 1] = gamma;
    st->alpha_hist[j & 1] = alpha;
  }
  double u[2] = {0.0, 0.0};   // r^T z, r^T r
  if (in) {
    double zn[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      // p, s and r are stored in Z; each is rounded once and used as stored
      pv[k] = (double)(Z)(zv[k] + beta * pv[k]);
      sw[k] = (double)(Z)(wv[k] + beta * sw[k]);
      p[3 * i + k] = (Z)pv[k];
      sv[3 * i + k] = (Z)sw[k];
      x[3 * i + k] = xv[k] + alpha * pv[k];
      rv[k] = (double)(Z)(rv[k] - alpha * sw[k]);
      r[3 * i + k] = (Z)rv[k];
    }
    apply3(m, rv, zn);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      zn[k] = (double)(Z)zn[k];
      z[3 * i + k] = (Z)zn[k];
      u[0] += rv[k] * zn[k];
      u[1] += rv[k] * rv[k];
    }
  }
  wg_sum_all<2>(u, lds_c);
  if (threadIdx.x == 0) {
    pb_out[blk] = u[0];
    pb_out[GS + blk] = u[1];
    pb_out[2 * GS + blk] = 0.0;
  }
}

// The stop test of iteration j alone (one workgroup), run at the end of a chunk.
__global__ __launch_bounds__(kWG) void k_pcg_check(int64_t j, const double* __restrict__ pb, unsigned gb,
                                                   PcgState* st, double rtol) {
  __shared__ double lds[3 * kWaves];
  const StateIn in_state = read_state(st, j);
  if (in_state.done) return;
  double t[3];
  all_sum<3>(pb, gb, lds, t);
  (void)stop_scalars(j, t, st, in_state, rtol);
}

constexpr int kFirstChunk = 16;
constexpr int kRateSpan = 8;   // iterations over which the host measures the residual's decay
constexpr int kRepeatMargin = 3;     // extra launches when a solve repeats the last one's shape
constexpr size_t kRepeatKeys = 64;   // remembered shapes
static_assert(kRateSpan < kRrRing, "the ring holds the span");
constexpr int kTimedReplays = 20;   // SpMV launches timed per PCG solve when kernel timing is on

int pcg(agc_context* c, const Matrix& a, const double* b, double* x, double rtol, int32_t max_iter, int32_t* iters,
        double* rel, bool x_zero) {
  const int32_t n = a.n;
  const int64_t n3 = 3 * (int64_t)n;
  *iters = 0;
  *rel = 0.0;
  if (n == 0) return AGC_OK;
  double* dinv = c->ws.get<double>("pcg.dinv", 6 * (int64_t)n);
  // z, r, p and s in the matrix's value type (see the top of this file)
  const bool f64 = a.dtype == AGC_F64;
  auto zvec = [&](const char* name) {
    return f64 ? (void*)c->ws.get<double>(name, n3) : (void*)c->ws.get<float>(std::string(name) + "32", n3);
  };
  void* z = zvec("pcg.z");
  void* r = zvec("pcg.r");
  void* p = zvec("pcg.p");
  void* sv = zvec("pcg.s");
  double* w = c->ws.get<double>("pcg.w", n3);
  const unsigned gr = blocks_for(n, kWG);
  const unsigned gs = blocks_for(a.nnzb, tile_of(a.dtype));
  // update partials, double-buffered by parity of j: iteration j reads pbs[j%2]
  double* pbs[2] = {c->ws.get<double>("pcg.pb0", 3 * part_stride(gr)),
                    c->ws.get<double>("pcg.pb1", 3 * part_stride(gr))};
  double* pa = c->ws.get<double>("pcg.pa", part_stride(gs));
  // the partials every update workgroup would read, summed over them
  const int64_t upd_reads = (int64_t)gr * (3 * (int64_t)gr + gs);
  const bool use_red = c->pcg_reduce < 0 ? upd_reads > kReduceWork : c->pcg_reduce == 1;
  double* red = use_red ? c->ws.get<double>("pcg.red", 4 * part_stride(kReduceSlices)) : nullptr;
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
  if (!x_zero) spmv(c, a, x, w);   // w = A x0
  if (a.dtype == AGC_F64)
    k_pcg_init<double><<<gr, kWG, 0, c->stream>>>(b, x_zero ? nullptr : w, dinv, n, x, (double*)r, (double*)z,
                                                  (double*)p, (double*)sv, pbs[0]);
  else
    k_pcg_init<float><<<gr, kWG, 0, c->stream>>>(b, x_zero ? nullptr : w, dinv, n, x, (float*)r, (float*)z,
                                                 (float*)p, (float*)sv, pbs[0]);
  AGC_LAUNCH_CHECK();
  k_pcg_check<<<1, kWG, 0, c->stream>>>(0, pbs[0], gr, st, rtol);
  AGC_LAUNCH_CHECK();

  // The host enqueues iterations in chunks and reads the device scalars (and
  // the block-Jacobi error word) in between.  After the first chunk, the
  // chunk length is the number of iterations the residual's current decay
  // (over the last kRateSpan iterations, from the ring of r^T r values) still
  // needs, with a margin, but at most the number already run: CG speeds up
  // as it goes, so an early rate overestimates, and a launch after
  // convergence, though it only reads a flag, still costs the host's enqueue
  // time, while a host round trip costs that of ~5-10 iterations.
  int64_t launched = 0;
  // a solve like the last one (rows within ~4%, same dtype, tolerance within
  // a quarter decade) starts with a chunk of its iteration count plus a
  // margin: usually one round trip
  const auto key = std::make_tuple((int32_t)floor(16.0 * log2((double)n)), a.dtype,
                                   (int32_t)floor(4.0 * log10(rtol > 0.0 ? rtol : 1e-300)));
  const auto last = c->pcg_last.find(key);
  int chunk = kFirstChunk;
  if (last != c->pcg_last.end() && last->second + kRepeatMargin > chunk)
    chunk = last->second + kRepeatMargin > kMaxChunk ? kMaxChunk : last->second + kRepeatMargin;
  for (;;) {
    for (int it = 0; it < chunk; ++it) {
      const int64_t j = launched + it;
      if (a.dtype == AGC_F64)
        k_pcg_spmv<double><<<gs, kWG, 0, c->stream>>>(a.ci(), a.ri(), (const double*)a.vals.p, a.nnzb, a.stride,
                                                      (const double*)z, w, carry, pa, st);
      else
        k_pcg_spmv<float><<<gs, kWG, 0, c->stream>>>(a.ci(), a.ri(), (const float*)a.vals.p, a.nnzb, a.stride,
                                                     (const float*)z, w, carry, pa, st);
      const double* pb_in = pbs[j & 1];
      const double* pa_in = pa;
      unsigned gin = gr, ga = gs;
      if (red) {
        k_pcg_reduce<<<kReduceSlices, kWG, 0, c->stream>>>(pb_in, gr, pa, gs, red);
        pb_in = red;
        pa_in = red + 3 * part_stride(kReduceSlices);
        gin = ga = kReduceSlices;
      }
      if (a.dtype == AGC_F64)
        k_pcg_update<double><<<gr, kWG, 0, c->stream>>>(j, a.rp(), n, w, carry, dinv, (double*)p, (double*)sv, x,
                                                        (double*)r, (double*)z, pa_in,
                                                        ga, pb_in, gin, pbs[(j + 1) & 1], st, rtol);
      else
        k_pcg_update<float><<<gr, kWG, 0, c->stream>>>(j, a.rp(), n, w, carry, dinv, (float*)p, (float*)sv, x,
                                                       (float*)r, (float*)z, pa_in,
                                                       ga, pb_in, gin, pbs[(j + 1) & 1], st, rtol);
    }
    launched += chunk;
    k_pcg_check<<<1, kWG, 0, c->stream>>>(launched, pbs[launched & 1], gr, st, rtol);
    AGC_LAUNCH_CHECK();
    AGC_HIP(hipMemcpyAsync(hs, st, sizeof(PcgState), hipMemcpyDeviceToHost, c->stream));
    AGC_HIP(hipMemcpyAsync(c->h_err, c->d_err, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
    AGC_HIP(hipStreamSynchronize(c->stream));
    if (*c->h_err) return AGC_ERR_NOT_SPD;   // a diagonal block without a Cholesky factor
    if (hs->done) break;
    // the device stops at max_iter; this only guards the host against a lost state
    if (launched > (int64_t)max_iter + 64) throw Error(AGC_ERR_DEVICE, "PCG state did not advance");
    double want = 2.0 * chunk;
    const int span = hs->iter < kRateSpan ? hs->iter : kRateSpan;
    const double rr_then = span > 0 ? hs->rr_ring[(hs->iter - span) % kRrRing] : 0.0;
    if (span > 0 && hs->rr > 0.0 && rr_then > hs->rr) {
      const double rate = log(hs->rr / rr_then) / (double)span;
      want = 1.1 * log(hs->tol2 / hs->rr) / rate + 2.0;
    }
    const int cap = launched < kFirstChunk ? kFirstChunk : (launched > kMaxChunk ? kMaxChunk : (int)launched);
    chunk = want < 4.0 ? 4 : (want > cap ? cap : (int)ceil(want));
  }
  if (c->kernel_timing && launched > 0) {
    // The SpMV kernel of the iterations, replayed back to back on the final
    // z between two events: its mean duration per launch.  The replays read a
    // state whose done flag is 0, so each does the flag read of an iteration
    // and none exits early; w, carry and pa are scratch by now.
    PcgState* live = c->ws.get<PcgState>("pcg.replay_state", 1);
    AGC_HIP(hipMemsetAsync(live, 0, sizeof(PcgState), c->stream));
    AGC_HIP(hipEventRecord(c->ev[6], c->stream));
    for (int r = 0; r < kTimedReplays; ++r) {
      if (a.dtype == AGC_F64)
        k_pcg_spmv<double><<<gs, kWG, 0, c->stream>>>(a.ci(), a.ri(), (const double*)a.vals.p, a.nnzb, a.stride,
                                                      (const double*)z, w, carry, pa, live);
      else
        k_pcg_spmv<float><<<gs, kWG, 0, c->stream>>>(a.ci(), a.ri(), (const float*)a.vals.p, a.nnzb, a.stride,
                                                     (const float*)z, w, carry, pa, live);
    }
    AGC_LAUNCH_CHECK();
    AGC_HIP(hipEventRecord(c->ev[7], c->stream));
    AGC_HIP(hipEventSynchronize(c->ev[7]));
    float ms = 0.f;
    AGC_HIP(hipEventElapsedTime(&ms, c->ev[6], c->ev[7]));
    c->spmv_ms += ms;
    c->spmv_n += kTimedReplays;
  }
  *iters = hs->iter;
  if (hs->done == 1) {
    if (c->pcg_last.size() >= kRepeatKeys && !c->pcg_last.count(key)) c->pcg_last.clear();
    c->pcg_last[key] = hs->iter;
  }
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

// r = b - y; partial sums of b^2 and r^2 per workgroup
__global__ __launch_bounds__(kWG) void k_resid_part(const double* __restrict__ b, const double* __restrict__ y,
                                                    double* __restrict__ r, int64_t n, double* __restrict__ part) {
  __shared__ double lds[2 * kWaves];
  double t[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG) {
    const double bi = b[i], ri = bi - y[i];
    r[i] = ri;
    t[0] += bi * bi;
    t[1] += ri * ri;
  }
  wg_sum_all<2>(t, lds);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = t[0];
    part[gridDim.x + blockIdx.x] = t[1];
  }
}

__global__ __launch_bounds__(kWG) void k_sum_part2(const double* __restrict__ part, unsigned n,
                                                   double* __restrict__ out) {
  __shared__ double lds[2 * kWaves];
  double t[2] = {0.0, 0.0};
  for (unsigned i = threadIdx.x; i < n; i += kWG) {
    t[0] += part[i];
    t[1] += part[n + i];
  }
  wg_sum_all<2>(t, lds);
  if (threadIdx.x == 0) {
    out[0] = t[0];
    out[1] = t[1];
  }
}

void residual_norms(agc_context* c, const double* b, const double* y, double* r, int64_t n3, double* bn,
                    double* rn) {
  const unsigned G = 512;
  double* part = c->ws.get<double>("resid.part", 2 * G + 2);
  k_resid_part<<<G, kWG, 0, c->stream>>>(b, y, r, n3, part);
  k_sum_part2<<<1, kWG, 0, c->stream>>>(part, G, part + 2 * G);
  AGC_LAUNCH_CHECK();
  double* h = (double*)c->h_pcg;   // pinned scratch; no PCG is in flight here
  AGC_HIP(hipMemcpyAsync(h, part + 2 * G, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  AGC_HIP(hipStreamSynchronize(c->stream));
  *bn = sqrt(h[0]);
  *rn = sqrt(h[1]);
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
