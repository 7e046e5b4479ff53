// The outer Newton loop of one implicit time step (Sec. 3, Eq. 1-2; Alg.
// overview), with no contact, barrier or friction terms: each iteration
// builds the fine gradient and an SPD Hessian proxy from the elements, tags
// edges by the Green strain increment against the previous iterate (Sec.
// 4.2, Eq. 3), solves the coarsened system (agc_solve: mapping, coarse
// assembly, PCG, prolongation, optional post-coarsening), and backtracks
// along the direction until the incremental potential decreases.
//
// The potential is divided by h^2 (same minimiser; its Hessian is the
// H = M/h^2 + K the linear solves take):
//   E(x) = sum_v m_v / (2 h^2) |x_v - xhat_v|^2 + sum_e V_e psi(F_e),
// with co-rotated elasticity psi(F) = mu |F - R|^2 + lam/2 (tr(R^T F) - 3)^2,
// R the rotation of the rotation-variant polar decomposition of F, exact
// first Piola stress P = 2 mu (F - R) + lam (tr(R^T F) - 3) R, and as the SPD
// proxy the Hessian with R held fixed, plus the element's lumped mass / h^2:
//   H_e[a][b] = V (2 mu (b_a . b_b) I + lam (R b_a)(R b_b)^T) + [a == b] rho V / (4 h^2) I,
// where F = sum_a x_a b_a^T (b_1..b_3 the rows of Dm^{-1}, b_0 = -(b_1 + b_2 + b_3)).
//
// One thread per element computes F, R (eigenvectors of F^T F by cyclic
// Jacobi rotations, then the left vectors from F), P, the element gradient,
// V psi and the 144 proxy entries.  Vertex gradients gather the element
// gradients through a vertex -> (element, corner) list sorted by element, so
// every sum has a fixed order; energies are summed by per-workgroup partials
// and one final workgroup, also in a fixed order.
#include <chrono>
#include <memory>

#include "internal.h"
#include "mat3.h"

namespace agc {
namespace {

constexpr int kMaxHalvings = 30;

// ------------------------------------------------------------ kernels

// b_a (12 per element, a-major) and the rest volume; a degenerate element or
// an id out of range sets kErrElem.
__global__ void k_nw_rest(const int32_t* __restrict__ tets, int64_t ne, const double* __restrict__ rest, int32_t n,
                          double* __restrict__ bvec, double* __restrict__ vol, unsigned* err) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
    int32_t t[4];
    bool ok = true;
    for (int a = 0; a < 4; ++a) {
      t[a] = tets[4 * e + a];
      ok = ok && t[a] >= 0 && t[a] < n;
    }
    if (!ok) {
      atomicOr(err, kErrElem);
      continue;
    }
    double d[3][3];   // columns X_k - X_0
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < 3; ++i) d[i][k] = rest[3 * (int64_t)t[k + 1] + i] - rest[3 * (int64_t)t[0] + i];
    // rows of Dm^{-1}: (d_1 x d_2, d_2 x d_0, d_0 x d_1) / det with d_k the columns
    double cr[3][3];
    for (int k = 0; k < 3; ++k) {
      const int p = (k + 1) % 3, q = (k + 2) % 3;
      cr[k][0] = d[1][p] * d[2][q] - d[2][p] * d[1][q];
      cr[k][1] = d[2][p] * d[0][q] - d[0][p] * d[2][q];
      cr[k][2] = d[0][p] * d[1][q] - d[1][p] * d[0][q];
    }
    const double det = d[0][0] * cr[0][0] + d[1][0] * cr[0][1] + d[2][0] * cr[0][2];
    if (!(fabs(det) > 0.0)) {
      atomicOr(err, kErrElem);
      continue;
    }
    double b[4][3];
    for (int k = 0; k < 3; ++k)
      for (int j = 0; j < 3; ++j) b[k + 1][j] = cr[k][j] / det;
    for (int j = 0; j < 3; ++j) b[0][j] = -(b[1][j] + b[2][j] + b[3][j]);
    for (int a = 0; a < 4; ++a)
      for (int j = 0; j < 3; ++j) bvec[12 * e + 3 * a + j] = b[a][j];
    vol[e] = fabs(det) / 6.0;
  }
}

// keys v and values e*4 + a of the vertex -> corner list
__global__ void k_nw_corners(const int32_t* __restrict__ tets, int64_t ne, uint32_t* __restrict__ key,
                             uint32_t* __restrict__ val) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < 4 * ne; s += (int64_t)gridDim.x * blockDim.x) {
    key[s] = (uint32_t)tets[s];
    val[s] = (uint32_t)s;
  }
}

// vptr[v] = the first sorted position whose key is >= v, for v in [0, n]:
// boundary i (between positions i - 1 and i) owns key[i - 1] < v <= key[i]
// (v from 0 at i = 0, up to n at i = m), so every v is written once.
__global__ void k_nw_vptr(const uint32_t* __restrict__ key, int64_t m, int32_t n, uint32_t* __restrict__ vptr) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= m; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t lo = i == 0 ? 0 : (int64_t)key[i - 1] + 1;
    const int64_t hi = i == m ? (int64_t)n : (int64_t)key[i];
    for (int64_t v = lo; v <= hi; ++v) vptr[v] = (uint32_t)i;
  }
}

// m_v = sum over the corners of v of rho V_e / 4, in element order
__global__ void k_nw_scale(const double* __restrict__ a, double s, int64_t n, double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = s * a[i];
}

__global__ void k_nw_mass(const uint32_t* __restrict__ vptr, const uint32_t* __restrict__ corner,
                          const double* __restrict__ vol, double rho, int32_t n, double* __restrict__ mass) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (uint32_t k = vptr[v]; k < vptr[v + 1]; ++k) s += rho * vol[corner[k] >> 2] / 4.0;
    mass[v] = s;
  }
}

// xhat = x_t + h v_t + h^2 f / m (the force term only where m > 0) and the
// previous state x_t - h v_t of the first iteration's tags
__global__ void k_nw_predict(const double* __restrict__ xt, const double* __restrict__ vt, const double* __restrict__ f,
                             const double* __restrict__ mass, double h, int32_t n, double* __restrict__ xhat,
                             double* __restrict__ xlast) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < 3 * (int64_t)n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const double m = mass[k / 3];
    double xh = xt[k] + h * vt[k];
    if (f && m > 0.0) xh += h * h * f[k] / m;
    xhat[k] = xh;
    xlast[k] = xt[k] - h * vt[k];
  }
}

struct Material {
  double mu, lam, rho, h;
};

// Per element: V psi into a per-workgroup partial; MODE >= 1 also the
// element gradient ge[e][12]; MODE 2 also the proxy blocks H[e][144].  For
// the blocks each thread leaves what its element's 144 entries need in LDS
// (R b_a, b_a, lam V, 2 mu V, the lumped mass / h^2), and the workgroup then
// writes its kWG consecutive blocks with coalesced 16-byte stores, each
// entry formed from LDS: a thread's own 144 stores would each touch a
// different 1152-byte block.
struct ElemCoef {
  double rb[12], b[12], lv, mv, mass;
};

__device__ __forceinline__ double proxy_entry(const ElemCoef& q, int row, int col) {
  const int a = row / 3, i = row - 3 * a, c = col / 3, j = col - 3 * c;
  // every product is formed symmetrically in (a, i) <-> (c, j), so the block
  // is bitwise symmetric
  double h = q.lv * (q.rb[3 * a + i] * q.rb[3 * c + j]);
  if (i == j) {
    const double bb = q.mv * (q.b[3 * a] * q.b[3 * c] + q.b[3 * a + 1] * q.b[3 * c + 1] + q.b[3 * a + 2] * q.b[3 * c + 2]);
    h += bb + (a == c ? q.mass : 0.0);
  }
  return h;
}

template <int MODE>
__global__ __launch_bounds__(kWG) void k_nw_elem(const double* __restrict__ x, const int32_t* __restrict__ tets,
                                                 const double* __restrict__ bvec, const double* __restrict__ vol,
                                                 int64_t ne, Material mt, double* __restrict__ ge,
                                                 double* __restrict__ H, double* __restrict__ epart) {
  __shared__ double lds[kWaves];
  __shared__ ElemCoef coef[MODE == 2 ? kWG : 1];
  const int64_t e0 = (int64_t)blockIdx.x * kWG;
  const int64_t e = e0 + threadIdx.x;
  double en = 0.0;
  if (e < ne) {
    double xa[4][3], b[4][3];
    for (int a = 0; a < 4; ++a) {
      const int64_t v = tets[4 * e + a];
      for (int i = 0; i < 3; ++i) {
        xa[a][i] = x[3 * v + i];
        b[a][i] = bvec[12 * e + 3 * a + i];
      }
    }
    double f[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) f[i][j] = xa[0][i] * b[0][j] + xa[1][i] * b[1][j] + xa[2][i] * b[2][j] + xa[3][i] * b[3][j];
    double r[3][3];
    polar_rotation(f, r);
    double tr = -3.0, d2 = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        tr += r[i][j] * f[i][j];
        d2 += (f[i][j] - r[i][j]) * (f[i][j] - r[i][j]);
      }
    const double V = vol[e];
    en = V * (mt.mu * d2 + 0.5 * mt.lam * tr * tr);
    if (MODE >= 1) {
      double p[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) p[i][j] = 2.0 * mt.mu * (f[i][j] - r[i][j]) + mt.lam * tr * r[i][j];
      for (int a = 0; a < 4; ++a)
        for (int i = 0; i < 3; ++i)
          ge[12 * e + 3 * a + i] = V * (p[i][0] * b[a][0] + p[i][1] * b[a][1] + p[i][2] * b[a][2]);
    }
    if (MODE == 2) {
      ElemCoef& q = coef[threadIdx.x];
      for (int a = 0; a < 4; ++a)
        for (int i = 0; i < 3; ++i) {
          q.rb[3 * a + i] = r[i][0] * b[a][0] + r[i][1] * b[a][1] + r[i][2] * b[a][2];
          q.b[3 * a + i] = b[a][i];
        }
      q.lv = mt.lam * V;
      q.mv = 2.0 * mt.mu * V;
      q.mass = mt.rho * V / (4.0 * mt.h * mt.h);
    }
  }
  if (MODE == 2) {
    __syncthreads();
    const int64_t cnt = ne - e0 < kWG ? ne - e0 : kWG;   // elements of this workgroup
    double2* dst = reinterpret_cast<double2*>(H + 144 * e0);
    for (int64_t k2 = threadIdx.x; k2 < 72 * cnt; k2 += kWG) {   // entries 2 k2 and 2 k2 + 1
      const int el = (int)(k2 / 72);
      const int k = (int)(2 * k2 - 144 * (int64_t)el);   // even: both entries lie in one row
      const int row = k / 12, col = k - 12 * row;
      const ElemCoef& q = coef[el];
      dst[k2] = make_double2(proxy_entry(q, row, col), proxy_entry(q, row, col + 1));
    }
  }
  const double s = wg_sum(en, lds);
  if (threadIdx.x == 0) epart[blockIdx.x] = s;
}

// Per vertex: the inertia energy m/(2h^2)|x - xhat|^2 into a per-workgroup
// partial; with g not null also g_v = m/h^2 (x - xhat) + the element
// gradients of its corners, in element order.
__global__ __launch_bounds__(kWG) void k_nw_vertex(const double* __restrict__ x, const double* __restrict__ xhat,
                                                   const double* __restrict__ mass, const uint32_t* __restrict__ vptr,
                                                   const uint32_t* __restrict__ corner, const double* __restrict__ ge,
                                                   int32_t n, double h, double* __restrict__ g,
                                                   double* __restrict__ vpart) {
  __shared__ double lds[kWaves];
  const int64_t v = (int64_t)blockIdx.x * kWG + threadIdx.x;
  double en = 0.0;
  if (v < n) {
    const double m = mass[v];
    double dx[3];
    for (int i = 0; i < 3; ++i) dx[i] = x[3 * v + i] - xhat[3 * v + i];
    en = m * (dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]) / (2.0 * h * h);
    if (g) {
      double s[3];
      for (int i = 0; i < 3; ++i) s[i] = m / (h * h) * dx[i];
      for (uint32_t k = vptr[v]; k < vptr[v + 1]; ++k) {
        const int64_t c = corner[k];   // e * 4 + a: ge[c * 3 + i]
        for (int i = 0; i < 3; ++i) s[i] += ge[3 * c + i];
      }
      for (int i = 0; i < 3; ++i) g[3 * v + i] = s[i];
    }
  }
  const double s = wg_sum(en, lds);
  if (threadIdx.x == 0) vpart[blockIdx.x] = s;
}

// out[0] = the element partials + the vertex partials, each in order
__global__ __launch_bounds__(kWG) void k_nw_total(const double* __restrict__ ep, unsigned gep, const double* __restrict__ vp,
                                                  unsigned gv, double* __restrict__ out) {
  __shared__ double lds[kWaves];
  double a = 0.0, b = 0.0;
  for (unsigned i = threadIdx.x; i < gep; i += kWG) a += ep[i];
  for (unsigned i = threadIdx.x; i < gv; i += kWG) b += vp[i];
  a = wg_sum(a, lds);
  b = wg_sum(b, lds);
  if (threadIdx.x == 0) out[0] = a + b;
}

// y = x0 - alpha s
__global__ void k_nw_step(const double* __restrict__ x0, const double* __restrict__ s, double alpha, int64_t n3,
                          double* __restrict__ y) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n3; k += (int64_t)gridDim.x * blockDim.x)
    y[k] = x0[k] - alpha * s[k];
}

// max |s| per workgroup, then over the partials (one workgroup)
__global__ __launch_bounds__(kWG) void k_nw_absmax(const double* __restrict__ s, int64_t n3, double* __restrict__ part) {
  __shared__ double lds[kWaves];
  double m = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * kWG + threadIdx.x; k < n3; k += (int64_t)gridDim.x * kWG) m = fmax(m, fabs(s[k]));
  for (int o = kWave / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if (lane_id() == 0) lds[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kWaves; ++w) t = fmax(t, lds[w]);
    part[blockIdx.x] = t;
  }
}
__global__ __launch_bounds__(kWG) void k_nw_absmax_final(const double* __restrict__ part, unsigned g, double* out) {
  __shared__ double lds[kWaves];
  double m = 0.0;
  for (unsigned i = threadIdx.x; i < g; i += kWG) m = fmax(m, part[i]);
  for (int o = kWave / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if (lane_id() == 0) lds[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kWaves; ++w) t = fmax(t, lds[w]);
    out[0] = t;
  }
}

}  // namespace
}  // namespace agc

struct agc_newton {
  int32_t n = 0;
  int64_t ne = 0, m = 0;
  const agc_mesh* mesh = nullptr;
  agc_tagger* tagger = nullptr;
  agc::Material mt{};
  agc::DevBuf edges, rest, bvec, vol, mass, vptr, corner;
  void release() {
    edges.release(); rest.release(); bvec.release(); vol.release(); mass.release(); vptr.release(); corner.release();
  }
  // releases the buffers and the tagger, also when creation fails half way
  ~agc_newton() {
    release();
    delete tagger;
  }
};

namespace agc {
namespace {

struct NwBufs {
  double *ge, *H, *g, *ep, *vp, *scal;
  unsigned gel, gvl;
};

NwBufs nw_bufs(agc_context* c, const agc_newton* nw, bool with_h) {
  NwBufs b;
  b.gel = blocks_for(nw->ne, kWG);
  b.gvl = blocks_for(nw->n, kWG);
  b.ge = c->ws.get<double>("nw.ge", 12 * nw->ne);
  b.H = with_h ? c->ws.get<double>("nw.H", 144 * nw->ne) : nullptr;
  b.g = c->ws.get<double>("nw.g", 3 * (int64_t)nw->n);
  b.ep = c->ws.get<double>("nw.ep", b.gel);
  b.vp = c->ws.get<double>("nw.vp", b.gvl);
  b.scal = c->ws.get<double>("nw.scal", 4);
  return b;
}

// E(x) [host]; synchronises
double nw_energy(agc_context* c, const agc_newton* nw, const NwBufs& b, const double* x, const double* xhat) {
  if (nw->ne > 0)
    k_nw_elem<0><<<b.gel, kWG, 0, c->stream>>>(x, (const int32_t*)nw->mesh->m.elem_verts.p, (const double*)nw->bvec.p,
                                                  (const double*)nw->vol.p, nw->ne, nw->mt, nullptr, nullptr, b.ep);
  k_nw_vertex<<<b.gvl, kWG, 0, c->stream>>>(x, xhat, (const double*)nw->mass.p, (const uint32_t*)nw->vptr.p,
                                            (const uint32_t*)nw->corner.p, nullptr, nw->n, nw->mt.h, nullptr, b.vp);
  k_nw_total<<<1, kWG, 0, c->stream>>>(b.ep, nw->ne > 0 ? b.gel : 0, b.vp, b.gvl, b.scal);
  AGC_LAUNCH_CHECK();
  double e = 0.0;
  AGC_HIP(hipMemcpyAsync(&e, b.scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  AGC_HIP(hipStreamSynchronize(c->stream));
  return e;
}

// g (and the proxy blocks H when b.H) at x
void nw_physics(agc_context* c, const agc_newton* nw, const NwBufs& b, const double* x, const double* xhat, double* g,
                double* H) {
  if (nw->ne > 0)
    if (H)
      k_nw_elem<2><<<b.gel, kWG, 0, c->stream>>>(x, (const int32_t*)nw->mesh->m.elem_verts.p, (const double*)nw->bvec.p,
                                                (const double*)nw->vol.p, nw->ne, nw->mt, b.ge, H, b.ep);
    else
      k_nw_elem<1><<<b.gel, kWG, 0, c->stream>>>(x, (const int32_t*)nw->mesh->m.elem_verts.p, (const double*)nw->bvec.p,
                                                (const double*)nw->vol.p, nw->ne, nw->mt, b.ge, nullptr, b.ep);
  k_nw_vertex<<<b.gvl, kWG, 0, c->stream>>>(x, xhat, (const double*)nw->mass.p, (const uint32_t*)nw->vptr.p,
                                            (const uint32_t*)nw->corner.p, b.ge, nw->n, nw->mt.h, g, b.vp);
  AGC_LAUNCH_CHECK();
}

double nw_absmax(agc_context* c, const double* s, int64_t n3) {
  const unsigned g = grid_blocks(n3 > 0 ? n3 : 1);
  double* part = c->ws.get<double>("nw.amax", g);
  double* out = c->ws.get<double>("nw.amax1", 1);
  k_nw_absmax<<<g, kWG, 0, c->stream>>>(s, n3, part);
  k_nw_absmax_final<<<1, kWG, 0, c->stream>>>(part, g, out);
  AGC_LAUNCH_CHECK();
  double h = 0.0;
  AGC_HIP(hipMemcpyAsync(&h, out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  AGC_HIP(hipStreamSynchronize(c->stream));
  return h;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace
}  // namespace agc

extern "C" {

agc_status agc_newton_create(agc_context* c, const agc_mesh* mesh, int64_t n_edges, const int32_t* edges,
                             const double* rest, const agc_material* mat, agc_newton** out) {
  using namespace agc;
  API_BEGIN(c)
  AGC_REQUIRE(out, "out is null");
  *out = nullptr;
  AGC_REQUIRE(mesh && mat && rest, "mesh, material or rest null");
  AGC_REQUIRE(n_edges >= 0 && (n_edges == 0 || edges), "edges null");
  AGC_REQUIRE(((uintptr_t)edges & 7) == 0, "edges must be 8-byte aligned");
  AGC_REQUIRE(mat->mu >= 0.0 && mat->lambda >= 0.0 && mat->rho > 0.0 && mat->h > 0.0, "bad material");
  const int32_t n = mesh->m.n_verts;
  const int64_t ne = mesh->m.n_elems;
  AGC_REQUIRE(4 * ne < (int64_t)UINT32_MAX, "too many elements");
  std::unique_ptr<agc_newton> nw(new agc_newton());
  nw->n = n;
  nw->ne = ne;
  nw->m = n_edges;
  nw->mesh = mesh;
  nw->mt = Material{mat->mu, mat->lambda, mat->rho, mat->h};
  int32_t* ed = (int32_t*)nw->edges.ensure(sizeof(int32_t) * 2 * (size_t)(n_edges > 0 ? n_edges : 1));
  if (n_edges > 0)
    AGC_HIP(hipMemcpyAsync(ed, edges, sizeof(int32_t) * 2 * (size_t)n_edges, hipMemcpyDeviceToDevice, c->stream));
  double* rs = (double*)nw->rest.ensure(sizeof(double) * 3 * (size_t)n);
  AGC_HIP(hipMemcpyAsync(rs, rest, sizeof(double) * 3 * (size_t)n, hipMemcpyDeviceToDevice, c->stream));
  const int32_t* tets = (const int32_t*)mesh->m.elem_verts.p;
  double* bv = (double*)nw->bvec.ensure(sizeof(double) * 12 * (size_t)(ne > 0 ? ne : 1));
  double* vol = (double*)nw->vol.ensure(sizeof(double) * (size_t)(ne > 0 ? ne : 1));
  err_reset(c);
  if (ne > 0) {
    k_nw_rest<<<grid_blocks(ne), kWG, 0, c->stream>>>(tets, ne, rs, n, bv, vol, c->d_err);
    AGC_LAUNCH_CHECK();
  }
  // vertex -> corner list, sorted by vertex, corners in element order (stable sort)
  const int64_t m4 = 4 * ne;
  uint32_t* vptr = (uint32_t*)nw->vptr.ensure(sizeof(uint32_t) * ((size_t)n + 1));
  uint32_t* corner = (uint32_t*)nw->corner.ensure(sizeof(uint32_t) * (size_t)(m4 > 0 ? m4 : 1));
  if (m4 > 0) {
    uint32_t* k1 = c->ws.get<uint32_t>("nw.k1", m4);
    uint32_t* k2 = c->ws.get<uint32_t>("nw.k2", m4);
    uint32_t* v2 = c->ws.get<uint32_t>("nw.v2", m4);
    k_nw_corners<<<grid_blocks(m4), kWG, 0, c->stream>>>(tets, ne, k1, corner);
    AGC_LAUNCH_CHECK();
    const bool alt = radix_sort_u32(c, k1, corner, k2, v2, m4, bits_for((uint64_t)(n > 0 ? n - 1 : 0)), "nw.sort");
    if (alt) {
      AGC_HIP(hipMemcpyAsync(k1, k2, sizeof(uint32_t) * m4, hipMemcpyDeviceToDevice, c->stream));
      AGC_HIP(hipMemcpyAsync(corner, v2, sizeof(uint32_t) * m4, hipMemcpyDeviceToDevice, c->stream));
    }
    k_nw_vptr<<<grid_blocks(m4 + 1), kWG, 0, c->stream>>>(k1, m4, n, vptr);
  } else {
    AGC_HIP(hipMemsetAsync(vptr, 0, sizeof(uint32_t) * ((size_t)n + 1), c->stream));
  }
  AGC_LAUNCH_CHECK();
  double* mass = (double*)nw->mass.ensure(sizeof(double) * (size_t)n);
  k_nw_mass<<<grid_blocks(n), kWG, 0, c->stream>>>(vptr, corner, vol, mat->rho, n, mass);
  AGC_LAUNCH_CHECK();
  err_throw(err_fetch(c));
  agc_tagger* tg = nullptr;
  const agc_status st = agc_tagger_create(c, n, ne, tets, rs, n_edges, ed, &tg);
  if (st != AGC_OK) throw Error(st, c->err.empty() ? "tagger" : c->err);
  nw->tagger = tg;
  *out = nw.release();
  API_END(c)
}

agc_status agc_newton_destroy(agc_context* c, agc_newton* nw) {
  if (!c || !nw) return AGC_ERR_INVALID_ARG;
  delete nw;
  return AGC_OK;
}

agc_status agc_newton_mass(agc_context* c, const agc_newton* nw, double* mass) {
  using namespace agc;
  API_BEGIN(c)
  AGC_REQUIRE(nw && mass, "null argument");
  AGC_HIP(hipMemcpyAsync(mass, nw->mass.p, sizeof(double) * (size_t)nw->n, hipMemcpyDeviceToDevice, c->stream));
  AGC_HIP(hipStreamSynchronize(c->stream));
  API_END(c)
}

agc_status agc_newton_physics(agc_context* c, const agc_newton* nw, const double* x, const double* x_hat, double* g,
                              double* elem_H, double* energy) {
  using namespace agc;
  API_BEGIN(c)
  AGC_REQUIRE(nw && x && x_hat, "null argument");
  AGC_REQUIRE(((uintptr_t)elem_H & 15) == 0, "elem_H must be 16-byte aligned");
  NwBufs b = nw_bufs(c, nw, false);
  if (g || elem_H) {
    nw_physics(c, nw, b, x, x_hat, g ? g : b.g, elem_H);
    AGC_HIP(hipStreamSynchronize(c->stream));
  }
  if (energy) *energy = nw_energy(c, nw, b, x, x_hat);
  API_END(c)
}

agc_status agc_newton_step(agc_context* c, agc_newton* nw, const agc_newton_opts* opts, const double* x_t,
                           const double* v_t, const double* f_ext, double* x_out, agc_newton_info* info) {
  using namespace agc;
  using clock = std::chrono::steady_clock;
  API_BEGIN(c)
  AGC_REQUIRE(nw && opts && x_t && v_t && x_out, "null argument");
  AGC_REQUIRE(opts->max_newton >= 1 && opts->eps_d >= 0.0 && opts->tag_threshold >= 0.0, "bad options");
  AGC_REQUIRE(opts->solve.affine_threshold == 0 || opts->coarsen, "affine embedding needs coarsen = 1");
  const int64_t n3 = 3 * (int64_t)nw->n;
  const double h = nw->mt.h;
  NwBufs b = nw_bufs(c, nw, true);
  double* xhat = c->ws.get<double>("nw.xhat", n3);
  double* xlast = c->ws.get<double>("nw.xlast", n3);
  double* xcur = c->ws.get<double>("nw.xcur", n3);
  double* xnew = c->ws.get<double>("nw.xnew", n3);
  double* sol = c->ws.get<double>("nw.sol", n3);
  uint8_t* tags = c->ws.get<uint8_t>("nw.tags", nw->m > 0 ? nw->m : 1);
  k_nw_predict<<<grid_blocks(n3), kWG, 0, c->stream>>>(x_t, v_t, f_ext, (const double*)nw->mass.p, h, nw->n, xhat,
                                                       xlast);
  AGC_LAUNCH_CHECK();
  AGC_HIP(hipMemcpyAsync(xcur, x_t, sizeof(double) * n3, hipMemcpyDeviceToDevice, c->stream));
  agc_newton_info inf{};
  double e_prev = nw_energy(c, nw, b, xcur, xhat);
  inf.energy0 = e_prev;
  agc_solve_opts so = opts->solve;
  so.coarsen = opts->coarsen ? 1 : 0;
  so.timing = 0;
  double* dlb = nullptr;   // the certified stop (target_err) needs a lower bound of the proxy's diagonal
  if (so.target_err > 0.0) {
    dlb = c->ws.get<double>("nw.dlb", nw->n);
    k_nw_scale<<<grid_blocks(nw->n), kWG, 0, c->stream>>>((const double*)nw->mass.p, 1.0 / (h * h), nw->n, dlb);
    AGC_LAUNCH_CHECK();
  }
  for (int it = 0; it < opts->max_newton; ++it) {
    auto t0 = clock::now();
    nw_physics(c, nw, b, xcur, xhat, b.g, b.H);
    AGC_HIP(hipStreamSynchronize(c->stream));
    inf.ms_physics += (float)ms_since(t0);
    t0 = clock::now();
    if (opts->coarsen) {
      const agc_status st = agc_tag_edges(c, nw->tagger, xcur, xlast, opts->tag_threshold, tags, nullptr);
      if (st != AGC_OK) throw Error(st, c->err);
      AGC_HIP(hipStreamSynchronize(c->stream));
    }
    inf.ms_tags += (float)ms_since(t0);
    t0 = clock::now();
    agc_problem pr{};
    pr.mesh = nw->mesh;
    pr.n_edges = nw->m;
    pr.edges = (const int32_t*)nw->edges.p;
    pr.tags = tags;
    pr.elem_H = b.H;
    pr.g = b.g;
    pr.rest = (const double*)nw->rest.p;
    pr.diag_lb = dlb;   // m_v / h^2: the proxy is M / h^2 plus positive semidefinite blocks
    agc_solve_info si{};
    const agc_status st = agc_solve(c, &pr, &so, sol, nullptr, &si);
    if (st != AGC_OK && st != AGC_ERR_NOT_CONVERGED) throw Error(st, c->err);
    inf.ms_solve += (float)ms_since(t0);
    inf.pcg_iters += si.pcg_iters;
    inf.coarse_nodes_sum += si.n_coarse;
    t0 = clock::now();
    const double d_inf = nw_absmax(c, sol, n3);   // the direction is d = -sol
    double alpha = 1.0, e_new = e_prev;
    int halv = 0;
    bool moved = true;
    for (;;) {
      k_nw_step<<<grid_blocks(n3), kWG, 0, c->stream>>>(xcur, sol, alpha, n3, xnew);
      AGC_LAUNCH_CHECK();
      e_new = nw_energy(c, nw, b, xnew, xhat);
      if (e_new < e_prev) break;
      if (++halv > kMaxHalvings) {
        moved = false;
        e_new = e_prev;
        break;
      }
      alpha *= 0.5;
    }
    inf.ms_line += (float)ms_since(t0);
    inf.halvings += halv;
    inf.newton_iters = it + 1;
    inf.d_inf = d_inf;
    if (moved) {
      std::swap(xlast, xcur);   // the old iterate becomes the previous one
      std::swap(xcur, xnew);
    }
    e_prev = e_new;
    if (d_inf / h <= opts->eps_d || !moved) break;
  }
  inf.energy = e_prev;
  AGC_HIP(hipMemcpyAsync(x_out, xcur, sizeof(double) * n3, hipMemcpyDeviceToDevice, c->stream));
  AGC_HIP(hipStreamSynchronize(c->stream));
  if (info) *info = inf;
  API_END(c)
}

}  // extern "C"
