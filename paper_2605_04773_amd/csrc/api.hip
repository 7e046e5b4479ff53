// The C ABI of libagc: argument checks, error mapping, and the orchestration
// of one coarsened Newton linear solve in the order of Alg. overview
// (mapping, coarse assembly, coarse solve, prolongation).
#include <cmath>
#include <cstring>

#include <cstdlib>

#include "internal.h"

struct agc_matrix {
  agc::Matrix m;
};

namespace {

using agc::Error;


__global__ void k_iota_i32(int32_t* __restrict__ v, int32_t n) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    v[k] = (int32_t)k;
}

template <class T>
__global__ void k_planes_to_aos(const T* __restrict__ planes, int64_t nnzb, int64_t stride, T* __restrict__ out) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnzb; k += (int64_t)gridDim.x * blockDim.x)
#pragma unroll
    for (int i = 0; i < 9; ++i) out[9 * k + i] = planes[(int64_t)i * stride + k];
}

unsigned gsb(int64_t n) {
  int64_t b = (n + agc::kWG - 1) / agc::kWG;
  if (b > 65536) b = 65536;
  return (unsigned)(b < 1 ? 1 : b);
}

void check_status(int st, const char* what) {
  if (st == AGC_OK) return;
  if (st == AGC_ERR_NOT_CONVERGED) throw Error(st, std::string(what) + ": PCG did not reach the tolerance");
  if (st == AGC_ERR_NOT_SPD) throw Error(st, std::string(what) + ": matrix not SPD (singular 3x3 diagonal block, p^T A p <= 0 or NaN)");
  throw Error(st, what);
}

struct Timer {
  agc_context* c;
  bool on;
  int idx = 0;
  Timer(agc_context* cc, bool enabled) : c(cc), on(enabled) {}
  void mark() {
    if (on) AGC_HIP(hipEventRecord(c->ev[idx++], c->stream));
  }
  float ms(int a, int b) {
    if (!on) return 0.f;
    float t = 0.f;
    AGC_HIP(hipEventSynchronize(c->ev[b]));
    AGC_HIP(hipEventElapsedTime(&t, c->ev[a], c->ev[b]));
    return t;
  }
};

void validate_opts(const agc_solve_opts* o) {
  AGC_REQUIRE(o, "opts is null");
  AGC_REQUIRE(o->precision == AGC_PREC_FP64 || o->precision == AGC_PREC_MIXED, "bad precision");
  AGC_REQUIRE(o->coarsen == 0 || o->coarsen == 1, "coarsen must be 0 or 1");
  AGC_REQUIRE(o->rtol > 0.0 && o->rtol < 1.0, "rtol must be in (0, 1)");
  AGC_REQUIRE(o->max_iter >= 1, "max_iter must be >= 1");
  AGC_REQUIRE(o->post_iters >= 0, "post_iters must be >= 0");
  AGC_REQUIRE(o->affine_threshold >= 0, "affine_threshold must be >= 0");
  AGC_REQUIRE(o->target_err >= 0.0 && o->target_err < 1.0, "target_err must be in [0, 1)");
  AGC_REQUIRE(o->target_err == 0.0 || o->affine_threshold == 0, "target_err needs affine_threshold = 0");
  if (o->precision == AGC_PREC_MIXED) {
    AGC_REQUIRE(o->inner_rtol > 0.0 && o->inner_rtol < 1.0, "inner_rtol must be in (0, 1)");
    AGC_REQUIRE(o->max_refine >= 1, "max_refine must be >= 1");
  }
}

void validate_problem(const agc_problem* p) {
  AGC_REQUIRE(p && p->mesh, "problem or mesh is null");
  AGC_REQUIRE(p->elem_H && p->g, "elem_H and g are required");
  AGC_REQUIRE(((uintptr_t)p->elem_H & 15) == 0, "elem_H must be 16-byte aligned");
  AGC_REQUIRE(p->n_edges >= 0, "n_edges < 0");
  AGC_REQUIRE(((uintptr_t)p->edges & 7) == 0, "edges must be 8-byte aligned");
  AGC_REQUIRE(p->n_contacts >= 0 && (p->n_contacts == 0 || (p->contact_verts && p->contact_H)),
              "contact elements need ids and blocks");
}

agc::Contacts contacts_of(const agc_problem* p) {
  agc::Contacts x;
  x.n = p->n_contacts;
  x.verts = p->contact_verts;
  x.H = p->contact_H;
  return x;
}

// Solves A_c x_c = b_c for the matrix assembled from the problem.
//   map == nullptr: fine system.  members/mkeys: sorted members of map.
// Returns the PCG iterations and refinement steps through the pointers.
struct Restrictor {
  agc_context* c;
  int32_t n, n_c;
  const int32_t* map;        // nullptr: identity
  const uint32_t* members;
  const uint32_t* mkeys;
  const agc::AffineMap* am = nullptr;   // set: affine embedding of the large aggregates
  // coarse 3x3 block rows
  int32_t blocks() const { return am ? am->n_flat : n_c; }
  // out = P^T v
  void apply(const double* v, double* out) const {
    if (am) agc::affine_restrict(c, n, *am, members, mkeys, v, out);
    else if (map) agc::restrict_sorted(c, n, n_c, members, mkeys, v, out);
    else AGC_HIP(hipMemcpyAsync(out, v, sizeof(double) * 3 * (size_t)n, hipMemcpyDeviceToDevice, c->stream));
  }
};

struct SolveResult {
  int32_t iters = 0, refine = 0;
  double rel = 0.0;
  int64_t nnzb = 0;
  bool converged = true;   // false: max_iter (or max_refine) ended the solve; x_c is its last iterate
};

// Iterations on the assembled coarse system in the context (solve_a64, and
// solve_a for the mixed path) with right-hand side b_c (workspace
// "solve.b"), from x_c = 0 (warm = false) or from the x_c given (warm =
// true), until the float64 relative residual is <= rtol or max_iter PCG
// iterations have run.  Leaves r_c = b_c - A_c x_c (float64) in the
// workspace ("solve.rc").
SolveResult coarse_iterate(agc_context* c, const agc_solve_opts* o, int64_t n3c, double* x_c, double rtol,
                           int32_t max_iter, bool warm) {
  SolveResult res;
  const bool mixed = o->precision == AGC_PREC_MIXED;
  agc::Matrix& A64 = c->solve_a64;
  res.nnzb = A64.nnzb;
  double* b_c = c->ws.get<double>("solve.b", n3c);
  double* y = c->ws.get<double>("solve.y", n3c);
  double* r_c = c->ws.get<double>("solve.rc", n3c);
  double bn = 0.0, rn = 0.0;
  if (!mixed) {
    int32_t it = 0;
    double rel = 0.0;
    const int st = agc::pcg(c, A64, b_c, x_c, rtol, max_iter, &it, &rel, !warm);
    if (st == AGC_ERR_NOT_CONVERGED) res.converged = false;
    else check_status(st, "coarse PCG");
    res.iters = it;
    // float64 residual of the returned iterate
    agc::spmv(c, A64, x_c, y);
    agc::residual_norms(c, b_c, y, r_c, n3c, &bn, &rn);
    res.rel = bn > 0 ? rn / bn : 0.0;
    return res;
  }
  // mixed: iterative refinement x_c += A32^{-1} (b_c - A64 x_c), the inner
  // solves on the float32 values with float64 vectors and inner products
  agc::Matrix& A32 = c->solve_a;
  double* e_c = c->ws.get<double>("solve.ec", n3c);
  double rel = 1.0;
  int32_t used = 0;
  int k0 = 0;
  if (warm) {   // refinement from the given iterate: its float64 residual first
    agc::spmv(c, A64, x_c, y);
    agc::residual_norms(c, b_c, y, r_c, n3c, &bn, &rn);
    rel = bn > 0 ? rn / bn : 0.0;
    k0 = 1;
  }
  for (int k = k0;; ++k) {
    if (rel <= rtol || (warm && bn == 0.0)) break;
    if (k - k0 >= o->max_refine || used >= max_iter) {   // x_c keeps the last refined iterate
      res.converged = false;
      break;
    }
    int32_t it = 0;
    double irel = 0.0;
    // the inner tolerance is relative to ||r_c||; never ask for more than rtol needs
    const double want = rtol / rel;
    const double itol = want > o->inner_rtol ? want : o->inner_rtol;
    const int st = agc::pcg(c, A32, k == 0 ? b_c : r_c, k == 0 ? x_c : e_c, itol, max_iter - used, &it, &irel,
                            true);
    used += it;
    if (st != AGC_OK && st != AGC_ERR_NOT_CONVERGED) check_status(st, "inner PCG");
    if (k > 0) agc::axpy_vec(c, x_c, e_c, 1.0, n3c);
    res.refine = k;
    agc::spmv(c, A64, x_c, y);
    agc::residual_norms(c, b_c, y, r_c, n3c, &bn, &rn);
    if (bn == 0.0) break;
    rel = rn / bn;
  }
  res.iters = used;
  res.rel = bn > 0 ? rel : 0.0;
  return res;
}

// rhs_fine: the fine vector whose restriction is the right-hand side (g, or w for the adjoint)
SolveResult coarse_solve(agc_context* c, const agc_problem* p, const agc_solve_opts* o, const Restrictor& R,
                         const double* rhs_fine, double* x_c, Timer* tm) {
  const agc::Mesh& mesh = p->mesh->m;
  const int64_t n3c = 3 * (int64_t)R.blocks();
  double* b_c = c->ws.get<double>("solve.b", n3c);
  R.apply(rhs_fine, b_c);
  // Both precisions assemble P^T H P once in float64 (the reduction sums in
  // float64); the mixed path also keeps the float32 rounding of the values
  // for its inner PCG.  The float64 matrix gives the float64 residuals.
  const bool mixed = o->precision == AGC_PREC_MIXED;
  agc::Matrix& A64 = c->solve_a64;
  agc::Matrix* A32 = mixed ? &c->solve_a : nullptr;
  const agc::Contacts x = contacts_of(p);
  if (R.am) {
    agc::assemble_coarse_affine(c, mesh, p->elem_H, *R.am, A64, A32, false, x);
  } else if (R.map) {
    agc::assemble_coarse(c, mesh, p->elem_H, AGC_F64, R.map, R.n_c, AGC_F64, A64, A32, false, x);
  } else if (x.n > 0) {
    // the fine system with this call's contact pairs: the coarse assembly with the identity map
    int32_t* ident = c->ws.get<int32_t>("solve.ident", mesh.n_verts);
    k_iota_i32<<<gsb(mesh.n_verts), agc::kWG, 0, c->stream>>>(ident, mesh.n_verts);
    AGC_LAUNCH_CHECK();
    agc::assemble_coarse(c, mesh, p->elem_H, AGC_F64, ident, mesh.n_verts, AGC_F64, A64, A32, false, x);
  } else {
    agc::assemble_fine(c, mesh, p->elem_H, AGC_F64, AGC_F64, A64, A32);
  }
  if (tm) tm->mark();
  return coarse_iterate(c, o, n3c, x_c, o->rtol, o->max_iter, false);
}

}  // namespace

extern "C" {

const char* agc_version(void) { return "agc 0.1 (gfx950)"; }

agc_status agc_create(agc_context** out, int32_t device, void* stream) {
  if (!out) return AGC_ERR_INVALID_ARG;
  *out = nullptr;
  agc_context* c = new (std::nothrow) agc_context();
  if (!c) return AGC_ERR_OUT_OF_MEMORY;
  c->device = device;
  c->stream = (hipStream_t)stream;
  if (const char* e = std::getenv("AGC_PCG_REDUCE")) {
    if (e[0] == '0' && e[1] == 0) c->pcg_reduce = 0;
    if (e[0] == '1' && e[1] == 0) c->pcg_reduce = 1;
  }
  try {
    int ndev = 0;
    AGC_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) throw Error(AGC_ERR_INVALID_ARG, "no such device");
    AGC_HIP(hipSetDevice(device));
    AGC_HIP(hipMalloc(&c->d_err, 256));
    AGC_HIP(hipHostMalloc(&c->h_err, 256, hipHostMallocDefault));
    AGC_HIP(hipMalloc(&c->d_pcg, sizeof(agc::PcgState)));
    AGC_HIP(hipHostMalloc(&c->h_pcg, sizeof(agc::PcgState), hipHostMallocDefault));
    for (auto& e : c->ev) AGC_HIP(hipEventCreate(&e));
    agc::noalloc_setup(device);
  } catch (const Error& e) {
    agc_destroy(c);
    return e.code;
  }
  *out = c;
  return AGC_OK;
}

agc_status agc_set_stream(agc_context* c, void* stream) {
  if (!c) return AGC_ERR_INVALID_ARG;
  c->stream = (hipStream_t)stream;
  return AGC_OK;
}

agc_status agc_set_allocator(agc_context* c, agc_alloc_fn alloc, agc_free_fn free_fn, void* user) {
  if (!c) return AGC_ERR_INVALID_ARG;
  if ((alloc == nullptr) != (free_fn == nullptr)) {
    c->err = "alloc and free must both be set or both be null";
    return AGC_ERR_INVALID_ARG;
  }
  c->alloc = agc::Allocator{alloc, free_fn, user};
  return AGC_OK;
}

agc_status agc_destroy(agc_context* c) {
  if (!c) return AGC_ERR_INVALID_ARG;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  c->solve_a.release();
  c->solve_a64.release();
  c->solve_fine.release();
  c->ws.release();
  if (c->d_err) (void)hipFree(c->d_err);
  if (c->h_err) (void)hipHostFree(c->h_err);
  if (c->d_pcg) (void)hipFree(c->d_pcg);
  if (c->h_pcg) (void)hipHostFree(c->h_pcg);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
  return AGC_OK;
}

const char* agc_last_error(const agc_context* c) { return c ? c->err.c_str() : "null context"; }

// ------------------------------------------------------------------ mesh

agc_status agc_mesh_create(agc_context* c, int32_t n_verts, int64_t n_elems, const int32_t* elem_verts,
                           agc_mesh** mesh) {
  API_BEGIN(c)
  AGC_REQUIRE(mesh && elem_verts, "null pointer");
  AGC_REQUIRE(n_verts >= 1 && n_elems >= 1, "empty mesh");
  *mesh = nullptr;
  agc_mesh* m = new agc_mesh();
  try {
    agc::mesh_build(c, m->m, n_verts, n_elems, elem_verts);
  } catch (...) {
    m->m.release();
    delete m;
    throw;
  }
  *mesh = m;
  API_END(c)
}

agc_status agc_mesh_destroy(agc_context* c, agc_mesh* mesh) {
  API_BEGIN(c)
  AGC_REQUIRE(mesh, "null mesh");
  AGC_HIP(hipStreamSynchronize(c->stream));
  mesh->m.release();
  delete mesh;
  API_END(c)
}

agc_status agc_mesh_info(const agc_mesh* mesh, int32_t* n_verts, int64_t* n_elems, int64_t* fine_nnzb) {
  if (!mesh) return AGC_ERR_INVALID_ARG;
  if (n_verts) *n_verts = mesh->m.n_verts;
  if (n_elems) *n_elems = mesh->m.n_elems;
  if (fine_nnzb) *fine_nnzb = mesh->m.ff_nnzb;
  return AGC_OK;
}

// ------------------------------------------------------------------- map

agc_status agc_aggregate(agc_context* c, int32_t n_verts, int64_t n_edges, const int32_t* edges,
                         const uint8_t* tags, int32_t* map, int32_t* n_coarse) {
  API_BEGIN(c)
  AGC_REQUIRE(n_verts >= 0 && n_edges >= 0, "negative size");
  AGC_REQUIRE(n_coarse, "n_coarse is null");
  AGC_REQUIRE(n_verts == 0 || map, "map is null");
  AGC_REQUIRE(n_edges == 0 || (edges && tags), "edges/tags null");
  AGC_REQUIRE(((uintptr_t)edges & 7) == 0, "edges must be 8-byte aligned");
  *n_coarse = agc::aggregate(c, n_verts, n_edges, edges, tags, map);
  API_END(c)
}

// ------------------------------------------------------------- assembly

static void restrict_api(agc_context* c, int32_t n, const int32_t* map, int32_t n_c, const double* v, double* v_c) {
  uint32_t* members = c->ws.get<uint32_t>("api.members", n);
  uint32_t* mkeys = c->ws.get<uint32_t>("api.mkeys", n);
  agc::group_members(c, n, map, n_c, members, mkeys);
  agc::err_throw(agc::err_fetch(c));
  agc::restrict_sorted(c, n, n_c, members, mkeys, v, v_c);
}

agc_status agc_assemble_coarse(agc_context* c, const agc_mesh* mesh, const void* elem_H, int32_t h_dtype,
                               const double* g, const int32_t* map, int32_t n_coarse, int32_t out_dtype,
                               agc_matrix** A_c, double* g_c) {
  API_BEGIN(c)
  AGC_REQUIRE(mesh && elem_H && map && A_c, "null pointer");
  AGC_REQUIRE(h_dtype == AGC_F64 || h_dtype == AGC_F32, "bad h_dtype");
  AGC_REQUIRE(out_dtype == AGC_F64 || out_dtype == AGC_F32, "bad out_dtype");
  AGC_REQUIRE(n_coarse >= 1 && n_coarse <= mesh->m.n_verts, "n_coarse out of range");
  *A_c = nullptr;
  agc_matrix* a = new agc_matrix();
  try {
    agc::assemble_coarse(c, mesh->m, elem_H, h_dtype, map, n_coarse, out_dtype, a->m);
    if (g && g_c) restrict_api(c, mesh->m.n_verts, map, n_coarse, g, g_c);
    AGC_HIP(hipStreamSynchronize(c->stream));
  } catch (...) {
    a->m.release();
    delete a;
    throw;
  }
  *A_c = a;
  API_END(c)
}

agc_status agc_assemble_coarse_affine(agc_context* c, const agc_mesh* mesh, const double* elem_H, const double* rest,
                                      const double* g, const int32_t* map, int32_t n_coarse, int32_t threshold,
                                      agc_matrix** A_c, double* g_c, int32_t* n3, int32_t* n12) {
  API_BEGIN(c)
  AGC_REQUIRE(mesh && elem_H && rest && map && A_c, "null pointer");
  AGC_REQUIRE(((uintptr_t)elem_H & 15) == 0, "elem_H must be 16-byte aligned");
  AGC_REQUIRE(n_coarse >= 1 && n_coarse <= mesh->m.n_verts, "n_coarse out of range");
  *A_c = nullptr;
  const int32_t n = mesh->m.n_verts;
  uint32_t* members = c->ws.get<uint32_t>("api.members", n);
  uint32_t* mkeys = c->ws.get<uint32_t>("api.mkeys", n);
  agc::group_members(c, n, map, n_coarse, members, mkeys);
  agc::err_throw(agc::err_fetch(c));
  agc::AffineMap am;
  agc::affine_classify(c, n, map, members, mkeys, n_coarse, threshold, rest, am);
  agc_matrix* a = new agc_matrix();
  try {
    agc::assemble_coarse_affine(c, mesh->m, elem_H, am, a->m);
    if (g && g_c) agc::affine_restrict(c, n, am, members, mkeys, g, g_c);
    AGC_HIP(hipStreamSynchronize(c->stream));
  } catch (...) {
    a->m.release();
    delete a;
    throw;
  }
  *A_c = a;
  if (n3) *n3 = am.n3;
  if (n12) *n12 = am.n12;
  API_END(c)
}

agc_status agc_assemble_fine(agc_context* c, const agc_mesh* mesh, const void* elem_H, int32_t h_dtype,
                             int32_t out_dtype, agc_matrix** H) {
  API_BEGIN(c)
  AGC_REQUIRE(mesh && elem_H && H, "null pointer");
  AGC_REQUIRE(h_dtype == AGC_F64 || h_dtype == AGC_F32, "bad h_dtype");
  AGC_REQUIRE(out_dtype == AGC_F64 || out_dtype == AGC_F32, "bad out_dtype");
  *H = nullptr;
  agc_matrix* a = new agc_matrix();
  try {
    agc::assemble_fine(c, mesh->m, elem_H, h_dtype, out_dtype, a->m);
    AGC_HIP(hipStreamSynchronize(c->stream));
  } catch (...) {
    a->m.release();
    delete a;
    throw;
  }
  *H = a;
  API_END(c)
}

agc_status agc_matrix_destroy(agc_context* c, agc_matrix* a) {
  API_BEGIN(c)
  AGC_REQUIRE(a, "null matrix");
  AGC_HIP(hipStreamSynchronize(c->stream));
  a->m.release();
  delete a;
  API_END(c)
}

agc_status agc_matrix_info(const agc_matrix* a, int32_t* n_rows, int64_t* nnzb, int32_t* dtype) {
  if (!a) return AGC_ERR_INVALID_ARG;
  if (n_rows) *n_rows = a->m.n;
  if (nnzb) *nnzb = a->m.nnzb;
  if (dtype) *dtype = a->m.dtype;
  return AGC_OK;
}

agc_status agc_matrix_copy(agc_context* c, const agc_matrix* a, int32_t* row_ptr, int32_t* col_idx, void* vals) {
  API_BEGIN(c)
  AGC_REQUIRE(a, "null matrix");
  const agc::Matrix& m = a->m;
  if (row_ptr)
    AGC_HIP(hipMemcpyAsync(row_ptr, m.rp(), sizeof(int32_t) * (m.n + 1), hipMemcpyDeviceToDevice, c->stream));
  if (col_idx && m.nnzb)
    AGC_HIP(hipMemcpyAsync(col_idx, m.ci(), sizeof(int32_t) * m.nnzb, hipMemcpyDeviceToDevice, c->stream));
  if (vals && m.nnzb) {
    if (m.dtype == AGC_F64)
      k_planes_to_aos<double><<<gsb(m.nnzb), agc::kWG, 0, c->stream>>>((const double*)m.vals.p, m.nnzb, m.stride,
                                                                       (double*)vals);
    else
      k_planes_to_aos<float><<<gsb(m.nnzb), agc::kWG, 0, c->stream>>>((const float*)m.vals.p, m.nnzb, m.stride,
                                                                      (float*)vals);
    AGC_LAUNCH_CHECK();
  }
  AGC_HIP(hipStreamSynchronize(c->stream));
  API_END(c)
}

agc_status agc_spmv(agc_context* c, const agc_matrix* a, const double* x, double* y) {
  API_BEGIN(c)
  AGC_REQUIRE(a && x && y, "null pointer");
  AGC_REQUIRE(x != y, "x and y must not alias");
  agc::spmv(c, a->m, x, y);
  API_END(c)
}

agc_status agc_time_spmv(agc_context* c, const agc_matrix* a, const double* x, double* y, int32_t reps,
                         float* avg_ms) {
  API_BEGIN(c)
  AGC_REQUIRE(a && x && y && avg_ms && reps >= 1, "bad argument");
  AGC_REQUIRE(x != y, "x and y must not alias");
  agc::spmv(c, a->m, x, y);   // warm
  AGC_HIP(hipEventRecord(c->ev[0], c->stream));
  for (int i = 0; i < reps; ++i) agc::spmv(c, a->m, x, y);
  AGC_HIP(hipEventRecord(c->ev[1], c->stream));
  AGC_HIP(hipEventSynchronize(c->ev[1]));
  float ms = 0.f;
  AGC_HIP(hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
  *avg_ms = ms / (float)reps;
  API_END(c)
}

// ------------------------------------------------------------------ PCG

agc_status agc_pcg(agc_context* c, const agc_matrix* a, const double* b, double* x, double rtol, int32_t max_iter,
                   agc_pcg_info* info) {
  API_BEGIN(c)
  AGC_REQUIRE(a && b && x, "null pointer");
  AGC_REQUIRE(rtol > 0.0 && rtol < 1.0, "rtol must be in (0, 1)");
  AGC_REQUIRE(max_iter >= 0, "max_iter < 0");
  int32_t it = 0;
  double rel = 0.0;
  const int st = agc::pcg(c, a->m, b, x, rtol, max_iter, &it, &rel);
  if (info) {
    info->iters = it;
    info->rel_res = rel;
  }
  check_status(st, "agc_pcg");
  API_END(c)
}

// ------------------------------------------------------ prolongation, P^T

agc_status agc_prolongate(agc_context* c, int32_t n_verts, const int32_t* map, int32_t n_coarse, const double* x_c,
                          double* x) {
  API_BEGIN(c)
  AGC_REQUIRE(n_verts >= 0 && n_coarse >= 0, "negative size");
  AGC_REQUIRE(n_verts == 0 || (map && x_c && x), "null pointer");
  agc::err_reset(c);
  agc::prolongate(c, n_verts, map, n_coarse, x_c, x);
  agc::err_throw(agc::err_fetch(c));
  API_END(c)
}

agc_status agc_restrict(agc_context* c, int32_t n_verts, const int32_t* map, int32_t n_coarse, const double* v,
                        double* v_c) {
  API_BEGIN(c)
  AGC_REQUIRE(n_verts >= 0 && n_coarse >= 0, "negative size");
  AGC_REQUIRE(n_verts == 0 || (map && v && v_c), "null pointer");
  if (n_verts > 0) restrict_api(c, n_verts, map, n_coarse, v, v_c);
  AGC_HIP(hipStreamSynchronize(c->stream));
  API_END(c)
}

// ------------------------------------------------------------ all in one

agc_status agc_solve(agc_context* c, const agc_problem* p, const agc_solve_opts* o, double* x, int32_t* map_out,
                     agc_solve_info* info) {
  API_BEGIN(c)
  validate_problem(p);
  validate_opts(o);
  AGC_REQUIRE(x, "x is null");
  const agc::Mesh& mesh = p->mesh->m;
  const int32_t n = mesh.n_verts;
  AGC_REQUIRE(o->coarsen == 0 || p->n_edges == 0 || (p->edges && p->tags), "edges/tags null");
  Timer tm(c, o->timing != 0);
  struct KernelTiming {   // on for this call only, also when it throws
    agc_context* c;
    ~KernelTiming() { c->kernel_timing = false; }
  } kt_scope{c};
  c->kernel_timing = o->timing >= 2;
  c->spmv_ms = 0.0;
  c->spmv_n = 0;
  tm.mark();                                                   // 0
  Restrictor R{c, n, n, nullptr, nullptr, nullptr};
  int32_t* map = nullptr;
  if (o->coarsen) {
    map = map_out ? map_out : c->ws.get<int32_t>("solve.map", n);
    R.n_c = agc::aggregate(c, n, p->n_edges, p->edges, p->tags, map);
    R.map = map;
    uint32_t* members = c->ws.get<uint32_t>("solve.members", n);
    uint32_t* mkeys = c->ws.get<uint32_t>("solve.mkeys", n);
    agc::group_members(c, n, map, R.n_c, members, mkeys);
    R.members = members;
    R.mkeys = mkeys;
  } else if (map_out) {
    k_iota_i32<<<gsb(n), agc::kWG, 0, c->stream>>>(map_out, n);
    AGC_LAUNCH_CHECK();
  }
  agc::AffineMap am;
  if (R.map && o->affine_threshold > 0) {
    agc::affine_classify(c, n, R.map, R.members, R.mkeys, R.n_c, o->affine_threshold, p->rest, am);
    R.am = &am;
  }
  tm.mark();                                                   // 1
  double* x_c = R.map ? c->ws.get<double>("solve.xc", 3 * (int64_t)R.blocks()) : x;
  SolveResult res = coarse_solve(c, p, o, R, p->g, x_c, &tm);  // marks 2 after assembly
  // certified error of P x_c; with target_err, more iterations until it holds
  double err_bound = -1.0;
  if (p->diag_lb && !R.am) {
    const int64_t n3c = 3 * (int64_t)R.blocks();
    const double* r_c = c->ws.get<double>("solve.rc", n3c);
    auto rel_bound = [&]() {
      const agc::Certificate ct = agc::certify(c, n, R.n_c, R.map, R.members, R.mkeys, p->diag_lb, x_c, r_c);
      return ct.x_norm > 0.0 ? ct.bound / ct.x_norm : (ct.bound > 0.0 ? INFINITY : 0.0);
    };
    err_bound = rel_bound();
    while (o->target_err > 0.0 && err_bound > o->target_err && res.converged && res.iters < o->max_iter) {
      const double f = o->target_err / err_bound;
      const double rtol2 = res.rel * (f < 0.01 ? 0.01 : (f > 0.5 ? 0.5 : f));
      const SolveResult more = coarse_iterate(c, o, n3c, x_c, rtol2, o->max_iter - res.iters, true);
      res.iters += more.iters;
      res.refine += more.refine;
      res.rel = more.rel;
      res.converged = more.converged;
      err_bound = rel_bound();
    }
    if (o->target_err > 0.0 && err_bound > o->target_err) res.converged = false;
  } else {
    AGC_REQUIRE(o->target_err == 0.0, "target_err needs prob.diag_lb");
  }
  tm.mark();                                                   // 3
  if (R.map) {
    agc::err_reset(c);
    if (R.am) agc::affine_prolongate(c, n, am, x_c, x);
    else agc::prolongate(c, n, R.map, R.n_c, x_c, x);
  }
  tm.mark();                                                   // 4
  // post-coarsening (Sec. 4.3): a few fine PCG iterations from x = P x_c
  int32_t post_done = 0;
  double fine_rel0 = 0.0, fine_rel = 0.0;
  if (o->post_iters > 0 && R.map) {
    agc::Matrix& F = c->solve_fine;
    // the coarse assembly just gathered the fine upper blocks of these element
    // blocks; this call's contact pairs join them through the coarse assembly
    // with the identity map
    const agc::Contacts xc = contacts_of(p);
    if (xc.n > 0) {
      int32_t* ident = c->ws.get<int32_t>("solve.ident", n);
      k_iota_i32<<<gsb(n), agc::kWG, 0, c->stream>>>(ident, n);
      AGC_LAUNCH_CHECK();
      agc::assemble_coarse(c, mesh, p->elem_H, AGC_F64, ident, n, AGC_F64, F, nullptr, true, xc);
    } else {
      agc::assemble_fine(c, mesh, p->elem_H, AGC_F64, AGC_F64, F, nullptr, true);
    }
    const int64_t n3 = 3 * (int64_t)n;
    double* y = c->ws.get<double>("post.y", n3);
    double* r = c->ws.get<double>("post.r", n3);
    double gn = 0.0;
    agc::spmv(c, F, x, y);
    agc::residual_norms(c, p->g, y, r, n3, &gn, &fine_rel0);
    fine_rel0 = gn > 0.0 ? fine_rel0 / gn : 0.0;
    double rel = 0.0;
    const int st = agc::pcg(c, F, p->g, x, o->rtol, o->post_iters, &post_done, &rel);
    if (st != AGC_OK && st != AGC_ERR_NOT_CONVERGED) check_status(st, "post-coarsening PCG");
    agc::spmv(c, F, x, y);
    agc::residual_norms(c, p->g, y, r, n3, &gn, &fine_rel);
    fine_rel = gn > 0.0 ? fine_rel / gn : 0.0;
  }
  tm.mark();                                                   // 5
  AGC_HIP(hipStreamSynchronize(c->stream));
  if (info) {
    info->n_coarse = R.n_c;
    info->nnzb = res.nnzb;
    info->pcg_iters = res.iters;
    info->refine_iters = res.refine;
    info->rel_res = res.rel;
    info->ms_aggregate = tm.ms(0, 1);
    info->ms_assemble = tm.ms(1, 2);
    info->ms_pcg = tm.ms(2, 3);
    info->ms_prolong = tm.ms(3, 4);
    info->spmv_launches = (int32_t)c->spmv_n;
    info->ms_spmv = (float)c->spmv_ms;
    info->n_affine = R.am ? am.n12 : 0;
    info->n_blocks = R.blocks();
    info->post_iters = post_done;
    info->fine_rel_res = fine_rel;
    info->fine_rel_res0 = fine_rel0;
    info->ms_post = tm.ms(4, 5);
    info->err_bound = err_bound;
  }
  if (!res.converged)
    throw Error(AGC_ERR_NOT_CONVERGED, "coarse PCG did not reach rtol (or target_err) within max_iter / max_refine: "
                                       "x holds P times the last coarse iterate");
  API_END(c)
}

agc_status agc_solve_backward(agc_context* c, const agc_problem* p, const agc_solve_opts* o, const int32_t* map,
                              int32_t n_coarse, const double* x, const double* w, double* dg, double* dH,
                              agc_solve_info* info) {
  API_BEGIN(c)
  validate_problem(p);
  validate_opts(o);
  AGC_REQUIRE(o->post_iters == 0 && o->affine_threshold == 0,
              "post_iters and affine_threshold must be 0 for the derivative of the coarsened solve");
  AGC_REQUIRE(x && w && dg, "null pointer");
  const agc::Mesh& mesh = p->mesh->m;
  const int32_t n = mesh.n_verts;
  Restrictor R{c, n, n, nullptr, nullptr, nullptr};
  if (o->coarsen) {
    AGC_REQUIRE(map, "map is null");
    AGC_REQUIRE(n_coarse >= 1 && n_coarse <= n, "n_coarse out of range");
    R.n_c = n_coarse;
    R.map = map;
    uint32_t* members = c->ws.get<uint32_t>("solve.members", n);
    uint32_t* mkeys = c->ws.get<uint32_t>("solve.mkeys", n);
    agc::group_members(c, n, map, n_coarse, members, mkeys);
    agc::err_throw(agc::err_fetch(c));
    R.members = members;
    R.mkeys = mkeys;
  }
  // lambda_c = A_c^{-1} P^T w (A_c symmetric, assembled again from the map)
  double* lam_c = R.map ? c->ws.get<double>("bwd.lc", 3 * (int64_t)R.n_c) : dg;
  SolveResult res = coarse_solve(c, p, o, R, w, lam_c, nullptr);
  if (R.map) {
    agc::err_reset(c);
    agc::prolongate(c, n, R.map, R.n_c, lam_c, dg);   // dL/dg = P lambda_c
  }
  if (dH) {                                            // dL/dH_e = -(S_e P lambda_c)(S_e x)^T
    agc::elem_outer(c, mesh, dg, x, dH);
    // then the call's contact elements (their ids were checked by the solve above)
    agc::elem_outer_list(c, p->contact_verts, p->n_contacts, dg, x, dH + 144 * mesh.n_elems);
  }
  agc::err_throw(agc::err_fetch(c));
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->n_coarse = R.n_c;
    info->nnzb = res.nnzb;
    info->pcg_iters = res.iters;
    info->refine_iters = res.refine;
    info->rel_res = res.rel;
  }
  if (!res.converged)
    throw Error(AGC_ERR_NOT_CONVERGED, "adjoint PCG did not reach rtol within max_iter / max_refine: dg and dH are "
                                       "those of the last coarse iterate");
  API_END(c)
}

}  // extern "C"
