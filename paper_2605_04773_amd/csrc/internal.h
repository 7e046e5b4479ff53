// Internal interfaces of libagc (not part of the ABI).
#pragma once

#include <map>
#include <tuple>

#include "common.h"

namespace agc {

// A BSR 3x3 matrix with full symmetric storage.  vals holds 9 planes:
// vals[(3r+s)*stride + k] is entry (r, s) of block k, so the nine loads of one
// block by consecutive lanes are each contiguous; stride is nnzb rounded up to
// a multiple of 64 so that every plane starts 256-byte aligned.  rowidx[k] is
// the block row of block k (used by the nonzero-balanced SpMV); diag[r] the
// position of the diagonal block of row r.
inline int64_t plane_stride(int64_t nnzb) { return (nnzb + 63) / 64 * 64; }

struct Matrix {
  int32_t n = 0;
  int64_t nnzb = 0;
  int64_t stride = 0;
  int32_t dtype = AGC_F64;
  DevBuf row_ptr, col, rowidx, diag, vals;
  // a matrix may borrow a static pattern (the fine matrix uses its mesh's)
  const int32_t *ext_rp = nullptr, *ext_ci = nullptr, *ext_ri = nullptr, *ext_dg = nullptr;
  int32_t* rp() const { return ext_rp ? (int32_t*)ext_rp : (int32_t*)row_ptr.p; }
  int32_t* ci() const { return ext_ci ? (int32_t*)ext_ci : (int32_t*)col.p; }
  int32_t* ri() const { return ext_ri ? (int32_t*)ext_ri : (int32_t*)rowidx.p; }
  int32_t* dg() const { return ext_dg ? (int32_t*)ext_dg : (int32_t*)diag.p; }
  // capacity for up to nb blocks; set_nnzb fixes the final count and stride
  void reserve(int32_t n_rows, int64_t nb, int32_t dt) {
    ext_rp = ext_ci = ext_ri = ext_dg = nullptr;
    row_ptr.ensure(sizeof(int32_t) * (size_t)(n_rows + 1));
    col.ensure(sizeof(int32_t) * (size_t)(plane_stride(nb) + 4));
    rowidx.ensure(sizeof(int32_t) * (size_t)(plane_stride(nb) + 4));
    diag.ensure(sizeof(int32_t) * (size_t)(n_rows + 1));
    reserve_values(n_rows, nb, dt);
  }
  void reserve_values(int32_t n_rows, int64_t nb, int32_t dt) {
    n = n_rows;
    dtype = dt;
    vals.ensure((dt == AGC_F64 ? 8 : 4) * 9 * (size_t)(plane_stride(nb) + 4));
    set_nnzb(nb);
  }
  void borrow_pattern(const int32_t* rp_, const int32_t* ci_, const int32_t* ri_, const int32_t* dg_) {
    ext_rp = rp_;
    ext_ci = ci_;
    ext_ri = ri_;
    ext_dg = dg_;
  }
  void set_nnzb(int64_t nb) {
    nnzb = nb;
    stride = plane_stride(nb);
  }
  void release() {
    row_ptr.release(); col.release(); rowidx.release(); diag.release(); vals.release();
    ext_rp = ext_ci = ext_ri = ext_dg = nullptr;
  }
};

// Static structure of a mesh.
struct Mesh {
  int32_t n_verts = 0;
  int64_t n_elems = 0;
  DevBuf elem_verts;     // private copy, [n_elems][4]
  // fine upper pattern (row <= col), sorted by (row, col)
  int64_t nf = 0;
  DevBuf fu_row, fu_col;
  DevBuf plan_ptr;       // [nf+1] into plan
  DevBuf plan;           // [10 n_elems]: e*16 + a*4 + b, sub-block (a,b) of H_e
  // full fine pattern from the upper one
  int64_t ff_nnzb = 0;
  DevBuf ff_row_ptr, ff_col, ff_rowidx, ff_src, ff_diag;   // src = upper*2 + transposed
  // Tables of the fine gather.  A piece is rows 3a..3a+2 of an element
  // block, a the local index of a vertex v of the element: the upper blocks
  // of row v read only the pieces of the elements around v.
  DevBuf piece_src;      // [4 n_elems] e*4 + a of each piece, rows in order, elements in order
  DevBuf pentry;         // [10 n_elems] u16: plan entry k as (piece within its workgroup) * 4 + b
  DevBuf wg_info;        // [n_wg][8] u32 per gather workgroup: first piece, pieces, blocks [f0, f1), plan [k0, k1)
  int64_t n_wg = 0;
  void release() {
    elem_verts.release(); fu_row.release(); fu_col.release(); plan_ptr.release(); plan.release();
    ff_row_ptr.release(); ff_col.release(); ff_rowidx.release(); ff_src.release(); ff_diag.release();
    piece_src.release(); pentry.release(); wg_info.release();
  }
};

constexpr int kMaxChunk = 256;   // PCG iterations enqueued between two host checks

// Device PCG scalars.
constexpr int kRrRing = 16;
struct PcgState {
  double rz_hist[2];              // gamma_j = r_j^T z_j, by parity of j
  double alpha_hist[2];           // alpha_j, by parity of j
  double rr, bb, tol2;
  int32_t iter, max_iter, done;   // done: 0 running, 1 converged, 2 max_iter, 3 breakdown
  int32_t pad;
  double rr_ring[kRrRing];        // r_j^T r_j at slot j % kRrRing (the host's convergence-rate estimate)
};

// ----------------------------------------------------------- primitives
// out[0..n] = exclusive scan of in[0..n), out[n] = total.  out may equal in.
void scan_u32(agc_context* c, const uint32_t* in, uint32_t* out, int64_t n, const std::string& tag);
// Stable LSD radix sort of (key, val) pairs on bits [0, nbits).  Returns true
// when the result ended in the *_alt arrays.
bool radix_sort_u64(agc_context* c, uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                    uint32_t* vals_alt, int64_t n, int nbits, const std::string& tag);
bool radix_sort_u32(agc_context* c, uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                    uint32_t* vals_alt, int64_t n, int nbits, const std::string& tag);

// error word helpers
void err_reset(agc_context* c);
unsigned err_fetch(agc_context* c);   // synchronises
void err_throw(unsigned bits);        // throws on a nonzero word

// out[0..n] = exclusive scan as scan_u32, with the caller's buffer of
// scan_sums_words(n) words for the tile sums (no workspace)
int64_t scan_sums_words(int64_t n);
void scan_u32_into(agc_context* c, const uint32_t* in, uint32_t* out, int64_t n, uint32_t* sums);

// ------------------------------------------------------------ aggregation
// Scratch of one aggregation of n vertices, carved from agg_scratch_words(n)
// 32-bit words by agg_scratch_carve (256-byte aligned base).
struct AggScratch {
  int32_t* parent = nullptr;     // [n]
  uint64_t* bits = nullptr;      // [nw]: root flags, 64 vertices per word
  uint32_t* lrank = nullptr;     // [nw]: roots in the words before, within a tile of 64 words
  uint32_t* tsum = nullptr;      // [tiles + 1]: roots per tile
  uint32_t* tp = nullptr;        // [tiles + 1]: exclusive prefix of tsum (very large n only)
  uint32_t* scan_sums = nullptr; // [scan_sums_words(tiles)]
  int64_t* bounds = nullptr;     // [vertex blocks + 1]: first edge of each block's range
};
int64_t agg_root_tiles(int32_t n);
int64_t agg_scratch_words(int32_t n);
AggScratch agg_scratch_carve(uint32_t* base, int32_t n);
// map and n_coarse with the given scratch; allocates nothing (synchronises)
int32_t aggregate_into(agc_context* c, int32_t n, int64_t m, const int32_t* edges, const uint8_t* tags,
                       int32_t* map, const AggScratch& s);
// device address of the no-allocation scratch array on `device` (current), looked up once per device
void noalloc_setup(int device);
// the same with scratch from the context's workspace
int32_t aggregate(agc_context* c, int32_t n, int64_t m, const int32_t* edges, const uint8_t* tags,
                  int32_t* map);
// Certified error of x = P x_c from its float64 residual r_c = b_c - A_c x_c
// and a lower bound d of H's diagonal per vertex (H >= diag(d) (x) I_3, e.g.
// the lumped masses over h^2): A_c >= diag(D_c) with D_c the sum of d over
// the members of c, so the error e_c satisfies ||e_c||_D <= ||r_c||_{D^-1},
// and ||P e_c||_2 <= ||P e_c||_d / sqrt(min d) = ||e_c||_D / sqrt(min d).
// map null: the fine system (D = d).  Synchronises; AGC_ERR_BAD_INPUT for a
// d_v that is not positive and finite.
struct Certificate {
  double bound = 0.0;    // bound on ||P x_c - P x_c*||_2
  double x_norm = 0.0;   // ||P x_c||_2
};
Certificate certify(agc_context* c, int32_t n, int32_t n_c, const int32_t* map, const uint32_t* members,
                    const uint32_t* mkeys, const double* d, const double* x_c, const double* r_c);
// members[k]: vertices sorted by (map, id); mkeys[k] = map[members[k]]
void group_members(agc_context* c, int32_t n, const int32_t* map, int32_t n_c, uint32_t* members,
                   uint32_t* mkeys);
// v_c[c] = sum over members of v (fixed order)
void restrict_sorted(agc_context* c, int32_t n, int32_t n_c, const uint32_t* members,
                     const uint32_t* mkeys, const double* v, double* v_c);
// x[v] = x_c[map[v]]; a map value outside [0, n_c) sets kErrMap and writes 0
void prolongate(agc_context* c, int32_t n, const int32_t* map, int32_t n_c, const double* x_c, double* x);

// --------------------------------------------------------- affine embedding
// Coarse nodes with more than `threshold` members carry 12 DoF (Eq. 4):
// x_f = sum_k Xbar_f[k] q_c[k] over four 3-blocks k, Xbar_f = (X, Y, Z, 1) the
// rest position in the aggregate's frame (origin at its smallest-id member).
// New node order: 3-DoF nodes first (canonical order), then 12-DoF nodes; a
// node's first flat 3-block is offset[c] (3-DoF: its new label; 12-DoF:
// n3 + 4 (label - n3)).
struct AffineMap {
  int32_t n_c = 0, n3 = 0, n12 = 0, n_flat = 0;
  const int32_t* map = nullptr;    // [n] canonical labels
  const double* rest = nullptr;    // [n][3] rest positions
  int32_t* newlab = nullptr;       // [n_c]
  int32_t* offset = nullptr;       // [n_c]
  int32_t* rep = nullptr;          // [n_c] smallest member id
};
// members/mkeys: from group_members (every label must have members)
void affine_classify(agc_context* c, int32_t n, const int32_t* map, const uint32_t* members,
                     const uint32_t* mkeys, int32_t n_c, int32_t threshold, const double* rest,
                     AffineMap& am);
// v_flat = P^T v (members/mkeys from group_members)
void affine_restrict(agc_context* c, int32_t n, const AffineMap& am, const uint32_t* members,
                     const uint32_t* mkeys, const double* v, double* v_flat);
// x = P x_flat; a map value outside [0, n_c) sets kErrMap and writes 0
void affine_prolongate(agc_context* c, int32_t n, const AffineMap& am, const double* x_flat, double* x);

// ------------------------------------------------------------- assembly
void mesh_build(agc_context* c, Mesh& m, int32_t n_verts, int64_t n_elems, const int32_t* ev);
// out32 (float64 output only, may be null) receives the same matrix rounded
// to float32; it borrows out's pattern, so out must outlive its use.
// reuse_upper: take the fine upper blocks that the last float64 assembly of
// the same element blocks left in the workspace instead of gathering them again
void assemble_fine(agc_context* c, const Mesh& m, const void* elem_h, int32_t h_dtype,
                   int32_t out_dtype, Matrix& out, Matrix* out32 = nullptr, bool reuse_upper = false);
// Per-call elements beside the mesh's (contact stencils found anew every
// Newton iteration): [n][4] ids and [n][144] float64 row-major blocks, keyed
// at the coarse level on each call instead of entering the static plan.
struct Contacts {
  int64_t n = 0;
  const int32_t* verts = nullptr;
  const double* H = nullptr;
};
// reuse_upper (float64 only): the fine upper blocks are already in the
// workspace (an assembly of the same element blocks just before)
void assemble_coarse(agc_context* c, const Mesh& m, const void* elem_h, int32_t h_dtype,
                     const int32_t* map, int32_t n_c, int32_t out_dtype, Matrix& out,
                     Matrix* out32 = nullptr, bool reuse_upper = false, const Contacts& x = Contacts{});
// A = P^T H P in the flat 3-block layout of `am` (float64 sums; out32 as for
// assemble_coarse)
void assemble_coarse_affine(agc_context* c, const Mesh& m, const double* elem_h, const AffineMap& am,
                            Matrix& out, Matrix* out32 = nullptr, bool reuse_upper = false,
                            const Contacts& x = Contacts{});
// dH_e = -(dg_e)(x_e)^T
void elem_outer(agc_context* c, const Mesh& m, const double* dg, const double* x, double* dh);
// the same over a list of elements ([ne][4] ids, checked by the caller)
void elem_outer_list(agc_context* c, const int32_t* ev, int64_t ne, const double* dg, const double* x, double* dh);

// ------------------------------------------------------------------ PCG
void spmv(agc_context* c, const Matrix& a, const double* x, double* y);
// returns status (AGC_OK / NOT_CONVERGED / NOT_SPD); *iters, *rel set.
// x holds x0 on entry, or x_zero says x0 = 0 (x is then output only).
int pcg(agc_context* c, const Matrix& a, const double* b, double* x, double rtol, int32_t max_iter,
        int32_t* iters, double* rel, bool x_zero = false);
// ||v||_2 of an [n][3] vector (float64, fixed order); synchronises
double norm2(agc_context* c, const double* v, int64_t n3, const std::string& tag);
void axpy_vec(agc_context* c, double* y, const double* x, double a, int64_t n3);
// r = b - y and the float64 norms of b and r (fixed order); synchronises
void residual_norms(agc_context* c, const double* b, const double* y, double* r, int64_t n3, double* bn,
                    double* rn);

}  // namespace agc

// --------------------------------------------------------------- context
struct agc_context {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  agc::Workspace ws;
  unsigned* d_err = nullptr;   // device error word for the current call
  unsigned* h_err = nullptr;   // pinned host mirror
  void* d_pcg = nullptr;       // device PCG state (agc::PcgState)
  void* h_pcg = nullptr;       // pinned host mirror
  hipEvent_t ev[8] = {};        // 0-5 phase timer, 6-7 SpMV replay timing
  bool kernel_timing = false;   // replay and time the PCG SpMV after each PCG solve
  double spmv_ms = 0.0;         // summed duration of the timed SpMV launches
  int64_t spmv_n = 0;
  // PCG partial-sum reduction between the SpMV and the update: -1 when the
  // system is large enough (the default), 0 never, 1 always; set at creation
  // from the environment variable AGC_PCG_REDUCE ("0" or "1"), for testing
  int pcg_reduce = -1;
  agc::Allocator alloc;         // device memory source of new buffers (agc_set_allocator)
  // iterations of the last PCG solve per (rows in ~4% steps, matrix dtype,
  // rtol in quarter decades): the first chunk of the next such solve
  // (chunking never changes the iterates)
  std::map<std::tuple<int32_t, int32_t, int32_t>, int32_t> pcg_last;
  agc::Matrix solve_a;         // matrices reused across agc_solve calls
  agc::Matrix solve_a64;
  agc::Matrix solve_fine;      // the fine system for post-coarsening
};

struct agc_mesh {
  agc::Mesh m;
};

// Static data of the strain-increment tags (tagging.hip); the destructor
// releases the device buffers, also when creation fails half way.
struct agc_tagger {
  int32_t n = 0;
  int64_t ne = 0, m = 0, nu = 0;
  agc::DevBuf tets, dminv, tedge, ekey, hot, count;
  void release() {
    tets.release(); dminv.release(); tedge.release(); ekey.release(); hot.release(); count.release();
  }
  ~agc_tagger() { release(); }
};

// Entry-point frame: a C++ exception never crosses the ABI; its message is
// kept in the context and its code returned.
#define API_BEGIN(ctx)                                \
  if (!(ctx)) return AGC_ERR_INVALID_ARG;             \
  (ctx)->err.clear();                                 \
  try {                                               \
    ::agc::AllocScope agc_alloc_scope_(&(ctx)->alloc);  \
    AGC_HIP(hipSetDevice((ctx)->device));

#define API_END(ctx)                                  \
  }                                                   \
  catch (const ::agc::Error& e) {                     \
    (ctx)->err = e.what();                            \
    return e.code;                                    \
  }                                                   \
  catch (const std::exception& e) {                   \
    (ctx)->err = e.what();                            \
    return AGC_ERR_DEVICE;                            \
  }                                                   \
  catch (...) {                                       \
    (ctx)->err = "unknown failure";                   \
    return AGC_ERR_DEVICE;                            \
  }                                                   \
  return AGC_OK;
