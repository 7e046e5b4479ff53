/*
 * agc.h - in-solve algebraic coarsening for one Newton linear solve of
 * implicit IPC, on AMD MI355X (gfx950).
 *
 * The method (Wang et al., "AGIPC: Adaptive In-Solve Algebraic Coarsening for
 * GPU IPC", SIGGRAPH 2026) replaces the Newton system H d = -g (Sec. 3,
 * Eq. 2) by a Galerkin coarse system built from per-edge collapse tags:
 *
 *   map  : fine vertex -> super-node, connected components of the graph of
 *          collapsible edges (Sec. 4.1; supplement Sec. 1, Alg. 1-2)
 *   A_c  = P^T H P,  b_c = P^T g      (Sec. 4.1, Galerkin equivalence)
 *   x_c  = A_c^{-1} b_c by 3x3 block-Jacobi PCG   (Alg. overview; Sec. 5.1)
 *   x    = P x_c                      (Sec. 4.3, prolongation)
 *
 * P is the 3n x 3n_c 0/1 matrix with P[3v+i][3 map(v)+i] = 1 (the paper's
 * restriction U is P^T).  The library returns x = P A_c^{-1} P^T g; the Newton
 * direction is d = -x.
 *
 * Conventions for every call:
 *  - Array arguments are DEVICE pointers unless marked [host].  They are
 *    owned by the caller, must stay valid until the call's work on the
 *    context's stream has finished, and are never freed by the library.
 *  - Work is enqueued on the context's HIP stream.  Calls that return a
 *    [host] value synchronise that stream before returning.
 *  - Every call returns an agc_status.  No C++ exception crosses this ABI.
 *    On a non-OK status agc_last_error() describes the failure.
 *  - Vectors of vertices are [n][3] float64, DoF order 3v+k.
 *  - A context is not thread-safe; use one context per host thread.
 *  - HIP errors (including a failed allocation) leave the context usable
 *    only for agc_destroy and agc_last_error.
 */
#ifndef AGC_H
#define AGC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t agc_status;
enum {
  AGC_OK = 0,
  AGC_ERR_INVALID_ARG = -1,   /* null pointer, negative size, bad enum: nothing was enqueued    */
  AGC_ERR_OUT_OF_MEMORY = -2, /* device allocation failed                                       */
  AGC_ERR_DEVICE = -3,        /* a HIP runtime call failed                                      */
  AGC_ERR_NOT_CONVERGED = -4, /* PCG hit max_iter: x holds the last iterate                     */
  AGC_ERR_NOT_SPD = -5,       /* a 3x3 diagonal block is not SPD, p^T A p <= 0, or NaN/Inf seen */
  AGC_ERR_BAD_INPUT = -6      /* device data out of range: vertex id, tag not 0/1, etc.         */
};

enum { AGC_F64 = 0, AGC_F32 = 1 };                 /* element / matrix value type */
enum { AGC_PREC_FP64 = 0, AGC_PREC_MIXED = 1 };    /* solve precision            */

typedef struct agc_context agc_context; /* owns workspace, binds one device + stream     */
typedef struct agc_mesh agc_mesh;       /* static element topology (built once per mesh) */
typedef struct agc_matrix agc_matrix;   /* assembled BSR 3x3 matrix, device resident     */

/* ---------------------------------------------------------------- context */

/* Creates a context on HIP device `device`, enqueuing on `stream` (a
 * hipStream_t; NULL = the legacy default stream).  *ctx receives the handle.
 * The environment variable AGC_PCG_REDUCE, read here, selects how the PCG
 * sums its per-workgroup partials: unset (or any other value) = by system
 * size, "0" = inside the update kernel always, "1" = in a separate reduction
 * kernel always.  The two differ only in summation order. */
agc_status agc_create(agc_context** ctx, int32_t device, void* stream);

/* Device memory for the buffers the context allocates from now on (its
 * workspace, the matrices it returns, and the meshes, taggers and Newton
 * handles created through it) comes from alloc(bytes, user) and goes back
 * through free(ptr, user), e.g. a framework's caching allocator, instead of
 * hipMalloc / hipFree; both NULL restores hipMalloc.  Buffers keep the
 * source they were allocated from.  Blocks are requested and returned in the
 * order of the context's stream: a stream-ordered allocator must serve that
 * stream.  alloc returning NULL gives AGC_ERR_OUT_OF_MEMORY.  The functions
 * must stay callable until every block they gave out has been returned
 * (agc_destroy, and the destroy call of each handle).  One of the two set
 * without the other gives AGC_ERR_INVALID_ARG. */
typedef void* (*agc_alloc_fn)(size_t bytes, void* user);
typedef void (*agc_free_fn)(void* ptr, void* user);
agc_status agc_set_allocator(agc_context* ctx, agc_alloc_fn alloc, agc_free_fn free_fn, void* user);
agc_status agc_set_stream(agc_context* ctx, void* stream);
/* Frees the context's workspace.  Matrices and meshes must be destroyed first. */
agc_status agc_destroy(agc_context* ctx);
/* [host] Text of the last failure on this context ("" if none).  Valid until
 * the next call on the context. */
const char* agc_last_error(const agc_context* ctx);
/* [host] Library version string. */
const char* agc_version(void);

/* ------------------------------------------------------------------- mesh */

/* Precomputes the static structure of a mesh of `n_elems` four-vertex
 * elements (tetrahedra, or point-triangle contact stencils).  In the method
 * the fine connectivity never changes between Newton iterations; only the
 * tags, the map and the values do (Sec. 4.1).  So the fine block pattern,
 * the order in which element sub-blocks are summed into each fine block, and
 * the vertex-element incidence are computed here once.
 *   elem_verts : [n_elems][4] int32, four distinct ids in [0, n_verts).
 * Returns AGC_ERR_BAD_INPUT if an id is out of range or repeated in an
 * element.  Synchronises the stream. */
agc_status agc_mesh_create(agc_context* ctx, int32_t n_verts, int64_t n_elems,
                           const int32_t* elem_verts, agc_mesh** mesh);
agc_status agc_mesh_destroy(agc_context* ctx, agc_mesh* mesh);
/* [host] sizes: vertices, elements, fine blocks in the full symmetric pattern. */
agc_status agc_mesh_info(const agc_mesh* mesh, int32_t* n_verts, int64_t* n_elems,
                         int64_t* fine_nnzb);

/* ---------------------------------------------- edge tags (before the map) */

/* Green-strain-increment criterion (Sec. 4.2 "Adaptive Coarsening
 * Criterion", Eq. 3).  For each tetrahedron, F = Ds Dm^{-1} (columns of Ds /
 * Dm: x_k - x_0 of the deformed / rest element, k = 1..3), G = (F^T F - I)/2,
 * and dG = G(x_cur) - G(x_prev) between two successive Newton iterates.  An
 * edge is tagged 0 (protected) when any tetrahedron containing it has
 * ||dG||_F > threshold, else 1 (collapsible); an edge in no tetrahedron, or a
 * self-loop, stays 1.
 *
 * The connectivity is static, so agc_tagger_create precomputes every
 * tetrahedron's Dm^{-1} and the position of each of its six edges in the
 * edge list; the tagger owns that device data until agc_tagger_destroy.
 *   tets  : [n_tets][4] int32 device, distinct ids in [0, n_verts).
 *   rest  : [n_verts][3] float64 device, rest positions.
 *   edges : [n_edges][2] int32 device, 8-byte aligned, the list agc_aggregate
 *           will receive (duplicates and self-loops allowed).
 * AGC_ERR_BAD_INPUT for an id out of range, a repeated vertex in a
 * tetrahedron or a rest tetrahedron of zero volume.  Synchronises. */
typedef struct agc_tagger agc_tagger;
agc_status agc_tagger_create(agc_context* ctx, int32_t n_verts, int64_t n_tets, const int32_t* tets,
                             const double* rest, int64_t n_edges, const int32_t* edges,
                             agc_tagger** out);
agc_status agc_tagger_destroy(agc_context* ctx, agc_tagger* tagger);

/* Tags for one Newton iteration.
 *   x_cur, x_prev : [n_verts][3] float64 device, positions at iterates i, i-1.
 *   threshold     : >= 0 (the paper uses 5e-5).
 *   tags          : [n_edges] uint8 device out.
 *   n_protected   : [host] out, number of tags 0; may be NULL (then the call
 *                   does not synchronise). */
agc_status agc_tag_edges(agc_context* ctx, const agc_tagger* tagger, const double* x_cur,
                         const double* x_prev, double threshold, uint8_t* tags,
                         int64_t* n_protected);

/* -------------------------------------------------------------- (a) map */

/* Fine-to-coarse aggregation (Sec. 4.1; supplement Sec. 1): super-nodes are
 * the connected components of the graph whose edges are the collapsible
 * ones.  Labels are canonical: component c is the c-th in increasing order of
 * its smallest vertex id, which is the order the supplement's elected-lane
 * popcount and group prefix sum produce (supplement Alg. 2, Sec. 1.3).
 *   edges    : [n_edges][2] int32 vertex ids, unordered; duplicates and
 *              self-loops allowed (a self-loop joins nothing); 8-byte
 *              aligned (AGC_ERR_INVALID_ARG otherwise).
 *   tags     : [n_edges] uint8, 1 = collapsible, 0 = protected.
 *   map      : [n_verts] int32 out.
 *   n_coarse : [host] out, number of super-nodes.  Synchronises.
 * AGC_ERR_BAD_INPUT if an id is outside [0, n_verts) or a tag is not 0/1
 * (map is then unspecified). */
agc_status agc_aggregate(agc_context* ctx, int32_t n_verts, int64_t n_edges,
                         const int32_t* edges, const uint8_t* tags,
                         int32_t* map, int32_t* n_coarse);

/* agc_aggregate for callers that cannot allocate device memory during the
 * call (code under graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments, results and errors as agc_aggregate; its
 * scratch is a fixed array of the library on each GPU (18.1 MB, held until
 * the process ends), so it allocates nothing, host or device.  n_verts must
 * be <= 4194304 (AGC_ERR_INVALID_ARG otherwise).  All calls on one GPU share
 * that array: calls that overlap in time on one GPU (from several threads,
 * contexts or streams) race and give wrong maps; serialise them. */
agc_status agc_aggregate_noalloc(agc_context* ctx, int32_t n_verts, int64_t n_edges,
                                 const int32_t* edges, const uint8_t* tags,
                                 int32_t* map, int32_t* n_coarse);

/* ---------------------------------------------------- (b) coarse system */

/* Galerkin coarse system (Sec. 4.1 "Algebraic Coarsening and System
 * Assembly"; supplement Sec. 2): A_c = P^T H P with H = sum_e S_e^T H_e S_e,
 * and g_c = P^T g.  Every 3x3 fine block (i, j) moves to (map i, map j) and
 * equal keys are summed in a fixed order (sorted keys, segmented reduction),
 * so results are bitwise reproducible.  The upper triangle is reduced and
 * mirrored, so A_c is exactly symmetric.
 *   elem_H   : [n_elems][144] row-major 12x12 blocks, DoF order 3a+k, of
 *              type h_dtype (AGC_F64 or AGC_F32); each must be symmetric.
 *   g        : [n_verts][3] float64, may be NULL (then g_c is not written).
 *   map      : [n_verts] int32 in [0, n_coarse) with every label used, as
 *              produced by agc_aggregate.
 *   out_dtype: AGC_F64 (sums in float64) or AGC_F32 (sums and storage in
 *              float32).
 *   A_c      : [host] out, a new matrix owned by the caller, freed with
 *              agc_matrix_destroy.
 *   g_c      : [n_coarse][3] float64 out, may be NULL. */
agc_status agc_assemble_coarse(agc_context* ctx, const agc_mesh* mesh,
                               const void* elem_H, int32_t h_dtype,
                               const double* g, const int32_t* map, int32_t n_coarse,
                               int32_t out_dtype, agc_matrix** A_c, double* g_c);

/* The coarse system with adaptive affine embedding (Sec. 4.2 "Adaptive
 * Affine Embedding", Eq. 4; supplement Sec. 2, Alg. 3-4): a coarse node
 * whose aggregate has more than `threshold` members carries 12 DoF,
 * x_f = sum_k Xbar_f[k] q_c[k] over four 3-blocks k with Xbar_f = (X, Y, Z, 1)
 * the homogeneous rest coordinate of member f in its aggregate's frame
 * (origin at the aggregate's smallest-id member: the same affine span as
 * global coordinates, with the four 3-blocks on comparable scales); every
 * other node keeps 3.
 * Nodes are reordered with the 3-DoF ones first (each group in canonical
 * label order); a 12-DoF node's four 3-blocks follow consecutively, so A_c
 * is a 3x3-block matrix of n3 + 4 n12 block rows (sums in float64).
 *   rest     : [n_verts][3] float64 rest positions.
 *   g        : [n_verts][3] float64, may be NULL.
 *   A_c      : [host] out, as for agc_assemble_coarse.
 *   g_c      : [n3 + 4 n12][3] float64 out, may be NULL.
 *   n3, n12  : [host] out, the node counts of each kind.  Synchronises. */
agc_status agc_assemble_coarse_affine(agc_context* ctx, const agc_mesh* mesh, const double* elem_H,
                                      const double* rest, const double* g, const int32_t* map,
                                      int32_t n_coarse, int32_t threshold, agc_matrix** A_c,
                                      double* g_c, int32_t* n3, int32_t* n12);

/* The fine matrix H itself (map = identity), the comparator of the method.
 * It shares the mesh's static block pattern: destroy it before the mesh. */
agc_status agc_assemble_fine(agc_context* ctx, const agc_mesh* mesh,
                             const void* elem_H, int32_t h_dtype, int32_t out_dtype,
                             agc_matrix** H);

agc_status agc_matrix_destroy(agc_context* ctx, agc_matrix* A);
/* [host] n_rows (block rows), nnzb (stored 3x3 blocks), dtype. */
agc_status agc_matrix_info(const agc_matrix* A, int32_t* n_rows, int64_t* nnzb, int32_t* dtype);
/* Copies the BSR arrays into caller buffers:
 *   row_ptr [n_rows+1] int32, col_idx [nnzb] int32 (sorted within a row),
 *   vals    [nnzb][9] row-major 3x3 blocks of the matrix dtype.
 * Any pointer may be NULL to skip that array. */
agc_status agc_matrix_copy(agc_context* ctx, const agc_matrix* A, int32_t* row_ptr,
                           int32_t* col_idx, void* vals);
/* y = A x on [n_rows][3] float64 vectors (float32 matrices are read as
 * float32 and multiplied in float64). */
agc_status agc_spmv(agc_context* ctx, const agc_matrix* A, const double* x, double* y);

/* --------------------------------------------------------- (c) PCG solve */

typedef struct {
  int32_t iters;    /* PCG iterations performed                          */
  double rel_res;   /* ||b - A x||_2 / ||b||_2 of the recurrence residual */
} agc_pcg_info;

/* 3x3 block-Jacobi preconditioned conjugate gradients (Alg. overview, solve
 * step; Sec. 5.1 "Preconditioners") on A x = b, A symmetric positive
 * definite.  x holds the initial guess on entry (zeros for the standard
 * start) and the result on exit.  Stops when the recurrence residual
 * satisfies ||r||_2 <= rtol ||b||_2 or after max_iter iterations
 * (AGC_ERR_NOT_CONVERGED, x = last iterate).  x, the product A z and every
 * inner product are float64.  The recurrence vectors r, z = D^{-1} r, p and
 * s = A p are stored in the matrix's value type: float64 for a float64
 * matrix; for a float32 matrix each is rounded to float32 once per update
 * and used as stored, so the residual behind the stop test and rel_res is
 * that float32 recurrence (its float64 true residual can differ by about the
 * float32 rounding of A x, relative to ||b||).  info may be NULL.
 * Synchronises. */
agc_status agc_pcg(agc_context* ctx, const agc_matrix* A, const double* b, double* x,
                   double rtol, int32_t max_iter, agc_pcg_info* info);

/* -------------------------------------------------- (d) prolongation, P^T */

/* x = P x_c: x[v] = x_c[map[v]] (Sec. 4.3; d_f = U^T d_c).  Bitwise copy. */
agc_status agc_prolongate(agc_context* ctx, int32_t n_verts, const int32_t* map,
                          int32_t n_coarse, const double* x_c, double* x);
/* v_c = P^T v: v_c[c] = sum of v over the members of c, summed in a fixed
 * order (Sec. 4.1, g_c = sum over child(c) of g_f).  Every label in
 * [0, n_coarse) must have a member (as agc_aggregate's maps do):
 * AGC_ERR_BAD_INPUT for a map value out of range or a label without members. */
agc_status agc_restrict(agc_context* ctx, int32_t n_verts, const int32_t* map,
                        int32_t n_coarse, const double* v, double* v_c);

/* ----------------------------------------------------------- all in one */

/* The arrays a problem points to are read during each call that takes the
 * problem (agc_solve, agc_solve_backward) and are not kept after it; the
 * caller keeps them valid and unchanged for the duration of those calls. */
typedef struct {
  const agc_mesh* mesh;    /* from agc_mesh_create                             */
  int64_t n_edges;         /* edge list for the aggregation                    */
  const int32_t* edges;    /* [n_edges][2] int32                               */
  const uint8_t* tags;     /* [n_edges] uint8                                  */
  const double* elem_H;    /* [n_elems][144] float64 element blocks, 16-byte
                              aligned (AGC_ERR_INVALID_ARG otherwise)         */
  const double* g;         /* [n_verts][3] float64 gradient                    */
  const double* rest;      /* [n_verts][3] float64 rest positions; needed only
                              with opts.affine_threshold > 0                  */
  const double* diag_lb;   /* [n_verts] float64 or NULL: d_v > 0 with
                              H >= diag(d) (x) I_3, e.g. the lumped masses
                              over h^2 when H = M / h^2 + K with K positive
                              semidefinite; enables the certified error
                              bound (agc_solve_info.err_bound)               */
  int64_t n_contacts;      /* elements of this call only, beside the mesh's:
                              the contact stencils the paper finds anew every
                              Newton iteration (Sec. 3; Alg. overview), each
                              a 12x12 block over 4 vertices whose pairs enter
                              the Galerkin sum on each call without the mesh's
                              static plan (0 = none; 10 n_contacts plus the
                              mesh's fine upper blocks stay below 2^30,
                              AGC_ERR_INVALID_ARG otherwise)                  */
  const int32_t* contact_verts; /* [n_contacts][4] int32, 4 distinct ids in
                              [0, n_verts) (AGC_ERR_BAD_INPUT otherwise)      */
  const double* contact_H; /* [n_contacts][144] float64 row-major, symmetric;
                              they join the affine-embedded system and the
                              fine system of post-coarsening too, and
                              agc_solve_backward returns their dL/dH after
                              the mesh's                                      */
} agc_problem;

typedef struct {
  int32_t precision;   /* AGC_PREC_FP64, or AGC_PREC_MIXED: float32 storage
                          and SpMV values in the inner PCG; float64
                          assembly sums, vectors, inner products, residuals
                          and iterative refinement                           */
  int32_t coarsen;     /* 1: aggregate by tags; 0: fine solve (map = identity) */
  double rtol;         /* target ||b_c - A_c x_c||_2 / ||b_c||_2 in float64    */
  int32_t max_iter;    /* PCG iteration cap (over all refinement steps)        */
  double inner_rtol;   /* mixed: relative tolerance of each inner PCG solve    */
  int32_t max_refine;  /* mixed: cap on inner solves (the first one and its
                          refinement steps)                                   */
  int32_t timing;      /* 1: fill the ms_* phase times of agc_solve_info;
                          2: also, after each PCG solve, replay its SpMV
                          kernel 20 times back to back between two HIP
                          events (spmv_launches, ms_spmv; the replays add
                          to ms_pcg)                                         */
  int32_t post_iters;  /* post-coarsening (Sec. 4.3): with coarsen = 1, at
                          most this many block-Jacobi PCG iterations on the
                          fine system H x = g from the prolongated x, in
                          float64, stopping early at rtol; 0 = off          */
  int32_t affine_threshold; /* > 0: aggregates with more members than this
                          get 12 DoF (adaptive affine embedding, as in
                          agc_assemble_coarse_affine; the paper uses 32);
                          0 = 3 DoF everywhere                               */
  double target_err;   /* > 0 (needs prob.diag_lb, affine_threshold = 0):
                          after reaching rtol, keep iterating from the
                          current iterate, with rtol tightened by the ratio
                          of the bound to the target, until err_bound <=
                          target_err (AGC_ERR_NOT_CONVERGED when max_iter
                          ends it first); 0 = stop at rtol                   */
} agc_solve_opts;

typedef struct {
  int32_t n_coarse;    /* super-nodes (n_verts when coarsen = 0)               */
  int64_t nnzb;        /* stored blocks of the solved matrix                   */
  int32_t pcg_iters;   /* PCG iterations over all refinement steps             */
  int32_t refine_iters;/* mixed: inner solves after the first, each on the
                          float64 residual b_c - A_c x_c (0 for FP64)        */
  double rel_res;      /* final float64 relative residual of the coarse system */
  float ms_aggregate, ms_assemble, ms_pcg, ms_prolong;  /* when timing >= 1   */
  int32_t spmv_launches;  /* when timing = 2: timed SpMV replay launches        */
  float ms_spmv;          /* when timing = 2: their summed duration            */
  int32_t post_iters;     /* post-coarsening iterations performed              */
  double fine_rel_res;    /* with post_iters > 0: ||g - H x||_2 / ||g||_2 of
                             the fine system before (fine_rel_res0) and after
                             post-coarsening, float64 matrix                  */
  double fine_rel_res0;
  float ms_post;          /* when timing >= 1: fine assembly + post PCG      */
  int32_t n_affine;       /* coarse nodes with 12 DoF                          */
  int32_t n_blocks;       /* 3x3 block rows of the coarse system: n_coarse
                             + 3 n_affine                                     */
  double err_bound;       /* with prob.diag_lb and affine_threshold = 0: a
                             bound on ||P x_c - x*||_2 / ||P x_c||_2, x* =
                             P A_c^-1 P^T g the exact coarsened solution (H^-1
                             g for coarsen = 0), from the float64 residual
                             r_c = b_c - A_c x_c: A_c >= diag(D_c) (x) I_3
                             with D_c the sum of d over the members of c, so
                             ||P e||_2 <= sqrt(sum_c |r_c|^2 / D_c / min d);
                             it bounds the coarse solve, before any
                             post-coarsening; -1 when not available          */
} agc_solve_info;

/* One Newton linear solve, steps in the order of Alg. overview (mapping,
 * coarse assembly, coarse solve, prolongation): x = P A_c^{-1} P^T g.
 *   x       : [n_verts][3] float64 out.
 *   map_out : [n_verts] int32 out, may be NULL.
 *   info    : [host] out, may be NULL.  Synchronises.
 * When the coarse PCG stops at max_iter (or the mixed refinement at
 * max_refine) before rtol, the remaining steps still run on the last coarse
 * iterate x_c: x = P x_c (then post-coarsening, if asked), info is filled,
 * and the call returns AGC_ERR_NOT_CONVERGED. */
agc_status agc_solve(agc_context* ctx, const agc_problem* prob, const agc_solve_opts* opts,
                     double* x, int32_t* map_out, agc_solve_info* info);

/* Derivatives of L(x) for x = agc_solve(...) given w = dL/dx:
 *   lambda_c = A_c^{-1} P^T w,  dL/dg = P lambda_c,
 *   dL/dH_e  = -(S_e P lambda_c)(S_e x)^T   (12x12, not symmetrised).
 * Only the map (and x) from the forward pass are needed; A_c is assembled
 * again, never stored.  dg: [n_verts][3] float64 out; dH: [n_elems +
 * n_contacts][144] float64 out, may be NULL: the mesh's elements, then the
 * problem's contact elements (whose blocks enter A_c as in agc_solve).
 * opts->precision selects the solve as in
 * agc_solve; opts->post_iters and opts->affine_threshold must be 0 (the
 * derivative is that of the 3-DoF coarsened solve).  The map must use every
 * label in [0, n_coarse) (AGC_ERR_BAD_INPUT otherwise).  A PCG stopped at
 * max_iter (or max_refine) still gives dg and dH from its last iterate, with
 * AGC_ERR_NOT_CONVERGED.  Synchronises. */
agc_status agc_solve_backward(agc_context* ctx, const agc_problem* prob,
                              const agc_solve_opts* opts, const int32_t* map, int32_t n_coarse,
                              const double* x, const double* w, double* dg, double* dH,
                              agc_solve_info* info);

/* ------------------------------------------------ the outer Newton loop */

/* One implicit time step's Newton loop (Sec. 3, Eq. 1-2; Alg. overview),
 * without contact, barrier or friction terms, on the tetrahedra of a mesh.
 * The incremental potential, divided by h^2, is
 *   E(x) = sum_v m_v / (2 h^2) |x_v - xhat_v|^2 + sum_e V_e psi(F_e),
 *   xhat = x^t + h v^t + h^2 M^{-1} f_ext,  m_v = sum of rho V_e / 4,
 * with co-rotated elasticity psi(F) = mu |F - R|^2 + lambda/2 (tr(R^T F) - 3)^2
 * (R the rotation of the rotation-variant polar decomposition of F).  The
 * Hessian proxy is the Hessian with every R held fixed plus the lumped mass
 * / h^2 (SPD).  Each iteration: gradient and proxy; edge tags from the Green
 * strain increment against the previous iterate (the first iteration takes
 * x^t - h v^t); the solve x = agc_solve(...) with d = -x; alpha = 1 halved
 * until E(x + alpha d) < E(x) (at most 30 halvings, after which the loop
 * stops without moving); stop when |d|_inf / h <= eps_d. */
typedef struct agc_newton agc_newton;
typedef struct { double mu, lambda, rho, h; } agc_material;   /* Lame parameters, density, time step */

/* rest: [n_verts][3] float64 rest positions, copied; edges: [n_edges][2]
 * int32 (8-byte aligned), copied.  The mesh must outlive the handle; its
 * elements are the tetrahedra.  A degenerate tetrahedron or an id out of
 * range gives AGC_ERR_INVALID_ARG.  Synchronises. */
agc_status agc_newton_create(agc_context* ctx, const agc_mesh* mesh, int64_t n_edges, const int32_t* edges,
                             const double* rest, const agc_material* mat, agc_newton** out);
agc_status agc_newton_destroy(agc_context* ctx, agc_newton* nw);

typedef struct {
  int32_t max_newton;    /* iteration cap                                      */
  double eps_d;          /* stop when |d|_inf / h <= eps_d                     */
  double tag_threshold;  /* Green strain increment threshold (paper: 5e-5)      */
  int32_t coarsen;       /* 1: tags from the strain increment; 0: fine solves    */
  agc_solve_opts solve;  /* options of every linear solve (timing is ignored)  */
} agc_newton_opts;

typedef struct {
  int32_t newton_iters;
  int32_t halvings;        /* line-search halvings over all iterations          */
  int32_t pcg_iters;       /* PCG iterations over all linear solves             */
  int64_t coarse_nodes_sum;/* sum over iterations of the coarse system size      */
  double energy0, energy;  /* E at x^t and at the result                        */
  double d_inf;            /* |d|_inf of the last direction                     */
  float ms_physics, ms_tags, ms_solve, ms_line;   /* host-timed phases          */
} agc_newton_info;

/* x_t, v_t: [n_verts][3] float64; f_ext: [n_verts][3] float64 or NULL;
 * x_out: [n_verts][3] float64 out (may not alias the inputs).  info may be
 * NULL.  Synchronises. */
agc_status agc_newton_step(agc_context* ctx, agc_newton* nw, const agc_newton_opts* opts, const double* x_t,
                           const double* v_t, const double* f_ext, double* x_out, agc_newton_info* info);

/* The pieces, for checking: the lumped masses m_v ([n_verts] out); at x with
 * the predicted positions x_hat, the gradient g ([n_verts][3] out, may be
 * NULL), the proxy blocks ([n_elems][144] float64 out, 16-byte aligned, may
 * be NULL) and E ([host] out, may be NULL).  Synchronise. */
agc_status agc_newton_mass(agc_context* ctx, const agc_newton* nw, double* mass);
agc_status agc_newton_physics(agc_context* ctx, const agc_newton* nw, const double* x, const double* x_hat,
                              double* g, double* elem_H, double* energy);

/* ------------------------------------------------------------- profiling */

/* Runs agc_spmv `reps` times between two HIP events on the context's stream
 * and returns the mean time of one launch in *avg_ms [host].  Synchronises. */
agc_status agc_time_spmv(agc_context* ctx, const agc_matrix* A, const double* x, double* y,
                         int32_t reps, float* avg_ms);

#ifdef __cplusplus
}
#endif
#endif /* AGC_H */
