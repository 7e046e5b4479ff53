"""Python binding of libagc: argument marshalling only.

Every function named ``agc_*`` here calls the C entry point of the same name
(declared in include/agc.h); all arithmetic runs in the HIP kernels of
libagc.so.  Tensors are torch tensors on the GPU; torch provides device memory
and the stream (the current torch stream is passed to the context).  There is
no CPU fallback: if the library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_float, c_int32, c_int64, c_void_p

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libagc.so")

AGC_OK = 0
AGC_ERR_INVALID_ARG = -1
AGC_ERR_OUT_OF_MEMORY = -2
AGC_ERR_DEVICE = -3
AGC_ERR_NOT_CONVERGED = -4
AGC_ERR_NOT_SPD = -5
AGC_ERR_BAD_INPUT = -6
AGC_F64, AGC_F32 = 0, 1
AGC_PREC_FP64, AGC_PREC_MIXED = 0, 1

EXPORTS = (
    "agc_create", "agc_set_stream", "agc_set_allocator", "agc_destroy", "agc_last_error", "agc_version",
    "agc_mesh_create", "agc_mesh_destroy", "agc_mesh_info", "agc_aggregate", "agc_aggregate_noalloc",
    "agc_assemble_coarse", "agc_assemble_fine", "agc_matrix_destroy", "agc_matrix_info",
    "agc_matrix_copy", "agc_spmv", "agc_pcg", "agc_prolongate", "agc_restrict", "agc_solve",
    "agc_solve_backward", "agc_time_spmv", "agc_tagger_create", "agc_tagger_destroy", "agc_tag_edges",
    "agc_assemble_coarse_affine", "agc_newton_create", "agc_newton_destroy", "agc_newton_step",
    "agc_newton_mass", "agc_newton_physics",
)


class AgcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class NotConverged(AgcError):
    pass


class NotSPD(AgcError):
    pass


class BadInput(AgcError):
    pass


class agc_problem(ctypes.Structure):
    _fields_ = [("mesh", c_void_p), ("n_edges", c_int64), ("edges", c_void_p), ("tags", c_void_p),
                ("elem_H", c_void_p), ("g", c_void_p), ("rest", c_void_p), ("diag_lb", c_void_p),
                ("n_contacts", c_int64), ("contact_verts", c_void_p), ("contact_H", c_void_p)]


class agc_solve_opts(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("coarsen", c_int32), ("rtol", c_double), ("max_iter", c_int32),
                ("inner_rtol", c_double), ("max_refine", c_int32), ("timing", c_int32), ("post_iters", c_int32),
                ("affine_threshold", c_int32), ("target_err", c_double)]


class agc_solve_info(ctypes.Structure):
    _fields_ = [("n_coarse", c_int32), ("nnzb", c_int64), ("pcg_iters", c_int32), ("refine_iters", c_int32),
                ("rel_res", c_double), ("ms_aggregate", c_float), ("ms_assemble", c_float),
                ("ms_pcg", c_float), ("ms_prolong", c_float), ("spmv_launches", c_int32), ("ms_spmv", c_float),
                ("post_iters", c_int32), ("fine_rel_res", c_double), ("fine_rel_res0", c_double), ("ms_post", c_float),
                ("n_affine", c_int32), ("n_blocks", c_int32), ("err_bound", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class agc_pcg_info(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("rel_res", c_double)]


class agc_material(ctypes.Structure):
    _fields_ = [("mu", c_double), ("lambda_", c_double), ("rho", c_double), ("h", c_double)]


class agc_newton_opts(ctypes.Structure):
    _fields_ = [("max_newton", c_int32), ("eps_d", c_double), ("tag_threshold", c_double), ("coarsen", c_int32),
                ("solve", agc_solve_opts)]


class agc_newton_info(ctypes.Structure):
    _fields_ = [("newton_iters", c_int32), ("halvings", c_int32), ("pcg_iters", c_int32),
                ("coarse_nodes_sum", c_int64), ("energy0", c_double), ("energy", c_double), ("d_inf", c_double),
                ("ms_physics", c_float), ("ms_tags", c_float), ("ms_solve", c_float), ("ms_line", c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, ctypes.c_size_t, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2605_04773_amd.build`")
    lib = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
    S = c_int32
    P = c_void_p
    sig = {
        "agc_create": (S, [POINTER(c_void_p), c_int32, P]),
        "agc_set_stream": (S, [P, P]),
        "agc_set_allocator": (S, [P, ALLOC_FN, FREE_FN, P]),
        "agc_destroy": (S, [P]),
        "agc_last_error": (c_char_p, [P]),
        "agc_version": (c_char_p, []),
        "agc_mesh_create": (S, [P, c_int32, c_int64, P, POINTER(c_void_p)]),
        "agc_mesh_destroy": (S, [P, P]),
        "agc_mesh_info": (S, [P, POINTER(c_int32), POINTER(c_int64), POINTER(c_int64)]),
        "agc_aggregate": (S, [P, c_int32, c_int64, P, P, P, POINTER(c_int32)]),
        "agc_aggregate_noalloc": (S, [P, c_int32, c_int64, P, P, P, POINTER(c_int32)]),
        "agc_tagger_create": (S, [P, c_int32, c_int64, P, P, c_int64, P, POINTER(c_void_p)]),
        "agc_tagger_destroy": (S, [P, P]),
        "agc_assemble_coarse_affine": (S, [P, P, P, P, P, P, c_int32, c_int32, POINTER(c_void_p), P,
                                           POINTER(c_int32), POINTER(c_int32)]),
        "agc_tag_edges": (S, [P, P, P, P, c_double, P, POINTER(c_int64)]),
        "agc_assemble_coarse": (S, [P, P, P, c_int32, P, P, c_int32, c_int32, POINTER(c_void_p), P]),
        "agc_assemble_fine": (S, [P, P, P, c_int32, c_int32, POINTER(c_void_p)]),
        "agc_matrix_destroy": (S, [P, P]),
        "agc_matrix_info": (S, [P, POINTER(c_int32), POINTER(c_int64), POINTER(c_int32)]),
        "agc_matrix_copy": (S, [P, P, P, P, P]),
        "agc_spmv": (S, [P, P, P, P]),
        "agc_pcg": (S, [P, P, P, P, c_double, c_int32, POINTER(agc_pcg_info)]),
        "agc_prolongate": (S, [P, c_int32, P, c_int32, P, P]),
        "agc_restrict": (S, [P, c_int32, P, c_int32, P, P]),
        "agc_solve": (S, [P, POINTER(agc_problem), POINTER(agc_solve_opts), P, P, POINTER(agc_solve_info)]),
        "agc_solve_backward": (S, [P, POINTER(agc_problem), POINTER(agc_solve_opts), P, c_int32, P, P, P, P,
                                   POINTER(agc_solve_info)]),
        "agc_time_spmv": (S, [P, P, P, P, c_int32, POINTER(c_float)]),
        "agc_newton_create": (S, [P, P, c_int64, P, P, POINTER(agc_material), POINTER(c_void_p)]),
        "agc_newton_destroy": (S, [P, P]),
        "agc_newton_step": (S, [P, P, POINTER(agc_newton_opts), P, P, P, P, POINTER(agc_newton_info)]),
        "agc_newton_mass": (S, [P, P, P]),
        "agc_newton_physics": (S, [P, P, P, P, P, P, POINTER(c_double)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def library_path() -> str:
    return LIB_PATH


def version() -> str:
    return _lib.agc_version().decode()


def _check(ctx, st):
    if st == AGC_OK:
        return
    msg = _lib.agc_last_error(ctx).decode() if ctx else "invalid argument"
    cls = {AGC_ERR_NOT_CONVERGED: NotConverged, AGC_ERR_NOT_SPD: NotSPD, AGC_ERR_BAD_INPUT: BadInput}.get(st, AgcError)
    raise cls(st, msg)


def _ptr(t):
    return c_void_p(0) if t is None else c_void_p(t.data_ptr())


def _dev(t, dtype, shape, name, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda" or (device is not None and t.device != device):
        raise ValueError(f"{name} must be on {device}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


# ---------------------------------------------------------------- handles

class Context:
    """An agc_context bound to one GPU and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        self.device = torch.device("cuda", device)
        s = torch.cuda.current_stream(self.device) if stream is None else stream
        self.stream = s
        h = c_void_p()
        _check(None, _lib.agc_create(byref(h), int(device), c_void_p(s.cuda_stream)))
        self.h = h

    def use_torch_allocator(self):
        """Route the device buffers the context allocates from now on through
        torch's caching allocator on its stream (agc_set_allocator).  Returns a
        dict counting the blocks requested and returned."""
        dev, stream = self.device, self.stream
        stats = {"alloc": 0, "free": 0, "bytes": 0}

        def _alloc(nbytes, _user):
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
            except RuntimeError:
                return None
            stats["alloc"] += 1
            stats["bytes"] += int(nbytes)
            return ptr

        def _free(ptr, _user):
            stats["free"] += 1
            torch.cuda.caching_allocator_delete(ptr)

        self._alloc_cbs = (ALLOC_FN(_alloc), FREE_FN(_free))   # kept alive with the context
        _check(self.h, _lib.agc_set_allocator(self.h, self._alloc_cbs[0], self._alloc_cbs[1], None))
        return stats

    def close(self):
        if getattr(self, "h", None):
            _lib.agc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    def __init__(self, ctx: Context, h, n_verts, n_elems, elem_verts):
        self.ctx, self.h, self.n_verts, self.n_elems = ctx, h, n_verts, n_elems
        self.elem_verts = elem_verts
        nv, ne, nnzb = c_int32(), c_int64(), c_int64()
        _lib.agc_mesh_info(h, byref(nv), byref(ne), byref(nnzb))
        self.fine_nnzb = nnzb.value

    def close(self):
        if getattr(self, "h", None) and self.ctx.h:
            _lib.agc_mesh_destroy(self.ctx.h, self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tagger:
    """Static data of the Green-strain-increment criterion for a tet mesh and an edge list."""

    def __init__(self, ctx: Context, h, n_verts, n_tets, n_edges):
        self.ctx, self.h, self.n_verts, self.n_tets, self.n_edges = ctx, h, n_verts, n_tets, n_edges

    def close(self):
        if getattr(self, "h", None) and self.ctx.h:
            _lib.agc_tagger_destroy(self.ctx.h, self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Matrix:
    def __init__(self, ctx: Context, h, keep=None):
        # keep: an object whose device memory the matrix uses (the mesh, whose
        # static pattern a fine matrix borrows), kept alive with it
        self.ctx, self.h, self._keep = ctx, h, keep
        n, nnzb, dt = c_int32(), c_int64(), c_int32()
        _lib.agc_matrix_info(h, byref(n), byref(nnzb), byref(dt))
        self.n_rows, self.nnzb, self.dtype = n.value, nnzb.value, dt.value

    def to_bsr(self):
        """(row_ptr int32 [n+1], col_idx int32 [nnzb], vals [nnzb, 3, 3]) copies on the device."""
        dev = self.ctx.device
        rp = torch.empty(self.n_rows + 1, dtype=torch.int32, device=dev)
        ci = torch.empty(max(self.nnzb, 1), dtype=torch.int32, device=dev)
        vt = torch.float64 if self.dtype == AGC_F64 else torch.float32
        vals = torch.empty((max(self.nnzb, 1), 3, 3), dtype=vt, device=dev)
        _check(self.ctx.h, _lib.agc_matrix_copy(self.ctx.h, self.h, _ptr(rp), _ptr(ci), _ptr(vals)))
        return rp, ci[: self.nnzb], vals[: self.nnzb]

    def close(self):
        if getattr(self, "h", None) and self.ctx.h:
            _lib.agc_matrix_destroy(self.ctx.h, self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------- entry points

def agc_mesh_create(ctx: Context, n_verts: int, elem_verts: torch.Tensor) -> Mesh:
    ne = elem_verts.shape[0]
    _dev(elem_verts, torch.int32, (ne, 4), "elem_verts", ctx.device)
    h = c_void_p()
    _check(ctx.h, _lib.agc_mesh_create(ctx.h, int(n_verts), int(ne), _ptr(elem_verts), byref(h)))
    return Mesh(ctx, h, int(n_verts), int(ne), elem_verts)


def agc_aggregate(ctx: Context, n_verts: int, edges: torch.Tensor, tags: torch.Tensor, map_out=None):
    m = edges.shape[0]
    _dev(edges, torch.int32, (m, 2), "edges", ctx.device)
    _dev(tags, torch.uint8, (m,), "tags", ctx.device)
    mp = torch.empty(n_verts, dtype=torch.int32, device=ctx.device) if map_out is None else map_out
    _dev(mp, torch.int32, (n_verts,), "map", ctx.device)
    nc = c_int32()
    _check(ctx.h, _lib.agc_aggregate(ctx.h, int(n_verts), int(m), _ptr(edges), _ptr(tags), _ptr(mp), byref(nc)))
    return mp, nc.value


def agc_aggregate_noalloc(ctx: Context, n_verts: int, edges: torch.Tensor, tags: torch.Tensor,
                          map_out: torch.Tensor):
    """agc_aggregate into the caller's map, with the library's fixed scratch (no allocation)."""
    m = edges.shape[0]
    _dev(edges, torch.int32, (m, 2), "edges", ctx.device)
    _dev(tags, torch.uint8, (m,), "tags", ctx.device)
    _dev(map_out, torch.int32, (n_verts,), "map", ctx.device)
    nc = c_int32()
    _check(ctx.h, _lib.agc_aggregate_noalloc(ctx.h, int(n_verts), int(m), _ptr(edges), _ptr(tags), _ptr(map_out),
                                             byref(nc)))
    return map_out, nc.value


def agc_assemble_coarse_affine(ctx: Context, mesh: Mesh, elem_H: torch.Tensor, rest: torch.Tensor, g,
                               map_: torch.Tensor, n_coarse: int, threshold: int):
    """(A_c, g_c [n3 + 4 n12, 3] or None, n3, n12): the affine-embedded coarse system (float64)."""
    _dev(elem_H, torch.float64, (mesh.n_elems, 144), "elem_H", ctx.device)
    _dev(rest, torch.float64, (mesh.n_verts, 3), "rest", ctx.device)
    _dev(map_, torch.int32, (mesh.n_verts,), "map", ctx.device)
    if g is not None:
        _dev(g, torch.float64, (mesh.n_verts, 3), "g", ctx.device)
    # g_c needs n3 + 4 n12 rows, known only after the call: a bound of 4 n_coarse rows
    g_c = torch.empty((4 * int(n_coarse), 3), dtype=torch.float64, device=ctx.device) if g is not None else None
    h = c_void_p()
    n3, n12 = c_int32(), c_int32()
    _check(ctx.h, _lib.agc_assemble_coarse_affine(ctx.h, mesh.h, _ptr(elem_H), _ptr(rest), _ptr(g), _ptr(map_),
                                                  int(n_coarse), int(threshold), byref(h), _ptr(g_c),
                                                  byref(n3), byref(n12)))
    nb = n3.value + 4 * n12.value
    return Matrix(ctx, h), (g_c[:nb] if g_c is not None else None), n3.value, n12.value


def agc_tagger_create(ctx: Context, n_verts: int, tets: torch.Tensor, rest: torch.Tensor,
                      edges: torch.Tensor) -> Tagger:
    ne, m = tets.shape[0], edges.shape[0]
    _dev(tets, torch.int32, (ne, 4), "tets", ctx.device)
    _dev(rest, torch.float64, (n_verts, 3), "rest", ctx.device)
    _dev(edges, torch.int32, (m, 2), "edges", ctx.device)
    h = c_void_p()
    _check(ctx.h, _lib.agc_tagger_create(ctx.h, int(n_verts), int(ne), _ptr(tets), _ptr(rest), int(m),
                                         _ptr(edges), byref(h)))
    return Tagger(ctx, h, int(n_verts), int(ne), int(m))


def agc_tag_edges(ctx: Context, tagger: Tagger, x_cur: torch.Tensor, x_prev: torch.Tensor, threshold: float,
                  tags_out=None, count=True):
    """(tags uint8 [n_edges] on the device, number protected or None)."""
    _dev(x_cur, torch.float64, (tagger.n_verts, 3), "x_cur", ctx.device)
    _dev(x_prev, torch.float64, (tagger.n_verts, 3), "x_prev", ctx.device)
    tags = torch.empty(tagger.n_edges, dtype=torch.uint8, device=ctx.device) if tags_out is None else tags_out
    _dev(tags, torch.uint8, (tagger.n_edges,), "tags", ctx.device)
    n = c_int64()
    _check(ctx.h, _lib.agc_tag_edges(ctx.h, tagger.h, _ptr(x_cur), _ptr(x_prev), float(threshold), _ptr(tags),
                                     byref(n) if count else None))
    return tags, (n.value if count else None)


def _h_dtype(t):
    if t.dtype == torch.float64:
        return AGC_F64
    if t.dtype == torch.float32:
        return AGC_F32
    raise ValueError("elem_H must be float64 or float32")


def agc_assemble_coarse(ctx: Context, mesh: Mesh, elem_H: torch.Tensor, g, map_: torch.Tensor, n_coarse: int,
                        out_dtype: int = AGC_F64):
    _dev(elem_H, elem_H.dtype, (mesh.n_elems, 144), "elem_H", ctx.device)
    hd = _h_dtype(elem_H)
    _dev(map_, torch.int32, (mesh.n_verts,), "map", ctx.device)
    g_c = None
    if g is not None:
        _dev(g, torch.float64, (mesh.n_verts, 3), "g", ctx.device)
        g_c = torch.empty((n_coarse, 3), dtype=torch.float64, device=ctx.device)
    h = c_void_p()
    _check(ctx.h, _lib.agc_assemble_coarse(ctx.h, mesh.h, _ptr(elem_H), hd, _ptr(g), _ptr(map_), int(n_coarse),
                                           int(out_dtype), byref(h), _ptr(g_c)))
    return Matrix(ctx, h), g_c


def agc_assemble_fine(ctx: Context, mesh: Mesh, elem_H: torch.Tensor, out_dtype: int = AGC_F64) -> Matrix:
    _dev(elem_H, elem_H.dtype, (mesh.n_elems, 144), "elem_H", ctx.device)
    h = c_void_p()
    _check(ctx.h, _lib.agc_assemble_fine(ctx.h, mesh.h, _ptr(elem_H), _h_dtype(elem_H), int(out_dtype), byref(h)))
    return Matrix(ctx, h, keep=mesh)


def agc_spmv(ctx: Context, A: Matrix, x: torch.Tensor, y=None) -> torch.Tensor:
    _dev(x, torch.float64, (A.n_rows, 3), "x", ctx.device)
    y = torch.empty_like(x) if y is None else y
    _dev(y, torch.float64, (A.n_rows, 3), "y", ctx.device)
    _check(ctx.h, _lib.agc_spmv(ctx.h, A.h, _ptr(x), _ptr(y)))
    return y


def agc_time_spmv(ctx: Context, A: Matrix, x: torch.Tensor, y: torch.Tensor, reps: int) -> float:
    _dev(x, torch.float64, (A.n_rows, 3), "x", ctx.device)
    _dev(y, torch.float64, (A.n_rows, 3), "y", ctx.device)
    ms = c_float()
    _check(ctx.h, _lib.agc_time_spmv(ctx.h, A.h, _ptr(x), _ptr(y), int(reps), byref(ms)))
    return ms.value


def agc_pcg(ctx: Context, A: Matrix, b: torch.Tensor, x: torch.Tensor, rtol: float, max_iter: int,
            raise_on_not_converged: bool = True):
    _dev(b, torch.float64, (A.n_rows, 3), "b", ctx.device)
    _dev(x, torch.float64, (A.n_rows, 3), "x", ctx.device)
    info = agc_pcg_info()
    st = _lib.agc_pcg(ctx.h, A.h, _ptr(b), _ptr(x), float(rtol), int(max_iter), byref(info))
    if st == AGC_ERR_NOT_CONVERGED and not raise_on_not_converged:
        return info
    _check(ctx.h, st)
    return info


def agc_prolongate(ctx: Context, map_: torch.Tensor, n_coarse: int, x_c: torch.Tensor, x=None) -> torch.Tensor:
    n = map_.shape[0]
    _dev(map_, torch.int32, (n,), "map", ctx.device)
    _dev(x_c, torch.float64, (n_coarse, 3), "x_c", ctx.device)
    x = torch.empty((n, 3), dtype=torch.float64, device=ctx.device) if x is None else x
    _dev(x, torch.float64, (n, 3), "x", ctx.device)
    _check(ctx.h, _lib.agc_prolongate(ctx.h, int(n), _ptr(map_), int(n_coarse), _ptr(x_c), _ptr(x)))
    return x


def agc_restrict(ctx: Context, map_: torch.Tensor, n_coarse: int, v: torch.Tensor) -> torch.Tensor:
    n = map_.shape[0]
    _dev(map_, torch.int32, (n,), "map", ctx.device)
    _dev(v, torch.float64, (n, 3), "v", ctx.device)
    out = torch.empty((n_coarse, 3), dtype=torch.float64, device=ctx.device)
    _check(ctx.h, _lib.agc_restrict(ctx.h, int(n), _ptr(map_), int(n_coarse), _ptr(v), _ptr(out)))
    return out


def make_opts(precision=AGC_PREC_FP64, coarsen=1, rtol=1e-10, max_iter=20000, inner_rtol=1e-4, max_refine=20,
              timing=0, post_iters=0, affine_threshold=0, target_err=0.0) -> agc_solve_opts:
    return agc_solve_opts(int(precision), int(coarsen), float(rtol), int(max_iter), float(inner_rtol),
                          int(max_refine), int(timing), int(post_iters), int(affine_threshold), float(target_err))


def make_problem(mesh: Mesh, edges, tags, elem_H, g, rest=None, diag_lb=None, contacts=None) -> agc_problem:
    """contacts: (verts [n][4] int32, H [n][144] float64) assembled on each call beside the mesh's elements."""
    ctx = mesh.ctx
    m = 0 if edges is None else edges.shape[0]
    if edges is not None:
        _dev(edges, torch.int32, (m, 2), "edges", ctx.device)
        _dev(tags, torch.uint8, (m,), "tags", ctx.device)
    _dev(elem_H, torch.float64, (mesh.n_elems, 144), "elem_H", ctx.device)
    _dev(g, torch.float64, (mesh.n_verts, 3), "g", ctx.device)
    if rest is not None:
        _dev(rest, torch.float64, (mesh.n_verts, 3), "rest", ctx.device)
    if diag_lb is not None:
        _dev(diag_lb, torch.float64, (mesh.n_verts,), "diag_lb", ctx.device)
    cv, ch = (None, None) if contacts is None else contacts
    nx = 0
    if cv is not None:
        nx = cv.shape[0]
        _dev(cv, torch.int32, (nx, 4), "contact_verts", ctx.device)
        _dev(ch, torch.float64, (nx, 144), "contact_H", ctx.device)
    prob = agc_problem(mesh.h, int(m), _ptr(edges), _ptr(tags), _ptr(elem_H), _ptr(g), _ptr(rest), _ptr(diag_lb),
                       int(nx), _ptr(cv), _ptr(ch))
    # The struct holds raw device pointers that every later call reads: it
    # keeps the tensors (and the mesh) alive, or a temporary passed here would
    # be freed and its memory handed to the next allocation of that size.
    prob._keep = (mesh, edges, tags, elem_H, g, rest, diag_lb, cv, ch)
    return prob


def agc_solve(ctx: Context, prob: agc_problem, opts: agc_solve_opts, x: torch.Tensor, map_out=None,
              raise_on_not_converged: bool = True):
    """Returns the agc_solve_info.  With raise_on_not_converged False, a solve
    stopped at max_iter / max_refine returns its info (x then holds P times the
    last coarse iterate) instead of raising NotConverged."""
    info = agc_solve_info()
    st = _lib.agc_solve(ctx.h, byref(prob), byref(opts), _ptr(x), _ptr(map_out), byref(info))
    if st == AGC_ERR_NOT_CONVERGED and not raise_on_not_converged:
        return info
    _check(ctx.h, st)
    return info


class Newton:
    """One implicit time step's Newton loop on the tetrahedra of a mesh (agc_newton_*)."""

    def __init__(self, ctx: Context, h, n_verts, n_elems, mesh=None):
        # the handle uses the mesh's static structure: the mesh is kept alive with it
        self.ctx, self.h, self.n_verts, self.n_elems, self.mesh = ctx, h, n_verts, n_elems, mesh

    def close(self):
        if getattr(self, "h", None) and self.ctx.h:
            _lib.agc_newton_destroy(self.ctx.h, self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def agc_newton_create(ctx: Context, mesh: Mesh, edges: torch.Tensor, rest: torch.Tensor, mu: float, lam: float,
                      rho: float, h: float) -> Newton:
    m = edges.shape[0]
    _dev(edges, torch.int32, (m, 2), "edges", ctx.device)
    _dev(rest, torch.float64, (mesh.n_verts, 3), "rest", ctx.device)
    mat = agc_material(float(mu), float(lam), float(rho), float(h))
    out = c_void_p()
    _check(ctx.h, _lib.agc_newton_create(ctx.h, mesh.h, int(m), _ptr(edges), _ptr(rest), byref(mat), byref(out)))
    return Newton(ctx, out, mesh.n_verts, mesh.n_elems, mesh)


def make_newton_opts(max_newton=50, eps_d=1e-3, tag_threshold=5e-5, coarsen=1, solve=None) -> agc_newton_opts:
    return agc_newton_opts(int(max_newton), float(eps_d), float(tag_threshold), int(coarsen),
                           solve if solve is not None else make_opts())


def agc_newton_step(ctx: Context, nw: Newton, opts: agc_newton_opts, x_t, v_t, f_ext=None, x_out=None):
    n = nw.n_verts
    _dev(x_t, torch.float64, (n, 3), "x_t", ctx.device)
    _dev(v_t, torch.float64, (n, 3), "v_t", ctx.device)
    if f_ext is not None:
        _dev(f_ext, torch.float64, (n, 3), "f_ext", ctx.device)
    x = torch.empty((n, 3), dtype=torch.float64, device=ctx.device) if x_out is None else x_out
    _dev(x, torch.float64, (n, 3), "x_out", ctx.device)
    info = agc_newton_info()
    _check(ctx.h, _lib.agc_newton_step(ctx.h, nw.h, byref(opts), _ptr(x_t), _ptr(v_t), _ptr(f_ext), _ptr(x),
                                       byref(info)))
    return x, info


def agc_newton_mass(ctx: Context, nw: Newton) -> torch.Tensor:
    m = torch.empty(nw.n_verts, dtype=torch.float64, device=ctx.device)
    _check(ctx.h, _lib.agc_newton_mass(ctx.h, nw.h, _ptr(m)))
    return m


def agc_newton_physics(ctx: Context, nw: Newton, x, x_hat, want_blocks=True):
    """(g [n,3], elem_H [n_e,144] or None, E) at x with predicted positions x_hat."""
    n = nw.n_verts
    _dev(x, torch.float64, (n, 3), "x", ctx.device)
    _dev(x_hat, torch.float64, (n, 3), "x_hat", ctx.device)
    g = torch.empty((n, 3), dtype=torch.float64, device=ctx.device)
    hb = torch.empty((nw.n_elems, 144), dtype=torch.float64, device=ctx.device) if want_blocks else None
    e = c_double()
    _check(ctx.h, _lib.agc_newton_physics(ctx.h, nw.h, _ptr(x), _ptr(x_hat), _ptr(g), _ptr(hb), byref(e)))
    return g, hb, e.value


def agc_solve_backward(ctx: Context, prob: agc_problem, opts: agc_solve_opts, map_, n_coarse: int, x, w, dg, dH):
    info = agc_solve_info()
    _check(ctx.h, _lib.agc_solve_backward(ctx.h, byref(prob), byref(opts), _ptr(map_), int(n_coarse), _ptr(x),
                                          _ptr(w), _ptr(dg), _ptr(dH), byref(info)))
    return info


# ------------------------------------------------------------- autograd

class AgcSolve(torch.autograd.Function):
    """x = P A_c^{-1} P^T g with A_c = sum_e (S_e P)^T H_e (S_e P); differentiable in g and H_e.

    forward(g [n,3] f64, elem_H [n_e,144] f64, mesh, edges, tags, opts,
            contact_verts [n_x,4] int32 = None, contact_H [n_x,144] f64 = None) -> x [n,3].
    The contact elements (this call's, beside the mesh's) are differentiable
    too.  Only the map (and x) are kept for backward; the coarse matrix is
    assembled again there.
    """

    @staticmethod
    def forward(fctx, g, elem_H, mesh, edges, tags, opts, contact_verts=None, contact_H=None):
        ctx = mesh.ctx
        g = g.contiguous()
        elem_H = elem_H.contiguous()
        contacts = None
        if contact_H is not None:
            contacts = (contact_verts.contiguous(), contact_H.contiguous())
        x = torch.empty_like(g)
        mp = torch.empty(mesh.n_verts, dtype=torch.int32, device=g.device)
        prob = make_problem(mesh, edges, tags, elem_H, g, contacts=contacts)
        info = agc_solve(ctx, prob, opts, x, mp)
        saved = (g, elem_H, mp, x) + (contacts if contacts is not None else ())
        fctx.save_for_backward(*saved)
        fctx.mesh, fctx.edges, fctx.tags, fctx.opts = mesh, edges, tags, opts
        fctx.n_coarse = info.n_coarse
        fctx.mark_non_differentiable(mp)
        return x

    @staticmethod
    def backward(fctx, dx):
        saved = fctx.saved_tensors
        g, elem_H, mp, x = saved[:4]
        contacts = (saved[4], saved[5]) if len(saved) > 4 else None
        mesh = fctx.mesh
        dx = dx.contiguous()
        dg = torch.empty_like(g)
        need_h = fctx.needs_input_grad[1]
        need_c = contacts is not None and fctx.needs_input_grad[7]
        n_e = elem_H.shape[0]
        n_x = contacts[1].shape[0] if contacts is not None else 0
        # the library writes dL/dH for the mesh's elements, then the contacts'
        dH = torch.empty((n_e + n_x, 144), dtype=torch.float64, device=g.device) if (need_h or need_c) else None
        prob = make_problem(mesh, fctx.edges, fctx.tags, elem_H, g, contacts=contacts)
        agc_solve_backward(mesh.ctx, prob, fctx.opts, mp, fctx.n_coarse, x, dx, dg, dH)
        d_mesh = dH[:n_e] if need_h else None
        d_contact = dH[n_e:] if need_c else None
        return dg, d_mesh, None, None, None, None, None, d_contact


def check_single_hip_runtime() -> list[str]:
    """Paths of libamdhip64 mapped into this process (expected: exactly one)."""
    libs = set()
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64" in line:
                libs.add(line.split()[-1])
    return sorted(libs)
