"""Oracle: Galerkin coarse system (test infrastructure only).

Sec. 4.1 "Algebraic Coarsening and System Assembly": every fine node's
gradient is added into its coarse node, g_c = sum over the children of c of
g_f, and every fine 3x3 Hessian block (i, j) is moved to (map i, map j) with
equal keys summed; the paper states this equals the Galerkin projection
H_c = U H U^T, g_c = U g with U the restriction defined by the map
(supplement Sec. 2 does the same from the already reduced fine blocks).

Here P = U^T is the 3n x 3n_c 0/1 matrix with P[3v+i, 3 map(v)+i] = 1, the
fine Hessian is H = sum_e S_e^T H_e S_e (S_e picks the 12 DoF of element e in
the order 3a+k), and the coarse system is A_c = P^T H P, b_c = P^T g.  The
coarse block pattern is every (map v_a, map v_b) over all elements and all
vertex pairs a, b of an element, kept even where values cancel.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def prolongation(map_: np.ndarray, n_c: int) -> sp.csr_matrix:
    """P with P[3v+i, 3 map(v)+i] = 1."""
    m = np.asarray(map_, dtype=np.int64)
    n = m.shape[0]
    rows = (3 * np.arange(n)[:, None] + np.arange(3)[None, :]).ravel()
    cols = (3 * m[:, None] + np.arange(3)[None, :]).ravel()
    return sp.csr_matrix((np.ones(3 * n), (rows, cols)), shape=(3 * n, 3 * n_c))


def element_dofs(elem_verts: np.ndarray) -> np.ndarray:
    """(n_e, 12) global DoF indices 3 v_a + k in local order 3a+k."""
    ev = np.asarray(elem_verts, dtype=np.int64)
    return (3 * ev[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)


def fine_hessian(n_verts: int, elem_verts, elem_H, chunk: int = 1 << 16) -> sp.csr_matrix:
    """H = sum_e S_e^T H_e S_e as a sparse 3n x 3n matrix (duplicates summed)."""
    dofs = element_dofs(elem_verts)
    hv = np.asarray(elem_H, dtype=np.float64).reshape(-1, 12, 12)
    total = None
    for s in range(0, dofs.shape[0], chunk):
        d = dofs[s:s + chunk]
        r = np.repeat(d, 12, axis=1).ravel()
        c = np.tile(d, (1, 12)).ravel()
        part = sp.coo_matrix((hv[s:s + chunk].ravel(), (r, c)), shape=(3 * n_verts, 3 * n_verts)).tocsr()
        total = part if total is None else total + part
    if total is None:
        total = sp.csr_matrix((3 * n_verts, 3 * n_verts))
    return total


def fine_matvec(elem_verts, elem_H, x, chunk: int = 1 << 18) -> np.ndarray:
    """H x = sum_e S_e^T (H_e (S_e x)) element by element, x of shape (n, 3)."""
    x = np.asarray(x, dtype=np.float64)
    ev = np.asarray(elem_verts, dtype=np.int64)
    hv = np.asarray(elem_H).reshape(-1, 12, 12)
    y = np.zeros(x.shape[0] * 3)
    for s in range(0, ev.shape[0], chunk):
        e = ev[s:s + chunk]
        ye = np.einsum("nij,nj->ni", hv[s:s + chunk].astype(np.float64), x[e].reshape(-1, 12))
        dofs = (3 * e[:, :, None] + np.arange(3)[None, None, :]).reshape(-1)
        y += np.bincount(dofs, weights=ye.reshape(-1), minlength=y.shape[0])
    return y.reshape(-1, 3)


def coarse_residual(elem_verts, elem_H, g, map_, n_c, x_c) -> np.ndarray:
    """b_c - A_c x_c = P^T (g - H P x_c) without assembling anything."""
    m = np.asarray(map_, dtype=np.int64)
    x = np.asarray(x_c, dtype=np.float64).reshape(-1, 3)[m]
    return restrict(m, n_c, np.asarray(g, dtype=np.float64) - fine_matvec(elem_verts, elem_H, x))


def coarse_system(n_verts: int, elem_verts, elem_H, g, map_, n_c):
    """A_c = P^T H P (sparse) and b_c = P^T g, shape (n_c, 3)."""
    p = prolongation(map_, n_c)
    h = fine_hessian(n_verts, elem_verts, elem_H)
    a_c = (p.T @ h @ p).tocsr()
    b_c = (p.T @ np.asarray(g, dtype=np.float64).reshape(-1)).reshape(-1, 3)
    return a_c, b_c


def restrict(map_, n_c, v) -> np.ndarray:
    """P^T v for v of shape (n, 3)."""
    return (prolongation(map_, n_c).T @ np.asarray(v, dtype=np.float64).reshape(-1)).reshape(-1, 3)


def prolongate(map_, x_c) -> np.ndarray:
    """P x_c, shape (n, 3)."""
    x_c = np.asarray(x_c, dtype=np.float64).reshape(-1, 3)
    return (prolongation(map_, x_c.shape[0]) @ x_c.reshape(-1)).reshape(-1, 3)


def coarse_pattern(elem_verts, map_, n_c):
    """Sorted unique block keys (row, col) = (map v_a, map v_b) over all elements and a, b."""
    m = np.asarray(map_, dtype=np.int64)[np.asarray(elem_verts, dtype=np.int64)]   # (n_e, 4)
    r = np.repeat(m, 4, axis=1).ravel()
    c = np.tile(m, (1, 4)).ravel()
    key = np.unique(r * n_c + c)
    return key // n_c, key % n_c


def coarse_rows(elem_verts, elem_H, map_, n_c, rows):
    """Selected block rows of A_c straight from the elements (for systems too big to assemble whole).

    Returns {(r, c): 3x3 block} for r in rows: the sum over every element e and
    local pair (a, b) with map(v_a) = r of the sub-block H_e[a, b] at column map(v_b).
    """
    rows = np.asarray(rows, dtype=np.int64)
    m = np.asarray(map_, dtype=np.int64)[np.asarray(elem_verts, dtype=np.int64)]       # (n_e, 4)
    want = np.zeros(n_c, dtype=bool)
    want[rows] = True
    sel = np.nonzero(want[m].any(axis=1))[0]
    he = np.asarray(elem_H, dtype=np.float64).reshape(-1, 4, 3, 4, 3)[sel]           # [e, a, i, b, j]
    ms = m[sel]
    out = {}
    for a in range(4):
        ra = ms[:, a]
        keep = want[ra]
        for b in range(4):
            key = ra[keep] * n_c + ms[keep, b]
            blocks = he[keep, a, :, b, :]
            uk, inv = np.unique(key, return_inverse=True)
            acc = np.zeros((uk.shape[0], 3, 3))
            np.add.at(acc, inv, blocks)
            for k, blk in zip(uk.tolist(), acc):
                out[(k // n_c, k % n_c)] = out.get((k // n_c, k % n_c), 0.0) + blk
    return out


def to_blocks(a: sp.spmatrix, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """Dense 3x3 blocks of a at the given block keys, shape (nnzb, 3, 3)."""
    a = a.tocsr()
    out = np.empty((rows.shape[0], 3, 3))
    for i in range(3):
        for j in range(3):
            out[:, i, j] = np.asarray(a[3 * rows + i, 3 * cols + j]).ravel()
    return out


def bsr_from_pattern(n_c: int, rows: np.ndarray, cols: np.ndarray):
    """row_ptr for block keys sorted by (row, col)."""
    row_ptr = np.zeros(n_c + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    return np.cumsum(row_ptr)


def dense_fine_hessian(n_verts, elem_verts, elem_H) -> np.ndarray:
    """Dense H by explicit scatter of every element block (tiny meshes)."""
    h = np.zeros((3 * n_verts, 3 * n_verts))
    dofs = element_dofs(elem_verts)
    hv = np.asarray(elem_H, dtype=np.float64).reshape(-1, 12, 12)
    for e in range(dofs.shape[0]):
        h[np.ix_(dofs[e], dofs[e])] += hv[e]
    return h


def dense_prolongation(map_, n_c) -> np.ndarray:
    m = np.asarray(map_, dtype=np.int64)
    p = np.zeros((3 * m.shape[0], 3 * n_c))
    for v in range(m.shape[0]):
        for i in range(3):
            p[3 * v + i, 3 * m[v] + i] = 1.0
    return p
