"""Oracle: adaptive affine embedding of large aggregates (test infrastructure only).

Definition (Sec. 4.2 "Adaptive Affine Embedding", Eq. 4; supplement Sec. 2,
Alg. 3-4): a coarse node whose aggregate has more than ``threshold`` fine
nodes carries 12 DoF instead of 3.  For such a node every member f has the
affine basis A_f = Xbar_f (x) I_3 (12 x 3), Xbar_f = (X, Y, Z, 1) its
homogeneous rest coordinate (here in the aggregate's frame: the origin at
its smallest-id member, which spans the same affine functions), and

    g_c = sum_f A_f g_f,        H_c = sum_f,f' A_f H_ff' A_f'^T,

that is, with the prolongation x_f = A_f^T q_c (q_c the node's 12 DoF), the
Galerkin product P^T H P and P^T g with this P.  3-DoF nodes keep x_f = x_c.

Ordering (supplement Alg. 3): 3-DoF nodes come first, in canonical label
order, then the 12-DoF nodes in canonical label order.  A 12-DoF node's 12
DoF are four consecutive 3-blocks k = 0..3, block k weighted by Xbar_f[k]
(supplement: global row n_3dof + (node - n_3dof) * 4 + K / 4), so the whole
coarse system is a 3x3-block matrix of n_3dof + 4 n_12dof block rows.

Written with scipy sparse matrices straight from the definition; the
Galerkin product, the restriction and the prolongation are the library
primitives.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import galerkin


def classify(map_: np.ndarray, n_c: int, threshold: int) -> dict:
    """Node DoF (3 or 12) by aggregate size, the new node order and block offsets.

    Returns new_label[c] (3-DoF nodes 0..n3-1, then 12-DoF nodes), the flat
    3-block offset of each node, n3, n12 and the number of flat 3-blocks."""
    size = np.bincount(map_, minlength=n_c)
    big = size > threshold
    n12 = int(big.sum())
    n3 = n_c - n12
    new_label = np.empty(n_c, np.int64)
    new_label[~big] = np.arange(n3)
    new_label[big] = n3 + np.arange(n12)
    offset = np.where(big, n3 + 4 * (new_label - n3), new_label)
    return {"big": big, "new_label": new_label, "offset": offset, "n3": n3, "n12": n12,
            "n_flat": n3 + 4 * n12}


def local_rest(map_: np.ndarray, rest: np.ndarray, n_c: int) -> np.ndarray:
    """Rest positions relative to the smallest-id member of each aggregate."""
    rep = np.full(n_c, map_.shape[0], np.int64)
    np.minimum.at(rep, map_, np.arange(map_.shape[0]))
    return rest - rest[rep[map_]]


def prolongation(map_: np.ndarray, rest: np.ndarray, cls: dict) -> sp.csr_matrix:
    """P (3n x 3 n_flat): I_3 into a 3-DoF node's block; A_f^T = Xbar_f^T (x) I_3 into a 12-DoF node's four blocks.

    Xbar_f is the homogeneous rest coordinate of f in its aggregate's frame (origin at
    the aggregate's smallest-id member): the same affine span as global coordinates,
    with the four 3-blocks of a node on comparable scales."""
    n = map_.shape[0]
    xbar = np.concatenate([local_rest(map_, rest, cls["big"].shape[0]), np.ones((n, 1))], axis=1)
    big = cls["big"][map_]
    off = cls["offset"][map_]
    rows, cols, vals = [], [], []
    f = np.flatnonzero(~big)                                        # x_f = x_c: one identity block
    for i in range(3):
        rows.append(3 * f + i)
        cols.append(3 * off[f] + i)
        vals.append(np.ones(f.size))
    f = np.flatnonzero(big)                                         # x_f = sum_k Xbar_f[k] q_c[k]
    for k in range(4):
        for i in range(3):
            rows.append(3 * f + i)
            cols.append(3 * (off[f] + k) + i)
            vals.append(xbar[f, k])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(3 * n, 3 * cls["n_flat"]))


def coarse_system(p: dict, map_: np.ndarray, n_c: int, threshold: int):
    """(A_c, b_c [n_flat, 3], cls, P) of the affine-embedded coarse system (Eq. 4)."""
    cls = classify(map_, n_c, threshold)
    pm = prolongation(map_, p["pos"], cls)
    h = galerkin.fine_hessian(p["n_verts"], p["elem_verts"], p["elem_H"])
    a_c = (pm.T @ h @ pm).tocsr()
    b_c = (pm.T @ p["g"].reshape(-1)).reshape(-1, 3)
    return a_c, b_c, cls, pm


def prolongate(pm: sp.spmatrix, x_c: np.ndarray) -> np.ndarray:
    return (pm @ x_c.reshape(-1)).reshape(-1, 3)
