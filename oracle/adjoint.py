"""Oracle: derivatives of the coarsened solve (test infrastructure only).

The solve maps (g, {H_e}) to x = P A_c^{-1} P^T g with A_c = sum_e (S_e P)^T H_e (S_e P)
(Sec. 4.1 Galerkin form; Sec. 4.3 prolongation).  For a loss L with
w = dL/dx:

* lambda_c = A_c^{-1} P^T w            (A_c is symmetric)
* dL/dg    = P lambda_c
* dL/dA_c  = -lambda_c x_c^T           (from x_c = A_c^{-1} b_c)
* dL/dH_e  = (S_e P)(dL/dA_c)(S_e P)^T = -(S_e P lambda_c)(S_e P x_c)^T, 12x12.

The map is piecewise constant in the inputs, so it carries no derivative.
"""
from __future__ import annotations

import numpy as np

from . import galerkin, solve as _solve


def adjoint(n_verts, elem_verts, elem_H, g, map_, n_c, w, dense: bool = False):
    """Returns (x, dL/dg (n,3), dL/dH (n_e,144)) using a direct coarse solve."""
    a_c, b_c = galerkin.coarse_system(n_verts, elem_verts, elem_H, g, map_, n_c)
    wb = galerkin.restrict(map_, n_c, w)
    if dense:
        ad = a_c.toarray()
        x_c = _solve.solve_dense(ad, b_c.reshape(-1)).reshape(-1, 3)
        lam_c = _solve.solve_dense(ad, wb.reshape(-1)).reshape(-1, 3)
    else:
        x_c = _solve.solve_sparse(a_c, b_c.reshape(-1)).reshape(-1, 3)
        lam_c = _solve.solve_sparse(a_c, wb.reshape(-1)).reshape(-1, 3)
    x = galerkin.prolongate(map_, x_c)
    dg = galerkin.prolongate(map_, lam_c)
    ev = np.asarray(elem_verts, dtype=np.int64)
    le = dg[ev].reshape(-1, 12)                 # S_e P lambda_c
    xe = x[ev].reshape(-1, 12)                  # S_e P x_c
    dh = -(le[:, :, None] * xe[:, None, :]).reshape(-1, 144)
    return x, dg, dh
