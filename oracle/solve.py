"""Oracle: the coarse linear solve and its error certificate (test infrastructure only).

Alg. overview, solve step: d_c = -H_c^{-1} g_c; the oracle returns
x_c = A_c^{-1} b_c (the caller negates).  Sec. 5.1 "Preconditioners" names the
3x3 block-Jacobi preconditioner as the standard GPU choice; ``pcg`` is the
textbook preconditioned conjugate gradient with that preconditioner, x0 = 0
unless given, stopping on the unpreconditioned relative residual
||b - A x||_2 / ||b||_2 (the paper's PCG stops on a relative residual norm,
Sec. 5, first paragraph).

Direct solves (dense Cholesky, sparse LU) give the exact answer up to
rounding and are the reference for small systems.

Error certificate: every element block here is K_e + (rho V_e / 4 h^2) I with
K_e positive semi-definite (elastic or contact), so A_c is bounded below by the
aggregated lumped mass over h^2.  Hence ||x_c - x_c*||_2 <= ||r||_2 / min_c(M_c/h^2),
a bound that holds at any size without knowing x_c*.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def solve_dense(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Cholesky solve; raises numpy/scipy LinAlgError when A is not SPD."""
    c = sla.cho_factor(np.asarray(a, dtype=np.float64), lower=True, check_finite=True)
    return sla.cho_solve(c, np.asarray(b, dtype=np.float64).reshape(-1)).reshape(np.shape(b))


def solve_sparse(a: sp.spmatrix, b: np.ndarray) -> np.ndarray:
    lu = spla.splu(sp.csc_matrix(a))
    return lu.solve(np.asarray(b, dtype=np.float64).reshape(-1)).reshape(np.shape(b))


def block_jacobi_inverse(a: sp.spmatrix) -> np.ndarray:
    """Inverses of the 3x3 diagonal blocks, shape (n, 3, 3); raises if a block is not SPD."""
    a = a.tocsr()
    n = a.shape[0] // 3
    d = np.empty((n, 3, 3))
    idx = np.arange(n)
    for i in range(3):
        for j in range(3):
            d[:, i, j] = np.asarray(a[3 * idx + i, 3 * idx + j]).ravel()
    np.linalg.cholesky(d)                   # raises LinAlgError for a non-SPD block
    return np.linalg.inv(d)


def pcg(a: sp.spmatrix, b: np.ndarray, rtol: float, max_iter: int, x0=None, callback=None):
    """Block-Jacobi PCG.  Returns (x, iterations, relative residual of the recurrence)."""
    a = a.tocsr()
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    dinv = block_jacobi_inverse(a)

    def prec(r):
        return np.einsum("nij,nj->ni", dinv, r.reshape(-1, 3)).reshape(-1)

    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64).reshape(-1).copy()
    r = b - a @ x
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x.reshape(-1, 3), 0, 0.0
    z = prec(r)
    p = z.copy()
    rz = r @ z
    it = 0
    rel = np.linalg.norm(r) / bnorm
    while rel > rtol and it < max_iter:
        q = a @ p
        pq = p @ q
        if not pq > 0.0:
            raise np.linalg.LinAlgError("p^T A p <= 0: matrix not SPD")
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        z = prec(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
        rel = np.linalg.norm(r) / bnorm
        if callback is not None:
            callback(it, x, r)
    return x.reshape(-1, 3), it, rel


def relative_residual(a: sp.spmatrix, b: np.ndarray, x: np.ndarray) -> float:
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    r = b - a @ np.asarray(x, dtype=np.float64).reshape(-1)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def mass_lower_bound(map_, n_c, vertex_mass, h) -> float:
    """min over coarse nodes of (aggregated lumped mass) / h^2: a lower bound on lambda_min(A_c)."""
    m_c = np.bincount(np.asarray(map_, dtype=np.int64), weights=vertex_mass, minlength=n_c)
    return float(m_c.min() / (h * h))


def certified_error(a: sp.spmatrix, b, x, lam_lo: float) -> float:
    """Upper bound on ||x - A^{-1} b||_2 from the residual and a lower eigenvalue bound."""
    r = np.asarray(b, dtype=np.float64).reshape(-1) - a @ np.asarray(x, dtype=np.float64).reshape(-1)
    return float(np.linalg.norm(r) / lam_lo)
