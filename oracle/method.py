"""Oracle: one coarsened Newton linear solve, steps in the order of Alg. overview (test infrastructure only).

1. map  <- fine-to-coarse mapping from the edge tags       (mapping step)
2. H_c, g_c <- Galerkin restriction of H and g              (coarse assembly step)
3. x_c  <- H_c^{-1} g_c                                     (coarse solve step)
4. x    <- P x_c                                            (prolongation, Sec. 4.3)
5. optionally, post-coarsening (Sec. 4.3): at most k block-Jacobi PCG
   iterations on the fine system H x = g started from x     (post_coarsen)

The Newton direction is d = -x.  With every tag 0 the map is the identity and
the result is the fine solve x = H^{-1} g.
"""
from __future__ import annotations

import numpy as np

from . import aggregate, galerkin, solve as _solve


def coarsened_solve(p: dict, solver: str = "sparse", rtol: float = 1e-13, max_iter: int = 100000,
                    tags=None) -> dict:
    n = p["n_verts"]
    t = p["tags"] if tags is None else tags
    m, n_c = aggregate.components(n, p["edges"], t)
    a_c, b_c = galerkin.coarse_system(n, p["elem_verts"], p["elem_H"], p["g"], m, n_c)
    if solver == "dense":
        x_c = _solve.solve_dense(a_c.toarray(), b_c.reshape(-1)).reshape(-1, 3)
        its = 0
    elif solver == "sparse":
        x_c = _solve.solve_sparse(a_c, b_c.reshape(-1)).reshape(-1, 3)
        its = 0
    elif solver == "pcg":
        x_c, its, _ = _solve.pcg(a_c, b_c, rtol, max_iter)
    else:
        raise ValueError(solver)
    x = galerkin.prolongate(m, x_c)
    return {"map": m, "n_c": n_c, "A_c": a_c, "b_c": b_c, "x_c": x_c, "x": x, "iters": its}


def fine_solve(p: dict, solver: str = "sparse", rtol: float = 1e-13, max_iter: int = 100000) -> dict:
    """The same steps with every edge protected (map = identity)."""
    return coarsened_solve(p, solver, rtol, max_iter, tags=np.zeros_like(p["tags"]))


def post_coarsen(p: dict, x0: np.ndarray, k: int, rtol: float = 0.0) -> tuple[np.ndarray, int]:
    """Post-coarsening (Sec. 4.3): PCG on the fine system H x = g from x0, at most
    k iterations (stopping earlier only when the relative residual reaches rtol).
    The textbook PCG loop of ``solve.pcg`` with the same block-Jacobi preconditioner."""
    h = galerkin.fine_hessian(p["n_verts"], p["elem_verts"], p["elem_H"])
    x, its, _ = _solve.pcg(h, p["g"], rtol, k, x0=x0)
    return x, its

