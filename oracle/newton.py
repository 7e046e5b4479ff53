"""Oracle: the outer Newton loop of one implicit time step (test infrastructure only).

Only tests/, the smoke check and the bench's CPU baseline may use this module.

What is computed (Sec. 3, Eq. 1-2, and the Newton loop of Alg. overview, with
no contact, barrier or friction terms):

* The incremental potential, divided by h^2 (same minimiser, and its Hessian
  is the H = M/h^2 + K of the linear solves):
      E(x) = sum_v m_v / (2 h^2) |x_v - xhat_v|^2 + sum_e V_e psi(F_e),
  xhat = x^t + h v^t + h^2 M^{-1} f_ext, m_v the lumped mass (rho V_e / 4 from
  every element of v).
* psi: co-rotated elasticity, psi(F) = mu |F - R|_F^2 + lam/2 (tr(R^T F) - 3)^2
  with R the rotation of the rotation-variant polar decomposition of F
  (from the SVD F = U S V^T with det U = det V = 1, the sign of det F carried
  by the smallest singular value).  The paper fixes no elastic model; this
  one has an SPD Hessian proxy without eigenvalue projection.
* dpsi/dF = 2 mu (F - R) + lam (tr(R^T F) - 3) R (exact: the terms from dR
  vanish at the polar R).
* SPD proxy of the Hessian (Sec. 3: "a symmetric positive definite proxy"):
  the Hessian with R held fixed, 2 mu I_9 + lam vec(R) vec(R)^T, mapped to
  the element's 12 DoF through F = sum_a x_a b_a^T (b_0 = -(b_1 + b_2 + b_3),
  b_i the rows of Dm^{-1}), plus the element's lumped mass / h^2 on its four
  vertex blocks:  H_e[a, b] = V (2 mu (b_a . b_b) I + lam (R b_a)(R b_b)^T)
                             + [a == b] rho V / (4 h^2) I.
* The loop (Alg. overview): E_prev = E(x); g, H at x; tags from the Green
  strain increment between x and the previous iterate (Sec. 4.2, Eq. 3; at
  the first iteration the previous state is x^t - h v^t); d = -P A_c^{-1} P^T g
  (the coarsened solve; every tag 0 gives the fine solve); alpha = 1, halved
  until E(x + alpha d) < E_prev; stop when |d|_inf / h <= eps_d.
"""
from __future__ import annotations

import numpy as np

from . import galerkin, method, tagging

MAX_HALVINGS = 30


def rest_shape(rest: np.ndarray, tets: np.ndarray):
    """Per element: Dm^{-1} (n_e, 3, 3), rest volume V (n_e,), and b_a (n_e, 4, 3)."""
    t = tets.astype(np.int64)
    dm = np.stack([rest[t[:, k]] - rest[t[:, 0]] for k in (1, 2, 3)], axis=-1)
    dminv = np.linalg.inv(dm)
    vol = np.abs(np.linalg.det(dm)) / 6.0
    b = np.empty((t.shape[0], 4, 3))
    b[:, 1:, :] = dminv               # row i-1 of Dm^{-1} for vertex i
    b[:, 0, :] = -dminv.sum(axis=1)
    return dminv, vol, b


def lumped_mass(n_verts: int, tets: np.ndarray, vol: np.ndarray, rho: float) -> np.ndarray:
    m = np.zeros(n_verts)
    for k in range(4):
        np.add.at(m, tets[:, k].astype(np.int64), rho * vol / 4.0)
    return m


def deformation_gradients(x: np.ndarray, tets: np.ndarray, b: np.ndarray) -> np.ndarray:
    """F = sum_a x_a b_a^T per element."""
    xs = x[tets.astype(np.int64)]                      # (n_e, 4, 3)
    return np.einsum("eai,eaj->eij", xs, b)


def polar_rotation(f: np.ndarray) -> np.ndarray:
    """Rotation of the rotation-variant polar decomposition (via SVD), per matrix."""
    u, _, vt = np.linalg.svd(f)
    du = np.linalg.det(u)
    dv = np.linalg.det(vt)
    u = u.copy()
    u[:, :, 2] *= du[:, None]             # det U = 1
    vt = vt.copy()
    vt[:, 2, :] *= dv[:, None]            # det V = 1 (the sign of det F moves to s_3)
    return u @ vt


def psi(f: np.ndarray, mu: float, lam: float) -> np.ndarray:
    r = polar_rotation(f)
    d = f - r
    tr = np.einsum("eij,eij->e", r, f) - 3.0
    return mu * np.einsum("eij,eij->e", d, d) + 0.5 * lam * tr * tr


def first_piola(f: np.ndarray, mu: float, lam: float) -> np.ndarray:
    r = polar_rotation(f)
    tr = np.einsum("eij,eij->e", r, f) - 3.0
    return 2.0 * mu * (f - r) + lam * tr[:, None, None] * r


def element_blocks(x, tets, b, vol, mu, lam, rho, h):
    """(n_e, 144) SPD proxy blocks, row-major 12x12 in DoF order 3a + k."""
    f = deformation_gradients(x, tets, b)
    r = polar_rotation(f)
    rb = np.einsum("eij,eaj->eai", r, b)                       # R b_a
    bb = np.einsum("eai,ebi->eab", b, b)                        # b_a . b_b
    n_e = tets.shape[0]
    blk = np.zeros((n_e, 4, 3, 4, 3))
    eye = np.eye(3)
    blk += (2.0 * mu * vol)[:, None, None, None, None] * bb[:, :, None, :, None] * eye[None, None, :, None, :]
    blk += (lam * vol)[:, None, None, None, None] * rb[:, :, :, None, None] * rb[:, None, None, :, :]
    for a in range(4):
        blk[:, a, :, a, :] += (rho * vol / (4.0 * h * h))[:, None, None] * eye
    return blk.reshape(n_e, 144)


def energy(x, x_hat, mass, tets, b, vol, mu, lam, h) -> float:
    dx = x - x_hat
    inertia = float(np.sum(mass * np.sum(dx * dx, axis=1))) / (2.0 * h * h)
    return inertia + float(np.sum(vol * psi(deformation_gradients(x, tets, b), mu, lam)))


def gradient(x, x_hat, mass, tets, b, vol, mu, lam, h) -> np.ndarray:
    p = first_piola(deformation_gradients(x, tets, b), mu, lam)
    ge = np.einsum("eij,eaj->eai", p, b) * vol[:, None, None]     # V P b_a
    g = (mass / (h * h))[:, None] * (x - x_hat)
    t = tets.astype(np.int64)
    for a in range(4):
        np.add.at(g, t[:, a], ge[:, a])
    return g


def predicted(x_t, v_t, f_ext, mass, h):
    xh = x_t + h * v_t
    if f_ext is not None:
        xh = xh + (h * h) * f_ext / mass[:, None]
    return xh


def affine_solve(sub: dict, rest: np.ndarray, threshold: int) -> tuple[np.ndarray, int]:
    """x = P A_c^{-1} P^T g with the adaptive affine embedding (Sec. 4.2, Eq. 4):
    aggregates of more than `threshold` members carry 12 DoF (oracle/affine.py),
    the coarse system solved directly.  Returns x and the number of 3x3 block rows."""
    from . import affine, aggregate
    from . import solve as _solve
    m, n_c = aggregate.components(sub["n_verts"], sub["edges"], sub["tags"])
    a_c, b_c, cls, pm = affine.coarse_system(dict(sub, pos=rest), m, n_c, threshold)
    x_c = _solve.solve_sparse(a_c, b_c.reshape(-1))
    return affine.prolongate(pm, x_c), int(cls["n_flat"])


def time_step(mesh: dict, mat: dict, x_t, v_t, f_ext=None, eps_d=1e-3, max_newton=50, tag_threshold=5e-5,
              coarsen=True, post_iters=0, affine_threshold=0, record=False):
    """One time step's Newton loop.  mesh: n_verts, rest, tets, edges; mat: mu, lam, rho, h.
    affine_threshold > 0: each solve uses the adaptive affine embedding of
    aggregates with more members than that (Sec. 4.2, Eq. 4).

    Returns x and a per-iteration log (energy before, step length, |d|_inf,
    n_c, the 3x3 block rows of the solve, the quadratic model's value along
    d; with record also the tags, the map, the strain increment norms and the
    iterate after the step)."""
    mu, lam, rho, h = mat["mu"], mat["lam"], mat["rho"], mat["h"]
    rest, tets, n = mesh["rest"], mesh["tets"], mesh["n_verts"]
    _, vol, b = rest_shape(rest, tets)
    mass = lumped_mass(n, tets, vol, rho)
    x_hat = predicted(x_t, v_t, f_ext, mass, h)
    x = x_t.copy()
    x_last = x_t - h * v_t
    log = []
    for _ in range(max_newton):
        e_prev = energy(x, x_hat, mass, tets, b, vol, mu, lam, h)
        g = gradient(x, x_hat, mass, tets, b, vol, mu, lam, h)
        blocks = element_blocks(x, tets, b, vol, mu, lam, rho, h)
        if coarsen:
            tags, norms = tagging.tag_edges(rest, x, x_last, tets, mesh["edges"], tag_threshold)
        else:
            tags = np.zeros(mesh["edges"].shape[0], np.uint8)
            norms = None
        sub = {"n_verts": n, "elem_verts": tets, "elem_H": blocks, "g": g, "edges": mesh["edges"], "tags": tags}
        r = method.coarsened_solve(sub, solver="sparse")
        xs, n_blocks = r["x"], r["n_c"]
        if affine_threshold > 0:
            xs, n_blocks = affine_solve(sub, rest, affine_threshold)
        if post_iters:
            xs, _ = method.post_coarsen(sub, xs, post_iters)
        d = -xs
        alpha, halvings = 1.0, 0
        while True:
            x_new = x + alpha * d
            e_new = energy(x_new, x_hat, mass, tets, b, vol, mu, lam, h)
            if e_new < e_prev:
                break
            halvings += 1
            if halvings > MAX_HALVINGS:
                x_new, e_new = x, e_prev
                break
            alpha *= 0.5
        d_inf = float(np.max(np.abs(d)))
        # the quadratic model of this iteration along d (Sec. 3, Eq. 2): g^T d + d^T H d / 2
        q = float(np.sum(g * d) + 0.5 * np.sum(d * galerkin.fine_matvec(tets, blocks, d)))
        entry = {"energy": e_prev, "energy_after": e_new, "alpha": alpha, "halvings": halvings,
                 "d_inf": d_inf, "n_c": r["n_c"], "n_blocks": n_blocks, "model": q}
        if record:
            entry.update(tags=tags, map=r["map"], norms=norms, x=x_new.copy())
        log.append(entry)
        x_last, x = x, x_new
        if d_inf / h <= eps_d or halvings > MAX_HALVINGS:
            break
    return x, log
