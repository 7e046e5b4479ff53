"""Pins of the Newton-loop oracle (Sec. 3, Eq. 1-2; Alg. overview), CPU only.

What fixes the oracle, independently of its own code:
* the polar rotation: R^T R = I, det R = 1, R^T F symmetric; for F = Q S with
  Q a rotation and S symmetric positive definite, R = Q; for a reflected F
  the sign goes to the smallest singular value (R proper, R^T F symmetric
  with one negative eigenvalue);
* psi: zero at rest, invariant under rotations of the deformed shape, the
  closed form 3 mu (s-1)^2 + 9 lam/2 (s-1)^2 for a uniform stretch s;
* dpsi/dF against central differences of psi;
* the SPD proxy: symmetric, positive definite, the exact Hessian of the
  energy with the element rotation held fixed (finite differences of that
  energy's gradient), mass part rho V / (4 h^2) I per vertex block;
* the total gradient against central differences of the total energy;
* the loop: energy decreases every iteration; the fine loop (every tag 0)
  ends with a gradient near zero; the coarsened one ends near the fine
  one's energy.
Planted mistakes (bottom) each trip one of these pins.
"""
import math

import numpy as np

from oracle import newton
from paper_2605_04773_amd import synth


def _rot(rng):
    return synth.random_rotations(rng, 1)[0]


def _small(n=3, seed=11):
    p = synth.grid_problem(n, seed, 0.6)
    return p


def _spd(rng, m=1):
    a = rng.standard_normal((m, 3, 3))
    return np.einsum("eij,ekj->eik", a, a) + 0.5 * np.eye(3)[None]


# ----------------------------------------------------------------- pins

def check_polar(polar):
    rng = np.random.default_rng(3)
    f = np.eye(3)[None] + 0.4 * rng.standard_normal((200, 3, 3))
    r = polar(f)
    assert np.allclose(np.einsum("eji,ejk->eik", r, r), np.eye(3)[None], atol=1e-12)
    assert np.allclose(np.linalg.det(r), 1.0, atol=1e-12)
    s = np.einsum("eji,ejk->eik", r, f)
    assert np.allclose(s, np.swapaxes(s, 1, 2), atol=1e-12)
    q = np.stack([_rot(rng) for _ in range(20)])
    sp = _spd(rng, 20)
    assert np.allclose(polar(q @ sp), q, atol=1e-11)
    # a reflected F: proper R, R^T F symmetric with exactly one negative eigenvalue
    refl = q @ sp @ np.diag([1.0, 1.0, -1.0])[None]
    r2 = polar(refl)
    assert np.allclose(np.linalg.det(r2), 1.0, atol=1e-12)
    s2 = np.einsum("eji,ejk->eik", r2, refl)
    assert np.allclose(s2, np.swapaxes(s2, 1, 2), atol=1e-11)
    ev = np.linalg.eigvalsh(0.5 * (s2 + np.swapaxes(s2, 1, 2)))
    assert np.all((ev < 0).sum(axis=1) == 1)


def check_psi(psi):
    mu, lam = 3.0, 7.0
    rng = np.random.default_rng(4)
    assert np.allclose(psi(np.stack([np.eye(3), _rot(rng)]), mu, lam), 0.0, atol=1e-13)
    f = np.eye(3)[None] + 0.3 * rng.standard_normal((50, 3, 3))
    q = np.stack([_rot(rng) for _ in range(50)])
    assert np.allclose(psi(q @ f, mu, lam), psi(f, mu, lam), rtol=1e-10, atol=1e-13)
    for s in (0.8, 1.0, 1.3):
        want = 3 * mu * (s - 1) ** 2 + 4.5 * lam * (s - 1) ** 2
        assert math.isclose(float(psi((s * np.eye(3))[None], mu, lam)[0]), want, rel_tol=1e-12, abs_tol=1e-14)


def check_piola(psi, piola):
    mu, lam = 3.0, 7.0
    rng = np.random.default_rng(5)
    f = np.eye(3)[None] + 0.3 * rng.standard_normal((20, 3, 3))
    p = piola(f, mu, lam)
    eps = 1e-6
    for i in range(3):
        for j in range(3):
            df = np.zeros((1, 3, 3))
            df[0, i, j] = eps
            fd = (psi(f + df, mu, lam) - psi(f - df, mu, lam)) / (2 * eps)
            assert np.allclose(p[:, i, j], fd, rtol=1e-6, atol=1e-7)


def _frozen_grad(x, tets, b, vol, r0, mu, lam):
    """Element gradients of the energy with rotations r0 held fixed."""
    f = newton.deformation_gradients(x, tets, b)
    tr = np.einsum("eij,eij->e", r0, f) - 3.0
    p = 2.0 * mu * (f - r0) + lam * tr[:, None, None] * r0
    return np.einsum("eij,eaj->eai", p, b) * vol[:, None, None]


def check_blocks(element_blocks):
    p = _small()
    mat = synth.material()
    mu, lam, rho, h = mat["mu"], mat["lam"], mat["rho"], mat["h"]
    rng = np.random.default_rng(6)
    tets = p["elem_verts"]
    _, vol, b = newton.rest_shape(p["pos"], tets)
    x = p["pos"] @ _rot(rng).T + 0.02 * rng.standard_normal(p["pos"].shape)
    blk = element_blocks(x, tets, b, vol, mu, lam, rho, h).reshape(-1, 12, 12)
    assert np.allclose(blk, np.swapaxes(blk, 1, 2), rtol=0, atol=1e-9 * np.abs(blk).max())
    assert np.linalg.eigvalsh(blk).min() > 0
    # exact Hessian of the frozen-rotation energy (finite differences; it is quadratic)
    r0 = newton.polar_rotation(newton.deformation_gradients(x, tets, b))
    dx = rng.standard_normal(x.shape)
    eps = 1e-4
    gp = _frozen_grad(x + eps * dx, tets, b, vol, r0, mu, lam)
    gm = _frozen_grad(x - eps * dx, tets, b, vol, r0, mu, lam)
    fd = ((gp - gm) / (2 * eps)).reshape(-1, 12)
    mass = np.zeros((tets.shape[0], 12, 12))
    for a in range(4):
        mass[:, 3 * a:3 * a + 3, 3 * a:3 * a + 3] = (rho * vol / (4 * h * h))[:, None, None] * np.eye(3)
    dxe = dx[tets.astype(np.int64)].reshape(-1, 12)
    hv = np.einsum("eij,ej->ei", blk - mass, dxe)
    assert np.allclose(hv, fd, rtol=1e-7, atol=1e-7 * np.abs(fd).max())


def check_gradient(gradient):
    p = _small()
    mat = synth.material()
    mu, lam, rho, h = mat["mu"], mat["lam"], mat["rho"], mat["h"]
    rng = np.random.default_rng(7)
    tets = p["elem_verts"]
    _, vol, b = newton.rest_shape(p["pos"], tets)
    mass = newton.lumped_mass(p["n_verts"], tets, vol, rho)
    x = p["pos"] + 0.01 * rng.standard_normal(p["pos"].shape)
    x_hat = p["pos"] + 0.005 * rng.standard_normal(p["pos"].shape)
    g = gradient(x, x_hat, mass, tets, b, vol, mu, lam, h)
    for _ in range(4):
        d = rng.standard_normal(x.shape)
        eps = 1e-7
        ep = newton.energy(x + eps * d, x_hat, mass, tets, b, vol, mu, lam, h)
        em = newton.energy(x - eps * d, x_hat, mass, tets, b, vol, mu, lam, h)
        fd = (ep - em) / (2 * eps)
        assert math.isclose(float(np.sum(g * d)), fd, rel_tol=1e-6)


def _newton_case(n=4):
    p = _small(n)
    mesh = {"n_verts": p["n_verts"], "rest": p["pos"], "tets": p["elem_verts"], "edges": p["edges"]}
    x_t, v_t, f = synth.newton_state(p, wave_speed=0.5)
    return p, mesh, x_t, v_t, f


def check_loop(time_step):
    p, mesh, x_t, v_t, f = _newton_case()
    mat = synth.material()
    xf, logf = time_step(mesh, mat, x_t, v_t, f, eps_d=1e-4, coarsen=False)
    xc, logc = time_step(mesh, mat, x_t, v_t, f, eps_d=1e-4, coarsen=True)
    for log in (logf, logc):
        assert all(it["energy_after"] < it["energy"] for it in log), "the line search must decrease E"
    _, vol, b = newton.rest_shape(p["pos"], p["elem_verts"])
    mass = newton.lumped_mass(p["n_verts"], p["elem_verts"], vol, mat["rho"])
    x_hat = newton.predicted(x_t, v_t, f, mass, mat["h"])
    args = (x_hat, mass, p["elem_verts"], b, vol, mat["mu"], mat["lam"], mat["h"])
    g0 = np.linalg.norm(newton.gradient(x_t, *args))
    assert np.linalg.norm(newton.gradient(xf, *args)) < 1e-4 * g0
    ef, ec = newton.energy(xf, *args), newton.energy(xc, *args)
    e0 = newton.energy(x_t, *args)
    assert ef <= ec and (ec - ef) < 1e-3 * (e0 - ef)
    assert len(logf) >= 2 and any(it["n_c"] < p["n_verts"] for it in logc)


def check_affine_loop(time_step):
    """The loop with the adaptive affine embedding (Sec. 4.2, Eq. 4): with the
    threshold above every aggregate it is the 3-DoF loop exactly; with a
    threshold of 8 its first solve, which sees the same tags and map as the
    3-DoF one, has 12-DoF nodes and lowers the quadratic model strictly more
    (its subspace contains the 3-DoF one; the iterations before it have no
    12-DoF node, so both loops reach it in the same state), every step lowers E, and the loop
    ends at the fine loop's minimum to 1e-3 of the energy drop."""
    p, mesh, x_t, v_t, f = _newton_case()
    mat = synth.material()
    xc, logc = newton.time_step(mesh, mat, x_t, v_t, f, eps_d=1e-4, coarsen=True)
    xb, logb = time_step(mesh, mat, x_t, v_t, f, eps_d=1e-4, coarsen=True, affine_threshold=10 ** 6)
    assert np.array_equal(xb, xc) and len(logb) == len(logc)
    xa, loga = time_step(mesh, mat, x_t, v_t, f, eps_d=1e-4, coarsen=True, affine_threshold=8)
    # the first iteration with a 12-DoF node: the iterations before it solve the same
    # 3-DoF systems (up to rounding), so both loops see the same state and map there
    k = next(i for i, it in enumerate(loga) if it["n_blocks"] > it["n_c"])
    assert k < len(logc) and loga[k]["n_c"] == logc[k]["n_c"]
    assert abs(loga[k]["energy"] - logc[k]["energy"]) <= 1e-12 * abs(logc[k]["energy"])
    assert loga[k]["model"] < logc[k]["model"] - 1e-9 * abs(logc[k]["model"])
    assert all(it["energy_after"] < it["energy"] for it in loga)
    xf, logf = newton.time_step(mesh, mat, x_t, v_t, f, eps_d=1e-4, coarsen=False)
    e0, ef = logf[0]["energy"], logf[-1]["energy_after"]
    assert loga[-1]["energy_after"] - ef <= 1e-3 * (e0 - ef)


def test_affine_loop():
    check_affine_loop(newton.time_step)


def test_mutant_affine_loop_ignores_the_embedding():
    """A loop that takes the 3-DoF solve whatever the threshold."""
    def time_step(mesh, mat, x_t, v_t, f, eps_d, coarsen, affine_threshold):
        x, log = newton.time_step(mesh, mat, x_t, v_t, f, eps_d=eps_d, coarsen=coarsen)
        for it in log:
            it["n_blocks"] = it["n_c"] + (3 if affine_threshold < 10 ** 6 else 0)
        return x, log
    assert _fails(check_affine_loop, time_step)


def test_polar():
    check_polar(newton.polar_rotation)


def test_psi():
    check_psi(newton.psi)


def test_piola():
    check_piola(newton.psi, newton.first_piola)


def test_blocks():
    check_blocks(newton.element_blocks)


def test_gradient():
    check_gradient(newton.gradient)


def test_loop():
    check_loop(newton.time_step)


# -------------------------------------------------------------- mutants

def _fails(fn, *a):
    try:
        fn(*a)
    except AssertionError:
        return True
    return False


def test_mutant_polar_without_sign_fix():
    def polar(f):
        u, _, vt = np.linalg.svd(f)
        return u @ vt                      # a reflection for det F < 0
    assert _fails(check_polar, polar)


def test_mutant_polar_transposed():
    assert _fails(check_polar, lambda f: np.swapaxes(newton.polar_rotation(f), 1, 2))


def test_mutant_psi_trace_without_rotation():
    def psi(f, mu, lam):
        r = newton.polar_rotation(f)
        d = f - r
        tr = np.einsum("eii->e", f) - 3.0   # tr F instead of tr R^T F: not rotation invariant
        return mu * np.einsum("eij,eij->e", d, d) + 0.5 * lam * tr * tr
    assert _fails(check_psi, psi)


def test_mutant_piola_sign():
    def piola(f, mu, lam):
        r = newton.polar_rotation(f)
        tr = np.einsum("eij,eij->e", r, f) - 3.0
        return 2.0 * mu * (f - r) - lam * tr[:, None, None] * r
    assert _fails(check_piola, newton.psi, piola)


def test_mutant_blocks_without_lambda():
    def blocks(x, tets, b, vol, mu, lam, rho, h):
        return newton.element_blocks(x, tets, b, vol, mu, 0.0, rho, h)
    assert _fails(check_blocks, blocks)


def test_mutant_blocks_rotation_transposed():
    def blocks(x, tets, b, vol, mu, lam, rho, h):
        f = newton.deformation_gradients(x, tets, b)
        ft = np.swapaxes(newton.polar_rotation(f), 1, 2)
        saved = newton.polar_rotation
        try:
            newton.polar_rotation = lambda _f: ft
            return newton.element_blocks(x, tets, b, vol, mu, lam, rho, h)
        finally:
            newton.polar_rotation = saved
    assert _fails(check_blocks, blocks)


def test_mutant_gradient_without_inertia():
    def gradient(x, x_hat, mass, tets, b, vol, mu, lam, h):
        return newton.gradient(x, x_hat, np.zeros_like(mass), tets, b, vol, mu, lam, h)
    assert _fails(check_gradient, gradient)


def test_mutant_loop_full_step_always():
    """A loop that takes alpha = 1 whatever the energy does."""
    def time_step(mesh, mat, x_t, v_t, f, eps_d, coarsen):
        x, log = newton.time_step(mesh, mat, x_t, v_t, f, eps_d=eps_d, coarsen=coarsen, max_newton=1)
        for it in log:
            it["energy_after"] = it["energy"] + 1.0
        return x, log
    assert _fails(check_loop, time_step)
