"""CPU checks of the synthetic input generator (mesh, element blocks, tags)."""
import math

import numpy as np
import pytest

from paper_2605_04773_amd import synth


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 3, 4), (8, 8, 8), (4, 8, 24)])
def test_mesh_counts_match_closed_forms(dims):
    nx, ny, nz = dims
    pos, tets = synth.box_mesh(nx, ny, nz, 0.1)
    edges = synth.mesh_edges(tets, pos.shape[0])
    c = synth.grid_counts(nx, ny, nz)
    assert pos.shape[0] == c["n_verts"]
    assert tets.shape[0] == c["n_tets"]
    # conforming face diagonals: one diagonal per cube face, no interior diagonal
    assert edges.shape[0] == c["n_edges"]
    vol, _ = synth.shape_gradients(pos, tets)
    assert np.isclose(vol.sum(), nx * ny * nz * 0.1 ** 3)
    d = pos[tets[:, 1:]] - pos[tets[:, :1]]
    assert (np.linalg.det(d) > 0).all()


def test_c_sizes():
    # vertex/element/edge counts quoted for the measured workloads
    assert synth.grid_counts(8, 8, 8) == {"n_verts": 729, "n_tets": 2560, "n_edges": 3672}
    assert synth.grid_counts(64, 64, 64)["n_verts"] == 274625
    assert synth.grid_counts(64, 64, 64)["n_tets"] == 1310720
    assert synth.grid_counts(128, 128, 128)["n_verts"] == 2146689
    assert synth.grid_counts(128, 128, 128)["n_edges"] == 12730752


def _tet_k0(seed=0):
    rng = np.random.default_rng(seed)
    pos = rng.standard_normal((4, 3))
    tets = np.array([[0, 1, 2, 3]], dtype=np.int32)
    if np.linalg.det(pos[1:] - pos[0]) < 0:
        tets = tets[:, [0, 1, 3, 2]]
    vol, grads = synth.shape_gradients(pos, tets)
    mu, lam = synth.lame()
    k0 = synth.linear_stiffness(vol, grads, mu, lam)[0].transpose(0, 2, 1, 3).reshape(12, 12)
    return pos, tets, vol[0], k0, mu, lam


def test_stiffness_energy_of_linear_field():
    """1/2 u^T K0 u equals V (mu eps:eps + lam/2 tr(eps)^2) for an affine displacement."""
    pos, tets, vol, k0, mu, lam = _tet_k0(3)
    rng = np.random.default_rng(7)
    for _ in range(5):
        grad_u = rng.standard_normal((3, 3))
        u = (pos[tets[0]] @ grad_u.T).reshape(-1)        # u(X) = G X at each vertex
        eps = 0.5 * (grad_u + grad_u.T)
        energy = vol * (mu * np.sum(eps * eps) + 0.5 * lam * np.trace(eps) ** 2)
        assert np.isclose(0.5 * u @ k0 @ u, energy, rtol=1e-12)


def test_stiffness_null_space():
    pos, tets, vol, k0, mu, lam = _tet_k0(5)
    for t in np.eye(3):
        assert np.abs(k0 @ np.tile(t, 4)).max() < 1e-9 * np.abs(k0).max()
    # infinitesimal rotation about the origin is also a zero-energy mode of K0
    w = np.array([0.3, -1.2, 0.7])
    u = np.cross(w[None, :], pos[tets[0]]).reshape(-1)
    assert np.abs(k0 @ u).max() < 1e-9 * np.abs(k0).max() * np.abs(u).max()
    assert np.linalg.eigvalsh(k0).min() > -1e-9 * np.abs(k0).max()


def test_rotations_orthonormal():
    r = synth.random_rotations(synth.rng_for(0, 0), 100)
    assert np.allclose(r @ np.swapaxes(r, 1, 2), np.eye(3), atol=1e-12)
    assert np.allclose(np.linalg.det(r), 1.0)


def test_c1_blocks_and_mass():
    p = synth.make_config("c1")
    h = p["elem_H"].reshape(-1, 12, 12)
    assert np.array_equal(h, np.swapaxes(h, 1, 2))                 # exactly symmetric
    assert np.linalg.eigvalsh(h).min() > 0                         # SPD (mass folded in)
    assert math.isclose(p["mass"].sum(), synth.DENSITY, rel_tol=1e-12)  # unit cube
    n_col = int(p["tags"].sum())
    assert n_col == math.floor(0.7 * p["edges"].shape[0])
    # the element mass term is rho V/(4 h^2) on the diagonal: H_e 1 (translation) = mass * 1
    vol, _ = synth.shape_gradients(p["pos"], p["elem_verts"])
    t = np.tile([1.0, 0.0, 0.0], 4)
    lhs = h @ t
    rhs = (synth.DENSITY * vol / (4 * p["h"] ** 2))[:, None] * t[None, :]
    assert np.allclose(lhs, rhs, rtol=1e-9, atol=1e-9 * np.abs(h).max())


def test_generator_is_deterministic():
    a = synth.grid_problem(3, 11, 0.5)
    b = synth.grid_problem(3, 11, 0.5)
    for k in ("edges", "tags", "elem_verts", "elem_H", "g"):
        assert np.array_equal(a[k], b[k])
    c = synth.grid_problem(3, 12, 0.5)
    assert not np.array_equal(a["g"], c["g"])


def test_rank_tags_ties_by_id():
    v = np.array([1.0, 0.0, 1.0, 0.0, 2.0])
    assert synth.rank_tags(v, 0.6).tolist() == [1, 1, 0, 1, 0]
