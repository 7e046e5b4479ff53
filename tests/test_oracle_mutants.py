"""Planted mistakes in copies of the oracle must trip the pins (CPU only).

Each mutant is a plausible slip - a wrong index, a transposed operand, a
dropped term, a wrong sign, a wrong order - applied to a local copy of an
oracle function.  The real oracle passes every pin (test_oracle.py); here each
mutant must fail at least one.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import aggregate, galerkin, solve
from paper_2605_04773_amd import synth
from tests import pins


@pytest.fixture(scope="module")
def c1():
    return synth.make_config("c1")


def _fails(fn, *a, **k):
    try:
        fn(*a, **k)
    except AssertionError:
        return True
    return False


def test_mutant_label_order_by_largest_member():
    def components_max(n, e, t):
        m, n_c = aggregate.components(n, e, t)
        last = np.zeros(n_c, np.int64)
        np.maximum.at(last, m, np.arange(n))
        rank = np.empty(n_c, np.int64)
        rank[np.argsort(last, kind="stable")] = np.arange(n_c)
        return rank[m], n_c
    hit = False
    for seed in range(10):
        rng = np.random.default_rng(seed)
        e, t = synth.random_graph(rng, 30, 40)
        m, n_c = components_max(30, e, t)
        hit |= _fails(pins.check_map_valid, 30, e, t, m, n_c)
    assert hit


def test_mutant_directed_edges_only():
    """Hooking only a->b for a < b on a path written backwards still connects; ignoring tags does not."""
    fx = pins.golden("hash_protected_singletons.json")
    e = np.array(fx["edges"])
    t = np.array(fx["tags"], np.uint8)
    m, n_c = aggregate.components(fx["n_nodes"], e, np.ones_like(t))     # mutant: tags ignored
    assert m.tolist() != fx["expected_map"]


def test_mutant_prolongation_shifted(c1):
    m, n_c = aggregate.components(c1["n_verts"], c1["edges"], c1["tags"])
    wrong = (m + 1) % n_c
    P = galerkin.prolongation(wrong, n_c)
    a_c, b_c = (P.T @ galerkin.fine_hessian(c1["n_verts"], c1["elem_verts"], c1["elem_H"]) @ P), \
        (P.T @ c1["g"].reshape(-1)).reshape(-1, 3)
    assert _fails(pins.check_energy_identity, a_c, b_c, c1["elem_verts"], c1["elem_H"], c1["g"], m, n_c)


def test_mutant_prolongation_component_swap(c1):
    """P[3v+i, 3c+(2-i)]: a transposed DoF index inside each vertex."""
    m, n_c = aggregate.components(c1["n_verts"], c1["edges"], c1["tags"])
    mm = np.asarray(m, np.int64)
    n = mm.shape[0]
    rows = (3 * np.arange(n)[:, None] + np.arange(3)[None, :]).ravel()
    cols = (3 * mm[:, None] + (2 - np.arange(3))[None, :]).ravel()
    P = sp.csr_matrix((np.ones(3 * n), (rows, cols)), shape=(3 * n, 3 * n_c))
    h = galerkin.fine_hessian(c1["n_verts"], c1["elem_verts"], c1["elem_H"])
    assert _fails(pins.check_energy_identity, P.T @ h @ P, (P.T @ c1["g"].reshape(-1)).reshape(-1, 3),
                  c1["elem_verts"], c1["elem_H"], c1["g"], m, n_c)


def test_mutant_wrong_dof_order(c1):
    """Element DoF taken as 4k+a instead of 3a+k."""
    m, n_c = aggregate.components(c1["n_verts"], c1["edges"], c1["tags"])
    ev = np.asarray(c1["elem_verts"], np.int64)
    dofs = (3 * ev[:, None, :] + np.arange(3)[None, :, None]).reshape(-1, 12)   # order k*4+a
    hv = c1["elem_H"].reshape(-1, 12, 12)
    r = np.repeat(dofs, 12, axis=1).ravel()
    c = np.tile(dofs, (1, 12)).ravel()
    n3 = 3 * c1["n_verts"]
    h = sp.coo_matrix((hv.ravel(), (r, c)), shape=(n3, n3)).tocsr()
    P = galerkin.prolongation(m, n_c)
    assert _fails(pins.check_energy_identity, P.T @ h @ P, galerkin.restrict(m, n_c, c1["g"]),
                  c1["elem_verts"], c1["elem_H"], c1["g"], m, n_c)


def test_mutant_dropped_element(c1):
    n = c1["n_verts"]
    m, n_c = aggregate.components(n, c1["edges"], np.ones_like(c1["tags"]))
    a_c, b_c = galerkin.coarse_system(n, c1["elem_verts"][:-1], c1["elem_H"][:-1], c1["g"], m, n_c)
    k = c1["elem_verts"].shape[0] * 144
    assert _fails(pins.check_all_collapsible_closed_form, a_c, b_c, c1["g"], synth.DENSITY, c1["h"], k,
                  np.abs(c1["elem_H"]).sum() / 9)


def test_mutant_adjoint_sign_and_transpose(c1):
    from oracle import adjoint
    p = synth.grid_problem(2, 5, 0.5)
    rng = np.random.default_rng(2)
    w = rng.standard_normal((p["n_verts"], 3))
    m, n_c = aggregate.components(p["n_verts"], p["edges"], p["tags"])
    x, dg, dh = adjoint.adjoint(p["n_verts"], p["elem_verts"], p["elem_H"], p["g"], m, n_c, w, dense=True)
    L = float(np.sum(w * x))
    assert _fails(pins.check_adjoint_identities, L, p["g"], dg, p["elem_H"], -dh)      # sign
    ev = np.asarray(p["elem_verts"], np.int64)
    wrong = -(dg[ev].reshape(-1, 12)[:, :, None] * dg[ev].reshape(-1, 12)[:, None, :]).reshape(-1, 144)
    assert _fails(pins.check_adjoint_identities, L, p["g"], dg, p["elem_H"], wrong)    # x_c -> lambda_c


def test_mutant_pcg_wrong_beta(c1):
    m, n_c = aggregate.components(c1["n_verts"], c1["edges"], c1["tags"])
    a_c, b_c = galerkin.coarse_system(c1["n_verts"], c1["elem_verts"], c1["elem_H"], c1["g"], m, n_c)
    x_star = solve.solve_dense(a_c.toarray(), b_c.reshape(-1))
    dinv = solve.block_jacobi_inverse(a_c)
    b = b_c.reshape(-1)
    x = np.zeros_like(b)
    r = b.copy()
    z = np.einsum("nij,nj->ni", dinv, r.reshape(-1, 3)).reshape(-1)
    p = z.copy()
    rz = r @ z
    for _ in range(200):                     # mutant: beta = rz_old / rz_new
        q = a_c @ p
        al = rz / (p @ q)
        x += al * p
        r -= al * q
        z = np.einsum("nij,nj->ni", dinv, r.reshape(-1, 3)).reshape(-1)
        rz_new = r @ z
        p = z + (rz / rz_new) * p
        rz = rz_new
    assert np.linalg.norm(x - x_star) > 1e-8 * np.linalg.norm(x_star)


def test_mutants_affine_node_order():
    """Three plausible slips in the affine node order each trip the Alg. 3 pin:
    12-DoF nodes first; no reorder at all (offsets by canonical label); and
    12-DoF nodes in reverse label order."""
    from oracle import affine
    m = np.repeat(np.arange(9), [6, 1, 2, 5, 1, 9, 3, 1, 7]).astype(np.int32)
    n_c, thr = 9, 4

    def twelve_first(map_, n, t):
        big = np.bincount(map_, minlength=n) > t
        n12 = int(big.sum())
        lab = np.empty(n, np.int64)
        lab[big] = np.arange(n12)
        lab[~big] = n12 + np.arange(n - n12)
        off = np.where(big, 4 * lab, 4 * n12 + (lab - n12))
        return {"new_label": lab, "offset": off, "n3": n - n12}

    def no_reorder(map_, n, t):
        big = np.bincount(map_, minlength=n) > t
        width = np.where(big, 4, 1)
        off = np.concatenate([[0], np.cumsum(width)[:-1]])
        return {"new_label": np.arange(n), "offset": off, "n3": int((~big).sum())}

    def reversed_12(map_, n, t):
        cls = affine.classify(map_, n, t)
        big = cls["big"]
        lab = cls["new_label"].copy()
        lab[big] = lab[big][::-1]
        off = np.where(big, cls["n3"] + 4 * (lab - cls["n3"]), lab)
        return {"new_label": lab, "offset": off, "n3": cls["n3"]}

    pins.check_affine_order(affine.classify, m, n_c, thr)
    for mutant in (twelve_first, no_reorder, reversed_12):
        assert _fails(pins.check_affine_order, mutant, m, n_c, thr), mutant.__name__
