"""Pins of the FP64 oracle against the paper's worked examples, closed forms,
invariants and brute force.  CPU only."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import adjoint, aggregate, galerkin, method, solve
from paper_2605_04773_amd import synth
from tests import pins


@pytest.fixture(scope="module")
def c1():
    return synth.make_config("c1")


@pytest.fixture(scope="module")
def tiny():
    return synth.grid_problem(2, 21, 0.5)


# =============================================================== aggregation

def test_golden_group4_indirect():
    fx = pins.golden("hash_group4_indirect.json")
    edges = pins.edges_from_direct_hashes(fx["direct_hashes"])
    tags = np.ones(edges.shape[0], np.uint8)
    h = aggregate.direct_hashes(4, edges, fx["group_size"])
    assert [pins.hash_str(x, 4) for x in h] == fx["direct_hashes"]
    _, _, _, closed = aggregate._one_level(4, edges, fx["group_size"])
    assert [pins.hash_str(x, 4) for x in closed] == fx["closed_hashes"]
    for fn in (aggregate.components, aggregate.components_bfs):
        m, n_c = fn(4, edges, tags)
        assert m.tolist() == fx["expected_map"] and n_c == fx["expected_n_coarse"]


def test_golden_protected_singletons():
    fx = pins.golden("hash_protected_singletons.json")
    e = np.array(fx["edges"])
    t = np.array(fx["tags"], np.uint8)
    col = e[t == 1]
    h = aggregate.direct_hashes(fx["n_nodes"], col, fx["group_size"])
    assert [pins.hash_str(x, 3) for x in h] == fx["expected_direct_hashes"]
    m, n_c, conv, _ = aggregate.hash_levels(fx["n_nodes"], e, t, fx["group_size"])
    assert conv and m.tolist() == fx["expected_map"] and n_c == fx["expected_n_coarse"]
    for fn in (aggregate.components, aggregate.components_bfs):
        m, n_c = fn(fx["n_nodes"], e, t)
        assert m.tolist() == fx["expected_map"] and n_c == fx["expected_n_coarse"]


@pytest.mark.parametrize("seed", range(30))
def test_components_three_ways(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 50))
    m_edges = int(rng.integers(0, 3 * n + 2))
    e, t = synth.random_graph(rng, n, m_edges, p_tag=rng.uniform(0, 1))
    if n == 0:
        e, t = np.zeros((0, 2), np.int32), np.zeros(0, np.uint8)
    a, na = aggregate.components(n, e, t)
    b, nb = aggregate.components_bfs(n, e, t)
    assert na == nb and np.array_equal(a, b)
    pins.check_map_valid(n, e, t, a, na)
    # the paper's group-hash procedure with one group spanning all nodes is an exact
    # connected-components algorithm, and its popcount labels are the canonical ones
    if n:
        c, nc, conv, _ = aggregate.hash_levels(n, e, t, group_size=max(n, 1))
        assert conv and nc == na and np.array_equal(c, a)


@pytest.mark.parametrize("gs", [3, 4, 8, 32])
def test_hash_levels_fixed_point_on_grid(gs):
    """All tags 1 on a connected mesh: the recursion ends in one node, Map(i) = 0 (supplement Sec. 1.3)."""
    pos, tets = synth.box_mesh(3, 3, 3, 1 / 3)
    e = synth.mesh_edges(tets, pos.shape[0])
    t = np.ones(e.shape[0], np.uint8)
    m, n_c, conv, _ = aggregate.hash_levels(pos.shape[0], e, t, gs)
    assert conv and n_c == 1 and not m.any()


@pytest.mark.parametrize("gs", [4, 8, 16, 32])
def test_hash_levels_match_canonical_when_converged(gs):
    """Where the level-wise recursion reaches its fixed point, its labels are the canonical map."""
    hits = 0
    for seed in range(40):
        p = synth.grid_problem(3, 100 + seed, 0.6)
        m, n_c, conv, _ = aggregate.hash_levels(p["n_verts"], p["edges"], p["tags"], gs)
        if conv:
            hits += 1
            a, na = aggregate.components(p["n_verts"], p["edges"], p["tags"])
            assert n_c == na and np.array_equal(m, a)
    assert hits >= 5


def test_map_special_cases(c1):
    n = c1["n_verts"]
    m, n_c = aggregate.components(n, c1["edges"], np.zeros_like(c1["tags"]))
    assert n_c == n and np.array_equal(m, np.arange(n))
    m, n_c = aggregate.components(n, c1["edges"], np.ones_like(c1["tags"]))
    assert n_c == 1 and not m.any()
    m, n_c = aggregate.components(n, c1["edges"], c1["tags"])
    pins.check_map_valid(n, c1["edges"], c1["tags"], m, n_c)
    rep = aggregate.representatives(m, n_c)
    assert (np.diff(rep) > 0).all() and rep[0] == 0


def test_aggregate_rejects_bad_input():
    with pytest.raises(ValueError):
        aggregate.components(3, np.array([[0, 3]]), np.array([1]))
    with pytest.raises(ValueError):
        aggregate.components(3, np.array([[0, 1]]), np.array([2]))


# =============================================================== Galerkin

def test_prolongation_pins(c1):
    m, n_c = aggregate.components(c1["n_verts"], c1["edges"], c1["tags"])
    pins.check_prolongation(galerkin.prolongation(m, n_c), m, n_c)
    pins.check_prolongation(galerkin.dense_prolongation(m, n_c), m, n_c)


def test_energy_identity(c1):
    m, n_c = aggregate.components(c1["n_verts"], c1["edges"], c1["tags"])
    a_c, b_c = galerkin.coarse_system(c1["n_verts"], c1["elem_verts"], c1["elem_H"], c1["g"], m, n_c)
    pins.check_energy_identity(a_c, b_c, c1["elem_verts"], c1["elem_H"], c1["g"], m, n_c)


def test_dense_and_sparse_agree(tiny):
    p = tiny
    m, n_c = aggregate.components(p["n_verts"], p["edges"], p["tags"])
    a_c, b_c = galerkin.coarse_system(p["n_verts"], p["elem_verts"], p["elem_H"], p["g"], m, n_c)
    hd = galerkin.dense_fine_hessian(p["n_verts"], p["elem_verts"], p["elem_H"])
    pd = galerkin.dense_prolongation(m, n_c)
    ad = pd.T @ hd @ pd
    assert np.allclose(a_c.toarray(), ad, rtol=0, atol=1e-9 * np.abs(ad).max())
    assert np.allclose(b_c.reshape(-1), pd.T @ p["g"].reshape(-1), rtol=0, atol=1e-12)


def test_coarse_spd_and_symmetric(c1):
    m, n_c = aggregate.components(c1["n_verts"], c1["edges"], c1["tags"])
    a_c, _ = galerkin.coarse_system(c1["n_verts"], c1["elem_verts"], c1["elem_H"], c1["g"], m, n_c)
    ad = a_c.toarray()
    assert np.abs(ad - ad.T).max() <= 1e-12 * np.abs(ad).max()
    np.linalg.cholesky(ad)


def test_coarse_pattern(c1):
    m, n_c = aggregate.components(c1["n_verts"], c1["edges"], c1["tags"])
    a_c, _ = galerkin.coarse_system(c1["n_verts"], c1["elem_verts"], c1["elem_H"], c1["g"], m, n_c)
    rows, cols = galerkin.coarse_pattern(c1["elem_verts"], m, n_c)
    key = set(zip(rows.tolist(), cols.tolist()))
    # every block with a nonzero entry is in the pattern, and the pattern is symmetric
    bsr = sp.bsr_matrix(a_c, blocksize=(3, 3))
    bsr.eliminate_zeros()
    for r in range(n_c):
        for k in range(bsr.indptr[r], bsr.indptr[r + 1]):
            if np.any(bsr.data[k] != 0):
                assert (r, int(bsr.indices[k])) in key
    assert all((c, r) in key for r, c in key)
    # the pattern is exactly the set of coarse pairs joined by some element
    ev = m[c1["elem_verts"]]
    brute = {(int(a), int(b)) for row in ev for a in row for b in row}
    assert brute == key


def test_coarse_rows_match_full_product(c1):
    m, n_c = aggregate.components(c1["n_verts"], c1["edges"], c1["tags"])
    a_c, _ = galerkin.coarse_system(c1["n_verts"], c1["elem_verts"], c1["elem_H"], c1["g"], m, n_c)
    ad = a_c.toarray()
    rows = [0, 1, n_c // 2, n_c - 1]
    blocks = galerkin.coarse_rows(c1["elem_verts"], c1["elem_H"], m, n_c, rows)
    pr, pc = galerkin.coarse_pattern(c1["elem_verts"], m, n_c)
    assert set(blocks) == {(r, c) for r, c in zip(pr.tolist(), pc.tolist()) if r in rows}
    for (r, c), blk in blocks.items():
        ref = ad[3 * r:3 * r + 3, 3 * c:3 * c + 3]
        assert np.allclose(blk, ref, rtol=0, atol=1e-9 * np.abs(ad).max())


def test_matrix_free_residual(c1):
    m, n_c = aggregate.components(c1["n_verts"], c1["edges"], c1["tags"])
    a_c, b_c = galerkin.coarse_system(c1["n_verts"], c1["elem_verts"], c1["elem_H"], c1["g"], m, n_c)
    rng = np.random.default_rng(4)
    x_c = rng.standard_normal((n_c, 3))
    r = galerkin.coarse_residual(c1["elem_verts"], c1["elem_H"], c1["g"], m, n_c, x_c)
    ref = b_c.reshape(-1) - a_c @ x_c.reshape(-1)
    assert np.allclose(r.reshape(-1), ref, rtol=0, atol=1e-9 * np.abs(a_c).max() * np.abs(x_c).max())
    h = galerkin.fine_hessian(c1["n_verts"], c1["elem_verts"], c1["elem_H"])
    xf = rng.standard_normal((c1["n_verts"], 3))
    assert np.allclose(galerkin.fine_matvec(c1["elem_verts"], c1["elem_H"], xf).reshape(-1), h @ xf.reshape(-1),
                       rtol=0, atol=1e-9 * np.abs(h).max() * np.abs(xf).max())


def test_all_collapsible_closed_form(c1):
    n = c1["n_verts"]
    m, n_c = aggregate.components(n, c1["edges"], np.ones_like(c1["tags"]))
    a_c, b_c = galerkin.coarse_system(n, c1["elem_verts"], c1["elem_H"], c1["g"], m, n_c)
    k = c1["elem_verts"].shape[0] * 144
    pins.check_all_collapsible_closed_form(a_c, b_c, c1["g"], synth.DENSITY, c1["h"], k,
                                           np.abs(c1["elem_H"]).sum() / 9)
    assert np.isclose(a_c[0, 0], 1e7, rtol=1e-9)


def test_identity_map_gives_fine_hessian(tiny):
    p = tiny
    n = p["n_verts"]
    m, n_c = aggregate.components(n, p["edges"], np.zeros_like(p["tags"]))
    a_c, b_c = galerkin.coarse_system(n, p["elem_verts"], p["elem_H"], p["g"], m, n_c)
    hd = galerkin.dense_fine_hessian(n, p["elem_verts"], p["elem_H"])
    assert np.allclose(a_c.toarray(), hd, rtol=0, atol=1e-9 * np.abs(hd).max())
    assert np.array_equal(b_c, p["g"])


# =============================================================== solve

def test_dense_solve_and_pcg(c1):
    r = method.coarsened_solve(c1, solver="dense")
    ad = r["A_c"].toarray()
    assert solve.relative_residual(r["A_c"], r["b_c"], r["x_c"]) < 1e-12
    x_p, its, rel = solve.pcg(r["A_c"], r["b_c"], 1e-13, 10000)
    assert rel <= 1e-13
    assert np.abs(x_p - r["x_c"]).max() <= 1e-8 * np.abs(r["x_c"]).max()
    assert np.array_equal(r["x"], r["x_c"][r["map"]])
    # x_c solves the Galerkin system: P^T H P x_c = P^T g, checked on the fine level
    h = galerkin.fine_hessian(c1["n_verts"], c1["elem_verts"], c1["elem_H"])
    res_c = galerkin.restrict(r["map"], r["n_c"], (h @ r["x"].reshape(-1)).reshape(-1, 3) - c1["g"])
    assert np.linalg.norm(res_c) <= 1e-11 * np.linalg.norm(r["b_c"])
    assert np.allclose(ad @ r["x_c"].reshape(-1), r["b_c"].reshape(-1), rtol=0, atol=1e-9 * np.abs(r["b_c"]).max())


def test_certified_bound_holds(c1):
    m, n_c = aggregate.components(c1["n_verts"], c1["edges"], c1["tags"])
    a_c, b_c = galerkin.coarse_system(c1["n_verts"], c1["elem_verts"], c1["elem_H"], c1["g"], m, n_c)
    x_star = solve.solve_dense(a_c.toarray(), b_c.reshape(-1))
    lam = solve.mass_lower_bound(m, n_c, c1["mass"], c1["h"])
    assert lam <= np.linalg.eigvalsh(a_c.toarray()).min() * (1 + 1e-12)
    seen = []

    def cb(it, x, r):
        err = np.linalg.norm(x - x_star)
        bound = np.linalg.norm(r) / lam
        seen.append((err, bound))
    solve.pcg(a_c, b_c, 1e-12, 1000, callback=cb)
    assert len(seen) > 3
    for err, bound in seen:
        assert err <= bound * (1 + 1e-6) + 1e-14


def test_all_collapsible_solution_closed_form(c1):
    t = np.ones_like(c1["tags"])
    r = method.coarsened_solve(c1, solver="dense", tags=t)
    expect = c1["g"].sum(axis=0) * c1["h"] ** 2 / synth.DENSITY
    assert np.allclose(r["x"], expect[None, :], rtol=1e-9, atol=0)


def test_no_collapsible_reduces_to_fine_solve(tiny):
    p = tiny
    hd = galerkin.dense_fine_hessian(p["n_verts"], p["elem_verts"], p["elem_H"])
    x_ref = np.linalg.solve(hd, p["g"].reshape(-1)).reshape(-1, 3)
    r = method.fine_solve(p, solver="dense")
    assert np.allclose(r["x"], x_ref, rtol=0, atol=1e-10 * np.abs(x_ref).max())


def test_pcg_block_diagonal_one_iteration():
    rng = np.random.default_rng(3)
    blocks = []
    for _ in range(10):
        q = rng.standard_normal((3, 3))
        blocks.append(q @ q.T + 3 * np.eye(3))
    a = sp.block_diag(blocks).tocsr()
    b = rng.standard_normal(30)
    x, its, rel = solve.pcg(a, b, 1e-14, 50)
    assert its == 1 and rel < 1e-13


def test_pcg_rejects_indefinite():
    a = sp.csr_matrix(np.diag([1.0, 1.0, -1.0]))
    with pytest.raises(np.linalg.LinAlgError):
        solve.pcg(a, np.ones(3), 1e-10, 10)


# =============================================================== adjoint

def _loss(p, g, elem_H, w, tags):
    m, n_c = aggregate.components(p["n_verts"], p["edges"], tags)
    a_c, b_c = galerkin.coarse_system(p["n_verts"], p["elem_verts"], elem_H, g, m, n_c)
    x_c = solve.solve_dense(a_c.toarray(), b_c.reshape(-1)).reshape(-1, 3)
    return float(np.sum(w * x_c[m]))


def test_adjoint_identities_and_fd(tiny):
    p = tiny
    rng = np.random.default_rng(9)
    w = rng.standard_normal((p["n_verts"], 3))
    m, n_c = aggregate.components(p["n_verts"], p["edges"], p["tags"])
    x, dg, dh = adjoint.adjoint(p["n_verts"], p["elem_verts"], p["elem_H"], p["g"], m, n_c, w, dense=True)
    L = float(np.sum(w * x))
    pins.check_adjoint_identities(L, p["g"], dg, p["elem_H"], dh)
    eps = 1e-6
    for _ in range(4):
        d = rng.standard_normal(p["g"].shape)
        d *= np.linalg.norm(p["g"]) / np.linalg.norm(d)
        fd = (_loss(p, p["g"] + eps * d, p["elem_H"], w, p["tags"])
              - _loss(p, p["g"] - eps * d, p["elem_H"], w, p["tags"])) / (2 * eps)
        an = float(np.sum(dg * d))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-12) + 1e-9 * abs(L)
    he = p["elem_H"].reshape(-1, 12, 12)
    for _ in range(4):
        d = rng.standard_normal(he.shape)
        d = 0.5 * (d + np.swapaxes(d, 1, 2))
        d *= (np.linalg.norm(he, axis=(1, 2)) / np.linalg.norm(d, axis=(1, 2)))[:, None, None]
        hp = (he + eps * d).reshape(-1, 144)
        hm = (he - eps * d).reshape(-1, 144)
        fd = (_loss(p, p["g"], hp, w, p["tags"]) - _loss(p, p["g"], hm, w, p["tags"])) / (2 * eps)
        an = float(np.sum(dh * d.reshape(-1, 144)))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-12) + 1e-9 * abs(L)


def test_adjoint_all_collapsible_closed_form(c1):
    rng = np.random.default_rng(1)
    w = rng.standard_normal((c1["n_verts"], 3))
    m, n_c = aggregate.components(c1["n_verts"], c1["edges"], np.ones_like(c1["tags"]))
    x, dg, dh = adjoint.adjoint(c1["n_verts"], c1["elem_verts"], c1["elem_H"], c1["g"], m, n_c, w, dense=True)
    expect = w.sum(axis=0) * c1["h"] ** 2 / synth.DENSITY
    assert np.allclose(dg, expect[None, :], rtol=1e-9, atol=0)


# ------------------------------------------------------- post-coarsening

def test_post_coarsen_is_cg_on_the_fine_system():
    """Pins of post_coarsen from what CG guarantees, not from its own loop:
    k = 0 returns x0; the H-norm error to the fine solution never grows; from
    the fine solution nothing moves; enough iterations reach the fine solution."""
    import scipy.sparse.linalg as spla
    from oracle import galerkin as _gal
    from oracle import method as _m
    p = synth.make_config("c1")
    co = _m.coarsened_solve(p, solver="sparse")
    h = _gal.fine_hessian(p["n_verts"], p["elem_verts"], p["elem_H"])
    x_star = spla.spsolve(h.tocsc(), p["g"].reshape(-1)).reshape(-1, 3)
    x0 = co["x"]
    x, its = _m.post_coarsen(p, x0, 0)
    assert its == 0 and np.array_equal(x, x0)

    def enorm(v):
        d = (v - x_star).reshape(-1)
        return float(np.sqrt(d @ (h @ d)))
    prev = enorm(x0)
    for k in (1, 2, 5, 10):
        x, its = _m.post_coarsen(p, x0, k)
        assert its == k
        e = enorm(x)
        assert e <= prev * (1 + 1e-12)
        prev = e
    assert prev < 0.5 * enorm(x0)                     # ten iterations do reduce the error
    x, _ = _m.post_coarsen(p, x_star, 3, rtol=1e-12)
    assert np.linalg.norm(x - x_star) <= 1e-9 * np.linalg.norm(x_star)
    x, its = _m.post_coarsen(p, x0, 2000, rtol=1e-13)
    assert np.linalg.norm(x - x_star) <= 1e-8 * np.linalg.norm(x_star)


# ------------------------------------------------------- affine embedding

def _affine_case(name="c1", threshold=32):
    from oracle import affine
    p = synth.make_config(name)
    m, n_c = aggregate.components(p["n_verts"], p["edges"], p["tags"])
    return p, m, n_c, affine.coarse_system(p, m, n_c, threshold)


def test_affine_reproduces_its_range():
    """Galerkin reproduction, independent of how P^T H P is formed: if the fine
    solution lies in range(P) (affine on every 12-DoF aggregate, constant on
    every other), the coarsened solve returns it exactly."""
    from oracle import affine
    p, m, n_c, (a_c, b_c, cls, pm) = _affine_case()
    assert cls["n12"] >= 1 and cls["n3"] >= 1
    rng = np.random.default_rng(3)
    y = rng.standard_normal(3 * cls["n_flat"])
    x_star = pm @ y
    h = galerkin.fine_hessian(p["n_verts"], p["elem_verts"], p["elem_H"])
    q = dict(p, g=(h @ x_star).reshape(-1, 3))
    a2, b2, _, pm2 = affine.coarse_system(q, m, n_c, 32)
    x_c = solve.solve_dense(a2.toarray(), b2.reshape(-1))
    x = affine.prolongate(pm2, x_c)
    assert np.linalg.norm(x.reshape(-1) - x_star) <= 1e-10 * np.linalg.norm(x_star)


def test_affine_moments_and_limits():
    """P^T P of a 12-DoF node is (sum_f Xbar_f Xbar_f^T) (x) I_3 (its rest moments);
    a threshold above every aggregate gives the plain 3-DoF system; the 12-DoF
    span contains the plain one (translations are the k = 3 block)."""
    from oracle import affine
    p, m, n_c, (a_c, b_c, cls, pm) = _affine_case()
    ptp = (pm.T @ pm).toarray()
    c = int(np.flatnonzero(cls["big"])[0])
    o = int(cls["offset"][c])
    mem = np.flatnonzero(m == c)
    xb = np.concatenate([p["pos"][mem] - p["pos"][mem.min()], np.ones((mem.size, 1))], axis=1)
    mom = xb.T @ xb
    blk = ptp[3 * o: 3 * o + 12, 3 * o: 3 * o + 12]
    assert np.allclose(blk, np.kron(mom, np.eye(3)), rtol=1e-13, atol=1e-13)
    a0, b0, cls0, _ = affine.coarse_system(p, m, n_c, 10 ** 9)
    assert cls0["n12"] == 0
    a_ref, b_ref = galerkin.coarse_system(p["n_verts"], p["elem_verts"], p["elem_H"], p["g"], m, n_c)
    assert abs(a0 - a_ref).max() <= 1e-9 * abs(a_ref).max() and np.allclose(b0, b_ref, rtol=1e-13, atol=1e-12)
    # energy: the affine-enriched solve lowers the quadratic model's minimum (a larger subspace)
    def energy(a, b):
        x = solve.solve_dense(a.toarray(), b.reshape(-1))
        return -0.5 * float(b.reshape(-1) @ x)
    assert energy(a_c, b_c) <= energy(a0, b0) + 1e-12 * abs(energy(a0, b0))
    # symmetric positive definite
    ev = np.linalg.eigvalsh(a_c.toarray())
    assert ev.min() > 0 and abs(a_c - a_c.T).max() <= 1e-9 * abs(a_c).max()


def test_affine_threshold_is_strict():
    """Only aggregates with MORE members than the threshold get 12 DoF (Eq. 4 text)."""
    from oracle import affine
    p = synth.make_config("c1")
    m, n_c = aggregate.components(p["n_verts"], p["edges"], p["tags"])
    big = int(np.bincount(m).max())
    assert affine.classify(m, n_c, big)["n12"] == 0
    assert affine.classify(m, n_c, big - 1)["n12"] >= 1


def test_affine_mutants_trip_the_pins():
    """Planted mistakes in a copy of the affine prolongation (the homogeneous
    coordinate in front; the translation block dropped) each break the moment pin."""
    from oracle import affine
    p = synth.make_config("c1")
    m, n_c = aggregate.components(p["n_verts"], p["edges"], p["tags"])
    cls = affine.classify(m, n_c, 32)
    c = int(np.flatnonzero(cls["big"])[0])
    o = int(cls["offset"][c])
    mem = np.flatnonzero(m == c)
    xb = np.concatenate([p["pos"][mem] - p["pos"][mem.min()], np.ones((mem.size, 1))], axis=1)
    want = np.kron(xb.T @ xb, np.eye(3))

    def moments_ok(pm):
        blk = (pm.T @ pm).toarray()[3 * o: 3 * o + 12, 3 * o: 3 * o + 12]
        return np.allclose(blk, want, rtol=1e-13, atol=1e-13)

    assert moments_ok(affine.prolongation(m, p["pos"], cls))
    good = affine.prolongation(m, p["pos"], cls).tocoo()
    rows, cols, vals = good.row, good.col, good.data.copy()
    # 1: (1, X, Y, Z) order: swap the weights of blocks k = 0 and k = 3
    blockk = (cols // 3 - cls["offset"][m[rows // 3]])
    in_big = cls["big"][m[rows // 3]]
    v1 = vals.copy()
    sel0, sel3 = in_big & (blockk == 0), in_big & (blockk == 3)
    v1[sel0], v1[sel3] = vals[sel3], vals[sel0]
    assert not moments_ok(sp.csr_matrix((v1, (rows, cols)), shape=good.shape))
    # 2: translation block dropped
    v2 = vals.copy()
    v2[sel3] = 0.0
    assert not moments_ok(sp.csr_matrix((v2, (rows, cols)), shape=good.shape))


def _interleaved_affine_map():
    """A hand-made map whose 12-DoF nodes (more than 4 members) sit at low,
    middle and high labels between 3-DoF nodes: sizes by label 6, 1, 2, 5, 1, 9, 3, 1, 7."""
    sizes = [6, 1, 2, 5, 1, 9, 3, 1, 7]
    return np.repeat(np.arange(len(sizes)), sizes).astype(np.int32), len(sizes), 4


def test_affine_node_order_follows_alg3():
    """The oracle's node classification and flat offsets equal those built from
    the supplement's Alg. 3 (sort keys i and i + n_c) and its row/column index
    formulas, on a map where 12-DoF nodes carry labels below 3-DoF ones, and
    on the 8^3 grid's map with thresholds that make one or several 12-DoF nodes."""
    from oracle import affine
    m, n_c, thr = _interleaved_affine_map()
    pins.check_affine_order(affine.classify, m, n_c, thr)
    cls = affine.classify(m, n_c, thr)
    # written out for this map: 3-DoF labels 1, 2, 4, 6, 7 -> 0..4; 12-DoF 0, 3, 5, 8 -> 5..8
    assert cls["new_label"].tolist() == [5, 0, 1, 6, 2, 7, 3, 4, 8]
    assert cls["offset"].tolist() == [5, 0, 1, 9, 2, 13, 3, 4, 17]
    p = synth.make_config("c1")
    mg, ncg = aggregate.components(p["n_verts"], p["edges"], p["tags"])
    for thr in (1, 3, 32):
        pins.check_affine_order(affine.classify, mg, ncg, thr)
