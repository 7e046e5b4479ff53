"""Pins of the Green-strain-increment tagging oracle (Sec. 4.2, Eq. 3), CPU only.

What fixes the oracle, independently of its own code:
* closed forms: an affine map x = A X + b has F = A on every element; a
  uniform stretch s has G = (s^2 - 1)/2 I, so two stretches differ by
  ||dG||_F = sqrt(3)/2 |s2^2 - s1^2|; a simple shear of amount k has
  ||G||_F = sqrt(2 k^2 + k^4) / 2 (and G is F^T F based, not F F^T: a shear
  with a rotation on the left leaves G unchanged);
* invariance: rigid motions of either state change no norm;
* the edge rule on hand-made meshes: the six edges of a hot element are
  protected, an edge shared with a cold element too, edges in no element and
  self-loops stay collapsible, duplicates agree;
* threshold monotonicity.
Planted mistakes (bottom) each trip one of these pins.
"""
import math

import numpy as np

from oracle import tagging
from paper_2605_04773_amd import synth


def _rot(rng):
    return synth.random_rotations(rng, 1)[0]


def _grid(n=3):
    pos, tets = synth.box_mesh(n, n, n, 1.0 / n)
    return pos, tets, synth.mesh_edges(tets, pos.shape[0])


# ----------------------------------------------------------------- pins

def check_affine_gradient(deformation_gradients):
    rng = np.random.default_rng(1)
    pos, tets, _ = _grid()
    a = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    x = pos @ a.T + rng.standard_normal(3)
    f = deformation_gradients(pos, x, tets)
    assert np.allclose(f, a[None], atol=1e-12), "F of an affine map must be its matrix"


def check_stretch_and_shear(strain_increment_norms):
    pos, tets, _ = _grid()
    s1, s2 = 1.01, 0.97
    got = strain_increment_norms(pos, s2 * pos, s1 * pos, tets)
    assert np.allclose(got, math.sqrt(3) / 2 * abs(s2 * s2 - s1 * s1), rtol=1e-11, atol=0)
    k = 0.02
    sh = pos.copy()
    sh[:, 0] += k * pos[:, 1]
    got = strain_increment_norms(pos, sh, pos, tets)       # previous state: the rest shape, G = 0
    assert np.allclose(got, 0.5 * math.sqrt(2 * k * k + k ** 4), rtol=1e-11, atol=0)
    # a rotation applied after the shear is a rigid motion: G, and every norm, unchanged
    rng = np.random.default_rng(5)
    r = _rot(rng)
    got_r = strain_increment_norms(pos, sh @ r.T, pos, tets)
    assert np.allclose(got_r, got, rtol=1e-10, atol=1e-15)
    # the same sheared shape under two different rotations: no strain increment
    # (G = (F^T F - I)/2 is blind to the rotation; F F^T is not)
    got_rr = strain_increment_norms(pos, sh @ _rot(rng).T, sh @ r.T, tets)
    assert np.max(got_rr) < 1e-13


def check_rigid_invariance(strain_increment_norms):
    rng = np.random.default_rng(2)
    pos, tets, _ = _grid()
    x1 = pos @ _rot(rng).T + rng.standard_normal(3)
    x2 = pos @ _rot(rng).T + rng.standard_normal(3)
    assert np.max(strain_increment_norms(pos, x2, x1, tets)) < 1e-13


def check_edge_rule(tag_edges):
    # two tets sharing the face (1, 2, 3); tet 0 = (0,1,2,3) deforms, tet 1 = (4,1,2,3) does not
    rest = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1], [5, 5, 5]], float)
    tets = np.array([[0, 1, 2, 3], [4, 1, 2, 3]], np.int32)
    x_prev = rest.copy()
    x_cur = rest.copy()
    x_cur[0] += [-0.01, 0.0, 0.0]            # moves vertex 0 only: only tet 0 strains
    edges = np.array([[1, 0], [0, 2], [3, 0], [1, 2], [2, 3], [1, 3], [4, 1], [4, 2], [4, 3],
                      [5, 0], [2, 2], [0, 1]], np.int32)
    tags, norms = tag_edges(rest, x_cur, x_prev, tets, edges, 1e-4)
    assert norms[0] > 1e-3 and norms[1] < 1e-14
    # tet 0's six edges (also the three it shares with tet 1) protected; tet 1's own
    # three edges, an edge in no element and a self-loop stay collapsible; the
    # duplicate (0, 1) agrees with (1, 0)
    assert tags.tolist() == [0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 0]
    # threshold above the norm: nothing protected
    tags, _ = tag_edges(rest, x_cur, x_prev, tets, edges, 2 * norms[0])
    assert tags.tolist() == [1] * len(edges)


def check_monotone(tag_edges):
    p = synth.make_config("c1")
    xp, xc = synth.deformation_states(p)
    prev = None
    for thr in (1e-6, 1e-5, 5e-5, 2e-4, 1e-3):
        tags, _ = tag_edges(p["pos"], xc, xp, p["elem_verts"], p["edges"], thr)
        if prev is not None:
            assert np.all(tags >= prev), "a larger threshold may only free edges"
        prev = tags


def test_affine_gradient():
    check_affine_gradient(tagging.deformation_gradients)


def test_stretch_and_shear():
    check_stretch_and_shear(tagging.strain_increment_norms)


def test_rigid_invariance():
    check_rigid_invariance(tagging.strain_increment_norms)


def test_edge_rule():
    check_edge_rule(tagging.tag_edges)


def test_monotone():
    check_monotone(tagging.tag_edges)


def test_synthetic_states_have_a_hot_region():
    """The generated iterates protect a minority of the edges and free the rest."""
    p = synth.make_config("c1")
    xp, xc = synth.deformation_states(p)
    tags, norms = tagging.tag_edges(p["pos"], xc, xp, p["elem_verts"], p["edges"], 5e-5)
    assert 0.02 < 1 - tags.mean() < 0.5
    assert norms.max() > 10 * 5e-5 and np.median(norms) < 5e-5


# -------------------------------------------------------------- mutants

def _fails(fn, *a):
    try:
        fn(*a)
    except AssertionError:
        return True
    return False


def _ds_dm(rest, x, tets):
    t = tets.astype(np.int64)
    dm = np.stack([rest[t[:, k]] - rest[t[:, 0]] for k in (1, 2, 3)], axis=-1)
    ds = np.stack([x[t[:, k]] - x[t[:, 0]] for k in (1, 2, 3)], axis=-1)
    return ds, dm


def _norms_from(grad_fn, strain_fn):
    def norms(rest, x_cur, x_prev, tets):
        d = strain_fn(grad_fn(rest, x_cur, tets)) - strain_fn(grad_fn(rest, x_prev, tets))
        return np.sqrt(np.sum(d * d, axis=(1, 2)))
    return norms


def test_mutant_gradient_operands_swapped():
    def grad(rest, x, tets):
        ds, dm = _ds_dm(rest, x, tets)
        return np.linalg.inv(dm) @ ds                      # Dm^-1 Ds instead of Ds Dm^-1
    assert _fails(check_affine_gradient, grad)


def test_mutant_gradient_rest_as_deformed():
    def grad(rest, x, tets):
        ds, dm = _ds_dm(rest, x, tets)
        return dm @ np.linalg.inv(ds)                      # inverse map
    assert _fails(check_affine_gradient, grad)


def test_mutant_strain_without_half():
    norms = _norms_from(tagging.deformation_gradients,
                        lambda f: np.swapaxes(f, -1, -2) @ f - np.eye(3))
    assert _fails(check_stretch_and_shear, norms)


def test_mutant_left_cauchy_green():
    norms = _norms_from(tagging.deformation_gradients,
                        lambda f: 0.5 * (f @ np.swapaxes(f, -1, -2) - np.eye(3)))   # F F^T
    assert _fails(check_stretch_and_shear, norms)


def test_mutant_small_strain():
    norms = _norms_from(tagging.deformation_gradients,
                        lambda f: 0.5 * (f + np.swapaxes(f, -1, -2)) - np.eye(3))   # linearised: not rotation invariant
    assert _fails(check_rigid_invariance, norms)


def test_mutant_protects_first_edge_only():
    def tag(rest, x_cur, x_prev, tets, edges, thr):
        norms = tagging.strain_increment_norms(rest, x_cur, x_prev, tets)
        hot = tets[norms > thr]
        prot = {(min(a, b), max(a, b)) for a, b in hot[:, :2].tolist()}
        tags = np.array([0 if (min(u, v), max(u, v)) in prot else 1 for u, v in edges.tolist()], np.uint8)
        return tags, norms
    assert _fails(check_edge_rule, tag)


def test_mutant_every_element_vote():
    """Protect only edges whose elements are all hot (an 'all' instead of an 'any')."""
    def tag(rest, x_cur, x_prev, tets, edges, thr):
        norms = tagging.strain_increment_norms(rest, x_cur, x_prev, tets)
        n = rest.shape[0]
        cold = tets[norms <= thr].astype(np.int64)
        pairs = np.concatenate([cold[:, [a, b]] for a in range(4) for b in range(a + 1, 4)], axis=0)
        free = set((np.minimum(pairs[:, 0], pairs[:, 1]) * n + np.maximum(pairs[:, 0], pairs[:, 1])).tolist())
        tags0, _ = tagging.tag_edges(rest, x_cur, x_prev, tets, edges, thr)
        keys = np.minimum(edges[:, 0], edges[:, 1]).astype(np.int64) * n + np.maximum(edges[:, 0], edges[:, 1])
        tags = np.array([1 if (k in free or t == 1) else 0 for k, t in zip(keys.tolist(), tags0.tolist())], np.uint8)
        return tags, norms
    assert _fails(check_edge_rule, tag)


def test_mutant_threshold_reversed():
    def tag(rest, x_cur, x_prev, tets, edges, thr):
        t, norms = tagging.tag_edges(rest, x_cur, x_prev, tets, edges, thr)
        return (1 - t).astype(np.uint8), norms
    assert _fails(check_edge_rule, tag)
