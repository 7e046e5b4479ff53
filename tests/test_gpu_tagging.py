"""GPU parity of agc_tagger_create / agc_tag_edges against the oracle (Sec. 4.2, Eq. 3).

Tags are bit-exact, except where floating point decides them at the
threshold: an element whose oracle norm lies within a relative 1e-9 of the
threshold may go either way (the two sides sum the nine squares in different
orders), so the edges of such elements are checked only for being 0 or 1.
None of the seeded workloads has such an element (the closest is 1.4e-6
away at 64^3), so in practice the comparison is exact."""
import numpy as np
import pytest

from oracle import tagging as otag
from paper_2605_04773_amd import synth
from tests.gpu_util import binding, log, problem

pytestmark = pytest.mark.gpu

THR = 5e-5


@pytest.fixture(scope="module")
def ctx():
    agc = binding()
    c = agc.Context(0)
    yield c
    c.close()


def _t(ctx, a, dt):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(ctx.device, dt)


def _gpu_tags(ctx, n, tets, rest, edges, x_cur, x_prev, thr):
    import torch
    agc = binding()
    tg = agc.agc_tagger_create(ctx, n, _t(ctx, tets, torch.int32), _t(ctx, rest, torch.float64),
                               _t(ctx, edges, torch.int32))
    tags, nprot = agc.agc_tag_edges(ctx, tg, _t(ctx, x_cur, torch.float64), _t(ctx, x_prev, torch.float64), thr)
    out = tags.cpu().numpy()
    tg.close()
    return out, nprot


def _compare(p, tets, x_cur, x_prev, got, thr=THR):
    ref, norms = otag.tag_edges(p["pos"], x_cur, x_prev, tets, p["edges"], thr)
    near = np.abs(norms - thr) <= 1e-9 * thr
    if near.any():
        hot = tets[near].astype(np.int64)
        n = p["n_verts"]
        pairs = np.concatenate([hot[:, [a, b]] for a in range(4) for b in range(a + 1, 4)], axis=0)
        amb = np.minimum(pairs[:, 0], pairs[:, 1]) * n + np.maximum(pairs[:, 0], pairs[:, 1])
        e = p["edges"].astype(np.int64)
        keys = np.minimum(e[:, 0], e[:, 1]) * n + np.maximum(e[:, 0], e[:, 1])
        free = ~np.isin(keys, amb)
    else:
        free = np.ones(ref.shape[0], bool)
    assert np.isin(got, [0, 1]).all()
    assert np.array_equal(got[free], ref[free])
    return ref


@pytest.mark.parametrize("name", ["c1", "c4", "c2", "c3"])
def test_tags_match_oracle(ctx, name):
    p = problem(name)
    log(f"[tag] {name}")
    tets = p["elem_verts"][: p.get("n_tets", p["elem_verts"].shape[0])]
    xp, xc = synth.deformation_states(p)
    got, nprot = _gpu_tags(ctx, p["n_verts"], tets, p["pos"], p["edges"], xc, xp, THR)
    _compare(p, tets, xc, xp, got)
    assert nprot == int((got == 0).sum())
    log(f"   protected {nprot} of {got.size} ({nprot / got.size:.3f})")
    assert 0 < nprot < got.size


def test_edge_rule_small_mesh(ctx):
    rest = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1], [5, 5, 5]], float)
    tets = np.array([[0, 1, 2, 3], [4, 1, 2, 3]], np.int32)
    x_prev = rest.copy()
    x_cur = rest.copy()
    x_cur[0] += [-0.01, 0.0, 0.0]
    edges = np.array([[1, 0], [0, 2], [3, 0], [1, 2], [2, 3], [1, 3], [4, 1], [4, 2], [4, 3],
                      [5, 0], [2, 2], [0, 1]], np.int32)
    got, nprot = _gpu_tags(ctx, 6, tets, rest, edges, x_cur, x_prev, 1e-4)
    assert got.tolist() == [0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 0] and nprot == 7
    got, nprot = _gpu_tags(ctx, 6, tets, rest, edges, x_cur, x_prev, 1.0)
    assert got.tolist() == [1] * 12 and nprot == 0


def test_rigid_motions_protect_nothing(ctx):
    p = problem("c4")
    rng = np.random.default_rng(7)
    r1, r2 = synth.random_rotations(rng, 2)
    x1 = p["pos"] @ r1.T + 0.3
    x2 = p["pos"] @ r2.T - 0.2
    got, nprot = _gpu_tags(ctx, p["n_verts"], p["elem_verts"], p["pos"], p["edges"], x2, x1, 1e-9)
    assert nprot == 0 and got.min() == 1


def test_tags_drive_the_map(ctx):
    """Tags from the tagger feed the aggregation: the map equals the oracle's
    components of the oracle's tags (the step before a1, then a1)."""
    import torch
    from oracle import aggregate as oagg
    agc = binding()
    p = problem("c4")
    xp, xc = synth.deformation_states(p)
    tg = agc.agc_tagger_create(ctx, p["n_verts"], _t(ctx, p["elem_verts"], torch.int32), _t(ctx, p["pos"], torch.float64),
                               _t(ctx, p["edges"], torch.int32))
    tags, _ = agc.agc_tag_edges(ctx, tg, _t(ctx, xc, torch.float64), _t(ctx, xp, torch.float64), THR, count=False)
    mp, nc = agc.agc_aggregate(ctx, p["n_verts"], _t(ctx, p["edges"], torch.int32), tags)
    ref_tags, _ = otag.tag_edges(p["pos"], xc, xp, p["elem_verts"], p["edges"], THR)
    m, nref = oagg.components(p["n_verts"], p["edges"], ref_tags)
    assert nc == nref and np.array_equal(mp.cpu().numpy(), m)
    # repeated calls: bitwise equal
    tags2, _ = agc.agc_tag_edges(ctx, tg, _t(ctx, xc, torch.float64), _t(ctx, xp, torch.float64), THR)
    assert torch.equal(tags, tags2)
    tg.close()


def test_bad_input(ctx):
    import torch
    agc = binding()
    rest = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0]], float)
    edges = np.array([[0, 1]], np.int32)
    flat = np.array([[0, 1, 2, 4]], np.int32)          # four coplanar rest points
    with pytest.raises(agc.BadInput):
        agc.agc_tagger_create(ctx, 5, _t(ctx, flat, torch.int32), _t(ctx, rest, torch.float64), _t(ctx, edges, torch.int32))
    rep = np.array([[0, 1, 1, 3]], np.int32)            # repeated vertex
    with pytest.raises(agc.BadInput):
        agc.agc_tagger_create(ctx, 5, _t(ctx, rep, torch.int32), _t(ctx, rest, torch.float64), _t(ctx, edges, torch.int32))
    good = np.array([[0, 1, 2, 3]], np.int32)
    far = np.array([[0, 9]], np.int32)                  # edge id out of range
    with pytest.raises(agc.BadInput):
        agc.agc_tagger_create(ctx, 5, _t(ctx, good, torch.int32), _t(ctx, rest, torch.float64), _t(ctx, far, torch.int32))
    # the context still works afterwards
    got, _ = _gpu_tags(ctx, 5, good, rest, edges, rest, rest, 0.0)
    assert got.tolist() == [1]
