"""GPU parity of agc_aggregate, agc_prolongate and agc_restrict against the oracle.

The map is integer work: it must match the oracle bit for bit."""
import numpy as np
import pytest

from oracle import aggregate as oagg
from oracle import galerkin as ogal
from paper_2605_04773_amd import synth
from tests.gpu_util import Dev, binding, gamma, log, problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    agc = binding()
    c = agc.Context(0)
    yield c
    c.close()


def _agg(ctx, n, edges, tags):
    import torch
    agc = binding()
    e = torch.from_numpy(np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)).to(ctx.device)
    t = torch.from_numpy(np.ascontiguousarray(tags, dtype=np.uint8).reshape(-1)).to(ctx.device)
    m, nc = agc.agc_aggregate(ctx, n, e, t)
    return m.cpu().numpy(), nc


@pytest.mark.parametrize("name", ["c1", "c4", "c3"])
def test_map_bit_exact(ctx, name):
    p = problem(name)
    log(f"[agg] {name}")
    m, nc = _agg(ctx, p["n_verts"], p["edges"], p["tags"])
    ref, nref = oagg.components(p["n_verts"], p["edges"], p["tags"])
    assert nc == nref
    assert np.array_equal(m, ref)


def test_map_full_size_c2(ctx):
    p = problem("c2")
    log("[agg] c2 full size")
    m, nc = _agg(ctx, p["n_verts"], p["edges"], p["tags"])
    ref, nref = oagg.components(p["n_verts"], p["edges"], p["tags"])
    assert nc == nref and np.array_equal(m, ref)


def _graphs():
    rng = np.random.default_rng(123)
    out = []
    for n, m in [(1, 0), (1, 3), (2, 1), (5, 0), (17, 40), (300, 200), (300, 900), (5000, 20000), (70000, 70000)]:
        e, t = synth.random_graph(rng, n, m, p_tag=rng.uniform(0.2, 0.9))
        out.append((f"rand{n}_{m}", n, e, t))
    n = 100_000            # a path written from the largest id down: long hook chains
    e = np.stack([np.arange(n - 1, 0, -1), np.arange(n - 2, -1, -1)], 1)
    out.append(("path_desc", n, e, np.ones(n - 1, np.uint8)))
    e = np.stack([np.zeros(n - 1, np.int64), np.arange(1, n)], 1)   # star around vertex 0
    out.append(("star", n, e, np.ones(n - 1, np.uint8)))
    e = np.stack([np.arange(n - 1), np.arange(1, n)], 1)            # path with every 7th edge protected
    out.append(("path_cut", n, e, (np.arange(n - 1) % 7 != 0).astype(np.uint8)))
    out.append(("dups_loops", 10, np.array([[1, 1], [2, 3], [3, 2], [2, 3], [9, 9], [0, 9]]),
                np.array([1, 1, 1, 0, 1, 1], np.uint8)))
    # the labelling sums the roots per tile of 4096 vertices; up to 4096 tiles
    # each workgroup sums the tiles before in LDS, beyond that one scan runs
    # first: the largest size of the one and the smallest of the other
    for n in (4096 * 4096, 4096 * 4096 + 1):
        e, t = synth.random_graph(rng, n, 2_000_000, p_tag=0.7)
        out.append((f"rand{n}_tiles", n, e, t))
    return out


@pytest.mark.parametrize("case", _graphs(), ids=lambda c: c[0])
def test_map_graphs(ctx, case):
    name, n, e, t = case
    log(f"[agg] graph {name}")
    m, nc = _agg(ctx, n, e, t)
    ref, nref = oagg.components(n, e, t)
    assert nc == nref and np.array_equal(m, ref)


@pytest.mark.parametrize("order", ["shuffled", "descending"])
def test_map_grid_edge_order(ctx, order):
    """The 32^3 grid's edges out of the sorted order the block pass reads as
    ranges: shuffled with half the pairs reversed, and sorted by smaller end
    descending; the map must not change."""
    p = problem("c4")
    rng = np.random.default_rng(11)
    if order == "shuffled":
        perm = rng.permutation(p["edges"].shape[0])
        e = p["edges"][perm].copy()
        flip = rng.random(e.shape[0]) < 0.5
        e[flip] = e[flip][:, ::-1]
    else:
        perm = np.argsort(-p["edges"].min(axis=1), kind="stable")
        e = p["edges"][perm]
    t = p["tags"][perm]
    log(f"[agg] c4 edges {order}")
    m, nc = _agg(ctx, p["n_verts"], e, t)
    ref, nref = oagg.components(p["n_verts"], p["edges"], p["tags"])
    assert nc == nref and np.array_equal(m, ref)


def test_map_all_or_nothing(ctx):
    p = problem("c4")
    m, nc = _agg(ctx, p["n_verts"], p["edges"], np.zeros_like(p["tags"]))
    assert nc == p["n_verts"] and np.array_equal(m, np.arange(p["n_verts"]))
    m, nc = _agg(ctx, p["n_verts"], p["edges"], np.ones_like(p["tags"]))
    assert nc == 1 and not m.any()            # every fine node maps to coarse node 0
    m, nc = _agg(ctx, 7, np.zeros((0, 2)), np.zeros(0))
    assert nc == 7 and np.array_equal(m, np.arange(7))


def test_map_deterministic(ctx):
    p = problem("c4")
    a, _ = _agg(ctx, p["n_verts"], p["edges"], p["tags"])
    for _ in range(3):
        b, _ = _agg(ctx, p["n_verts"], p["edges"], p["tags"])
        assert np.array_equal(a, b)


def test_bad_input(ctx):
    agc = binding()
    with pytest.raises(agc.BadInput):
        _agg(ctx, 4, np.array([[0, 1], [2, 3]]), np.array([1, 2]))
    with pytest.raises(agc.BadInput):
        _agg(ctx, 4, np.array([[0, 1], [2, 4]]), np.array([1, 0]))
    with pytest.raises(agc.BadInput):
        _agg(ctx, 4, np.array([[-1, 1]]), np.array([0]))


def test_prolongate_bit_exact(ctx):
    import torch
    agc = binding()
    p = problem("c4")
    ref, nref = oagg.components(p["n_verts"], p["edges"], p["tags"])
    rng = np.random.default_rng(5)
    x_c = rng.standard_normal((nref, 3))
    mp = torch.from_numpy(ref).to(ctx.device)
    x = agc.agc_prolongate(ctx, mp, nref, torch.from_numpy(x_c).to(ctx.device))
    assert np.array_equal(x.cpu().numpy(), ogal.prolongate(ref, x_c))
    bad = mp.clone()
    bad[3] = nref
    with pytest.raises(agc.BadInput):
        agc.agc_prolongate(ctx, bad, nref, torch.from_numpy(x_c).to(ctx.device))


@pytest.mark.parametrize("name", ["c1", "c4", "c2"])
def test_restrict_within_summation_bound(ctx, name):
    import torch
    agc = binding()
    p = problem(name)
    ref, nref = oagg.components(p["n_verts"], p["edges"], p["tags"])
    v = p["g"]
    out = agc.agc_restrict(ctx, torch.from_numpy(ref).to(ctx.device), nref,
                           torch.from_numpy(v).to(ctx.device)).cpu().numpy()
    exact = ogal.restrict(ref, nref, v)
    sizes = np.bincount(ref, minlength=nref)
    absum = ogal.restrict(ref, nref, np.abs(v))
    bound = gamma(2 * sizes.max()) * absum
    assert (np.abs(out - exact) <= bound + 1e-300).all()


def test_restrict_deterministic(ctx):
    import torch
    agc = binding()
    p = problem("c2")
    ref, nref = oagg.components(p["n_verts"], p["edges"], p["tags"])
    mp = torch.from_numpy(ref).to(ctx.device)
    v = torch.from_numpy(p["g"]).to(ctx.device)
    a = agc.agc_restrict(ctx, mp, nref, v)
    b = agc.agc_restrict(ctx, mp, nref, v)
    assert torch.equal(a, b)


def test_restrict_rejects_unused_label(ctx):
    """A map that leaves a label in [0, n_coarse) without members is rejected
    (BAD_INPUT), by agc_restrict and by agc_assemble_coarse's g_c, rather than
    shifting the sums of every later label; a map that uses every label passes."""
    import torch
    agc = binding()
    p = problem("c1")
    ref, nref = oagg.components(p["n_verts"], p["edges"], p["tags"])
    v = torch.from_numpy(p["g"]).to(ctx.device)
    gap = ref.astype(np.int64)
    gap[gap >= 5] += 1                       # label 5 unused, n_coarse one larger
    mp = torch.from_numpy(gap.astype(np.int32)).to(ctx.device)
    with pytest.raises(agc.BadInput):
        agc.agc_restrict(ctx, mp, nref + 1, v)
    short = ref.astype(np.int32)              # n_coarse one too large: the last label unused
    with pytest.raises(agc.BadInput):
        agc.agc_restrict(ctx, torch.from_numpy(short).to(ctx.device), nref + 1, v)
    d = Dev(ctx, p)
    with pytest.raises(agc.AgcError):
        agc.agc_assemble_coarse(ctx, d.mesh, d.eh, d.g, mp, nref + 1)
    out = agc.agc_restrict(ctx, torch.from_numpy(ref).to(ctx.device), nref, v)
    assert np.allclose(out.cpu().numpy(), ogal.restrict(ref, nref, p["g"]), rtol=1e-12, atol=1e-12)
