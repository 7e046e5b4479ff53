"""agc_aggregate_noalloc (the aggregation whose scratch is the library's
fixed device array) against agc_aggregate, bit for bit, on two calls in a
row, the second with a smaller input; with the torch allocator routed
through the context, the call requests no device memory."""
import numpy as np
import pytest

from oracle import aggregate as oagg
from paper_2605_04773_amd import synth
from tests.gpu_util import binding, log, problem

pytestmark = pytest.mark.gpu


def _graph(seed, n, m):
    rng = np.random.default_rng(seed)
    edges, tags = synth.random_graph(rng, n, m, p_tag=0.6)
    return n, edges, tags


def test_noalloc_matches_aggregate_twice():
    import torch
    agc = binding()
    ctx = agc.Context(0)
    stats = ctx.use_torch_allocator()
    dev = ctx.device
    p = problem("c4")
    cases = [("32^3 grid", p["n_verts"], p["edges"], p["tags"]), ("random multigraph",) + _graph(7, 5000, 12000)]
    for name, n, e_np, t_np in cases:
        log(f"[noalloc] {name}: {n} vertices, {e_np.shape[0]} edges")
        edges = torch.from_numpy(np.ascontiguousarray(e_np)).to(dev, torch.int32)
        tags = torch.from_numpy(np.ascontiguousarray(t_np)).to(dev, torch.uint8)
        ref, nref = agc.agc_aggregate(ctx, n, edges, tags)
        out = torch.full((n,), -7, dtype=torch.int32, device=dev)
        before = dict(stats)
        out, nc = agc.agc_aggregate_noalloc(ctx, n, edges, tags, out)
        torch.cuda.synchronize()
        assert stats == before, "agc_aggregate_noalloc requested device memory"
        assert nc == nref
        assert torch.equal(out, ref)
        m_orc, n_orc = oagg.components(n, e_np, t_np)
        assert nc == n_orc and np.array_equal(out.cpu().numpy(), m_orc)
    ctx.close()


def test_noalloc_rejects_oversize():
    import torch
    agc = binding()
    ctx = agc.Context(0)
    e = torch.zeros((1, 2), dtype=torch.int32, device=ctx.device)
    t = torch.zeros(1, dtype=torch.uint8, device=ctx.device)
    n = (1 << 22) + 1
    mp = torch.empty(n, dtype=torch.int32, device=ctx.device)
    with pytest.raises(agc.AgcError, match="4194304"):
        agc.agc_aggregate_noalloc(ctx, n, e, t, mp)
    ctx.close()
