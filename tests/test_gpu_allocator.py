"""agc_set_allocator: a context whose device buffers come from torch's caching
allocator gives bitwise the results of one using hipMalloc, returns every
block it took, and reports an allocator that gives no memory."""
import pytest

from tests.gpu_util import Dev, binding, log, problem

pytestmark = pytest.mark.gpu


def _solve(ctx, d):
    import torch
    agc = binding()
    x = torch.empty((d.p["n_verts"], 3), dtype=torch.float64, device=ctx.device)
    mp = torch.empty(d.p["n_verts"], dtype=torch.int32, device=ctx.device)
    info = agc.agc_solve(ctx, d.problem(), agc.make_opts(precision=agc.AGC_PREC_MIXED, rtol=1e-7, post_iters=3),
                         x, mp)
    torch.cuda.synchronize()
    return x, mp, info


def test_torch_allocator_same_results():
    import torch
    agc = binding()
    p = problem("c4")
    ref_ctx = agc.Context(0)
    d_ref = Dev(ref_ctx, p)
    x_ref, m_ref, _ = _solve(ref_ctx, d_ref)
    ctx = agc.Context(0)
    stats = ctx.use_torch_allocator()
    before = torch.cuda.memory_allocated()
    d = Dev(ctx, p)
    x, m, info = _solve(ctx, d)
    x2, _, _ = _solve(ctx, d)        # a second call reuses the workspace
    log(f"[alloc] {stats['alloc']} blocks, {stats['bytes'] / 2**20:.1f} MiB through torch; "
        f"torch holds {(torch.cuda.memory_allocated() - before) / 2**20:.1f} MiB more")
    assert stats["alloc"] > 0 and torch.cuda.memory_allocated() > before
    assert torch.equal(x, x_ref) and torch.equal(m, m_ref) and torch.equal(x2, x)
    d.mesh.close()
    ctx.close()
    assert stats["free"] == stats["alloc"]
    d_ref.mesh.close()
    ref_ctx.close()


def test_allocator_errors():
    import torch
    agc = binding()
    ctx = agc.Context(0)
    alloc_only = agc.ALLOC_FN(lambda n, u: None)
    st = agc._lib.agc_set_allocator(ctx.h, alloc_only, agc.FREE_FN(), None)
    assert st == agc.AGC_ERR_INVALID_ARG
    # an allocator that gives nothing: the call fails with AGC_ERR_OUT_OF_MEMORY ...
    nothing = (agc.ALLOC_FN(lambda n, u: None), agc.FREE_FN(lambda ptr, u: None))
    assert agc._lib.agc_set_allocator(ctx.h, nothing[0], nothing[1], None) == agc.AGC_OK
    p = problem("tiny")
    ev = torch.from_numpy(p["elem_verts"]).to(ctx.device, torch.int32)
    with pytest.raises(agc.AgcError) as ei:
        agc.agc_mesh_create(ctx, p["n_verts"], ev)
    assert ei.value.code == agc.AGC_ERR_OUT_OF_MEMORY
    # ... and with hipMalloc restored the context works
    assert agc._lib.agc_set_allocator(ctx.h, agc.ALLOC_FN(), agc.FREE_FN(), None) == agc.AGC_OK
    mesh = agc.agc_mesh_create(ctx, p["n_verts"], ev)
    mesh.close()
    ctx.close()
