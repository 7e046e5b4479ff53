"""GPU parity of the adjoint (agc_solve_backward / AgcSolve autograd) against
the oracle gradient, central finite differences and the exact identities
L = <dL/dg, g> and sum_e <dL/dH_e, H_e> = -L."""
import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import aggregate as oagg
from paper_2605_04773_amd import synth
from tests.gpu_util import Dev, binding, log, problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    agc = binding()
    c = agc.Context(0)
    yield c
    c.close()


def _forward_backward(ctx, d, w, opts, g=None, eh=None):
    import torch
    agc = binding()
    g = d.g if g is None else g
    eh = d.eh if eh is None else eh
    gg = g.clone().requires_grad_(True)
    hh = eh.clone().requires_grad_(True)
    x = agc.AgcSolve.apply(gg, hh, d.mesh, d.edges, d.tags, opts)
    L = (x * w).sum()
    L.backward()
    torch.cuda.synchronize()
    return x.detach(), float(L), gg.grad, hh.grad


@pytest.mark.parametrize("name", ["tiny", "c1", "c4"])
def test_gradient_matches_oracle(ctx, name):
    import torch
    agc = binding()
    p = problem(name)
    d = Dev(ctx, p)
    w_np = synth.adjoint_seed(p)
    w = torch.from_numpy(w_np).to(ctx.device)
    log(f"[adj] {name}")
    x, L, dg, dh = _forward_backward(ctx, d, w, agc.make_opts(rtol=1e-12, max_iter=20000))
    m, nc = oagg.components(p["n_verts"], p["edges"], p["tags"])
    xr, dgr, dhr = oadj.adjoint(p["n_verts"], p["elem_verts"], p["elem_H"], p["g"], m, nc, w_np,
                                dense=p["n_verts"] < 1000)
    dg, dh = dg.cpu().numpy(), dh.cpu().numpy()
    assert np.linalg.norm(dg - dgr) <= 1e-6 * np.linalg.norm(dgr)
    assert np.linalg.norm(dh - dhr) <= 1e-6 * np.linalg.norm(dhr)
    # exact identities, with the GPU's own forward value of L
    lin = float(np.sum(dg * p["g"]))
    euler = float(np.sum(dh * p["elem_H"]))
    assert abs(lin - L) <= 1e-8 * abs(L) + 1e-12 * np.abs(dg * p["g"]).sum()
    assert abs(euler + L) <= 1e-8 * abs(L) + 1e-12 * np.abs(dh * p["elem_H"]).sum()


def test_gradient_mixed_precision(ctx):
    import torch
    agc = binding()
    p = problem("c4")
    d = Dev(ctx, p)
    w_np = synth.adjoint_seed(p)
    w = torch.from_numpy(w_np).to(ctx.device)
    x, L, dg, dh = _forward_backward(ctx, d, w, agc.make_opts(precision=agc.AGC_PREC_MIXED, rtol=1e-8))
    m, nc = oagg.components(p["n_verts"], p["edges"], p["tags"])
    _, dgr, dhr = oadj.adjoint(p["n_verts"], p["elem_verts"], p["elem_H"], p["g"], m, nc, w_np)
    assert np.linalg.norm(dg.cpu().numpy() - dgr) <= 1e-5 * np.linalg.norm(dgr)
    assert np.linalg.norm(dh.cpu().numpy() - dhr) <= 1e-5 * np.linalg.norm(dhr)


def test_central_differences(ctx):
    """Central differences of the GPU forward at the 32^3 grid (eps = 1e-6,
    relative): 16 random directions of g (||d|| = ||g||) and 16 random
    symmetric element perturbations (||D_e||_F = ||H_e||_F per element).
    Every +/- solve runs the same fixed number of PCG iterations (the count
    that reaches rtol 1e-13 on the unperturbed system; the library is asked
    for an unreachable 1e-16 and stops at max_iter), so the differences are
    not polluted by differing stop points."""
    import torch
    agc = binding()
    p = problem("c4")
    d = Dev(ctx, p)
    rng = np.random.default_rng(4)
    w = torch.from_numpy(synth.adjoint_seed(p)).to(ctx.device)
    x, L, dg, dh = _forward_backward(ctx, d, w, agc.make_opts(rtol=1e-13, max_iter=20000))
    probe = agc.agc_solve(ctx, d.problem(), agc.make_opts(rtol=1e-13, max_iter=20000), torch.empty_like(d.g))
    fixed = agc.make_opts(rtol=1e-16, max_iter=probe.pcg_iters)
    log(f"[fd] 32^3: {probe.pcg_iters} PCG iterations per solve, L = {L:.6e}")

    def loss(g, eh):
        xx = torch.empty_like(g)
        prob = agc.make_problem(d.mesh, d.edges, d.tags, eh, g)
        info = agc.agc_solve(ctx, prob, fixed, xx, raise_on_not_converged=False)
        assert info.pcg_iters == probe.pcg_iters
        return float((xx * w).sum())

    eps = 1e-6
    worst = 0.0
    for _ in range(16):
        dd = rng.standard_normal(p["g"].shape)
        dd *= np.linalg.norm(p["g"]) / np.linalg.norm(dd)
        dt = torch.from_numpy(dd).to(ctx.device)
        fd = (loss(d.g + eps * dt, d.eh) - loss(d.g - eps * dt, d.eh)) / (2 * eps)
        an = float((dg * dt).sum())
        worst = max(worst, abs(fd - an) / (abs(an) + 1e-300))
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-8 * abs(L)
    he = p["elem_H"].reshape(-1, 12, 12)
    hn = np.linalg.norm(he, axis=(1, 2))
    for _ in range(16):
        dd = rng.standard_normal(he.shape)
        dd = 0.5 * (dd + np.swapaxes(dd, 1, 2))
        dd *= (hn / np.linalg.norm(dd, axis=(1, 2)))[:, None, None]
        dt = torch.from_numpy(dd.reshape(-1, 144)).to(ctx.device)
        del dd
        fd = (loss(d.g, d.eh + eps * dt) - loss(d.g, d.eh - eps * dt)) / (2 * eps)
        an = float((dh * dt).sum())
        worst = max(worst, abs(fd - an) / (abs(an) + 1e-300))
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-8 * abs(L)
    log(f"   worst relative FD mismatch over 32 directions: {worst:.2e}")


def test_backward_keeps_only_the_map(ctx):
    import torch
    agc = binding()
    p = problem("tiny")
    d = Dev(ctx, p)
    g = d.g.clone().requires_grad_(True)
    x = agc.AgcSolve.apply(g, d.eh, d.mesh, d.edges, d.tags, agc.make_opts(rtol=1e-12))
    saved = x.grad_fn.saved_tensors
    shapes = sorted(tuple(t.shape) for t in saved)
    # g, elem_H, map and x: no coarse matrix is kept
    assert shapes == sorted([tuple(d.g.shape), tuple(d.eh.shape), (p["n_verts"],), tuple(d.g.shape)])
    assert any(t.dtype == torch.int32 for t in saved)
