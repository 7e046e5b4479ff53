"""The certified error bound of agc_solve (info.err_bound, opts.target_err).

With H = M / h^2 + K (K positive semidefinite), d = m / h^2 is a lower
bound of H's diagonal, A_c = P^T H P >= diag(D_c) (x) I_3 with D_c the
aggregated d, and the error of x = P x_c against the exact coarsened solution
x* = P A_c^-1 P^T g is at most sqrt(sum_c |r_c|^2 / D_c / min d).

* The reported bound equals that formula evaluated with the oracle's own
  (matrix-free) residual of the returned iterate, and it bounds the true
  error against the oracle's direct solve (8^3, 32^3; coarsened and fine;
  FP64 and mixed).
* target_err: from a loose rtol the solve continues until the bound is at
  or below the target, and then the true error is too.
* Without diag_lb the bound is -1; target_err without diag_lb, a diag_lb
  entry that is not positive, and target_err with the affine embedding are
  rejected.
"""
import numpy as np
import pytest

from oracle import aggregate as oagg
from oracle import galerkin as ogal
from oracle import method
from tests.gpu_util import Dev, binding, log, problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    agc = binding()
    c = agc.Context(0)
    yield c
    c.close()


_devs, _refs = {}, {}


def dev(ctx, name):
    if name not in _devs:
        _devs[name] = Dev(ctx, problem(name))
    return _devs[name]


def reference(name, coarsen):
    """x* from the oracle's direct solve of its own coarse (or fine) system."""
    key = (name, coarsen)
    if key not in _refs:
        p = problem(name)
        r = method.coarsened_solve(p, solver="dense" if name == "c1" else "sparse") if coarsen else \
            method.fine_solve(p, solver="dense" if name == "c1" else "sparse")
        _refs[key] = (r["x"], r["map"], r["n_c"])
    return _refs[key]


def oracle_bound(p, m, nc, x):
    """The bound's formula with the oracle's matrix-free residual of x's coarse iterate (absolute)."""
    x_c = x[oagg.representatives(m, nc)]
    r_c = ogal.coarse_residual(p["elem_verts"], p["elem_H"], p["g"], m, nc, x_c)
    d = p["mass"] / p["h"] ** 2
    dc = np.bincount(m, weights=d, minlength=nc)
    return np.sqrt(np.sum(np.sum(r_c * r_c, axis=1) / dc) / d.min())


def solve(ctx, d, **kw):
    import torch
    agc = binding()
    p = d.p
    dlb = kw.pop("diag_lb", d.t(p["mass"] / p["h"] ** 2, torch.float64))
    prob = agc.make_problem(d.mesh, d.edges, d.tags, d.eh, d.g, d.rest, diag_lb=dlb)
    n = p["n_verts"]
    x = torch.empty((n, 3), dtype=torch.float64, device=ctx.device)
    mp = torch.empty(n, dtype=torch.int32, device=ctx.device)
    info = agc.agc_solve(ctx, prob, agc.make_opts(max_iter=50000, **kw), x, mp)
    return x.cpu().numpy(), mp.cpu().numpy(), info


@pytest.mark.parametrize("name", ["c1", "c4"])
@pytest.mark.parametrize("coarsen", [1, 0])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bound_formula_and_validity(ctx, name, coarsen, precision):
    agc = binding()
    d = dev(ctx, name)
    p = d.p
    x_ref, m_ref, nc_ref = reference(name, coarsen)
    prec = agc.AGC_PREC_MIXED if precision == "mixed" else agc.AGC_PREC_FP64
    for rtol in (1e-4, 1e-7):
        x, mp, info = solve(ctx, d, coarsen=coarsen, precision=prec, rtol=rtol)
        m, nc = (m_ref, nc_ref) if coarsen else (np.arange(p["n_verts"]), p["n_verts"])
        if coarsen:
            assert np.array_equal(mp, m_ref)
        true_err = np.linalg.norm(x - x_ref) / np.linalg.norm(x)
        ob = oracle_bound(p, m, nc, x) / np.linalg.norm(x)
        log(f"[cert] {name} coarsen={coarsen} {precision} rtol {rtol:g}: err_bound {info.err_bound:.3e} "
            f"oracle formula {ob:.3e} true error {true_err:.3e}")
        assert abs(info.err_bound - ob) <= 1e-4 * ob
        assert true_err <= info.err_bound * (1 + 1e-9)


@pytest.mark.parametrize("name", ["c1", "c4"])
@pytest.mark.parametrize("coarsen", [1, 0])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_target_err(ctx, name, coarsen, precision):
    agc = binding()
    d = dev(ctx, name)
    x_ref, _, _ = reference(name, coarsen)
    prec = agc.AGC_PREC_MIXED if precision == "mixed" else agc.AGC_PREC_FP64
    for target in (1e-5, 1e-9):
        x, _, info = solve(ctx, d, coarsen=coarsen, precision=prec, rtol=1e-2, target_err=target)
        true_err = np.linalg.norm(x - x_ref) / np.linalg.norm(x)
        log(f"[cert] {name} coarsen={coarsen} {precision} target {target:g}: err_bound {info.err_bound:.3e} "
            f"true {true_err:.3e} iters {info.pcg_iters} rel_res {info.rel_res:.2e}")
        assert info.err_bound <= target
        assert true_err <= target


def test_no_bound_and_bad_arguments(ctx):
    import torch
    agc = binding()
    d = dev(ctx, "c1")
    p = d.p
    prob = agc.make_problem(d.mesh, d.edges, d.tags, d.eh, d.g, d.rest)
    x = torch.empty((p["n_verts"], 3), dtype=torch.float64, device=ctx.device)
    info = agc.agc_solve(ctx, prob, agc.make_opts(rtol=1e-8), x)
    assert info.err_bound == -1.0
    with pytest.raises(agc.AgcError):
        agc.agc_solve(ctx, prob, agc.make_opts(rtol=1e-8, target_err=1e-6), x)
    bad = d.t(p["mass"] / p["h"] ** 2, torch.float64)
    bad[5] = 0.0
    with pytest.raises(agc.BadInput):
        solve(ctx, d, rtol=1e-8, diag_lb=bad)
    with pytest.raises(agc.AgcError):
        solve(ctx, d, rtol=1e-8, target_err=1e-6, affine_threshold=32)
