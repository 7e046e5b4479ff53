"""Contact elements given per call (agc_problem.contact_*) instead of in the
mesh's static plan: the paper finds contact stencils anew every Newton
iteration and adds their Hessian blocks to the fine system before
coarsening (Sec. 3; Alg. overview).

Rows of deformable cuboids with point-triangle barrier blocks between
neighbours (the contact workload's recipe at two small sizes): the mesh holds
the tetrahedra only and the contact elements come with the problem.  The map
is bit-exact against the oracle's components; the FP64 solutions (coarsened,
and fine with coarsen = 0) match the oracle's direct solve of the system
with every element; the mixed solution is within 1e-5; the solution equals
the one with the contacts in the static plan to rounding; post-coarsening
iterates on the fine system with the contacts; the adjoint gives dL/dH for
the contacts after the tets'; the affine embedding takes them; the certified
bound holds; malformed contacts are rejected.
"""
import numpy as np
import pytest

from oracle import aggregate as oagg
from oracle import method
from paper_2605_04773_amd import synth
from tests.gpu_util import binding, log
from tests.gpu_util import problem as gpu_problem

pytestmark = pytest.mark.gpu

CASES = {"small": dict(n_bodies=4, body=(2, 3, 4), n_contacts=300),
         "medium": dict(n_bodies=12, body=(3, 5, 8), n_contacts=6000)}


@pytest.fixture(scope="module")
def ctx():
    agc = binding()
    c = agc.Context(0)
    yield c
    c.close()


_state = {}


def setup(ctx, name):
    if name in _state:
        return _state[name]
    import torch
    agc = binding()
    p = synth.contact_problem(17, **CASES[name])
    nt = p["n_tets"]
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(ctx.device, dt)
    d = {"p": p, "t": t,
         "mesh_tets": agc.agc_mesh_create(ctx, p["n_verts"], t(p["elem_verts"][:nt], torch.int32)),
         "mesh_all": agc.agc_mesh_create(ctx, p["n_verts"], t(p["elem_verts"], torch.int32)),
         "edges": t(p["edges"], torch.int32), "tags": t(p["tags"], torch.uint8),
         "eh_tets": t(p["elem_H"][:nt], torch.float64), "eh_all": t(p["elem_H"], torch.float64),
         "cv": t(p["elem_verts"][nt:], torch.int32), "ch": t(p["elem_H"][nt:], torch.float64),
         "g": t(p["g"], torch.float64), "rest": t(p["pos"], torch.float64),
         "dlb": t(p["mass"] / p["h"] ** 2, torch.float64)}
    solver = "dense" if name == "small" else "sparse"
    d["ref_c"] = method.coarsened_solve(p, solver=solver)
    d["ref_f"] = method.fine_solve(p, solver=solver)
    _state[name] = d
    return d


def solve(ctx, d, per_call=True, **kw):
    import torch
    agc = binding()
    p = d["p"]
    if per_call:
        prob = agc.make_problem(d["mesh_tets"], d["edges"], d["tags"], d["eh_tets"], d["g"], d["rest"],
                                diag_lb=d["dlb"], contacts=(d["cv"], d["ch"]))
    else:
        prob = agc.make_problem(d["mesh_all"], d["edges"], d["tags"], d["eh_all"], d["g"], d["rest"],
                                diag_lb=d["dlb"])
    x = torch.empty((p["n_verts"], 3), dtype=torch.float64, device=ctx.device)
    mp = torch.empty(p["n_verts"], dtype=torch.int32, device=ctx.device)
    info = agc.agc_solve(ctx, prob, agc.make_opts(max_iter=100000, **kw), x, mp)
    return x.cpu().numpy(), mp.cpu().numpy(), info


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name", list(CASES))
def test_coarsened_fp64_and_mixed(ctx, name):
    agc = binding()
    d = setup(ctx, name)
    ref = d["ref_c"]
    x, mp, info = solve(ctx, d, rtol=1e-12)
    m_ref, nc_ref = oagg.components(d["p"]["n_verts"], d["p"]["edges"], d["p"]["tags"])
    assert info.n_coarse == nc_ref and np.array_equal(mp, m_ref)
    e64 = rel(x, ref["x"])
    xs, _, info_s = solve(ctx, d, per_call=False, rtol=1e-12)
    xm, _, info_m = solve(ctx, d, precision=agc.AGC_PREC_MIXED, rtol=1e-9)
    log(f"[contacts] {name}: n_c {info.n_coarse}, nnzb {info.nnzb} (static plan {info_s.nnzb}); FP64 error {e64:.2e}, "
        f"vs static plan {rel(x, xs):.2e}, mixed {rel(xm, ref['x']):.2e}; bound {info.err_bound:.2e}")
    assert info.nnzb == info_s.nnzb
    assert e64 <= 1e-8
    assert rel(x, xs) <= 1e-10
    assert rel(xm, ref["x"]) <= 1e-5
    assert np.linalg.norm(x - ref["x"]) / np.linalg.norm(x) <= info.err_bound * (1 + 1e-9)


@pytest.mark.parametrize("name", list(CASES))
def test_fine_with_contacts(ctx, name):
    d = setup(ctx, name)
    x, mp, info = solve(ctx, d, coarsen=0, rtol=1e-12)
    xs, _, info_s = solve(ctx, d, per_call=False, coarsen=0, rtol=1e-12)
    e = rel(x, d["ref_f"]["x"])
    log(f"[contacts] {name} fine: nnzb {info.nnzb} (static {info_s.nnzb}) error {e:.2e} vs static {rel(x, xs):.2e}")
    assert np.array_equal(mp, np.arange(d["p"]["n_verts"]))
    assert info.nnzb == info_s.nnzb
    assert e <= 1e-8 and rel(x, xs) <= 1e-10
    agc = binding()
    xm, _, _ = solve(ctx, d, coarsen=0, precision=agc.AGC_PREC_MIXED, rtol=1e-9)
    log(f"[contacts] {name} fine mixed: error {rel(xm, d['ref_f']['x']):.2e}")
    assert rel(xm, d["ref_f"]["x"]) <= 1e-5


@pytest.mark.parametrize("name", list(CASES))
def test_post_coarsening_with_contacts(ctx, name):
    """Post-coarsening (Sec. 4.3) with the contacts given per call: k fine
    PCG iterations from x = P x_c on the fine system with every element.  The
    oracle's textbook PCG from the GPU's own x0 gives the same x (1e-9), and
    so does the static plan with the contacts in the mesh (1e-10)."""
    d = setup(ctx, name)
    k = 10
    x0, _, _ = solve(ctx, d, rtol=1e-9)
    x, _, info = solve(ctx, d, rtol=1e-9, post_iters=k)
    xs, _, _ = solve(ctx, d, per_call=False, rtol=1e-9, post_iters=k)
    ref, its = method.post_coarsen(d["p"], x0, k)
    log(f"[contacts] {name} post-coarsening: fine residual {info.fine_rel_res0:.3e} -> {info.fine_rel_res:.3e}; "
        f"x vs oracle {rel(x, ref):.2e}, vs static plan {rel(x, xs):.2e}")
    assert info.post_iters == k and its == k
    assert rel(x, ref) <= 1e-9 and rel(x, xs) <= 1e-10
    assert info.fine_rel_res < info.fine_rel_res0


@pytest.mark.parametrize("name", list(CASES))
def test_adjoint_with_contacts(ctx, name):
    """agc_solve_backward with the contacts given per call: dL/dg and dL/dH
    for every element (the tets, then the contacts) against the oracle's
    adjoint of the system with every element, and the exact identities
    L = <dL/dg, g> and sum_e <dL/dH_e, H_e> = -L."""
    import torch
    from oracle import adjoint as oadj
    agc = binding()
    d = setup(ctx, name)
    p = d["p"]
    n, ne = p["n_verts"], p["elem_verts"].shape[0]
    w_np = np.random.default_rng(29).standard_normal((n, 3))
    w = torch.from_numpy(w_np).to(ctx.device)
    prob = agc.make_problem(d["mesh_tets"], d["edges"], d["tags"], d["eh_tets"], d["g"], d["rest"],
                            contacts=(d["cv"], d["ch"]))
    opts = agc.make_opts(rtol=1e-12, max_iter=100000)
    x = torch.empty((n, 3), dtype=torch.float64, device=ctx.device)
    mp = torch.empty(n, dtype=torch.int32, device=ctx.device)
    info = agc.agc_solve(ctx, prob, opts, x, mp)
    dg = torch.empty_like(x)
    dh = torch.full((ne, 144), float("nan"), dtype=torch.float64, device=ctx.device)
    agc.agc_solve_backward(ctx, prob, opts, mp, info.n_coarse, x, w, dg, dh)
    m, nc = oagg.components(n, p["edges"], p["tags"])
    _, dgr, dhr = oadj.adjoint(n, p["elem_verts"], p["elem_H"], p["g"], m, nc, w_np, dense=name == "small")
    dg, dh = dg.cpu().numpy(), dh.cpu().numpy()
    nt = p["n_tets"]
    e_g = np.linalg.norm(dg - dgr) / np.linalg.norm(dgr)
    e_t = np.linalg.norm(dh[:nt] - dhr[:nt]) / np.linalg.norm(dhr[:nt])
    e_c = np.linalg.norm(dh[nt:] - dhr[nt:]) / np.linalg.norm(dhr[nt:])
    log(f"[contacts] {name} adjoint: dg {e_g:.2e}, dH tets {e_t:.2e}, dH contacts {e_c:.2e}")
    assert e_g <= 1e-6 and e_t <= 1e-6 and e_c <= 1e-6
    L = float(np.sum(x.cpu().numpy() * w_np))
    lin = float(np.sum(dg * p["g"]))
    euler = float(np.sum(dh * p["elem_H"]))
    assert abs(lin - L) <= 1e-8 * abs(L) + 1e-12 * np.abs(dg * p["g"]).sum()
    assert abs(euler + L) <= 1e-8 * abs(L) + 1e-12 * np.abs(dh * p["elem_H"]).sum()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_affine_with_contacts(ctx, name, precision):
    """The adaptive affine embedding (Sec. 4.2, Eq. 4) with the contacts given
    per call: node counts as the oracle's classification; FP64 at rtol 1e-10:
    the oracle's coarse residual P^T (g - H x) of the system with every
    element <= 1e-8 of P^T g; the error against the oracle's direct solve <=
    1e-5; the same solution as with the contacts in the static plan (1e-10)."""
    from oracle import affine as oaff
    from oracle import galerkin as ogal
    from oracle import solve as osol
    agc = binding()
    d = setup(ctx, name)
    p = d["p"]
    thr = 16   # every aggregate above it spans 3-D (a planar one would make the embedded system singular)
    m, nc = oagg.components(p["n_verts"], p["edges"], p["tags"])
    a_c, b_c, cls, pm = oaff.coarse_system(p, m, nc, thr)
    x_ref = oaff.prolongate(pm, osol.solve_sparse(a_c, b_c.reshape(-1)))
    prec = agc.AGC_PREC_MIXED if precision == "mixed" else agc.AGC_PREC_FP64
    rtol = 1e-10 if precision == "fp64" else 1e-7
    x, mp, info = solve(ctx, d, precision=prec, rtol=rtol, affine_threshold=thr)
    xs, _, info_s = solve(ctx, d, per_call=False, precision=prec, rtol=rtol, affine_threshold=thr)
    err = rel(x, x_ref)
    log(f"[contacts] {name} affine {precision}: n12 {info.n_affine}, block rows {info.n_blocks}, error {err:.2e}, "
        f"vs static plan {rel(x, xs):.2e}")
    assert np.array_equal(mp, m)
    assert info.n_affine == cls["n12"] > 0 and info.n_blocks == cls["n_flat"] == info_s.n_blocks
    if precision == "fp64":
        h = ogal.fine_hessian(p["n_verts"], p["elem_verts"], p["elem_H"])
        r_c = pm.T @ (p["g"].reshape(-1) - h @ x.reshape(-1))
        assert np.linalg.norm(r_c) <= 1e-8 * np.linalg.norm(b_c)
        assert rel(x, xs) <= 1e-10
    assert err <= 1e-5


def test_autograd_with_contacts(ctx):
    """AgcSolve with the contacts given per call: the gradients of g, of the
    mesh's element blocks and of the contact blocks against the oracle's
    adjoint of the system with every element."""
    import torch
    from oracle import adjoint as oadj
    agc = binding()
    d = setup(ctx, "small")
    p = d["p"]
    n, nt = p["n_verts"], p["n_tets"]
    w_np = np.random.default_rng(31).standard_normal((n, 3))
    w = torch.from_numpy(w_np).to(ctx.device)
    g = d["g"].clone().requires_grad_(True)
    eh = d["eh_tets"].clone().requires_grad_(True)
    ch = d["ch"].clone().requires_grad_(True)
    x = agc.AgcSolve.apply(g, eh, d["mesh_tets"], d["edges"], d["tags"], agc.make_opts(rtol=1e-12, max_iter=100000),
                           d["cv"], ch)
    (x * w).sum().backward()
    torch.cuda.synchronize()
    m, nc = oagg.components(n, p["edges"], p["tags"])
    xr, dgr, dhr = oadj.adjoint(n, p["elem_verts"], p["elem_H"], p["g"], m, nc, w_np, dense=True)
    log(f"[contacts] autograd: x {rel(x.detach().cpu().numpy(), xr):.2e}, dg {rel(g.grad.cpu().numpy(), dgr):.2e}, "
        f"dH tets {rel(eh.grad.cpu().numpy(), dhr[:nt]):.2e}, dH contacts {rel(ch.grad.cpu().numpy(), dhr[nt:]):.2e}")
    assert rel(x.detach().cpu().numpy(), xr) <= 1e-8
    assert rel(g.grad.cpu().numpy(), dgr) <= 1e-6
    assert rel(eh.grad.cpu().numpy(), dhr[:nt]) <= 1e-6
    assert rel(ch.grad.cpu().numpy(), dhr[nt:]) <= 1e-6


def test_contact_set_changes_between_calls(ctx):
    """One context, one tet plan, three calls whose contact sets shrink
    (all 300, the first 120, none) and a fourth with all of them again: each
    solution matches the oracle's direct solve with the tets and that call's
    contacts (the coarse assembly's buffers are sized per call)."""
    import torch
    agc = binding()
    d = setup(ctx, "small")
    p, nt = d["p"], d["p"]["n_tets"]
    n = p["n_verts"]
    x = torch.empty((n, 3), dtype=torch.float64, device=ctx.device)
    for k in (300, 120, 0, 300):
        q = dict(p, elem_verts=p["elem_verts"][:nt + k], elem_H=p["elem_H"][:nt + k])
        ref = method.coarsened_solve(q, solver="dense")["x"]
        contacts = (d["cv"][:k].contiguous(), d["ch"][:k].contiguous()) if k else None
        prob = agc.make_problem(d["mesh_tets"], d["edges"], d["tags"], d["eh_tets"], d["g"], d["rest"],
                                contacts=contacts)
        agc.agc_solve(ctx, prob, agc.make_opts(rtol=1e-12, max_iter=100000), x)
        e = rel(x.cpu().numpy(), ref)
        log(f"[contacts] {k} contacts per call: error {e:.2e}")
        assert e <= 1e-8


def test_rejected(ctx):
    import torch
    agc = binding()
    d = setup(ctx, "small")
    p = d["p"]
    bad = d["cv"].clone()
    bad[3, 2] = bad[3, 1]                       # a repeated vertex
    prob = agc.make_problem(d["mesh_tets"], d["edges"], d["tags"], d["eh_tets"], d["g"], contacts=(bad, d["ch"]))
    x = torch.empty((p["n_verts"], 3), dtype=torch.float64, device=ctx.device)
    with pytest.raises(agc.BadInput):
        agc.agc_solve(ctx, prob, agc.make_opts(rtol=1e-8), x)
    bad = d["cv"].clone()
    bad[7, 0] = p["n_verts"]                    # out of range
    prob = agc.make_problem(d["mesh_tets"], d["edges"], d["tags"], d["eh_tets"], d["g"], contacts=(bad, d["ch"]))
    with pytest.raises(agc.BadInput):
        agc.agc_solve(ctx, prob, agc.make_opts(rtol=1e-8), x)
    prob = agc.make_problem(d["mesh_tets"], d["edges"], d["tags"], d["eh_tets"], d["g"], d["rest"],
                            contacts=(d["cv"], d["ch"]))
    # the context still works
    x2, _, _ = solve(ctx, d, rtol=1e-10)
    assert rel(x2, d["ref_c"]["x"]) <= 1e-7


_full = {}


def _full_row(ctx):
    """The contact row at full size: a plan of the tets alone, the contact blocks per call."""
    if "d" not in _full:
        import torch
        agc = binding()
        p = gpu_problem("c3")
        nt = p["n_tets"]
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(ctx.device, dt)
        ev, eh = t(p["elem_verts"], torch.int32), t(p["elem_H"], torch.float64)
        _full["d"] = {"p": p, "mesh": agc.agc_mesh_create(ctx, p["n_verts"], ev[:nt].contiguous()),
                      "edges": t(p["edges"], torch.int32), "tags": t(p["tags"], torch.uint8),
                      "eh": eh[:nt].contiguous(), "cv": ev[nt:].contiguous(), "ch": eh[nt:].contiguous(),
                      "g": t(p["g"], torch.float64), "rest": t(p["pos"], torch.float64)}
    return _full["d"]


def _full_solve(ctx, d, **kw):
    import torch
    agc = binding()
    prob = agc.make_problem(d["mesh"], d["edges"], d["tags"], d["eh"], d["g"], d["rest"], contacts=(d["cv"], d["ch"]))
    n = d["p"]["n_verts"]
    x = torch.empty((n, 3), dtype=torch.float64, device=ctx.device)
    mp = torch.empty(n, dtype=torch.int32, device=ctx.device)
    info = agc.agc_solve(ctx, prob, agc.make_opts(max_iter=50000, **kw), x, mp)
    return x.cpu().numpy(), mp.cpu().numpy(), info


@pytest.mark.parametrize("mode", ["fp64", "mixed", "fine_fp64"])
def test_full_size_contact_row(ctx, mode):
    """The contact row at full size (108,000 vertices, 368,640 tets, 250,000
    contact blocks given per call): the map is the oracle's; in FP64 at rtol
    1e-10 the oracle's matrix-free residual with every element is <= 1e-8; at
    rtol 1e-7 the error against an FP64 reference that the oracle certifies
    (residual and mass bound <= 1e-8) is <= 1e-5, the bars of the static plan."""
    from tests.test_gpu_solve import _certified
    agc = binding()
    d = _full_row(ctx)
    p = d["p"]
    coarsen = 0 if mode.startswith("fine") else 1
    if coarsen:
        m, nc = oagg.components(p["n_verts"], p["edges"], p["tags"])
    else:
        m, nc = np.arange(p["n_verts"], dtype=np.int32), p["n_verts"]
    key = ("ref", coarsen)
    if key not in _full:
        x_ref, mp, info = _full_solve(ctx, d, coarsen=coarsen, rtol=1e-12)
        cert, _ = _certified(p, m, nc, x_ref)
        log(f"[contacts] full row reference coarsen={coarsen}: iters {info.pcg_iters} certified {cert:.2e}")
        assert np.array_equal(mp, m) and cert <= 1e-8
        _full[key] = x_ref
    x_ref = _full[key]
    if mode != "mixed":
        x, mp, info = _full_solve(ctx, d, coarsen=coarsen, rtol=1e-10)
        _, res = _certified(p, m, nc, x)
        log(f"[contacts] full row {mode} rtol 1e-10: iters {info.pcg_iters} oracle residual {res:.2e}")
        assert np.array_equal(mp, m) and res <= 1e-8
    prec = agc.AGC_PREC_MIXED if mode == "mixed" else agc.AGC_PREC_FP64
    x, mp, info = _full_solve(ctx, d, coarsen=coarsen, precision=prec, rtol=1e-7)
    err = rel(x, x_ref)
    log(f"[contacts] full row {mode} rtol 1e-7: iters {info.pcg_iters} error {err:.2e}")
    assert np.array_equal(mp, m) and err <= 1e-5
