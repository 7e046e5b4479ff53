"""GPU parity of the outer Newton loop (agc_newton_*) against the oracle (Sec. 3, Eq. 1-2; Alg. overview).

Per element and per vertex (masses, gradient, proxy blocks, energy): against
oracle/newton.py at deformed states that include inverted elements, to
rounding (relative 1e-10 of each quantity's scale; the rotation comes from
two different methods, Jacobi on F^T F here and an SVD in the oracle).  The
loop: with float64 solves to 1e-12 both sides take the same directions, so
the per-iteration energies and step lengths agree and the results agree to
1e-9 of the displacement.  The coarsened loop, with and without the affine
embedding, is compared iteration by iteration (tags, map, iterate, energy)
on a case whose strain increments keep clear of the threshold, and by its
final energy elsewhere."""
import numpy as np
import pytest

from oracle import newton as onw
from paper_2605_04773_amd import synth
from tests.gpu_util import binding, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    agc = binding()
    c = agc.Context(0)
    yield c
    c.close()


_cases = {}


def case(ctx, n):
    """(p, device tensors, Newton handle) of an n^3 grid."""
    if n not in _cases:
        import torch
        agc = binding()
        p = synth.grid_problem(n, 40 + n, 0.6)
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(ctx.device, dt)
        d = {"ev": t(p["elem_verts"], torch.int32), "edges": t(p["edges"], torch.int32),
             "rest": t(p["pos"], torch.float64), "t": t}
        d["mesh"] = agc.agc_mesh_create(ctx, p["n_verts"], d["ev"])
        m = synth.material()
        d["nw"] = agc.agc_newton_create(ctx, d["mesh"], d["edges"], d["rest"], m["mu"], m["lam"], m["rho"], m["h"])
        _cases[n] = (p, d)
    return _cases[n]


def _oracle_parts(p):
    m = synth.material()
    _, vol, b = onw.rest_shape(p["pos"], p["elem_verts"])
    mass = onw.lumped_mass(p["n_verts"], p["elem_verts"], vol, m["rho"])
    return m, vol, b, mass


@pytest.mark.parametrize("n", [3, 8])
def test_mass(ctx, n):
    agc = binding()
    p, d = case(ctx, n)
    _, _, _, mass = _oracle_parts(p)
    got = agc.agc_newton_mass(ctx, d["nw"]).cpu().numpy()
    assert np.allclose(got, mass, rtol=1e-14, atol=0)


@pytest.mark.parametrize("n", [3, 8])
@pytest.mark.parametrize("state", ["spun", "crushed"])
def test_physics(ctx, n, state):
    import torch
    agc = binding()
    p, d = case(ctx, n)
    m, vol, b, mass = _oracle_parts(p)
    rng = np.random.default_rng(100 + n)
    rot = synth.random_rotations(rng, 1)[0]
    x = p["pos"] @ rot.T + 0.3
    if state == "spun":
        x = x + 0.02 / n * rng.standard_normal(x.shape)
    else:   # large deformation: some elements inverted
        x = x + 0.6 / n * rng.standard_normal(x.shape)
    x_hat = p["pos"] + 0.01 * rng.standard_normal(x.shape)
    f = onw.deformation_gradients(x, p["elem_verts"], b)
    n_inv = int((np.linalg.det(f) < 0).sum())
    log(f"[newton physics] n={n} {state}: {n_inv} inverted of {f.shape[0]}")
    if state == "crushed":
        assert n_inv > 0
    g, hb, e = agc.agc_newton_physics(ctx, d["nw"], d["t"](x, torch.float64), d["t"](x_hat, torch.float64))
    g, hb = g.cpu().numpy(), hb.cpu().numpy()
    args = (x_hat, mass, p["elem_verts"], b, vol, m["mu"], m["lam"], m["h"])
    g_ref = onw.gradient(x, *args)
    e_ref = onw.energy(x, *args)
    h_ref = onw.element_blocks(x, p["elem_verts"], b, vol, m["mu"], m["lam"], m["rho"], m["h"])
    assert abs(e - e_ref) <= 1e-11 * abs(e_ref)
    assert np.abs(g - g_ref).max() <= 1e-10 * np.abs(g_ref).max()
    assert np.abs(hb - h_ref).max() <= 1e-10 * np.abs(h_ref).max()
    hb3 = hb.reshape(-1, 12, 12)
    assert np.array_equal(hb3, np.swapaxes(hb3, 1, 2))


def _run(ctx, n, coarsen, precision="fp64", **kw):
    import torch
    agc = binding()
    p, d = case(ctx, n)
    x_t, v_t, f = synth.newton_state(p, wave_speed=0.5)
    solve = agc.make_opts(rtol=1e-12, coarsen=1) if precision == "fp64" else \
        agc.make_opts(precision=agc.AGC_PREC_MIXED, rtol=1e-7)
    opts = agc.make_newton_opts(eps_d=kw.get("eps_d", 1e-4), coarsen=coarsen, solve=solve)
    t = lambda a: d["t"](a, torch.float64)
    x, info = agc.agc_newton_step(ctx, d["nw"], opts, t(x_t), t(v_t), t(f))
    return p, x.cpu().numpy(), info, (x_t, v_t, f)


@pytest.mark.parametrize("n", [4, 8])
def test_fine_loop_matches_oracle(ctx, n):
    p, x, info, (x_t, v_t, f) = _run(ctx, n, coarsen=0)
    mesh = {"n_verts": p["n_verts"], "rest": p["pos"], "tets": p["elem_verts"], "edges": p["edges"]}
    x_ref, log_ref = onw.time_step(mesh, synth.material(), x_t, v_t, f, eps_d=1e-4, coarsen=False)
    log(f"[newton fine] n={n}: gpu {info.newton_iters} iters E {info.energy0:.6g} -> {info.energy:.10g}; "
        f"oracle {len(log_ref)} iters E -> {log_ref[-1]['energy_after']:.10g}")
    assert info.newton_iters == len(log_ref)
    assert info.halvings == sum(it["halvings"] for it in log_ref)
    assert abs(info.energy0 - log_ref[0]["energy"]) <= 1e-11 * abs(log_ref[0]["energy"])
    assert abs(info.energy - log_ref[-1]["energy_after"]) <= 1e-9 * abs(log_ref[0]["energy"])
    disp = np.abs(x_ref - x_t).max()
    assert np.abs(x - x_ref).max() <= 1e-9 * disp


@pytest.mark.parametrize("n", [4, 8])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_coarsened_loop(ctx, n, precision):
    p, x, info, (x_t, v_t, f) = _run(ctx, n, coarsen=1, precision=precision)
    mesh = {"n_verts": p["n_verts"], "rest": p["pos"], "tets": p["elem_verts"], "edges": p["edges"]}
    mat = synth.material()
    x_ref, log_ref = onw.time_step(mesh, mat, x_t, v_t, f, eps_d=1e-4, coarsen=True)
    xf_ref, logf = onw.time_step(mesh, mat, x_t, v_t, f, eps_d=1e-4, coarsen=False)
    e0, ef = logf[0]["energy"], logf[-1]["energy_after"]
    log(f"[newton coarsened] n={n} {precision}: gpu {info.newton_iters} iters, mean coarse size "
        f"{info.coarse_nodes_sum / info.newton_iters:.0f} of {p['n_verts']}, E -> {info.energy:.10g}; oracle "
        f"{len(log_ref)} iters E -> {log_ref[-1]['energy_after']:.10g}; fine minimum {ef:.10g}")
    assert info.energy < info.energy0
    assert abs(info.energy - log_ref[-1]["energy_after"]) <= 1e-6 * (e0 - ef)
    assert info.energy - ef <= 1e-3 * (e0 - ef)
    assert info.coarse_nodes_sum < info.newton_iters * p["n_verts"]
    if precision == "fp64":
        assert abs(info.newton_iters - len(log_ref)) <= 1


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_affine_embedded_loop(ctx, precision):
    """The paper's main variant inside the loop: aggregates of more than 8
    vertices get 12 DoF.  It must still end at the fine loop's minimum."""
    import torch
    agc = binding()
    p, d = case(ctx, 8)
    x_t, v_t, f = synth.newton_state(p, wave_speed=0.5)
    solve = agc.make_opts(rtol=1e-12, affine_threshold=8) if precision == "fp64" else \
        agc.make_opts(precision=agc.AGC_PREC_MIXED, rtol=1e-7, affine_threshold=8)
    opts = agc.make_newton_opts(eps_d=1e-4, coarsen=1, solve=solve)
    t = lambda a: d["t"](a, torch.float64)
    x, info = agc.agc_newton_step(ctx, d["nw"], opts, t(x_t), t(v_t), t(f))
    mesh = {"n_verts": p["n_verts"], "rest": p["pos"], "tets": p["elem_verts"], "edges": p["edges"]}
    _, logf = onw.time_step(mesh, synth.material(), x_t, v_t, f, eps_d=1e-4, coarsen=False)
    e0, ef = logf[0]["energy"], logf[-1]["energy_after"]
    log(f"[newton affine] {precision}: {info.newton_iters} iters, mean coarse size "
        f"{info.coarse_nodes_sum / info.newton_iters:.0f}, E -> {info.energy:.10g}; fine minimum {ef:.10g}")
    assert info.energy < info.energy0
    assert info.energy - ef <= 1e-3 * (e0 - ef)
    # the embedding was active: some solve had a 12-DoF node (a coarse system smaller than the fine one)
    assert info.coarse_nodes_sum < info.newton_iters * p["n_verts"]
    # with the threshold above every aggregate the loop is the 3-DoF one, bit for bit
    big = agc.make_opts(rtol=1e-12, affine_threshold=10**6) if precision == "fp64" else \
        agc.make_opts(precision=agc.AGC_PREC_MIXED, rtol=1e-7, affine_threshold=10**6)
    plain = agc.make_opts(rtol=1e-12) if precision == "fp64" else agc.make_opts(precision=agc.AGC_PREC_MIXED, rtol=1e-7)
    xa, ia = agc.agc_newton_step(ctx, d["nw"], agc.make_newton_opts(eps_d=1e-4, coarsen=1, solve=big), t(x_t), t(v_t),
                                 t(f))
    xb, ib = agc.agc_newton_step(ctx, d["nw"], agc.make_newton_opts(eps_d=1e-4, coarsen=1, solve=plain), t(x_t),
                                 t(v_t), t(f))
    assert torch.equal(xa, xb) and ia.newton_iters == ib.newton_iters


@pytest.mark.parametrize("affine", [0, 8])
def test_coarsened_loop_per_iteration(ctx, affine):
    """The coarsened loop (FP64 solves to 1e-12), iteration by iteration,
    against the oracle's loop of the same path (affine > 0: aggregates of
    more than `affine` vertices carry 12 DoF, Sec. 4.2 Eq. 4).  After k
    iterations (a run with max_newton = k) the GPU iterate is the oracle's
    within 1e-9 of the displacement, and so is the energy; the tags of
    iteration k, from the library's tagger on the GPU's iterates k-1 and
    k-2, are the oracle's bit for bit, and so is the map agc_aggregate makes
    of them.  No element's strain increment in the oracle's iterates lies
    within 1e-6 of the threshold (checked), so rounding decides no tag."""
    import torch
    agc = binding()
    p, d = case(ctx, 8)
    mat = synth.material()
    h, thr = mat["h"], 5e-5
    x_t, v_t, f = synth.newton_state(p, wave_speed=0.5)
    mesh = {"n_verts": p["n_verts"], "rest": p["pos"], "tets": p["elem_verts"], "edges": p["edges"]}
    _, lg = onw.time_step(mesh, mat, x_t, v_t, f, eps_d=1e-4, coarsen=True, affine_threshold=affine, record=True)
    margin = min(float(np.min(np.abs(it["norms"] - thr))) / thr for it in lg)
    assert margin > 1e-6
    assert any(it["n_c"] < p["n_verts"] for it in lg)
    if affine:
        assert any(it["n_blocks"] > it["n_c"] for it in lg)
    t = lambda a: d["t"](a, torch.float64)
    tagger = agc.agc_tagger_create(ctx, p["n_verts"], d["ev"], d["rest"], d["edges"])
    disp = max(float(np.abs(it["x"] - x_t).max()) for it in lg)
    solve = agc.make_opts(rtol=1e-12, affine_threshold=affine)
    prev2, prev = x_t - h * v_t, x_t
    for k in range(1, len(lg) + 1):
        ref = lg[k - 1]
        tags, _ = agc.agc_tag_edges(ctx, tagger, t(prev), t(prev2), thr)
        assert np.array_equal(tags.cpu().numpy(), ref["tags"]), f"tags of iteration {k}"
        mp, nc = agc.agc_aggregate(ctx, p["n_verts"], d["edges"], tags)
        assert nc == ref["n_c"] and np.array_equal(mp.cpu().numpy(), ref["map"]), f"map of iteration {k}"
        opts = agc.make_newton_opts(max_newton=k, eps_d=1e-4, coarsen=1, solve=solve)
        x, info = agc.agc_newton_step(ctx, d["nw"], opts, t(x_t), t(v_t), t(f))
        xk = x.cpu().numpy()
        err = float(np.abs(xk - ref["x"]).max()) / disp
        log(f"[newton per-iteration] affine={affine} k={k}: n_c {nc} blocks {ref['n_blocks']} halvings "
            f"{ref['halvings']} x vs oracle {err:.1e} of the displacement")
        assert info.newton_iters == k
        assert err <= 1e-9
        assert abs(info.energy - ref["energy_after"]) <= 1e-9 * abs(lg[0]["energy"])
        prev2, prev = prev, xk
    tagger.close()


def test_bad_input(ctx):
    import torch
    agc = binding()
    p, d = case(ctx, 3)
    m = synth.material()
    with pytest.raises(agc.AgcError):
        agc.agc_newton_create(ctx, d["mesh"], d["edges"], d["rest"], m["mu"], m["lam"], -1.0, m["h"])
    flat = d["rest"].clone()
    flat[:, 2] = 0.0            # every element degenerate
    with pytest.raises(agc.AgcError):
        agc.agc_newton_create(ctx, d["mesh"], d["edges"], flat, m["mu"], m["lam"], m["rho"], m["h"])
    x_t, v_t, f = synth.newton_state(p)
    t = lambda a: d["t"](a, torch.float64)
    with pytest.raises(agc.AgcError):
        agc.agc_newton_step(ctx, d["nw"], agc.make_newton_opts(max_newton=0), t(x_t), t(v_t), t(f))
    # the handle still works
    x, info = agc.agc_newton_step(ctx, d["nw"], agc.make_newton_opts(eps_d=1e-3), t(x_t), t(v_t), None)
    assert info.newton_iters >= 1 and info.energy < info.energy0


def test_handle_keeps_its_mesh(ctx):
    """The Newton handle uses its mesh's static structure: the binding keeps
    the mesh alive while only the handle refers to it (a collected mesh
    would be destroyed under the handle)."""
    import gc
    import torch
    agc = binding()
    p = synth.grid_problem(3, 77, 0.6)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(ctx.device, dt)
    m = synth.material()
    nw = agc.agc_newton_create(ctx, agc.agc_mesh_create(ctx, p["n_verts"], t(p["elem_verts"], torch.int32)),
                               t(p["edges"], torch.int32), t(p["pos"], torch.float64), m["mu"], m["lam"], m["rho"],
                               m["h"])
    gc.collect()
    assert nw.mesh is not None and nw.mesh.h is not None
    x_t, v_t, f = synth.newton_state(p, wave_speed=0.5)
    x, info = agc.agc_newton_step(ctx, nw, agc.make_newton_opts(eps_d=1e-3), t(x_t, torch.float64),
                                  t(v_t, torch.float64), t(f, torch.float64))
    assert info.newton_iters >= 1 and info.energy < info.energy0
    nw.close()
