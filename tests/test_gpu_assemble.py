"""GPU parity of agc_assemble_coarse / agc_assemble_fine / agc_spmv against the oracle.

Pattern: bit-exact.  Values: within the Higham bound gamma_K * sum|terms| per
entry, K the number of summed terms (at most 16 per element).  Symmetry of the
stored matrix: exact."""
import numpy as np
import pytest

from oracle import aggregate as oagg
from oracle import galerkin as ogal
from tests.gpu_util import U32, Dev, binding, bsr_numpy, gamma, log, problem, to_scipy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    agc = binding()
    c = agc.Context(0)
    yield c
    c.close()


_devs = {}


def dev(ctx, name):
    if name not in _devs:
        _devs[name] = Dev(ctx, problem(name), f32=True)
    return _devs[name]


def _check_exact_symmetry(rp, ci, vals):
    n = rp.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    pos = {(int(r), int(c)): k for k, (r, c) in enumerate(zip(rows, ci))}
    for k, (r, c) in enumerate(zip(rows.tolist(), ci.tolist())):
        kt = pos[(c, r)]
        assert np.array_equal(vals[k], vals[kt].T), (r, c)


@pytest.mark.parametrize("name", ["tiny", "c1", "c4"])
def test_coarse_matches_oracle(ctx, name):
    import torch
    agc = binding()
    d = dev(ctx, name)
    p = d.p
    log(f"[asm] coarse {name}")
    mp, nc = agc.agc_aggregate(ctx, p["n_verts"], d.edges, d.tags)
    A, g_c = agc.agc_assemble_coarse(ctx, d.mesh, d.eh, d.g, mp, nc)
    m = mp.cpu().numpy()
    rp, ci, vals = bsr_numpy(A)
    # pattern bit-exact: sorted keys per row equal the oracle's key set
    pr, pc = ogal.coarse_pattern(p["elem_verts"], m, nc)
    assert np.array_equal(rp, ogal.bsr_from_pattern(nc, pr, pc))
    assert np.array_equal(ci, pc)
    # values within the summation bound
    a_ref, b_ref = ogal.coarse_system(p["n_verts"], p["elem_verts"], p["elem_H"], p["g"], m, nc)
    a_abs, _ = ogal.coarse_system(p["n_verts"], p["elem_verts"], np.abs(p["elem_H"]), p["g"], m, nc)
    ref_blocks = ogal.to_blocks(a_ref, pr, pc)
    abs_blocks = ogal.to_blocks(a_abs, pr, pc)
    K = 16 * p["elem_verts"].shape[0]
    assert (np.abs(vals - ref_blocks) <= 2 * gamma(K) * abs_blocks).all()
    _check_exact_symmetry(rp, ci, vals)
    # g_c = P^T g
    gb = gamma(2 * np.bincount(m).max()) * ogal.restrict(m, nc, np.abs(p["g"]))
    assert (np.abs(g_c.cpu().numpy() - b_ref) <= gb + 1e-300).all()
    # float32 sums and storage: within the float32 bound of the exact values
    A32, _ = agc.agc_assemble_coarse(ctx, d.mesh, d.eh, None, mp, nc, out_dtype=agc.AGC_F32)
    rp32, ci32, v32 = bsr_numpy(A32)
    assert np.array_equal(rp32, rp) and np.array_equal(ci32, ci)
    assert (np.abs(v32 - ref_blocks) <= 2 * gamma(K, U32) * abs_blocks + U32 * np.abs(ref_blocks)).all()
    _check_exact_symmetry(rp32, ci32, v32)
    # float32 element input, float32 sums
    A32b, _ = agc.agc_assemble_coarse(ctx, d.mesh, d.eh32, None, mp, nc, out_dtype=agc.AGC_F32)
    v32b = bsr_numpy(A32b)[2]
    assert (np.abs(v32b - ref_blocks) <= 2 * gamma(K + 1, U32) * abs_blocks + U32 * np.abs(ref_blocks)).all()
    del torch


@pytest.mark.parametrize("name", ["tiny", "c1", "c4"])
def test_fine_matches_oracle(ctx, name):
    agc = binding()
    d = dev(ctx, name)
    p = d.p
    log(f"[asm] fine {name}")
    H = agc.agc_assemble_fine(ctx, d.mesh, d.eh)
    assert d.mesh.fine_nnzb == p["n_verts"] + 2 * p["edges"].shape[0]
    rp, ci, vals = bsr_numpy(H)
    ident = np.arange(p["n_verts"])
    pr, pc = ogal.coarse_pattern(p["elem_verts"], ident, p["n_verts"])
    assert np.array_equal(ci, pc) and np.array_equal(rp, ogal.bsr_from_pattern(p["n_verts"], pr, pc))
    h_ref = ogal.fine_hessian(p["n_verts"], p["elem_verts"], p["elem_H"])
    h_abs = ogal.fine_hessian(p["n_verts"], p["elem_verts"], np.abs(p["elem_H"]))
    ref = ogal.to_blocks(h_ref, pr, pc)
    ab = ogal.to_blocks(h_abs, pr, pc)
    assert (np.abs(vals - ref) <= 2 * gamma(64) * ab).all()
    _check_exact_symmetry(rp, ci, vals)


def _max_plan(p):
    """Largest number of element sub-blocks summed into one fine block."""
    ev = p["elem_verts"].astype(np.int64)
    a, b = np.triu_indices(4)
    va, vb = ev[:, a], ev[:, b]
    key = np.minimum(va, vb).ravel() * p["n_verts"] + np.maximum(va, vb).ravel()
    return int(np.unique(key, return_counts=True)[1].max())


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_coarse_full_size_sampled(ctx, name):
    """Full size (64^3 grid; 96-body contact row): pattern bit-exact; values of
    sampled rows (incl. the longest row) vs per-row oracle."""
    agc = binding()
    d = dev(ctx, name)
    p = d.p
    log(f"[asm] {name} full size")
    mp, nc = agc.agc_aggregate(ctx, p["n_verts"], d.edges, d.tags)
    for dt in (agc.AGC_F64, agc.AGC_F32):
        A, _ = agc.agc_assemble_coarse(ctx, d.mesh, d.eh, None, mp, nc, out_dtype=dt)
        m = mp.cpu().numpy()
        rp, ci, vals = bsr_numpy(A)
        pr, pc = ogal.coarse_pattern(p["elem_verts"], m, nc)
        assert np.array_equal(ci, pc) and np.array_equal(rp, ogal.bsr_from_pattern(nc, pr, pc))
        lens = np.diff(rp)
        rng = np.random.default_rng(0)
        rows = sorted(set(rng.choice(nc, 60, replace=False).tolist()) | {int(np.argmax(lens)), 0, nc - 1})
        blocks = ogal.coarse_rows(p["elem_verts"], p["elem_H"], m, nc, rows)
        ablocks = ogal.coarse_rows(p["elem_verts"], np.abs(p["elem_H"]), m, nc, rows)
        # Every entry is summed along a tree whose depth is bounded by the
        # plan length of a fine block, the in-tile scan and carries (< 24)
        # and the cross-tile fix-up (< 24 + tiles/256); so the error is at
        # most gamma_D sum|terms| (plus one rounding of each term to float32).
        depth = _max_plan(p) + 48 + (d.mesh.fine_nnzb // (256 * 256) + 1)
        u = gamma(depth) if dt == agc.AGC_F64 else gamma(depth, U32) + U32
        for r in rows:
            for k in range(rp[r], rp[r + 1]):
                ref = blocks[(r, int(ci[k]))]
                assert (np.abs(vals[k] - ref) <= u * ablocks[(r, int(ci[k]))]).all(), (r, int(ci[k]), dt)
        del A


@pytest.mark.parametrize("name", ["c1", "c4"])
def test_spmv_matches_scipy(ctx, name):
    import torch
    agc = binding()
    d = dev(ctx, name)
    p = d.p
    mp, nc = agc.agc_aggregate(ctx, p["n_verts"], d.edges, d.tags)
    for mat in (agc.agc_assemble_coarse(ctx, d.mesh, d.eh, None, mp, nc)[0], agc.agc_assemble_fine(ctx, d.mesh, d.eh)):
        S = to_scipy(mat)
        rng = np.random.default_rng(1)
        x = rng.standard_normal((mat.n_rows, 3))
        y = agc.agc_spmv(ctx, mat, torch.from_numpy(x).to(ctx.device)).cpu().numpy().reshape(-1)
        ref = S @ x.reshape(-1)
        absr = abs(S) @ np.abs(x.reshape(-1))
        lens = np.diff(mat.to_bsr()[0].cpu().numpy())
        assert (np.abs(y - ref) <= gamma(3 * lens.max() + 8) * absr + 1e-300).all()


def test_assembly_deterministic(ctx):
    agc = binding()
    d = dev(ctx, "c4")
    mp, nc = agc.agc_aggregate(ctx, d.p["n_verts"], d.edges, d.tags)
    ref = bsr_numpy(agc.agc_assemble_coarse(ctx, d.mesh, d.eh, None, mp, nc)[0])
    for _ in range(2):
        got = bsr_numpy(agc.agc_assemble_coarse(ctx, d.mesh, d.eh, None, mp, nc)[0])
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)


def test_mesh_rejects_bad_elements(ctx):
    import torch
    agc = binding()
    ev = torch.tensor([[0, 1, 2, 3], [0, 1, 2, 2]], dtype=torch.int32, device=ctx.device)
    with pytest.raises(agc.BadInput):
        agc.agc_mesh_create(ctx, 4, ev)
    ev = torch.tensor([[0, 1, 2, 4]], dtype=torch.int32, device=ctx.device)
    with pytest.raises(agc.BadInput):
        agc.agc_mesh_create(ctx, 4, ev)


@pytest.mark.parametrize("h_dtype", ["f64", "f32"])
def test_fine_gather_paths_agree(ctx, h_dtype):
    """The fine gather stages the element blocks around each row in LDS; a
    row around more elements than fit, and element blocks that are not
    16-byte aligned, are gathered from global memory instead.  Here one
    vertex lies in 300 tetrahedra (a row over the limit) and the others in a
    few: the sums match the oracle's to rounding, and the aligned (staged)
    and misaligned (global) calls agree bit for bit."""
    import torch
    agc = binding()
    rng = np.random.default_rng(11)
    k, nv = 300, 201
    ev = np.empty((k, 4), np.int64)
    ev[:, 0] = 0
    for e in range(k):   # every other vertex in 4 or 5 elements
        ev[e, 1:] = 1 + (3 * e + np.arange(3)) % (nv - 1)
    a = rng.standard_normal((k, 12, 12))
    eh = (a + np.swapaxes(a, 1, 2)).reshape(k, 144)
    tdt = torch.float64 if h_dtype == "f64" else torch.float32
    if h_dtype == "f32":
        eh = eh.astype(np.float32).astype(np.float64)   # the values the float32 call sees
    mesh = agc.agc_mesh_create(ctx, nv, torch.from_numpy(ev.astype(np.int32)).to(ctx.device))
    aligned = torch.from_numpy(eh).to(ctx.device, tdt)
    flat = torch.zeros(k * 144 + 1, dtype=tdt, device=ctx.device)
    flat[1:] = aligned.reshape(-1)
    shifted = flat[1:].view(k, 144)
    assert aligned.data_ptr() % 16 == 0 and shifted.data_ptr() % 16 != 0
    h1 = agc.agc_assemble_fine(ctx, mesh, aligned)
    h2 = agc.agc_assemble_fine(ctx, mesh, shifted)
    rp, ci, vals = bsr_numpy(h1)
    rp2, ci2, vals2 = bsr_numpy(h2)
    assert np.array_equal(rp, rp2) and np.array_equal(ci, ci2) and np.array_equal(vals, vals2)
    ident = np.arange(nv)
    pr, pc = ogal.coarse_pattern(ev, ident, nv)
    assert np.array_equal(ci, pc)
    ref = ogal.to_blocks(ogal.fine_hessian(nv, ev, eh), pr, pc)
    ab = ogal.to_blocks(ogal.fine_hessian(nv, ev, np.abs(eh)), pr, pc)
    log(f"[asm] gather paths {h_dtype}: row 0 sums {np.diff(rp)[0]} blocks of up to {k} sub-blocks")
    assert (np.abs(vals - ref) <= 2 * gamma(k + 16) * ab).all()
    h1.close()
    h2.close()
    mesh.close()
