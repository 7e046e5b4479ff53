"""Seeded synthetic inputs for one Newton linear solve of implicit elastodynamics.

This module builds the *inputs* of the in-solve coarsening path: a tetrahedral
mesh, its edge list, per-element 12x12 Hessian blocks, the per-DoF gradient,
the per-edge collapse tags, and (for the contact case) point-triangle barrier
blocks.  It holds none of the arithmetic of the coarsening method (no
aggregation, no Galerkin product, no solve); both the GPU library and the CPU
oracle consume what it returns.

The paper solves H d = -grad E with H an SPD proxy of the incremental
potential's Hessian (Sec. 3, Eq. 1-2): H = M/h^2 + (elastic Hessian) +
(contact Hessian).  Here the elastic part of every tetrahedron is the
co-rotated linear-elastic stiffness R K0 R^T at a random per-element rotation,
and the lumped mass rho*V/4 per element vertex, divided by h^2, is folded into
the element block so that every element block is SPD on its own.

Edge tags follow the paper's tag semantics (Sec. 4.1; supplement Sec. 1.1):
1 = collapsible, 0 = protected.  A smooth random field stands in for the
Green-strain-increment criterion (Sec. 4.2, Eq. 3): an edge is collapsible
when the mean of the field at its two endpoints ranks among the lowest
``frac`` of all edges.

Random streams: ``np.random.default_rng(SeedSequence([seed, stream]))`` with
stream 0 rotations, 1 field, 2 gradient, 3 adjoint seed w, 4 finite-difference
directions, 5 jitter, 6 contact, 7 drift, 8 deformation states.
"""
from __future__ import annotations

import math
import os

import numpy as np

YOUNG = 1.0e5
POISSON = 0.4
DENSITY = 1000.0
H_STEP = 1.0e-2

S_ROT, S_FIELD, S_GRAD, S_W, S_FD, S_JITTER, S_CONTACT, S_DRIFT, S_STATES, S_NEWTON = range(10)
GRAVITY = 9.8


def rng_for(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(stream)]))


def lame(young: float = YOUNG, poisson: float = POISSON) -> tuple[float, float]:
    mu = young / (2.0 * (1.0 + poisson))
    lam = young * poisson / ((1.0 + poisson) * (1.0 - 2.0 * poisson))
    return mu, lam


# --------------------------------------------------------------------------
# mesh
# --------------------------------------------------------------------------

# corner code c = dx + 2*dy + 4*dz inside one cube
_C = {(0, 0, 0): 0, (1, 0, 0): 1, (0, 1, 0): 2, (1, 1, 0): 3,
      (0, 0, 1): 4, (1, 0, 1): 5, (0, 1, 1): 6, (1, 1, 1): 7}


def _tets(spec):
    return np.array([[_C[tuple(int(ch) for ch in v)] for v in t.split()] for t in spec], dtype=np.int64)


# 5-tet split without an interior diagonal; odd cubes use the mirror split so
# that the face diagonals of neighbouring cubes coincide.
_EVEN = _tets(["000 110 101 011", "100 000 110 101", "010 110 000 011",
               "001 101 011 000", "111 011 101 110"])
_ODD = _tets(["100 010 001 111", "000 100 010 001", "110 010 100 111",
              "101 001 111 100", "011 111 001 010"])


def box_mesh(nx: int, ny: int, nz: int, cell: float, origin=(0.0, 0.0, 0.0)):
    """Vertices and tets of an nx*ny*nz grid of cubes (edge ``cell``), 5 tets per cube.

    Vertex id = i + (nx+1)*(j + (ny+1)*k).  Tets are positively oriented.
    """
    vx, vy, vz = nx + 1, ny + 1, nz + 1
    k, j, i = np.meshgrid(np.arange(vz), np.arange(vy), np.arange(vx), indexing="ij")
    pos = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64) * cell
    pos += np.asarray(origin, dtype=np.float64)[None, :]

    ck, cj, ci = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    corner = np.empty((ci.size, 8), dtype=np.int64)
    for (dx, dy, dz), c in _C.items():
        corner[:, c] = (ci + dx) + vx * ((cj + dy) + vy * (ck + dz))
    odd = ((ci + cj + ck) & 1).astype(bool)
    table = np.where(odd[:, None, None], _ODD[None], _EVEN[None])        # (ncube,5,4)
    tets = np.take_along_axis(corner[:, None, :], table, axis=2).reshape(-1, 4)

    d = pos[tets[:, 1:]] - pos[tets[:, :1]]
    neg = np.linalg.det(d) < 0
    tets[neg] = tets[neg][:, [0, 1, 3, 2]]
    return pos, tets.astype(np.int32)


def mesh_edges(tets: np.ndarray, n_verts: int) -> np.ndarray:
    """Unique undirected edges of a tet mesh as sorted (lo, hi) int32 pairs."""
    t = tets.astype(np.int64)
    pairs = np.concatenate([t[:, [a, b]] for a in range(4) for b in range(a + 1, 4)], axis=0)
    lo = pairs.min(axis=1)
    hi = pairs.max(axis=1)
    key = np.unique(lo * n_verts + hi)
    return np.stack([key // n_verts, key % n_verts], axis=1).astype(np.int32)


def grid_counts(nx: int, ny: int, nz: int) -> dict:
    """Closed-form sizes of the 5-tet grid (used by the tests)."""
    nv = (nx + 1) * (ny + 1) * (nz + 1)
    axis = nx * (ny + 1) * (nz + 1) + (nx + 1) * ny * (nz + 1) + (nx + 1) * (ny + 1) * nz
    diag = nx * ny * (nz + 1) + nx * (ny + 1) * nz + (nx + 1) * ny * nz
    return {"n_verts": nv, "n_tets": 5 * nx * ny * nz, "n_edges": axis + diag}


# --------------------------------------------------------------------------
# element blocks
# --------------------------------------------------------------------------

def shape_gradients(pos: np.ndarray, tets: np.ndarray):
    """Per-tet volume and gradients of the 4 linear shape functions, (n,) and (n,4,3)."""
    x = pos[tets]
    dm = np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=-1)
    vol = np.abs(np.linalg.det(dm)) / 6.0
    inv = np.linalg.inv(dm)                 # rows: grad N_1..N_3
    grads = np.empty((tets.shape[0], 4, 3))
    grads[:, 1:] = inv
    grads[:, 0] = -inv.sum(axis=1)
    return vol, grads


def linear_stiffness(vol, grads, mu, lam):
    """Rest-pose linear-elastic stiffness blocks K0[n,a,b] (3x3), psi = mu eps:eps + lam/2 tr(eps)^2."""
    gg = np.einsum("nai,nbi->nab", grads, grads)
    eye = np.eye(3)
    k = mu * gg[:, :, :, None, None] * eye
    k = k + mu * np.einsum("nbm,nap->nabmp", grads, grads)
    k = k + lam * np.einsum("nam,nbp->nabmp", grads, grads)
    return k * vol[:, None, None, None, None]


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform rotations from normalised 4-D Gaussian quaternions (Shoemake)."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    r = np.empty((n, 3, 3))
    r[:, 0, 0] = 1 - 2 * (y * y + z * z)
    r[:, 0, 1] = 2 * (x * y - z * w)
    r[:, 0, 2] = 2 * (x * z + y * w)
    r[:, 1, 0] = 2 * (x * y + z * w)
    r[:, 1, 1] = 1 - 2 * (x * x + z * z)
    r[:, 1, 2] = 2 * (y * z - x * w)
    r[:, 2, 0] = 2 * (x * z - y * w)
    r[:, 2, 1] = 2 * (y * z + x * w)
    r[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def elastic_blocks(pos, tets, rot, mu, lam, rho, h, out=None, chunk=1 << 11, progress=None, workers=None):
    """12x12 row-major element blocks (DoF order 3a+k): R K0 R^T + rho V/(4 h^2) I, symmetrised.

    Chunks of elements are independent (the rotations are drawn beforehand),
    so they are computed on a pool of threads; the result does not depend on
    the pool.  ``progress(done, total)`` is called after every 1024 chunks, when given."""
    from concurrent.futures import ThreadPoolExecutor
    n = tets.shape[0]
    if out is None:
        out = np.empty((n, 144), dtype=np.float64)

    def one(s):
        e = slice(s, min(n, s + chunk))
        vol, grads = shape_gradients(pos, tets[e])
        # R K0 R^T from the rotated gradients q_a = R grad N_a (R R^T = I):
        # block (a,b) = V (mu (grad N_a . grad N_b) I + mu q_b q_a^T + lam q_a q_b^T)
        # elementwise products summed in a fixed order (no BLAS: the same bits in every thread)
        r = rot[e]
        q = (grads[:, :, None, 0] * r[:, None, :, 0] + grads[:, :, None, 1] * r[:, None, :, 1]
             + grads[:, :, None, 2] * r[:, None, :, 2])                # (m,4,3): q_a = R grad N_a
        gg = (grads[:, :, None, 0] * grads[:, None, :, 0] + grads[:, :, None, 1] * grads[:, None, :, 1]
              + grads[:, :, None, 2] * grads[:, None, :, 2])           # (m,4,4)
        blk = (mu * q.transpose(0, 2, 1)[:, None, :, :, None]) * q[:, :, None, None, :]
        blk += (lam * q)[:, :, :, None, None] * q[:, None, None, :, :]
        idx = np.arange(3)
        blk[:, :, idx, :, idx] += mu * gg[None]                        # (3,m,4,4) on the k = l diagonal
        blk *= vol[:, None, None, None, None]
        blk = blk.reshape(-1, 12, 12)
        blk[:, np.arange(12), np.arange(12)] += (rho * vol / (4.0 * h * h))[:, None]
        blk = 0.5 * (blk + np.swapaxes(blk, 1, 2))
        out[e] = blk.reshape(-1, 144)

    starts = list(range(0, n, chunk))
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        for ci, _ in enumerate(ex.map(one, starts)):
            if progress is not None and ci % 1024 == 0 and ci > 0:
                progress(starts[ci], n)
    return out


def lumped_mass(tets, vol, rho, n_verts):
    return np.bincount(tets.ravel().astype(np.int64), weights=np.repeat(rho * vol / 4.0, 4),
                       minlength=n_verts)


# --------------------------------------------------------------------------
# tags
# --------------------------------------------------------------------------

def fourier_field(rng: np.random.Generator, n_modes: int = 4):
    """Smooth scalar field: sum of n_modes cosines, 1-3 cycles per unit length."""
    amp = rng.standard_normal(n_modes)
    d = rng.standard_normal((n_modes, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    k = d * rng.uniform(1.0, 3.0, size=(n_modes, 1))
    phase = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    return {"amp": amp, "k": k, "phase": phase}


def eval_field(field, pos, shift=None):
    """The field at each position, summed in a fixed order without BLAS (whose
    rounding can depend on how many threads call it), so that tags drawn from
    it are the same on every host and in every thread."""
    p = pos if shift is None else pos - shift[None, :]
    out = np.zeros(p.shape[0])
    for m in range(field["amp"].shape[0]):
        k = field["k"][m]
        arg = 2.0 * math.pi * (p[:, 0] * k[0] + p[:, 1] * k[1] + p[:, 2] * k[2]) + field["phase"][m]
        out += field["amp"][m] * np.cos(arg)
    return out


def rank_tags(values: np.ndarray, frac: float) -> np.ndarray:
    """1 for the floor(frac*E) edges with the smallest value (ties by edge id), else 0."""
    order = np.argsort(values, kind="stable")
    tags = np.zeros(values.shape[0], dtype=np.uint8)
    tags[order[: int(math.floor(frac * values.shape[0]))]] = 1
    return tags


def edge_tags(field, pos, edges, frac, shift=None):
    f = eval_field(field, pos, shift)
    return rank_tags(0.5 * (f[edges[:, 0]] + f[edges[:, 1]]), frac)


# --------------------------------------------------------------------------
# problems
# --------------------------------------------------------------------------

def grid_problem(n: int, seed: int, frac: float, young: float = YOUNG, poisson: float = POISSON,
                 rho: float = DENSITY, h: float = H_STEP, log=None) -> dict:
    """Unit cube as an n^3 grid of cubes, 5 tets each, co-rotated stiffness + lumped mass.

    ``log(message)`` receives a line after each generation step, when given."""
    say = log if log is not None else (lambda m: None)
    pos, tets = box_mesh(n, n, n, 1.0 / n)
    nv = pos.shape[0]
    edges = mesh_edges(tets, nv)
    say(f"mesh: {nv} vertices, {tets.shape[0]} tets, {edges.shape[0]} edges")
    mu, lam = lame(young, poisson)
    rot = random_rotations(rng_for(seed, S_ROT), tets.shape[0])
    elem_h = elastic_blocks(pos, tets, rot, mu, lam, rho, h,
                            progress=lambda d, t: say(f"element blocks {d}/{t}"))
    say("element blocks done")
    vol, _ = shape_gradients(pos, tets)
    field = fourier_field(rng_for(seed, S_FIELD))
    tags = edge_tags(field, pos, edges, frac)
    g = rng_for(seed, S_GRAD).standard_normal((nv, 3))
    return {
        "name": f"grid{n}", "n_verts": nv, "pos": pos, "edges": edges, "tags": tags,
        "elem_verts": tets, "elem_H": elem_h, "g": g, "h": h,
        "mass": lumped_mass(tets, vol, rho, nv), "field": field, "frac": frac, "seed": seed,
    }


def boundary_triangles(tets: np.ndarray, on_face: np.ndarray) -> np.ndarray:
    """Faces of the tets whose three vertices all satisfy on_face[v] (one per boundary triangle)."""
    t = tets.astype(np.int64)
    faces = np.concatenate([t[:, [0, 1, 2]], t[:, [0, 1, 3]], t[:, [0, 2, 3]], t[:, [1, 2, 3]]], axis=0)
    keep = on_face[faces].all(axis=1)
    f = np.sort(faces[keep], axis=1)
    return np.unique(f, axis=0)


def contact_blocks(rng: np.random.Generator, n: int) -> np.ndarray:
    """Point-triangle barrier blocks J^T diag(s) J: J ~ N(0,1) 3x12, s_i = 10^U(2,6) per row."""
    j = rng.standard_normal((n, 3, 12))
    s = 10.0 ** rng.uniform(2.0, 6.0, size=(n, 3))
    blk = np.einsum("nik,ni,nil->nkl", j, s, j)
    return (0.5 * (blk + np.swapaxes(blk, 1, 2))).reshape(n, 144)


def contact_problem(seed: int, n_bodies: int = 96, body=(4, 8, 24), n_contacts: int = 250_000,
                    frac_range=(0.2, 0.9), young: float = YOUNG, poisson: float = POISSON,
                    rho: float = DENSITY, h: float = H_STEP) -> dict:
    """A row of deformable cuboids pressed together, with point-triangle barrier blocks.

    Bodies are body[0] x body[1] x body[2] grids of cubes of edge 1/8 m, 5 tets
    per cube, the short axis along the row (x), gap 1/16 m, each body shifted
    by U(-1/16, 1/16) m in y and z.  Contact elements [p, t0, t1, t2] pair a
    vertex of one body's facing face with a triangle of the neighbouring
    body's facing face whose centroid lies within 1.5 cube edges in (y, z),
    both directions; n_contacts of all such candidates are drawn without
    replacement.  Each body gets its own collapsible fraction q_b ~
    U(frac_range) of its edges (ranked by the smooth field); afterwards every
    edge touching a contact element's vertex is protected.
    """
    nx, ny, nz = body
    cell = 1.0 / 8.0
    gap = 1.0 / 16.0
    rng_j = rng_for(seed, S_JITTER)
    jitter = rng_j.uniform(-gap, gap, size=(n_bodies, 2))
    pos0, tets0 = box_mesh(nx, ny, nz, cell)
    nvb = pos0.shape[0]
    edges0 = mesh_edges(tets0, nvb)
    pos = np.concatenate([pos0 + np.array([b * (nx * cell + gap), jitter[b, 0], jitter[b, 1]])
                          for b in range(n_bodies)])
    tets = np.concatenate([tets0 + b * nvb for b in range(n_bodies)]).astype(np.int32)
    nv = pos.shape[0]

    # facing faces and their candidate pairs
    tri_lo = boundary_triangles(tets0, np.isclose(pos0[:, 0], 0.0))            # -x face of a body
    tri_hi = boundary_triangles(tets0, np.isclose(pos0[:, 0], nx * cell))      # +x face
    v_lo = np.flatnonzero(np.isclose(pos0[:, 0], 0.0))
    v_hi = np.flatnonzero(np.isclose(pos0[:, 0], nx * cell))
    cand = []
    for b in range(n_bodies - 1):
        for pts, tri, pb, tb in ((v_hi, tri_lo, b, b + 1), (v_lo, tri_hi, b + 1, b)):
            p_yz = pos[pts + pb * nvb, 1:]
            c_yz = pos[tri + tb * nvb][:, :, 1:].mean(axis=1)
            d2 = ((p_yz[:, None, :] - c_yz[None, :, :]) ** 2).sum(axis=2)
            ip, it = np.nonzero(d2 <= (1.5 * cell) ** 2)
            cand.append(np.concatenate([(pts[ip] + pb * nvb)[:, None], tri[it] + tb * nvb], axis=1))
    cand = np.concatenate(cand).astype(np.int32)
    rng_c = rng_for(seed, S_CONTACT)
    pick = np.sort(rng_c.choice(cand.shape[0], size=min(n_contacts, cand.shape[0]), replace=False))
    contacts = cand[pick]

    mu, lam = lame(young, poisson)
    rot = random_rotations(rng_for(seed, S_ROT), tets.shape[0])
    elem_h = np.concatenate([elastic_blocks(pos, tets, rot, mu, lam, rho, h),
                             contact_blocks(rng_c, contacts.shape[0])])
    vol, _ = shape_gradients(pos, tets)

    rng_f = rng_for(seed, S_FIELD)
    field = fourier_field(rng_f)
    fracs = rng_f.uniform(frac_range[0], frac_range[1], size=n_bodies)
    f = eval_field(field, pos)
    edges = np.concatenate([edges0 + b * nvb for b in range(n_bodies)]).astype(np.int32)
    tags = np.concatenate([rank_tags(0.5 * (f[edges0[:, 0] + b * nvb] + f[edges0[:, 1] + b * nvb]), fracs[b])
                           for b in range(n_bodies)])
    touched = np.zeros(nv, dtype=bool)
    touched[contacts.ravel()] = True
    tags[touched[edges[:, 0]] | touched[edges[:, 1]]] = 0

    g = rng_for(seed, S_GRAD).standard_normal((nv, 3))
    return {
        "name": "contact", "n_verts": nv, "pos": pos, "edges": edges, "tags": tags,
        "elem_verts": np.concatenate([tets, contacts]).astype(np.int32), "elem_H": elem_h, "g": g, "h": h,
        "mass": lumped_mass(tets, vol, rho, nv), "field": field, "frac": fracs, "seed": seed,
        "n_tets": tets.shape[0], "n_contacts": contacts.shape[0], "body_verts": nvb,
    }


def drift_fraction(p: dict, delta: float, sample=None) -> float:
    """Fraction of edge tags that change when the field moves by delta along p's drift
    direction (on the edge subset ``sample``, ranked within it, when given)."""
    u = p["drift_dir"]
    edges = p["edges"] if sample is None else p["edges"][sample]
    t0 = edge_tags(p["field"], p["pos"], edges, p["frac"])
    t1 = edge_tags(p["field"], p["pos"], edges, p["frac"], shift=delta * u)
    return float(np.mean(t1 != t0))


def calibrate_drift(p: dict, target: float = 0.10, iters: int = 16, max_sample: int = 1 << 20) -> float:
    """Step length delta whose one-step tag flip fraction is about ``target`` (bisection on
    the host over a seeded sample of at most max_sample edges)."""
    m = p["edges"].shape[0]
    sample = None
    if m > max_sample:
        sample = np.sort(rng_for(p["seed"], S_DRIFT).choice(m, size=max_sample, replace=False))
    lo, hi = 0.0, 1.0
    while drift_fraction(p, hi, sample) < target and hi < 64.0:
        hi *= 2.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if drift_fraction(p, mid, sample) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def drift_tags(p: dict, it: int) -> np.ndarray:
    """Tags of system ``it`` of a drifting sequence: the field advected by it * delta along the
    seeded direction (a stand-in for the activity moving between Newton iterations)."""
    shift = it * p["drift_delta"] * p["drift_dir"]
    return edge_tags(p["field"], p["pos"], p["edges"], p["frac"], shift=shift)


def with_drift(p: dict, target: float = 0.10) -> dict:
    u = rng_for(p["seed"], S_DRIFT).standard_normal(3)
    p["drift_dir"] = u / np.linalg.norm(u)
    p["drift_delta"] = calibrate_drift(p, target)
    return p


def deformation_states(p: dict, wave_amp: float = 2e-4, wave_cycles: float = 3.0, width: float = 0.15,
                       background: float = 1e-6) -> tuple[np.ndarray, np.ndarray]:
    """Positions at two successive Newton iterates (previous, current) of the mesh of p.

    Both are rigid motions (a random rotation about the body's centre plus a
    translation, different for the two states) of the rest shape plus a
    displacement field: a smooth background of amplitude ``background`` at
    one cycle per unit length, changing between the two states, and in the
    current state an elastic wave packet of amplitude ``wave_amp`` with
    ``wave_cycles`` cycles per unit length under a Gaussian envelope of width
    ``width`` around a random point.  The Green strain increment is then
    large inside the packet and small elsewhere (rigid motions leave G
    unchanged).
    """
    rng = rng_for(p["seed"], S_STATES)
    rest = p["pos"]
    c = rest.mean(axis=0)
    lo, hi = rest.min(axis=0), rest.max(axis=0)

    def smooth(k_dir, phase):
        arg = 2.0 * math.pi * (rest @ k_dir) + phase
        return np.sin(arg)[:, None] * rng.standard_normal(3)[None, :]

    def rigid(x):
        r = random_rotations(rng, 1)[0]
        return (x - c) @ r.T + c + rng.uniform(-0.1, 0.1, size=3)

    d1 = rng.standard_normal(3)
    d1 /= np.linalg.norm(d1)
    d2 = rng.standard_normal(3)
    d2 /= np.linalg.norm(d2)
    u_prev = background * smooth(d1, rng.uniform(0, 2 * math.pi))
    u_cur = background * smooth(d2, rng.uniform(0, 2 * math.pi))
    centre = lo + rng.uniform(0.25, 0.75, size=3) * (hi - lo)
    kw = rng.standard_normal(3)
    kw *= wave_cycles / np.linalg.norm(kw)
    env = np.exp(-np.sum((rest - centre) ** 2, axis=1) / (width * width))
    pol = rng.standard_normal(3)
    pol /= np.linalg.norm(pol)
    u_cur = u_cur + wave_amp * (env * np.sin(2.0 * math.pi * (rest @ kw)))[:, None] * pol[None, :]
    return rigid(rest + u_prev), rigid(rest + u_cur)


def material(young: float = YOUNG, poisson: float = POISSON, rho: float = DENSITY, h: float = H_STEP) -> dict:
    mu, lam = lame(young, poisson)
    return {"mu": mu, "lam": lam, "rho": rho, "h": h}


def newton_state(p: dict, spin: float = 1.0, wave_speed: float = 0.2, wave_cycles: float = 3.0,
                 width: float = 0.15, gravity: bool = True):
    """Start of one implicit time step on the mesh of p: positions x^t (the rest
    shape), velocities v^t (a rigid spin of ``spin`` rad/s about a random axis
    through the centre plus a transverse elastic wave packet of peak speed
    ``wave_speed`` m/s, ``wave_cycles`` cycles per unit length, Gaussian
    envelope of width ``width`` around a random point) and external forces
    f_ext (gravity on the lumped masses, or None).  The strain increment is
    then large inside the packet and near zero elsewhere."""
    rng = rng_for(p["seed"], S_NEWTON)
    rest = p["pos"]
    c = rest.mean(axis=0)
    lo, hi = rest.min(axis=0), rest.max(axis=0)
    axis = rng.standard_normal(3)
    axis /= np.linalg.norm(axis)
    v = spin * np.cross(axis[None, :], rest - c)
    centre = lo + rng.uniform(0.25, 0.75, size=3) * (hi - lo)
    kw = rng.standard_normal(3)
    kw *= wave_cycles / np.linalg.norm(kw)
    pol = np.cross(kw, rng.standard_normal(3))
    pol /= np.linalg.norm(pol)
    env = np.exp(-np.sum((rest - centre) ** 2, axis=1) / (width * width))
    v = v + wave_speed * (env * np.sin(2.0 * math.pi * (rest @ kw)))[:, None] * pol[None, :]
    f = None
    if gravity:
        f = np.zeros_like(rest)
        f[:, 1] = -GRAVITY * p["mass"]
    return rest.copy(), v, f


# The measured workloads.
CONFIGS = {
    "c1": dict(n=8, seed=1, frac=0.7),      # 729 vertices, 2560 tets, FP64, PCG rtol 1e-10
    "c2": dict(n=64, seed=2, frac=0.6),     # 274,625 vertices, 1.31M tets, FP64 and mixed
    "c3": dict(contact=True, seed=3),       # 96 bodies, 108,000 vertices, 368,640 tets + 250k contacts
    "c4": dict(n=32, seed=4, frac=0.7),     # 35,937 vertices, adjoint
    "c5": dict(n=128, seed=5, frac=0.6, drift=True),   # 2.15M vertices, 10 drifting systems
}


def make_config(name: str, log=None) -> dict:
    c = CONFIGS[name]
    if c.get("contact"):
        p = contact_problem(c["seed"])
    else:
        p = grid_problem(c["n"], c["seed"], c["frac"], log=log)
    if c.get("drift"):
        with_drift(p)
        if log is not None:
            log(f"drift step {p['drift_delta']:.4g} along {np.round(p['drift_dir'], 3).tolist()}")
    p["name"] = name
    return p


def adjoint_seed(p: dict) -> np.ndarray:
    return rng_for(p["seed"], S_W).standard_normal((p["n_verts"], 3))


def random_graph(rng: np.random.Generator, n: int, m: int, p_tag: float = 0.5):
    """Random multigraph with self-loops and duplicates, for aggregation tests."""
    if n == 0:
        return np.zeros((0, 2), np.int32), np.zeros(0, np.uint8)
    e = rng.integers(0, n, size=(m, 2)).astype(np.int32)
    t = (rng.random(m) < p_tag).astype(np.uint8)
    return e, t
