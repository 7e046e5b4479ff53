"""Helpers for the GPU parity tests: device copies of a synthetic problem and
conversions of library outputs for comparison with the oracle."""
from __future__ import annotations

import functools
import sys

import numpy as np
import scipy.sparse as sp

from paper_2605_04773_amd import synth

U64 = np.finfo(np.float64).eps / 2
U32 = np.finfo(np.float32).eps / 2


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gamma(k, u=U64):
    return k * u / (1 - k * u)


def binding():
    from paper_2605_04773_amd import agc   # raises if libagc.so is missing
    return agc


@functools.lru_cache(maxsize=None)
def problem(name: str) -> dict:
    """The named synthetic problem, generated once per test process (treat as read-only)."""
    log(f"[gen] {name}")
    if name == "tiny":
        return synth.grid_problem(2, 21, 0.5)
    if name == "g3":
        return synth.grid_problem(3, 33, 0.6)
    return synth.make_config(name)


class Dev:
    """A synthetic problem copied to the GPU with its mesh handle."""

    def __init__(self, ctx, p, f32=False):
        import torch
        agc = binding()
        self.p = p
        self.ctx = ctx
        dev = ctx.device
        self.t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)
        self.edges = self.t(p["edges"], torch.int32)
        self.tags = self.t(p["tags"], torch.uint8)
        self.ev = self.t(p["elem_verts"], torch.int32)
        self.eh = self.t(p["elem_H"], torch.float64)
        self.eh32 = self.eh.to(torch.float32) if f32 else None
        self.g = self.t(p["g"], torch.float64)
        self.rest = self.t(p["pos"], torch.float64)
        self.mesh = agc.agc_mesh_create(ctx, p["n_verts"], self.ev)

    def problem(self, tags=None):
        agc = binding()
        return agc.make_problem(self.mesh, self.edges, self.tags if tags is None else tags, self.eh, self.g,
                                self.rest)


def to_scipy(mat) -> sp.csr_matrix:
    rp, ci, vals = mat.to_bsr()
    v = vals.double().cpu().numpy()
    n = mat.n_rows
    return sp.bsr_matrix((v, ci.cpu().numpy(), rp.cpu().numpy()), shape=(3 * n, 3 * n)).tocsr()


def bsr_numpy(mat):
    rp, ci, vals = mat.to_bsr()
    return rp.cpu().numpy().astype(np.int64), ci.cpu().numpy().astype(np.int64), vals.double().cpu().numpy()
