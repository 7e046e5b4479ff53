"""Checks that pin the oracle to facts fixed by the paper and by mathematics.

Each ``check_*`` raises AssertionError when the pin does not hold.  The
oracle tests run them against the oracle; the mutant tests run them against
copies of the oracle with a planted mistake and expect them to fail.
"""
from __future__ import annotations

import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def hash_str(h: int, width: int) -> str:
    """Bit string with lane 0 as the rightmost character."""
    return format(h, "0{}b".format(width))


def edges_from_direct_hashes(strings):
    """Collapsible edges implied by direct hashes (bit u of node v set, u != v)."""
    width = len(strings[0])
    edges = set()
    for v, s in enumerate(strings):
        h = int(s, 2)
        for u in range(width):
            if u != v and (h >> u) & 1:
                edges.add((min(u, v), max(u, v)))
    return np.array(sorted(edges), dtype=np.int64)


# --------------------------------------------------------------------- aggregation

def check_map_valid(n, edges, tags, m, n_c):
    """Labels constant along collapsible edges, reps increasing, components connected."""
    m = np.asarray(m, dtype=np.int64)
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    tags = np.asarray(tags).reshape(-1)
    assert m.shape == (n,)
    if n == 0:
        assert n_c == 0
        return
    assert m.min() == 0 and m.max() == n_c - 1
    col = edges[tags == 1]
    assert (m[col[:, 0]] == m[col[:, 1]]).all(), "collapsible edge joins two aggregates"
    first = np.full(n_c, n, dtype=np.int64)
    np.minimum.at(first, m, np.arange(n))
    assert (np.diff(first) > 0).all(), "labels not ordered by smallest member id"
    # each aggregate is connected through collapsible edges (union-find over col)
    parent = np.arange(n)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a
    for a, b in col.tolist():
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    roots = np.array([find(v) for v in range(n)])
    # same aggregate <=> same union-find root
    assert len(np.unique(roots)) == n_c
    pair = np.unique(np.stack([roots, m], 1), axis=0)
    assert pair.shape[0] == n_c, "aggregate split or merged across components"


# --------------------------------------------------------------------- Galerkin

def check_prolongation(P, m, n_c):
    """P^T 1 = aggregate sizes (per DoF) and P^T P = diag(sizes)."""
    sizes = np.bincount(np.asarray(m, dtype=np.int64), minlength=n_c)
    ones = np.ones(P.shape[0])
    assert np.array_equal(P.T @ ones, np.repeat(sizes, 3).astype(float))
    ptp = (P.T @ P)
    ptp = ptp.toarray() if hasattr(ptp, "toarray") else ptp
    assert np.array_equal(ptp, np.diag(np.repeat(sizes, 3).astype(float)))


def element_bilinear(elem_verts, elem_H, u, v):
    """sum_e (S_e u)^T H_e (S_e v) for fine vectors u, v of shape (n, 3); no assembled matrix."""
    ev = np.asarray(elem_verts, dtype=np.int64)
    ue = np.asarray(u)[ev].reshape(-1, 12)
    ve = np.asarray(v)[ev].reshape(-1, 12)
    he = np.asarray(elem_H).reshape(-1, 12, 12)
    return float(np.einsum("ni,nij,nj->", ue, he, ve))


def check_energy_identity(A_c, b_c, elem_verts, elem_H, g, m, n_c, seed=0, rtol=1e-11):
    """z^T A_c y = sum_e (S_e P z)^T H_e (S_e P y) and y^T b_c = (P y)^T g."""
    rng = np.random.default_rng(seed)
    m = np.asarray(m, dtype=np.int64)
    for _ in range(3):
        y = rng.standard_normal((n_c, 3))
        z = rng.standard_normal((n_c, 3))
        lhs = z.reshape(-1) @ (A_c @ y.reshape(-1))
        rhs = element_bilinear(elem_verts, elem_H, z[m], y[m])
        scale = element_bilinear(elem_verts, np.abs(np.asarray(elem_H)), np.abs(z[m]), np.abs(y[m]))
        assert abs(lhs - rhs) <= rtol * scale, (lhs, rhs)
        lb = y.reshape(-1) @ np.asarray(b_c).reshape(-1)
        rb = float(np.sum(y[m] * g))
        assert abs(lb - rb) <= rtol * float(np.sum(np.abs(y[m] * g)))


def check_all_collapsible_closed_form(A_c, b_c, g, total_mass, h, n_terms_bound, abs_scale):
    """tau = 1 on a connected body: A_c = (M_tot/h^2) I_3 and b_c = sum g (translations are K-null)."""
    a = A_c.toarray() if hasattr(A_c, "toarray") else np.asarray(A_c)
    assert a.shape == (3, 3)
    u = np.finfo(np.float64).eps / 2
    gamma = n_terms_bound * u / (1 - n_terms_bound * u)
    assert np.abs(a - (total_mass / h ** 2) * np.eye(3)).max() <= gamma * abs_scale * 4
    assert np.allclose(np.asarray(b_c).reshape(3), np.asarray(g).sum(axis=0), rtol=0, atol=1e-9 * np.abs(g).sum())


# --------------------------------------------------------------------- adjoint

def check_adjoint_identities(L, g, dg, elem_H, dH, rtol=1e-10):
    """Linearity in g: L = <dL/dg, g>.  Degree -1 homogeneity in H: sum_e <dL/dH_e, H_e> = -L."""
    lin = float(np.sum(dg * g))
    assert abs(lin - L) <= rtol * max(abs(L), np.abs(dg * g).sum()), (lin, L)
    euler = float(np.sum(np.asarray(dH).reshape(-1) * np.asarray(elem_H).reshape(-1)))
    assert abs(euler + L) <= rtol * max(abs(L), np.abs(np.asarray(dH).reshape(-1) * np.asarray(elem_H).reshape(-1)).sum()), (euler, L)


# --------------------------------------------------------------- affine order

def supplement_node_order(sizes, threshold):
    """Node order and flat 3-block offsets built from the supplement's Alg. 3
    and its index formulas, without the oracle.

    Alg. 3: a node with more than ``threshold`` members is a 12-DoF node and
    gets the sort key i + n_c, any other node the key i; a pair sort of
    (key, node index) puts the 3-DoF nodes first, each kind in label order;
    a node's new label is its position in that sorted order.  The row index
    formula of the supplement (Sec. 2, after Alg. 4) places sub-block K of a
    12-DoF node at r = n3 + (new - n3) * 4 + floor(K / 4) and its column at
    c = n3 + (new - n3) * 4 + K % 4; a 3-DoF node's global index is its new
    label.  Returns (new_label, offset, n3) with offset the first flat
    3-block of every node."""
    sizes = np.asarray(sizes)
    n_c = sizes.shape[0]
    keys = [i + n_c if sizes[i] > threshold else i for i in range(n_c)]
    indices = sorted(range(n_c), key=lambda i: keys[i])      # the SortPairs step (keys are distinct)
    new_label = [0] * n_c
    for pos, i in enumerate(indices):
        new_label[i] = pos
    n3 = sum(1 for i in range(n_c) if sizes[i] <= threshold)
    offset = []
    for i in range(n_c):
        if sizes[i] > threshold:
            rows = {n3 + (new_label[i] - n3) * 4 + K // 4 for K in range(16)}
            cols = {n3 + (new_label[i] - n3) * 4 + K % 4 for K in range(16)}
            assert rows == cols and len(rows) == 4
            offset.append(min(rows))
        else:
            offset.append(new_label[i])
    return np.array(new_label), np.array(offset), n3


def check_affine_order(classify, map_, n_c, threshold):
    """classify(map, n_c, threshold)['new_label' / 'offset' / 'n3'] follow Alg. 3
    and the supplement's index formulas; the flat 3-blocks tile [0, n3 + 4 n12)."""
    sizes = np.bincount(np.asarray(map_, dtype=np.int64), minlength=n_c)
    want_lab, want_off, want_n3 = supplement_node_order(sizes, threshold)
    cls = classify(np.asarray(map_), n_c, threshold)
    assert int(cls["n3"]) == want_n3, "3-DoF node count"
    assert np.array_equal(np.asarray(cls["new_label"]), want_lab), "node order differs from Alg. 3"
    assert np.array_equal(np.asarray(cls["offset"]), want_off), "flat offsets differ from the index formulas"
    big = sizes > threshold
    width = np.where(big, 4, 1)
    cover = np.zeros(want_n3 + 4 * int(big.sum()), np.int64)
    for c in range(n_c):
        cover[want_off[c]: want_off[c] + width[c]] += 1
    assert (cover == 1).all(), "flat 3-blocks overlap or leave gaps"
