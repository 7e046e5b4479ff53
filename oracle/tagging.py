"""Oracle: the Green-strain-increment edge tags (test infrastructure only).

Definition (Sec. 4.2 "Adaptive Coarsening Criterion", Eq. 3): for every
element, with F its deformation gradient and G = (F^T F - I) / 2 its Green
strain, the increment between two successive Newton iterates is
dG = G_i - G_{i-1}.  An edge is protected (tag 0) when any element that
contains it has ||dG||_F above the threshold; every other edge stays
collapsible (tag 1), including an edge that no element contains.

For a linear tetrahedron F = Ds Dm^{-1}, where the columns of Ds (Dm) are the
edge vectors x_1 - x_0, x_2 - x_0, x_3 - x_0 of the deformed (rest) element.
Everything here is float64 and written for reading, not speed: the element
loop is numpy over all elements, the edge rule is a plain set lookup.
"""
from __future__ import annotations

import numpy as np


def deformation_gradients(rest: np.ndarray, x: np.ndarray, tets: np.ndarray) -> np.ndarray:
    """F of every tetrahedron, (n_e, 3, 3): Ds Dm^{-1}."""
    t = tets.astype(np.int64)
    dm = np.stack([rest[t[:, k]] - rest[t[:, 0]] for k in (1, 2, 3)], axis=-1)
    ds = np.stack([x[t[:, k]] - x[t[:, 0]] for k in (1, 2, 3)], axis=-1)
    return ds @ np.linalg.inv(dm)


def green_strain(f: np.ndarray) -> np.ndarray:
    """G = (F^T F - I) / 2 for a stack of F."""
    return 0.5 * (np.swapaxes(f, -1, -2) @ f - np.eye(3))


def strain_increment_norms(rest: np.ndarray, x_cur: np.ndarray, x_prev: np.ndarray,
                           tets: np.ndarray) -> np.ndarray:
    """||G_i - G_{i-1}||_F per element (Eq. 3)."""
    g_cur = green_strain(deformation_gradients(rest, x_cur, tets))
    g_prev = green_strain(deformation_gradients(rest, x_prev, tets))
    d = g_cur - g_prev
    return np.sqrt(np.sum(d * d, axis=(1, 2)))


def tag_edges(rest: np.ndarray, x_cur: np.ndarray, x_prev: np.ndarray, tets: np.ndarray,
              edges: np.ndarray, threshold: float) -> tuple[np.ndarray, np.ndarray]:
    """Edge tags (1 collapsible, 0 protected) and the per-element norms.

    The six edges of every element over the threshold form the protected set;
    an edge of the list is protected when its (unordered) pair is in it."""
    n = int(max(rest.shape[0], 1))
    norms = strain_increment_norms(rest, x_cur, x_prev, tets)
    hot = tets[norms > threshold].astype(np.int64)
    pairs = np.concatenate([hot[:, [a, b]] for a in range(4) for b in range(a + 1, 4)], axis=0)
    protected = np.minimum(pairs[:, 0], pairs[:, 1]) * n + np.maximum(pairs[:, 0], pairs[:, 1])
    e = edges.astype(np.int64)
    keys = np.minimum(e[:, 0], e[:, 1]) * n + np.maximum(e[:, 0], e[:, 1])
    tags = np.where(np.isin(keys, protected), 0, 1).astype(np.uint8)
    tags[e[:, 0] == e[:, 1]] = 1          # a self-loop lies in no element
    return tags, norms
