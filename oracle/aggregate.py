"""Oracle: fine-to-coarse aggregation (test infrastructure only).

Definition (Sec. 4.1 "Adaptive Coarsening via Edge Collapse"): fine nodes are
coalesced into one super-node exactly when a path of collapsible edges
(tag 1) joins them.  The supplement's hashing scheme (Sec. 1, Alg. 1-2) finds
these components group by group and applies itself recursively "until a
minimal set of DoF is obtained" (Sec. 1.2), so at its fixed point the
super-nodes are the connected components of the graph of collapsible edges.

Label order (supplement Alg. 2 and Sec. 1.3): inside a group the coarse index
of a node is the number of elected (lowest-lane) members below it, and the
global index adds an exclusive prefix sum over groups.  Groups are contiguous
id ranges, so coarse ids are increasing in the smallest fine id of each
component, and every level of the recursion keeps that order.  The canonical
map is therefore: sort the components by their smallest vertex id; the label
of a component is its position in that order.

Three implementations live here:
* ``components``      - scipy's connected components, relabelled canonically
                        (the library routine serves as the graph step);
* ``components_bfs``  - breadth-first search in plain Python (small inputs);
* ``hash_levels``     - the supplement's group-hash procedure (Alg. 1 direct
                        neighbour bits, Alg. 2 bitwise-OR closure, elected-lane
                        popcount and group prefix sum), repeated level by
                        level on the coarse graph (small inputs).
"""
from __future__ import annotations

from collections import deque

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg


def _collapsible(n_verts: int, edges: np.ndarray, tags: np.ndarray) -> np.ndarray:
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    tags = np.asarray(tags).reshape(-1)
    if edges.shape[0] != tags.shape[0]:
        raise ValueError("edges and tags differ in length")
    if edges.size and (edges.min() < 0 or edges.max() >= n_verts):
        raise ValueError("edge endpoint out of range")
    if tags.size and not np.isin(tags, (0, 1)).all():
        raise ValueError("tags must be 0 or 1")
    return edges[tags == 1]


def canonical_labels(raw: np.ndarray) -> tuple[np.ndarray, int]:
    """Relabel arbitrary component ids so that labels follow the smallest member id."""
    n = raw.shape[0]
    if n == 0:
        return np.zeros(0, np.int32), 0
    first = {}
    out = np.empty(n, np.int32)
    nxt = 0
    for v in range(n):                      # v ascending: first visit = smallest member
        r = int(raw[v])
        if r not in first:
            first[r] = nxt
            nxt += 1
        out[v] = first[r]
    return out, nxt


def components(n_verts: int, edges, tags) -> tuple[np.ndarray, int]:
    """Canonical fine-to-coarse map via a library connected-components step."""
    col = _collapsible(n_verts, edges, tags)
    if n_verts == 0:
        return np.zeros(0, np.int32), 0
    g = sp.coo_matrix((np.ones(col.shape[0]), (col[:, 0], col[:, 1])), shape=(n_verts, n_verts))
    _, raw = csg.connected_components(g, directed=False)
    # vectorised canonical relabel: rank of each component's smallest vertex
    n_c = int(raw.max()) + 1
    first_v = np.full(n_c, n_verts, dtype=np.int64)
    np.minimum.at(first_v, raw, np.arange(n_verts))
    order = np.argsort(first_v, kind="stable")
    rank = np.empty(n_c, np.int64)
    rank[order] = np.arange(n_c)
    return rank[raw].astype(np.int32), n_c


def components_bfs(n_verts: int, edges, tags) -> tuple[np.ndarray, int]:
    """Same map by breadth-first search, visiting start vertices in id order."""
    col = _collapsible(n_verts, edges, tags)
    adj = [[] for _ in range(n_verts)]
    for a, b in col.tolist():
        adj[a].append(b)
        adj[b].append(a)
    out = np.full(n_verts, -1, np.int32)
    label = 0
    for s in range(n_verts):
        if out[s] >= 0:
            continue
        out[s] = label
        q = deque([s])
        while q:
            u = q.popleft()
            for w in adj[u]:
                if out[w] < 0:
                    out[w] = label
                    q.append(w)
        label += 1
    return out, label


# ---------------------------------------------------------------------------
# The supplement's group-hash procedure (small inputs only).
# ---------------------------------------------------------------------------

def direct_hashes(n_nodes: int, col_edges: np.ndarray, group_size: int) -> list[int]:
    """Supplement Alg. 1: own lane bit plus the lane bits of collapsible neighbours in the same group."""
    h = [1 << (v % group_size) for v in range(n_nodes)]
    for a, b in np.asarray(col_edges, dtype=np.int64).reshape(-1, 2).tolist():
        if a == b or a // group_size != b // group_size:
            continue
        h[a] |= 1 << (b % group_size)
        h[b] |= 1 << (a % group_size)
    return h


def _one_level(n_nodes: int, col_edges: np.ndarray, group_size: int):
    """Supplement Alg. 2 for every group: OR-closure, elected lanes, popcount index, group prefix sum."""
    h = direct_hashes(n_nodes, col_edges, group_size)
    n_groups = (n_nodes + group_size - 1) // group_size
    closed = list(h)
    local = [0] * n_nodes
    counts = [0] * n_groups
    for grp in range(n_groups):
        lo, hi = grp * group_size, min(n_nodes, (grp + 1) * group_size)
        for v in range(lo, hi):
            lane = v % group_size
            con = h[v]
            visited = 1 << lane
            while True:
                todo = visited ^ con                      # visited is a subset of con
                if todo == 0:
                    break
                nxt = (todo & -todo).bit_length() - 1          # first set bit
                visited |= 1 << nxt
                con |= h[lo + nxt]
            closed[v] = con
        elected = 0
        for v in range(lo, hi):
            lane = v % group_size
            if closed[v] & ((1 << lane) - 1) == 0:           # lowest lane of its component
                elected |= 1 << lane
        counts[grp] = bin(elected).count("1")
        for v in range(lo, hi):
            lane = v % group_size
            # index = elected lanes below the first set bit of v's closed hash
            # (supplement Sec. 1.3: the first '1' of the hash fixes the order)
            first = (closed[v] & -closed[v]).bit_length() - 1
            local[v] = bin(elected & ((1 << first) - 1)).count("1")
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    m = np.array([offsets[v // group_size] + local[v] for v in range(n_nodes)], dtype=np.int64)
    return m, int(offsets[-1]), h, closed


def hash_levels(n_verts: int, edges, tags, group_size: int, max_levels: int = 64):
    """Apply the group-hash step level by level on the coarse graph.

    Returns (map, n_coarse, converged, per-level direct hashes).  Converged means
    that no collapsible edge joins two different coarse nodes any more; only then
    is the result the fixed point the paper describes.
    """
    col = _collapsible(n_verts, edges, tags)
    fine_to = np.arange(n_verts, dtype=np.int64)
    n_nodes = n_verts
    cur = col.copy()
    levels = []
    for _ in range(max_levels):
        cur = cur[cur[:, 0] != cur[:, 1]] if cur.size else cur
        if cur.shape[0] == 0:
            return fine_to.astype(np.int32), n_nodes, True, levels
        m, n_next, h, _ = _one_level(n_nodes, cur, group_size)
        levels.append(h)
        if n_next == n_nodes:
            return fine_to.astype(np.int32), n_nodes, False, levels
        fine_to = m[fine_to]
        cur = m[cur]
        n_nodes = n_next
    return fine_to.astype(np.int32), n_nodes, False, levels


def sizes(map_: np.ndarray, n_c: int) -> np.ndarray:
    return np.bincount(np.asarray(map_, dtype=np.int64), minlength=n_c)


def representatives(map_: np.ndarray, n_c: int) -> np.ndarray:
    """rep[c] = smallest fine vertex of aggregate c."""
    rep = np.full(n_c, np.iinfo(np.int64).max, dtype=np.int64)
    np.minimum.at(rep, np.asarray(map_, dtype=np.int64), np.arange(map_.shape[0]))
    return rep
