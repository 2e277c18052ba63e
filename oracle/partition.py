"""Disjoint partitions of the active nodes (paper Section 3).

The paper partitions the 6-neighbour graph of Sigma_A with METIS (Section 3.1),
a third-party tool that is not part of this work. The partitions used here are
integer-only coordinate splits of the same node set:

* octant: part = 4[i >= n0//2] + 2[j >= n1//2] + [k >= n2//2] (box-centre
  planes, nodes on a plane go to the upper side);
* recursive coordinate bisection (RCB): split the current node set along the
  axis of largest index extent (ties x < y < z), ordering nodes by (index on
  that axis, L); the left group takes the first floor(|S| W_l / W) nodes where
  W_l is the weight of the floor(n/2) left parts and W of all n parts (unit
  weights for plain RCB, seeded target weights for weighted RCB). Left parts
  get the lower ids. Weight sums are accumulated left to right.
* recursive graph bisection of the same 6-neighbour graph (a stand-in for the
  graph partitioner of Section 3.1): as RCB, but the current node set is
  ordered by breadth-first distance, inside the subgraph it induces, from a
  pseudo-peripheral node (two sweeps: from the lowest band index to the
  farthest node, lowest index on ties, then from there), ties by band index;
  nodes it cannot reach come last. After the cut, pieces of the right group
  cut off from its largest connected piece (ties: the piece holding the lowest
  band index) join the left group, so both halves of a connected set stay
  connected (the left group is a breadth-first ball plus pieces touching it).

Interface alignment (Section 3.2): a node with an active FD neighbour in
another part moves to the part of the grid node nearest to its closest point
(the node x~ with index floor((CP - lo)/h + 1/2) per axis) when that part
differs; all moves of a pass are made at once; p + 1 passes.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, shortest_path


def octant_partition(band):
    n0, n1, n2 = band.shape
    ijk = band.ijk[: band.n_act]
    return (4 * (ijk[:, 0] >= n0 // 2) + 2 * (ijk[:, 1] >= n1 // 2)
            + (ijk[:, 2] >= n2 // 2)).astype(np.int64)


def rcb_partition(band, n_parts, weights=None):
    if n_parts < 1:
        raise ValueError("n_parts must be >= 1")
    na = band.n_act
    if n_parts > na:
        raise ValueError("more parts than active nodes")
    ijk = band.ijk[:na]
    L = band.lin[:na]
    part = np.full(na, -1, dtype=np.int64)
    w = None if weights is None else [float(x) for x in weights]
    if w is not None and len(w) != n_parts:
        raise ValueError("need one weight per part")

    stack = [(np.arange(na, dtype=np.int64), 0, n_parts)]
    while stack:
        idx, first, n = stack.pop()
        if n == 1:
            part[idx] = first
            continue
        sub = ijk[idx]
        ext = sub.max(axis=0) - sub.min(axis=0)
        axis = int(np.argmax(ext))
        order = np.lexsort((L[idx], sub[:, axis]))
        srt = idx[order]
        nl = n // 2
        if w is None:
            cut = (len(srt) * nl) // n
        else:
            wl = 0.0
            for q in range(first, first + nl):
                wl += w[q]
            wt = 0.0
            for q in range(first, first + n):
                wt += w[q]
            cut = int(math.floor(float(len(srt)) * wl / wt))
        stack.append((srt[:cut], first, nl))
        stack.append((srt[cut:], first + nl, n - nl))
    assert (part >= 0).all()
    return part


def _active_graph(band):
    na = band.n_act
    rows = np.repeat(np.arange(na), 6)
    cols = band.nbr.reshape(-1)
    keep = cols < na
    return sp.csr_matrix((np.ones(int(keep.sum())), (rows[keep], cols[keep])), shape=(na, na))


def _bfs_distance(G, idx, start):
    """Hop distance from start (a position in idx) inside the subgraph on idx."""
    sub = G[idx][:, idx]
    return shortest_path(sub, unweighted=True, directed=False, indices=start)


def graph_partition(band, n_parts, weights=None):
    if n_parts < 1:
        raise ValueError("n_parts must be >= 1")
    na = band.n_act
    if n_parts > na:
        raise ValueError("more parts than active nodes")
    w = None if weights is None else [float(x) for x in weights]
    if w is not None and len(w) != n_parts:
        raise ValueError("need one weight per part")
    G = _active_graph(band)
    part = np.full(na, -1, dtype=np.int64)
    stack = [(np.arange(na, dtype=np.int64), 0, n_parts)]
    while stack:
        idx, first, n = stack.pop()
        if n == 1:
            part[idx] = first
            continue
        # idx is sorted by band index; position 0 is the lowest index
        d = _bfs_distance(G, idx, 0)
        far = int(np.argmax(np.where(np.isfinite(d), d, -1.0)))  # first maximum: lowest index
        d = _bfs_distance(G, idx, far)
        key = np.where(np.isfinite(d), d, float(na + 1))
        order = np.lexsort((idx, key))
        srt = idx[order]
        nl = n // 2
        if w is None:
            cut = (len(srt) * nl) // n
        else:
            wl = 0.0
            for q in range(first, first + nl):
                wl += w[q]
            wt = 0.0
            for q in range(first, first + n):
                wt += w[q]
            cut = int(math.floor(float(len(srt)) * wl / wt))
        left, right = np.sort(srt[:cut]), np.sort(srt[cut:])
        if len(right):
            ncomp, lab = connected_components(G[right][:, right], directed=False)
            if ncomp > 1:
                size = np.bincount(lab, minlength=ncomp)
                first_pos = np.array([np.flatnonzero(lab == c)[0] for c in range(ncomp)])
                keep = min(range(ncomp), key=lambda c: (-size[c], first_pos[c]))
                left = np.sort(np.concatenate([left, right[lab != keep]]))
                right = right[lab == keep]
        stack.append((left, first, nl))
        stack.append((right, first + nl, n - nl))
    assert (part >= 0).all()
    return part


def nearest_grid_node(band):
    """Band index of the grid node nearest to each active node's closest point."""
    na = band.n_act
    t = (band.cp[:na] - band.lo) / band.h
    ijk = np.floor(t + 0.5).astype(np.int64)
    n0, n1, n2 = band.shape
    L = (ijk[:, 0] * n1 + ijk[:, 1]) * n2 + ijk[:, 2]
    q = band.index_of(L)
    if (q < 0).any() or (q >= na).any():
        raise ValueError("a closest point's nearest grid node is not active")
    return q


def align_interfaces(band, part, passes):
    part = np.array(part, dtype=np.int64)
    n_parts = int(part.max()) + 1
    na = band.n_act
    xbar = nearest_grid_node(band)
    nbr = band.nbr
    for _ in range(passes):
        iface = np.zeros(na, dtype=bool)
        for e in range(6):
            y = nbr[:, e]
            ok = y < na
            iface[ok] |= part[y[ok]] != part[ok]
        target = part[xbar]
        move = iface & (target != part)
        part = np.where(move, target, part)
    if (np.bincount(part, minlength=n_parts) == 0).any():
        raise ValueError("a part is empty after alignment")
    return part
