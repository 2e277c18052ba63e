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
"""

from __future__ import annotations

import math

import numpy as np


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
