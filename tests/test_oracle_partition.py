"""Pins of the oracle's coordinate partitions."""

import numpy as np
import pytest

import cpm_inputs as ci
import oracle


@pytest.fixture(scope="module")
def band():
    return oracle.build_band(ci.Sphere(), 0.1, 3, [-2.0] * 3, [2.0] * 3)


def test_octant_symmetry(band):
    part = oracle.octant_partition(band)
    cnt = np.bincount(part, minlength=8)
    # the sphere is centred on the node that defines the planes; nodes on a plane go
    # to the upper side, so the count depends only on how many upper sides a part has
    assert cnt[1] == cnt[2] == cnt[4]
    assert cnt[3] == cnt[5] == cnt[6]
    assert cnt[0] < cnt[1] < cnt[3] < cnt[7]
    assert cnt.sum() == band.n_act


@pytest.mark.parametrize("n", [2, 3, 7, 64])
def test_rcb_balance_and_separation(band, n):
    part = oracle.rcb_partition(band, n)
    cnt = np.bincount(part, minlength=n)
    assert cnt.sum() == band.n_act
    assert cnt.max() - cnt.min() <= 1
    if n == 2:
        ijk = band.ijk[: band.n_act]
        ext = ijk.max(0) - ijk.min(0)
        ax = int(np.argmax(ext))
        assert ijk[part == 0, ax].max() <= ijk[part == 1, ax].min()


def test_weighted_rcb_sizes(band):
    w = ci.wrcb_weights(16, seed=2)
    part = oracle.rcb_partition(band, 16, weights=w)
    cnt = np.bincount(part, minlength=16)
    target = band.n_act * w / w.sum()
    assert np.all(np.abs(cnt - target) <= 5)
    assert cnt.sum() == band.n_act


# ---- graph bisection and interface alignment (Sections 3.1, 3.2) --------------

from collections import deque

import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


def _bfs_brute(band, members, start):
    """Plain queue BFS over the 6-neighbour graph restricted to `members`."""
    na = band.n_act
    mem = set(int(q) for q in members)
    dist = {int(start): 0}
    dq = deque([int(start)])
    while dq:
        u = dq.popleft()
        for y in band.nbr[u]:
            y = int(y)
            if y < na and y in mem and y not in dist:
                dist[y] = dist[u] + 1
                dq.append(y)
    return dist


def test_graph_bfs_distance_matches_a_queue_bfs():
    from oracle.partition import _active_graph, _bfs_distance
    b = oracle.build_band(ci.Torus(1.0, 0.4), 0.1, 2, [-2.0] * 3, [2.0] * 3)
    G = _active_graph(b)
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(b.n_act, b.n_act // 2, replace=False))
    for start in (0, 17, len(idx) - 1):
        d = _bfs_distance(G, idx, start)
        ref = _bfs_brute(b, idx, idx[start])
        for pos, q in enumerate(idx):
            want = ref.get(int(q), np.inf)
            assert d[pos] == want


@pytest.mark.parametrize("surf,h", [(ci.Sphere(), 0.1), (ci.Torus(1.0, 0.4), 0.05)])
def test_graph_partition_sizes_and_connected_parts(surf, h):
    b = oracle.build_band(surf, h, 3, [-2.0] * 3, [2.0] * 3)
    n = 16
    part = oracle.graph_partition(b, n)
    sizes = np.bincount(part, minlength=n)
    assert sizes.sum() == b.n_act and sizes.max() <= 1.25 * sizes.min()
    from oracle.partition import _active_graph
    G = _active_graph(b)
    for j in range(n):
        idx = np.flatnonzero(part == j)
        ncomp, _ = connected_components(G[idx][:, idx], directed=False)
        assert ncomp == 1, (j, ncomp)


def test_graph_partition_weighted_cut_rule():
    b = oracle.build_band(ci.Sphere(), 0.1, 3, [-2.0] * 3, [2.0] * 3)
    w = ci.wrcb_weights(6, seed=2)
    part = oracle.graph_partition(b, 6, weights=w)
    sizes = np.bincount(part, minlength=6)
    # the first split gives floor(N * (w0+w1+w2)/sum(w)) nodes to parts 0..2,
    # plus the few pieces cut off from the right group
    want = int(np.floor(b.n_act * (w[0] + w[1] + w[2]) / w.sum()))
    assert want <= sizes[:3].sum() <= want + 0.02 * b.n_act


def _align_brute(band, part, passes):
    na = band.n_act
    part = [int(x) for x in part]
    xbar = []
    for q in range(na):
        g = [int(np.floor((band.cp[q, a] - band.lo[a]) / band.h + 0.5)) for a in range(3)]
        L = (g[0] * band.shape[1] + g[1]) * band.shape[2] + g[2]
        xbar.append(int(band.index_of(np.array([L]))[0]))
    for _ in range(passes):
        new = list(part)
        for q in range(na):
            iface = any(int(y) < na and part[int(y)] != part[q] for y in band.nbr[q])
            if iface and part[xbar[q]] != part[q]:
                new[q] = part[xbar[q]]
        part = new
    return np.array(part)


@pytest.mark.parametrize("method", ["rcb", "graph"])
def test_alignment_matches_brute_force(method):
    b = oracle.build_band(ci.Torus(1.0, 0.4), 0.1, 2, [-2.0] * 3, [2.0] * 3)
    part0 = oracle.rcb_partition(b, 7) if method == "rcb" else oracle.graph_partition(b, 7)
    for passes in (1, 3):
        np.testing.assert_array_equal(oracle.align_interfaces(b, part0, passes), _align_brute(b, part0, passes))


def test_alignment_leaves_normal_planes_and_single_parts_alone():
    b = oracle.build_band(ci.Sphere(), 0.1, 3, [-2.0] * 3, [2.0] * 3)
    one = np.zeros(b.n_act, dtype=np.int64)
    np.testing.assert_array_equal(oracle.align_interfaces(b, one, 4), one)
    # octant planes pass through the sphere's centre and contain its normals:
    # only nodes whose nearest-grid-node rounding crosses a plane move
    oc = oracle.octant_partition(b)
    moved = (oracle.align_interfaces(b, oc, 4) != oc).mean()
    assert moved < 0.03
