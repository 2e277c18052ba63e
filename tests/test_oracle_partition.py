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
