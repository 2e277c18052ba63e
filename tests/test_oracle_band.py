"""Pins of the oracle's band and extension rows (paper Section 2.1)."""

import json
import os

import numpy as np
import pytest

import cpm_inputs as ci
import oracle
from oracle.band import lagrange_weights_1d

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_sphere_band_counts.json")


def _paper_counts():
    with open(GOLD) as fh:
        return json.load(fh)


@pytest.mark.parametrize("inv_h", [50, 100, 125, 175, 200, 250])
def test_paper_active_counts(inv_h):
    """The six sphere band sizes printed in Sections 6.2 and 6.6 (p = 2); the
    finest take about a minute each."""
    g = _paper_counts()
    b = oracle.build_band(ci.Sphere(), 1.0 / inv_h, g["p"], [-1.2] * 3, [1.2] * 3,
                          band_factor=g["band_factor"])
    assert b.n_act == g["counts"][str(inv_h)]


def test_lagrange_basis_properties():
    s = np.linspace(-0.5, 3.5, 41)
    for p in (2, 3):
        w = lagrange_weights_1d(s, p)
        # partition of unity and exact reproduction of monomials s^q, q <= p
        for q in range(p + 1):
            np.testing.assert_allclose(w @ (np.arange(p + 1.0) ** q), s ** q, rtol=1e-13, atol=1e-12)
        # Kronecker delta at the nodes
        np.testing.assert_array_equal(lagrange_weights_1d(np.arange(p + 1.0), p), np.eye(p + 1))
    # cubic weights at s = 1.5 are the classic (-1, 9, 9, -1)/16
    np.testing.assert_allclose(lagrange_weights_1d(np.array([1.5]), 3)[0],
                               np.array([-1, 9, 9, -1]) / 16.0, rtol=0, atol=1e-16)


@pytest.fixture(scope="module")
def sphere01():
    return oracle.build_band(ci.Sphere(), 0.1, 3, [-2.0] * 3, [2.0] * 3)


@pytest.fixture(scope="module")
def torus():
    return oracle.build_band(ci.Torus(1.0, 0.4), 0.05, 3, [-2.0] * 3, [2.0] * 3)


def test_band_sets(sphere01):
    b = sphere01
    na = b.n_act
    # sorted, disjoint
    assert np.all(np.diff(b.lin[:na]) > 0) and np.all(np.diff(b.lin[na:]) > 0)
    assert len(np.intersect1d(b.lin[:na], b.lin[na:])) == 0
    # actives: exactly the tube |  |x| - 1 | <= sqrt(12) h  (sphere distance in closed form)
    r = np.linalg.norm(b.xyz, axis=1)
    assert np.all(np.abs(r[:na] - 1.0) <= np.sqrt(12.0) * 0.1 + 1e-12)
    # ghosts: exactly the 6-neighbour shell of the actives
    shell = set(b.nbr.ravel().tolist()) - set(range(na))
    assert shell == set(range(na, b.n_total))
    # every stencil column is active and the stencil sits at base..base+p
    assert b.cols.max() < na
    off = np.stack(np.meshgrid(*([np.arange(4)] * 3), indexing="ij"), -1).reshape(-1, 3)
    np.testing.assert_array_equal(b.ijk[b.cols], b.base[:, None, :] + off[None, :, :])


def test_band_sphere_counts_tiny():
    # sizes of two tiny bands computed independently of the builder:
    # count grid nodes with | |x| - 1 | <= sqrt(12) h by brute force
    for h in (0.2, 0.15):
        n = int(round(4 / h)) + 1
        g = -2.0 + np.arange(n) * h
        X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
        r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
        brute = int(np.count_nonzero(np.abs(r - 1.0) <= np.sqrt(12.0) * h + 1e-13))
        b = oracle.build_band(ci.Sphere(), h, 3, [-2.0] * 3, [2.0] * 3)
        assert b.n_act == brute


def _poly(x, e):
    return x[:, 0] ** e[0] * x[:, 1] ** e[1] * x[:, 2] ** e[2]


@pytest.mark.parametrize("which", ["sphere", "torus"])
def test_extension_reproduces_polynomials(which, sphere01, torus):
    b = sphere01 if which == "sphere" else torus
    E = oracle.extension_matrix(b)
    np.testing.assert_allclose(E @ np.ones(b.n_act), 1.0, rtol=0, atol=1e-13)
    for e in [(1, 0, 0), (0, 2, 1), (3, 3, 3), (2, 0, 3)]:
        q = _poly(b.xyz[: b.n_act], e)
        np.testing.assert_allclose(E @ q, _poly(b.cp, e), rtol=1e-11, atol=1e-11)


def test_extension_degree2_reproduces_quadratics():
    b = oracle.build_band(ci.Sphere(), 0.1, 2, [-2.0] * 3, [2.0] * 3)
    E = oracle.extension_matrix(b)
    for e in [(2, 2, 2), (1, 2, 0)]:
        np.testing.assert_allclose(E @ _poly(b.xyz[: b.n_act], e), _poly(b.cp, e), atol=1e-12)
    # a cubic term is not reproduced by quadratic interpolation
    assert np.abs(E @ _poly(b.xyz[: b.n_act], (3, 0, 0)) - _poly(b.cp, (3, 0, 0))).max() > 1e-6


def test_band_errors():
    with pytest.raises(ValueError):
        oracle.build_band(ci.Sphere(), 0.1, 4, [-2.0] * 3, [2.0] * 3)
    with pytest.raises(ValueError):
        oracle.build_band(ci.Sphere(), 0.1, 3, [-1.2] * 3, [1.2] * 3)  # ghosts leave the box
