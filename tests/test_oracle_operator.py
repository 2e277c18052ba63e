"""Pins of the oracle's stabilised CPM operator (paper Section 2.1)."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import cpm_inputs as ci
import oracle


@pytest.fixture(scope="module")
def band():
    return oracle.build_band(ci.Sphere(), 0.1, 3, [-2.0] * 3, [2.0] * 3)


def test_constants_and_quadratics(band):
    b = band
    c = 1.7
    A = oracle.stabilized_operator(b, c)
    # E 1 = 1 and Delta^h annihilates constants, so A 1 = c 1
    np.testing.assert_allclose(A @ np.ones(b.n_act), c, rtol=1e-12)
    # the 7-point Laplacian is exact on quadratics: Delta(x^2 + 2y^2 - z^2) = 2 + 4 - 2
    L = oracle.laplacian_matrix(b)
    q = b.xyz[:, 0] ** 2 + 2 * b.xyz[:, 1] ** 2 - b.xyz[:, 2] ** 2
    np.testing.assert_allclose(L @ q, 4.0, rtol=1e-9)
    # and exact-zero on linear functions
    np.testing.assert_allclose(L @ (3 * b.xyz[:, 0] - b.xyz[:, 2]), 0.0, atol=1e-9)


def test_operator_row_structure(band):
    # A = (c + 6/h^2) I - (1/h^2) N E, with N the 6-neighbour sum: check on a random vector
    b = band
    c = 0.5
    A = oracle.stabilized_operator(b, c)
    E = oracle.extension_matrix(b)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(b.n_act)
    ex = E @ x
    y = (c + 6 / b.h ** 2) * x - ex[b.nbr].sum(axis=1) / b.h ** 2
    np.testing.assert_allclose(A @ x, y, rtol=1e-12, atol=1e-9)


def test_spherical_harmonic_convergence():
    # Delta_S Y_l^m = -l(l+1) Y_l^m on the unit sphere: u = Y solves (c - Delta_S) u = (c + l(l+1)) Y.
    c = 1.0
    errs = []
    hs = [0.1, 0.05, 0.025]
    for h in hs:
        b = oracle.build_band(ci.Sphere(), h, 3, [-2.0] * 3, [2.0] * 3)
        A = oracle.stabilized_operator(b, c)
        cp = b.cp[: b.n_act]
        u_ex = ci.real_sph_harm(3, 1, cp) + 0.5 * ci.real_sph_harm(2, -2, cp)
        f = (c + 12) * ci.real_sph_harm(3, 1, cp) + 0.5 * (c + 6) * ci.real_sph_harm(2, -2, cp)
        u, info = spla.gmres(A, f, rtol=1e-12, restart=200, maxiter=200)
        assert info == 0
        errs.append(np.abs(u - u_ex).max())
    orders = np.log(np.array(errs[:-1]) / np.array(errs[1:])) / np.log(2.0)
    # second order: every observed order >= 1.7, the finest pair within 2 +- 0.6
    assert np.all(orders > 1.7) and abs(orders[-1] - 2.0) < 0.6, (errs, orders)


def test_tiny_dense_solve():
    # brute force: dense solve of the whole system on the h=0.2 band equals the sparse solve
    b = oracle.build_band(ci.Sphere(), 0.2, 3, [-2.0] * 3, [2.0] * 3)
    A = oracle.stabilized_operator(b, 1.0)
    f = ci.rhs_sphere_y20(b.cp[: b.n_act], 1.0)
    u1 = np.linalg.solve(A.toarray(), f)
    u2 = spla.spsolve(A.tocsc(), f)  # SuperLU, a second, sparse factorisation
    np.testing.assert_allclose(u1, u2, rtol=1e-10, atol=1e-12)


def test_c_must_be_positive(band):
    with pytest.raises(ValueError):
        oracle.stabilized_operator(band, 0.0)
