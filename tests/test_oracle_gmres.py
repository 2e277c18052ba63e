"""Pins of the oracle's FGMRES against textbook dense solves."""

import numpy as np

from oracle import fgmres


def _system(n=60, seed=0):
    rng = np.random.default_rng(seed)
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    return A, b


def test_matches_dense_solve_unrestarted():
    A, b = _system()
    x, info = fgmres(lambda v: A @ v, b, tol=1e-13, restart=80)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-11, atol=1e-12)
    assert info["converged"] and info["cycles"] == 1
    h = np.array(info["history"])
    assert np.all(np.diff(h) <= 1e-15)


def test_restarted_and_preconditioned():
    A, b = _system(seed=1)
    x_ref = np.linalg.solve(A, b)
    x, info = fgmres(lambda v: A @ v, b, tol=1e-12, restart=5)
    assert info["cycles"] > 1
    np.testing.assert_allclose(x, x_ref, rtol=1e-10, atol=1e-11)
    D = np.diag(1.0 / np.diag(A))
    x2, _ = fgmres(lambda v: A @ v, b, M=lambda v: D @ v, tol=1e-12, restart=5)
    np.testing.assert_allclose(x2, x_ref, rtol=1e-10, atol=1e-11)


def test_exact_preconditioner_one_iteration():
    A, b = _system(seed=2)
    Ainv = np.linalg.inv(A)
    x, info = fgmres(lambda v: A @ v, b, M=lambda v: Ainv @ v, tol=1e-12)
    assert info["iters"] == 1
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-11)


def test_zero_rhs():
    A, _ = _system()
    x, info = fgmres(lambda v: A @ v, np.zeros(60))
    assert info["converged"] and not x.any()


def test_max_iter_reports_not_converged():
    A, b = _system(seed=3)
    x, info = fgmres(lambda v: A @ v, b, tol=1e-14, restart=3, max_iter=4)
    assert not info["converged"] and info["iters"] == 4
