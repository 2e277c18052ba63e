"""Pins of the oracle's FGMRES against textbook dense solves."""

import numpy as np

from oracle import fgmres, gmres_left


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


def test_left_gmres_minimises_the_preconditioned_residual_over_the_krylov_space():
    """Without restarts, iterate k is the x in K_k(M^{-1}A, M^{-1}b) that minimises
    ||M^{-1}(b - A x)|| (the definition of GMRES on the left-preconditioned
    system): checked by a least-squares solve on the explicit Krylov basis."""
    A, b = _system(n=40, seed=4)
    D = np.diag(1.0 / (np.diag(A) + np.linspace(0.0, 1.0, 40)))  # a non-trivial M^{-1}
    Mb = D @ b
    MA = D @ A
    for k in (1, 2, 3, 5, 8):
        x, info = gmres_left(lambda v: A @ v, b, lambda v: D @ v, tol=1e-30, restart=50, max_iter=k)
        assert info["iters"] == k and info["cycles"] == 1
        K = np.stack([np.linalg.matrix_power(MA, q) @ Mb for q in range(k)], axis=1)
        Q, _ = np.linalg.qr(K)
        c, *_ = np.linalg.lstsq(MA @ Q, Mb, rcond=None)
        x_ref = Q @ c
        np.testing.assert_allclose(x, x_ref, rtol=1e-9, atol=1e-11)
        # and the history is that minimum's preconditioned residual
        assert abs(info["history"][-1] - np.linalg.norm(Mb - MA @ x_ref) / np.linalg.norm(Mb)) < 1e-10


def test_left_gmres_stopping_rule_and_exact_preconditioner():
    A, b = _system(seed=5)
    D = np.diag(1.0 / np.diag(A))
    x, info = gmres_left(lambda v: A @ v, b, lambda v: D @ v, tol=1e-6, restart=5)
    assert info["converged"] and info["cycles"] > 1
    r = np.linalg.norm(D @ (b - A @ x)) / np.linalg.norm(D @ b)
    assert r <= 1e-6 and abs(r - info["relres"]) < 1e-15
    assert info["relres_true"] == np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    # with M = A^{-1} the preconditioned operator is the identity: one iteration
    Ainv = np.linalg.inv(A)
    x, info = gmres_left(lambda v: A @ v, b, lambda v: Ainv @ v, tol=1e-12)
    assert info["iters"] == 1
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-11)
    # zero right-hand side, and max_iter
    x, info = gmres_left(lambda v: A @ v, np.zeros(60), lambda v: v)
    assert info["converged"] and not x.any()
    x, info = gmres_left(lambda v: A @ v, b, lambda v: v, tol=1e-14, restart=3, max_iter=4)
    assert not info["converged"] and info["iters"] == 4
