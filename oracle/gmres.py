"""Restarted flexible GMRES with right preconditioning (the Krylov acceleration of
paper Section 2.2, where the Schwarz operator preconditions GMRES).

Reading: the paper writes the preconditioned system as M^{-1} A u = M^{-1} f
and stops on a 10^6 reduction of the residual norm without fixing the GMRES
variant. Here: FGMRES(m), right preconditioning, modified Gram-Schmidt,
Givens rotations, x0 = 0; a cycle stops when the rotated residual estimate
falls to tol ||f||; the solve stops when the true residual ||f - A x|| does.
Right preconditioning makes the monitored residual the true one, so FP32 and
FP64 preconditioners are compared at equal final accuracy.

gmres_left is the paper's own formulation, kept for comparisons with its
iteration counts: GMRES(m) on M^{-1} A x = M^{-1} b stopping on a reduction of
the preconditioned residual.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.linalg


def fgmres(A, b, M=None, tol=1e-8, restart=30, max_iter=1000):
    """Solve A x = b. A and M are callables on 1-D arrays. Returns (x, info)."""
    b = np.asarray(b, dtype=np.float64)
    n = len(b)
    if M is None:
        def M(v):
            return v
    bnorm = float(np.linalg.norm(b))
    x = np.zeros(n)
    info = {"iters": 0, "cycles": 0, "history": [], "converged": False}
    if bnorm == 0.0:
        info.update(converged=True, relres=0.0)
        return x, info
    r = b.copy()
    beta = bnorm
    while True:
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k_used = 0
        for k in range(restart):
            Z[k] = M(V[k])
            w = A(Z[k])
            for i in range(k + 1):
                H[i, k] = np.dot(V[i], w)
                w = w - H[i, k] * V[i]
            hk1 = float(np.linalg.norm(w))
            H[k + 1, k] = hk1
            if hk1 > 0.0:
                V[k + 1] = w / hk1
            for i in range(k):
                a, bb = H[i, k], H[i + 1, k]
                H[i, k] = cs[i] * a + sn[i] * bb
                H[i + 1, k] = -sn[i] * a + cs[i] * bb
            den = math.hypot(H[k, k], H[k + 1, k])
            cs[k] = H[k, k] / den
            sn[k] = H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            k_used = k + 1
            info["iters"] += 1
            info["history"].append(abs(g[k + 1]) / bnorm)
            if abs(g[k + 1]) <= tol * bnorm or info["iters"] >= max_iter or hk1 == 0.0:
                break
        y = scipy.linalg.solve_triangular(H[:k_used, :k_used], g[:k_used])
        x = x + Z[:k_used].T @ y
        r = b - A(x)
        beta = float(np.linalg.norm(r))
        info["cycles"] += 1
        if beta <= tol * bnorm:
            info["converged"] = True
            break
        if info["iters"] >= max_iter:
            break
    info["relres"] = beta / bnorm
    return x, info


def gmres_left(A, b, M, tol=1e-6, restart=30, max_iter=1000):
    """GMRES(m) on the left-preconditioned system M^{-1} A x = M^{-1} b, the form
    the paper gives for the Schwarz-preconditioned Krylov solve (Section 2.2),
    with the paper's stopping rule (Section 6): the 2-norm of the (preconditioned)
    residual reduced by the factor 1/tol, i.e. ||M^{-1}(b - A x)|| <= tol ||M^{-1} b||.
    x0 = 0, modified Gram-Schmidt, Givens rotations; a cycle stops on the
    rotated estimate, the solve on the recomputed preconditioned residual.
    A and M are callables on 1-D arrays. Returns (x, info); info["relres"] is
    the preconditioned ratio, info["relres_true"] = ||b - A x|| / ||b||."""
    b = np.asarray(b, dtype=np.float64)
    n = len(b)
    x = np.zeros(n)
    r = M(b)
    beta0 = float(np.linalg.norm(r))
    info = {"iters": 0, "cycles": 0, "history": [], "converged": False}
    if beta0 == 0.0:
        info.update(converged=True, relres=0.0, relres_true=0.0)
        return x, info
    beta = beta0
    while True:
        V = np.zeros((restart + 1, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k_used = 0
        for k in range(restart):
            w = M(A(V[k]))
            for i in range(k + 1):
                H[i, k] = np.dot(V[i], w)
                w = w - H[i, k] * V[i]
            hk1 = float(np.linalg.norm(w))
            H[k + 1, k] = hk1
            if hk1 > 0.0:
                V[k + 1] = w / hk1
            for i in range(k):
                a, bb = H[i, k], H[i + 1, k]
                H[i, k] = cs[i] * a + sn[i] * bb
                H[i + 1, k] = -sn[i] * a + cs[i] * bb
            den = math.hypot(H[k, k], H[k + 1, k])
            cs[k] = H[k, k] / den
            sn[k] = H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            k_used = k + 1
            info["iters"] += 1
            info["history"].append(abs(g[k + 1]) / beta0)
            if abs(g[k + 1]) <= tol * beta0 or info["iters"] >= max_iter or hk1 == 0.0:
                break
        y = scipy.linalg.solve_triangular(H[:k_used, :k_used], g[:k_used])
        x = x + V[:k_used].T @ y
        r = M(b - A(x))
        beta = float(np.linalg.norm(r))
        info["cycles"] += 1
        if beta <= tol * beta0:
            info["converged"] = True
            break
        if info["iters"] >= max_iter:
            break
    info["relres"] = beta / beta0
    info["relres_true"] = float(np.linalg.norm(b - A(x)) / np.linalg.norm(b))
    return x, info
