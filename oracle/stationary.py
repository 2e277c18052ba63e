"""(O)RAS as a stationary solver (paper Section 2.2, eq. algRAS):
u^{n+1} = u^n + M^{-1} (f - A u^n), u^0 = 0, stopped when the residual
2-norm has dropped below tol ||f||."""

from __future__ import annotations

import numpy as np


def stationary(A, f, M, tol=1e-8, max_iter=1000):
    """A, M: callables on 1-D arrays. Returns (u, info)."""
    f = np.asarray(f, dtype=np.float64)
    u = np.zeros_like(f)
    fn = float(np.linalg.norm(f))
    info = {"iters": 0, "history": [], "converged": fn == 0.0}
    if fn == 0.0:
        info["relres"] = 0.0
        return u, info
    r = f - A(u)
    while True:
        u = u + M(r)
        info["iters"] += 1
        r = f - A(u)
        rel = float(np.linalg.norm(r)) / fn
        info["history"].append(rel)
        if rel <= tol:
            info["converged"] = True
            break
        if info["iters"] >= max_iter or not np.isfinite(rel):
            break
    info["relres"] = rel
    return u, info
