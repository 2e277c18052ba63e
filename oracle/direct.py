"""Direct solution of the global CPM system (the plain definition u = A^{-1} f
of the model problem (c - Delta_S) u = f, Section 1, with A of Section 2.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every Schwarz-preconditioned Krylov solve of the paper converges to this
vector (Section 6.1 compares the domain-decomposition solution with the direct
one), so it is the reference the iterative results are held against. The sparse
LU factorisation (SuperLU with a fill-reducing column order) is one library
step; a few rounds of iterative refinement, each r = f - A u then
u <- u + LU^{-1} r, bring the residual to the rounding level of A itself.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def sparse_direct_solve(A, f, refine=2):
    """Return (u, relres history) for A u = f by sparse LU plus `refine`
    refinement rounds; the history holds ||f - A u|| / ||f|| after the solve
    and after every round."""
    f = np.asarray(f, dtype=np.float64)
    lu = spla.splu(A.tocsc(), permc_spec="COLAMD")
    u = lu.solve(f)
    fn = float(np.linalg.norm(f))
    hist = [float(np.linalg.norm(f - A @ u)) / fn]
    for _ in range(refine):
        r = f - A @ u
        u = u + lu.solve(r)
        hist.append(float(np.linalg.norm(f - A @ u)) / fn)
    return u, hist
