"""Write the reference solution of the benchmark-size sphere problem.

Unit sphere, closest point x/|x|, grid h = 0.025 on [-2, 2]^3, tricubic
extension (N_A = 139,886), c = 1, f = sum_{l<=4,|m|<=l} (c + l(l+1)) a_lm
Y_l^m(CP(x)) with a_lm ~ N(0,1) from seed 1 (the benchmark's first
right-hand side). u = A^{-1} f by the oracle's sparse direct solve with
iterative refinement (Section 1 problem, Section 2.1 operator). The solution
does not depend on the Schwarz preconditioner, so one file serves every
Robin weight and factor precision.

Calls only the oracle and the shared input generators. Takes about seven
minutes and 40 GB of memory:
    python tests/golden/make_sphere_h0025_solution.py
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import cpm_inputs as ci  # noqa: E402
import oracle  # noqa: E402
from oracle.direct import sparse_direct_solve  # noqa: E402

H, C, SEED = 0.025, 1.0, 1
OUT = os.path.join(HERE, "sphere_h0025_seed1_solution.npz")


def main():
    t0 = time.time()
    b = oracle.build_band(ci.Sphere(), H, 3, [-2.0] * 3, [2.0] * 3)
    A = oracle.stabilized_operator(b, C)
    f = ci.rhs_sphere_random_sh(b.cp[: b.n_act], C, seed=SEED)[0]
    u, hist = sparse_direct_solve(A, f, refine=2)
    meta = {"surface": "unit sphere", "h": H, "degree": 3, "box": [-2.0, 2.0], "c": C,
            "rhs": "seeded random spherical harmonics l<=4", "seed": SEED, "n_act": int(b.n_act),
            "solver": "oracle.direct.sparse_direct_solve (SuperLU, 2 refinement rounds)",
            "relres_history": hist, "seconds": time.time() - t0}
    np.savez_compressed(OUT, u=u, lin=b.lin[: b.n_act], meta=json.dumps(meta))
    print(json.dumps(meta))


if __name__ == "__main__":
    main()
