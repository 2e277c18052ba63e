"""CPU FP64 oracle for the Schwarz-preconditioned closest point method solve.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or call anything here; the library in
``paper_1909_08734_amd`` never does, and the oracle imports nothing from it.
Both sides share only the seeded inputs in ``cpm_inputs``.

The oracle is a plain, slow, obviously correct restatement of May, Haynes and
Ruuth, "Schwarz solvers and preconditioners for the closest point method"
(arXiv:1909.08734), in float64 numpy/scipy. Each function cites the section or
equation it follows. Library primitives (sparse products, LAPACK LU, sorting)
serve as single steps; no blocking, fusion or reordering is added.

Readings taken where the paper is silent or ambiguous are listed in the module
that uses them and collected in the repository's design notes.
"""

from .band import Band, build_band, lagrange_weights_1d  # noqa: F401
from .operator import (  # noqa: F401
    extension_matrix,
    laplacian_matrix,
    stabilized_operator,
)
from .partition import octant_partition, rcb_partition, graph_partition, align_interfaces  # noqa: F401
from .schwarz import Decomposition, decompose, local_matrix, Preconditioner  # noqa: F401
from .gmres import fgmres, gmres_left  # noqa: F401
from .stationary import stationary  # noqa: F401
