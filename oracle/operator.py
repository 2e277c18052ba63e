"""Global CPM operator (paper Section 2.1, equation for the stabilised
discretisation, and the model problem (c - Delta_S) u = f of Section 1).

* E in R^{N_T x N_A}: row i holds the (p+1)^3 tensor-product weights that
  interpolate active values at CP_S(x_i).
* Delta^h in R^{N_A x N_T}: the 7-point second-order Laplacian on the band.
* Stabilised Laplace-Beltrami: Delta_S^h = -(2d/h^2) I + (Delta^h + (2d/h^2) I) E
  with d = 3. The identity inside the bracket is [I 0] (it selects the active
  rows of E), the one outside is the N_A identity.
* A = c I - Delta_S^h.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def extension_matrix(band):
    """E as a CSR matrix, N_T x N_A."""
    p = band.p
    n = band.n_total
    wx = band.wts[:, 0, :]
    wy = band.wts[:, 1, :]
    wz = band.wts[:, 2, :]
    w = (wx[:, :, None, None] * wy[:, None, :, None]) * wz[:, None, None, :]
    w = w.reshape(n, (p + 1) ** 3)
    rows = np.repeat(np.arange(n), (p + 1) ** 3)
    return sp.csr_matrix((w.ravel(), (rows, band.cols.ravel())), shape=(n, band.n_act))


def laplacian_matrix(band):
    """Delta^h as a CSR matrix, N_A x N_T (7-point stencil, spacing h)."""
    na = band.n_act
    h2 = band.h * band.h
    rows = np.concatenate([np.arange(na), np.repeat(np.arange(na), 6)])
    cols = np.concatenate([np.arange(na), band.nbr.ravel()])
    vals = np.concatenate([np.full(na, -6.0 / h2), np.full(6 * na, 1.0 / h2)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(na, band.n_total))


def stabilized_operator(band, c):
    """A = c I - Delta_S^h as a CSR matrix, N_A x N_A."""
    if not c > 0:
        raise ValueError("c must be positive")
    na = band.n_act
    d = 3
    s = 2.0 * d / (band.h * band.h)
    I_A = sp.identity(na, format="csr")
    I_AT = sp.csr_matrix((np.ones(na), (np.arange(na), np.arange(na))),
                         shape=(na, band.n_total))
    E = extension_matrix(band)
    lap_s = -s * I_A + (laplacian_matrix(band) + s * I_AT) @ E
    return (c * I_A - lap_s).tocsr()
