"""Computational band of the closest point method (paper Section 2.1).

* Grid: uniform spacing h, node (i, j, k) at lo + (i, j, k) h, linear index
  L = (i n1 + j) n2 + k.
* Active nodes Sigma_A: the tube-radius construction, every node whose distance
  to its closest point is at most r_A = rho h. Default rho = sqrt(3)(p+1)/2,
  the smallest radius that contains every interpolation stencil of a point on
  the surface, so that the extension only references active nodes.
* Ghost nodes Sigma_G: nodes needed to complete the 7-point stencils of the
  active nodes that are not active themselves.
* Extension rows: tensor-product Lagrange interpolation of degree p at
  CP_S(x) (Section 2.1, Figure 1); the weight of stencil node (a, b, c) is the
  product of the three one-dimensional weights.

Readings (the paper does not fix them):
* the tube radius is rho h with rho^2 = 0.75 (p+1)^2 unless overridden;
* a stencil whose nodes are not all active pulls them into Sigma_A (closure);
* stencil placement: for odd p the CP lies in the central cell
  (base = floor(t) - (p-1)/2), for even p the central node is the nearest node
  (base = floor(t + 1/2) - p/2), with t = (cp - lo)/h per axis;
* ordering: actives sorted by L, then ghosts sorted by L;
* the FD neighbour order is (x-, x+, y-, y+, z-, z+).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def grid_shape(lo, hi, h):
    return tuple(int(np.floor((hi[a] - lo[a]) / h + 0.5)) + 1 for a in range(3))


def lagrange_weights_1d(s, p):
    """Lagrange basis l_m(s) = prod_{q != m} (s - q)/(m - q) on nodes 0..p.

    Same polynomial as the barycentric form the paper cites; for integer s it
    is exactly the Kronecker delta.
    """
    s = np.asarray(s, dtype=np.float64)
    w = np.ones(s.shape + (p + 1,))
    for m in range(p + 1):
        for q in range(p + 1):
            if q != m:
                w[..., m] *= (s - q) / float(m - q)
    return w


@dataclass
class Band:
    lo: np.ndarray
    h: float
    p: int
    shape: tuple
    n_act: int
    n_ghost: int
    lin: np.ndarray      # (N_T,) int64: actives sorted, then ghosts sorted
    ijk: np.ndarray      # (N_T, 3) int64
    xyz: np.ndarray      # (N_T, 3) node coordinates
    cp: np.ndarray       # (N_T, 3) closest points
    nrm: np.ndarray      # (N_T, 3) unit normals at the closest points
    nbr: np.ndarray      # (N_A, 6) int64 band indices of the FD neighbours
    base: np.ndarray     # (N_T, 3) int64 first stencil index per axis
    wts: np.ndarray      # (N_T, 3, p+1) one-dimensional weights
    cols: np.ndarray     # (N_T, (p+1)^3) int64 band indices of stencil nodes (c fastest)

    @property
    def n_total(self):
        return self.n_act + self.n_ghost

    def index_of(self, L):
        """Band index of linear grid indices (-1 if not in the band)."""
        L = np.asarray(L, dtype=np.int64)
        act = self.lin[: self.n_act]
        gh = self.lin[self.n_act:]
        out = np.full(L.shape, -1, dtype=np.int64)
        pa = np.searchsorted(act, L)
        ina = (pa < len(act)) & (act[np.minimum(pa, len(act) - 1)] == L)
        out[ina] = pa[ina]
        if len(gh):
            pg = np.searchsorted(gh, L)
            ing = (~ina) & (pg < len(gh)) & (gh[np.minimum(pg, len(gh) - 1)] == L)
            out[ing] = self.n_act + pg[ing]
        return out


def _coords(lo, h, ijk):
    ijk = np.asarray(ijk, dtype=np.int64).reshape(-1, 3)
    x = np.empty(ijk.shape, dtype=np.float64)
    for a in range(3):
        x[:, a] = lo[a] + ijk[:, a].astype(np.float64) * h
    return x


def _ijk_of(L, shape):
    n0, n1, n2 = shape
    L = np.asarray(L, dtype=np.int64)
    return np.stack([L // (n1 * n2), (L // n2) % n1, L % n2], axis=1)


def _lin_of(ijk, shape):
    n0, n1, n2 = shape
    return (ijk[:, 0] * n1 + ijk[:, 1]) * n2 + ijk[:, 2]


def _dist2(x, cp):
    d0 = x[:, 0] - cp[:, 0]
    d1 = x[:, 1] - cp[:, 1]
    d2 = x[:, 2] - cp[:, 2]
    return (d0 * d0 + d1 * d1) + d2 * d2


def _stencil_base(cp, lo, h, p):
    t = np.empty(cp.shape)
    for a in range(3):
        t[:, a] = (cp[:, a] - lo[a]) / h
    if p % 2 == 1:
        base = np.floor(t).astype(np.int64) - (p - 1) // 2
    else:
        base = np.floor(t + 0.5).astype(np.int64) - p // 2
    s = t - base.astype(np.float64)
    return base, s


def _stencil_lin(base, p, shape):
    """Linear indices of the (p+1)^3 stencil nodes, ordered (a, b, c), c fastest."""
    off = np.arange(p + 1)
    a, b, c = np.meshgrid(off, off, off, indexing="ij")
    ii = base[:, 0:1] + a.reshape(1, -1)
    jj = base[:, 1:2] + b.reshape(1, -1)
    kk = base[:, 2:3] + c.reshape(1, -1)
    n0, n1, n2 = shape
    inside = (ii >= 0) & (ii < n0) & (jj >= 0) & (jj < n1) & (kk >= 0) & (kk < n2)
    if not inside.all():
        raise ValueError("interpolation stencil leaves the grid box")
    return (ii * n1 + jj) * n2 + kk


_NB_OFFSETS = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]],
                       dtype=np.int64)


def _neighbour_ijk(ijk, shape):
    nb = ijk[:, None, :] + _NB_OFFSETS[None, :, :]
    inside = np.all((nb >= 0) & (nb < np.array(shape)[None, None, :]), axis=2)
    return nb, inside


def build_band(surface, h, p, lo, hi, band_factor=None):
    """Tube-radius band with ghosts and extension rows (Section 2.1)."""
    if p not in (2, 3):
        raise ValueError("degree must be 2 or 3")
    if not h > 0:
        raise ValueError("h must be positive")
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    shape = grid_shape(lo, hi, h)
    n0, n1, n2 = shape
    rho2 = 0.75 * (p + 1) ** 2 if band_factor is None else float(band_factor) * float(band_factor)
    r2 = rho2 * (h * h)

    # Active nodes: every grid node within the tube radius (slab by slab).
    jj, kk = np.meshgrid(np.arange(n1, dtype=np.int64), np.arange(n2, dtype=np.int64),
                         indexing="ij")
    jj = jj.ravel()
    kk = kk.ravel()
    act = []
    for i in range(n0):
        ijk = np.stack([np.full(jj.shape, i, dtype=np.int64), jj, kk], axis=1)
        x = _coords(lo, h, ijk)
        cp, _ = surface.cp(x)
        d2 = _dist2(x, cp)
        sel = d2 <= r2
        act.append(_lin_of(ijk[sel], shape))
    act = np.unique(np.concatenate(act))

    # Ghosts and stencil closure.
    while True:
        aijk = _ijk_of(act, shape)
        nb, inside = _neighbour_ijk(aijk, shape)
        if not inside.all():
            raise ValueError("ghost node outside the grid box")
        nbL = _lin_of(nb.reshape(-1, 3), shape)
        ghosts = np.setdiff1d(np.unique(nbL), act)
        rows = np.concatenate([act, ghosts])
        rx = _coords(lo, h, _ijk_of(rows, shape))
        rcp, _ = surface.cp(rx)
        if not np.all(np.isfinite(rcp)):
            raise ValueError("closest point undefined at a band node")
        base, _ = _stencil_base(rcp, lo, h, p)
        sl = _stencil_lin(base, p, shape)
        missing = np.setdiff1d(np.unique(sl), act)
        if missing.size == 0:
            break
        act = np.union1d(act, missing)

    lin = np.concatenate([act, ghosts])
    ijk = _ijk_of(lin, shape)
    xyz = _coords(lo, h, ijk)
    cp, nrm = surface.cp(xyz)
    base, s = _stencil_base(cp, lo, h, p)
    wts = lagrange_weights_1d(s, p)

    band = Band(lo=lo, h=float(h), p=p, shape=shape, n_act=len(act), n_ghost=len(ghosts),
                lin=lin, ijk=ijk, xyz=xyz, cp=cp, nrm=nrm, nbr=None, base=base, wts=wts,
                cols=None)
    nb, _ = _neighbour_ijk(ijk[: len(act)], shape)
    band.nbr = band.index_of(_lin_of(nb.reshape(-1, 3), shape)).reshape(-1, 6)
    band.cols = band.index_of(_stencil_lin(base, p, shape))
    assert (band.nbr >= 0).all()
    assert (band.cols >= 0).all() and (band.cols < band.n_act).all()
    return band


def surface_distance_radius(p, band_factor=None):
    """Tube radius in units of h."""
    return np.sqrt(0.75 * (p + 1) ** 2) if band_factor is None else float(band_factor)
