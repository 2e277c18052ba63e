"""Overlapping Schwarz preconditioner for the CPM system (paper Sections 2.2, 4, 5).

M^{-1} = sum_j  R~_j^T A_j^{-1} R_j   (restricted additive Schwarz, eq. algRAS)

Node sets per subdomain j (Section 4.1, 4.2):
* Sigma~_j: disjoint part j of the active nodes.
* Sigma_j: Sigma~_j grown by N_O breadth-first layers over the 6-neighbour graph
  restricted to Sigma_A; F_j is the last layer added.
* Sigma_j^G: global ghost nodes among the FD neighbours of Sigma_j.
* B_j (the active part of Sigma_j^BC): active nodes outside Sigma_j that are FD
  neighbours of Sigma_j or columns of the extension rows of Sigma_j u Sigma_j^G.

Local operator (Section 5, eq. localOP), taken literally:
  A_j = (c + 2d/h^2) I - (2d/h^2 + Delta_j^h) [E_j ; T_j]
with the local extension [E_j; T_j] (rows of E for Sigma_j u Sigma_j^G, rows
T_j for B_j) and the local 7-point Laplacian Delta_j^h, which has rows only at
Sigma_j (the stencils of B_j nodes are not complete in the local problem).
So the rows of B_j read (c + 2d/h^2) u_b - (2d/h^2) (T_j u)_b = 0, with zero
right-hand side (Section 5).
* RAS (Dirichlet, Section 5.1): T_j = [0 I], so c u_b = 0; the B unknowns are
  identically zero and are dropped (local size |Sigma_j|).
* ORAS (Robin, Section 5.2, eq. robfo): (T_j u)_b = u(CP_{S_j}(x_b)) / (1 + alpha_b d_b.q_b),
  where CP_{S_j}(x_b) is the closest point among Lambda_j = CP(F_j)
  (eq. locCP; exhaustive argmin, smallest band index on ties), u at that point
  is interpolated with the extension row of the final-layer node x* it came
  from, and d_b.q_b = |d_b - (d_b.n)n| with d_b = x_b - CP(x*), n the surface
  normal there (eq. naConorm; zero when d_b is parallel to n).
* Cross points (Section 5.2.2): active nodes whose active FD neighbours lie in
  at least two parts other than their own; B nodes within 2 N_O grid units of
  any cross point (integer squared distance, inclusive) use alpha_cross.
Local right-hand side: [r|_{Sigma_j}; 0]. Local solves use LU with partial
pivoting (Section 5). Prolongation keeps only Sigma~_j (each node written once).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg
import scipy.sparse as sp

RAS = "RAS"
ORAS = "ORAS"


@dataclass
class Subdomain:
    tilde: np.ndarray          # sorted band indices of the disjoint part
    sigma: np.ndarray          # sorted band indices of Sigma_j
    final: np.ndarray          # sorted band indices of the last overlap layer
    ghost: np.ndarray          # sorted band indices of Sigma_j^G
    bnd: np.ndarray            # sorted band indices of B_j
    xstar: np.ndarray = None   # (|B_j|,) band index of the final-layer node chosen for b
    s: np.ndarray = None       # (|B_j|,) d_b . q_b
    alpha: np.ndarray = None   # (|B_j|,) Robin weight per B node

    def local_size(self, kind):
        return len(self.sigma) + (len(self.bnd) if kind == ORAS else 0)


@dataclass
class Decomposition:
    kind: str
    overlap: int
    alpha: float
    alpha_cross: float
    part: np.ndarray
    cross: np.ndarray                   # bool mask over actives
    subs: list = field(default_factory=list)


def cross_points(band, part):
    """Actives with active FD neighbours in >= 2 parts other than their own."""
    na = band.n_act
    nb = band.nbr
    p_nb = np.where(nb < na, part[np.minimum(nb, na - 1)], -1)
    own = part[:, None]
    p_nb = np.where(p_nb == own, -1, p_nb)
    srt = np.sort(p_nb, axis=1)
    distinct = (srt >= 0) & np.concatenate(
        [np.ones((na, 1), dtype=bool), srt[:, 1:] != srt[:, :-1]], axis=1)
    return distinct.sum(axis=1) >= 2


def _grow(band, mask):
    na = band.n_act
    nb = band.nbr
    nb_in = np.where(nb < na, mask[np.minimum(nb, na - 1)], False)
    return mask | nb_in.any(axis=1)


def decompose(band, part, overlap, kind, alpha=0.0, alpha_cross=0.0, only=None):
    """Node sets of every subdomain (or of the subdomains listed in `only`;
    the others are left as None). Cross points always use the whole partition."""
    if kind not in (RAS, ORAS):
        raise ValueError("kind must be RAS or ORAS")
    if overlap < 0 or (kind == ORAS and overlap < 1):
        raise ValueError("overlap must be >= 1 for ORAS (>= 0 for RAS)")
    na = band.n_act
    part = np.asarray(part, dtype=np.int64)
    n_sub = int(part.max()) + 1
    cross = cross_points(band, part)
    cross_ijk = band.ijk[:na][cross]
    dec = Decomposition(kind=kind, overlap=overlap, alpha=float(alpha),
                        alpha_cross=float(alpha_cross), part=part, cross=cross)
    for j in range(n_sub):
        if only is not None and j not in only:
            dec.subs.append(None)
            continue
        mask = part == j
        tilde = np.flatnonzero(mask)
        prev = mask
        for _ in range(overlap):
            prev = mask
            mask = _grow(band, mask)
        sigma = np.flatnonzero(mask)
        final = np.flatnonzero(mask & ~prev) if overlap > 0 else tilde
        nbs = band.nbr[sigma].ravel()
        ghost = np.unique(nbs[nbs >= na])
        cand = np.concatenate([nbs[nbs < na], band.cols[sigma].ravel(), band.cols[ghost].ravel()])
        bnd = np.setdiff1d(np.unique(cand), sigma)
        sd = Subdomain(tilde=tilde, sigma=sigma, final=final, ghost=ghost, bnd=bnd)
        if kind == ORAS and len(bnd) == 0:
            sd.xstar = np.zeros(0, dtype=np.int64)
            sd.s = np.zeros(0)
            sd.alpha = np.zeros(0)
        elif kind == ORAS:
            if len(final) == 0:
                raise ValueError("subdomain has boundary nodes but no final overlap layer")
            xb = band.xyz[bnd]
            cf = band.cp[final]
            d0 = xb[:, 0:1] - cf[None, :, 0]
            d1 = xb[:, 1:2] - cf[None, :, 1]
            d2 = xb[:, 2:3] - cf[None, :, 2]
            dist2 = (d0 * d0 + d1 * d1) + d2 * d2
            xstar = final[np.argmin(dist2, axis=1)]
            y = band.cp[xstar]
            nrm = band.nrm[xstar]
            d = xb - y
            dn = (d[:, 0] * nrm[:, 0] + d[:, 1] * nrm[:, 1]) + d[:, 2] * nrm[:, 2]
            t = d - dn[:, None] * nrm
            s = np.sqrt((t[:, 0] * t[:, 0] + t[:, 1] * t[:, 1]) + t[:, 2] * t[:, 2])
            a = np.full(len(bnd), float(alpha))
            if alpha_cross > 0 and len(cross_ijk):
                r2 = (2 * overlap) ** 2
                bijk = band.ijk[bnd]
                near = np.zeros(len(bnd), dtype=bool)
                for c0 in range(0, len(cross_ijk), 4096):
                    cj = cross_ijk[c0:c0 + 4096]
                    dd = bijk[:, None, :] - cj[None, :, :]
                    near |= ((dd * dd).sum(axis=2) <= r2).any(axis=1)
                a[near] = float(alpha_cross)
            sd.xstar, sd.s, sd.alpha = xstar, s, a
        dec.subs.append(sd)
    return dec


def local_matrix(band, dec, j, c):
    """Dense A_j following eq. localOP with the readings in the module docstring."""
    sd = dec.subs[j]
    kind = dec.kind
    h2 = band.h * band.h
    sig = c + 6.0 / h2
    m = len(sd.sigma)
    nbnd = len(sd.bnd)
    n_unk = m + nbnd                      # unknowns [Sigma_j ; B_j] before dropping
    # Extended local nodes X = [Sigma_j ; Sigma_j^G ; B_j].
    X = np.concatenate([sd.sigma, sd.ghost, sd.bnd])
    xpos = np.full(band.n_total, -1, dtype=np.int64)
    xpos[X] = np.arange(len(X))
    upos = np.full(band.n_total, -1, dtype=np.int64)
    upos[sd.sigma] = np.arange(m)
    upos[sd.bnd] = m + np.arange(nbnd)

    E = _extension_rows(band, np.concatenate([sd.sigma, sd.ghost]), upos, n_unk)
    if kind == ORAS:
        T = _extension_rows(band, sd.xstar, upos, n_unk)
        T = sp.diags(1.0 / (1.0 + sd.alpha * sd.s)) @ T
    else:
        T = sp.csr_matrix((np.ones(nbnd), (np.arange(nbnd), m + np.arange(nbnd))),
                          shape=(nbnd, n_unk))
    ext = sp.vstack([E, T]).tocsr()       # [E_j ; T_j], |X| x n_unk

    # Delta_j^h on the rows of Sigma_j: -6/h^2 at the node, 1/h^2 at each neighbour.
    nbx = xpos[band.nbr[sd.sigma]]
    assert (nbx >= 0).all()
    rows = np.concatenate([np.arange(m), np.repeat(np.arange(m), 6)])
    cols = np.concatenate([np.arange(m), nbx.ravel()])
    vals = np.concatenate([np.full(m, -6.0 / h2), np.full(6 * m, 1.0 / h2)])
    lap = sp.csr_matrix((vals, (rows, cols)), shape=(m, len(X)))
    sel = sp.csr_matrix((np.ones(m), (np.arange(m), np.arange(m))), shape=(m, len(X)))
    I_mu = sp.csr_matrix((np.ones(m), (np.arange(m), np.arange(m))), shape=(m, n_unk))
    top = sig * I_mu - ((6.0 / h2) * sel + lap) @ ext

    if kind == ORAS:
        # B rows: Delta_j^h has no row there, leaving (c + 6/h^2) u_b - (6/h^2) (T_j u)_b
        I_bu = sp.csr_matrix((np.ones(nbnd), (np.arange(nbnd), m + np.arange(nbnd))),
                             shape=(nbnd, n_unk))
        bot = sig * I_bu - (6.0 / h2) * T
        A = sp.vstack([top, bot]).toarray()
    else:
        A = top.toarray()[:, :m]
    return A


def _extension_rows(band, nodes, upos, n_unk):
    p = band.p
    k = (p + 1) ** 3
    wx = band.wts[nodes, 0, :]
    wy = band.wts[nodes, 1, :]
    wz = band.wts[nodes, 2, :]
    w = ((wx[:, :, None, None] * wy[:, None, :, None]) * wz[:, None, None, :]).reshape(-1, k)
    cols = upos[band.cols[nodes]]
    assert (cols >= 0).all(), "extension stencil leaves the local node set"
    rows = np.repeat(np.arange(len(nodes)), k)
    return sp.csr_matrix((w.ravel(), (rows, cols.ravel())), shape=(len(nodes), n_unk))


class Preconditioner:
    """z = M^{-1} v with LU-factored local operators (Section 5)."""

    def __init__(self, band, dec, c, subs=None):
        self.band = band
        self.dec = dec
        self.c = float(c)
        self.which = list(range(len(dec.subs))) if subs is None else list(subs)
        self.lu = {}
        for j in self.which:
            self.lu[j] = scipy.linalg.lu_factor(local_matrix(band, dec, j, c),
                                                check_finite=False)

    def local_solve(self, j, v):
        sd = self.dec.subs[j]
        n = sd.local_size(self.dec.kind)
        rhs = np.zeros(n)
        rhs[: len(sd.sigma)] = v[sd.sigma]
        return scipy.linalg.lu_solve(self.lu[j], rhs, check_finite=False)

    def apply(self, v):
        """M^{-1} v; entries of parts not factored here are left as NaN."""
        v = np.asarray(v, dtype=np.float64)
        z = np.full(self.band.n_act, np.nan)
        for j in self.which:
            sd = self.dec.subs[j]
            e = self.local_solve(j, v)
            z[sd.tilde] = e[np.searchsorted(sd.sigma, sd.tilde)]
        return z
