"""Closest point method on a circular arc with a Dirichlet end and a Robin end
(Section 5.2.1, order-of-accuracy test of eq. robfo; Table 1).

TEST INFRASTRUCTURE ONLY (see the package docstring). A plain float64
restatement, in two dimensions, of the pieces the three-dimensional oracle
uses, so that the first-order Robin row can be checked on a problem with a
known solution:

* surface: the arc theta in [0, 2] of the unit circle; the closest point of a
  grid node is the radial projection when its polar angle lies in [0, 2],
  otherwise the nearer end point;
* band: grid nodes lo + (i, j) h within rho h of the arc, rho = sqrt(2)(p+1)/2,
  closed under the interpolation stencils, plus the 4-neighbour ghost layer;
* extension rows: tensor-product Lagrange interpolation of degree p at the
  closest point (Section 2.1), except for nodes whose closest point is an end:
  - theta = 0, Dirichlet u = 0 to second order by the mirror point: the row
    is minus the interpolation row at CP(2 CP(x) - x) (odd reflection
    through the end point);
  - theta = 2, the Robin condition du/dq + alpha u = 0 by eq. robfo: the row
    is the interpolation row at the end point divided by 1 + alpha d.q, with
    d = x - CP(x) and q the outward unit tangent at the end;
* operator: the stabilised form of eq. impLapBel in two dimensions,
  A = c I - (-(4/h^2) I + (Delta^h + (4/h^2) [I 0]) E~), i.e. row i is
  (c + 4/h^2) e_i - h^-2 sum over the 4 grid neighbours of their rows of E~.

The error is measured at the active nodes whose closest point lies inside the
arc, against the exact solution of (1 - Delta_S) u = 1 - theta^2, u(0) = 0,
u'(2) + u(2) = 0.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .band import lagrange_weights_1d

THETA_END = 2.0


def exact_solution(theta):
    """u(theta) = cosh(theta) + (9 e^-2 - 1) sinh(theta) - theta^2 - 1."""
    return np.cosh(theta) + (9.0 * np.exp(-2.0) - 1.0) * np.sinh(theta) - theta ** 2 - 1.0


def closest_point(x):
    """Closest points on the arc and a code per point: 0 interior, 1 the end
    theta = 0, 2 the end theta = 2. Also returns the polar angle of the point."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 2)
    phi = np.arctan2(x[:, 1], x[:, 0])
    inside = (phi >= 0.0) & (phi <= THETA_END)
    p0 = np.array([1.0, 0.0])
    p2 = np.array([np.cos(THETA_END), np.sin(THETA_END)])
    d0 = np.hypot(x[:, 0] - p0[0], x[:, 1] - p0[1])
    d2 = np.hypot(x[:, 0] - p2[0], x[:, 1] - p2[1])
    code = np.where(inside, 0, np.where(d0 <= d2, 1, 2))
    theta = np.where(inside, phi, np.where(code == 1, 0.0, THETA_END))
    cp = np.stack([np.cos(theta), np.sin(theta)], axis=1)
    return cp, code, theta


def _interp_rows(pts, lo, h, p):
    """Stencil base (i, j) and 1-D weights of the degree-p interpolation at pts."""
    t = (pts - lo) / h
    if p % 2 == 1:
        base = np.floor(t).astype(np.int64) - (p - 1) // 2
    else:
        base = np.floor(t + 0.5).astype(np.int64) - p // 2
    s = t - base
    return base, lagrange_weights_1d(s[:, 0], p), lagrange_weights_1d(s[:, 1], p)


def solve_arc(h, p=3, alpha=1.0, c=1.0, lo=-2.0):
    """Assemble and solve the arc problem at grid spacing h. Returns a dict with
    the band size, the max error over interior-closest-point actives and the
    solution."""
    n = int(round(4.0 / h)) + 1
    rho = np.sqrt(2.0) * (p + 1) / 2.0
    lo2 = np.array([lo, lo])
    q_end = np.array([-np.sin(THETA_END), np.cos(THETA_END)])  # outward tangent at theta = 2
    p0 = np.array([1.0, 0.0])

    def key(ij):
        return ij[:, 0] * n + ij[:, 1]

    def coords(ij):
        return lo2 + ij * h

    # active nodes: within rho h of the arc
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ij_all = np.stack([ii.ravel(), jj.ravel()], axis=1)
    x_all = coords(ij_all)
    cp_all, _, _ = closest_point(x_all)
    dist = np.hypot(x_all[:, 0] - cp_all[:, 0], x_all[:, 1] - cp_all[:, 1])
    active = set(key(ij_all[dist <= rho * h]).tolist())

    def interp_points(keys):
        """The points each row of E~ interpolates at, and the row's scale."""
        ij = np.stack([np.array(keys) // n, np.array(keys) % n], axis=1)
        x = coords(ij)
        cp, code, _ = closest_point(x)
        pts = cp.copy()
        scale = np.ones(len(keys))
        m1 = code == 1
        if m1.any():  # mirror point through the Dirichlet end
            xm = 2.0 * p0 - x[m1]
            pts[m1] = closest_point(xm)[0]
            scale[m1] = -1.0
        m2 = code == 2
        if m2.any():  # eq. robfo at the Robin end
            d = x[m2] - cp[m2]
            scale[m2] = 1.0 / (1.0 + alpha * (d @ q_end))
        return pts, scale

    def stencil_keys(pts):
        base, _, _ = _interp_rows(pts, lo2, h, p)
        out = []
        for a in range(p + 1):
            for b in range(p + 1):
                out.append(key(base + np.array([a, b])))
        return np.concatenate(out)

    # closure: every interpolation stencil (of actives and ghosts) is active
    while True:
        act = np.array(sorted(active))
        aij = np.stack([act // n, act % n], axis=1)
        nb = np.concatenate([key(aij + d) for d in ([1, 0], [-1, 0], [0, 1], [0, -1])])
        ghosts = np.setdiff1d(nb, act)
        rows = np.concatenate([act, ghosts])
        pts, _ = interp_points(rows.tolist())
        missing = np.setdiff1d(stencil_keys(pts), act)
        if missing.size == 0:
            break
        active.update(missing.tolist())

    na = len(act)
    index = {k: q for q, k in enumerate(rows.tolist())}
    pts, scale = interp_points(rows.tolist())
    base, wx, wy = _interp_rows(pts, lo2, h, p)
    # E~ (rows: actives then ghosts; columns: actives)
    er, ec, ev = [], [], []
    for a in range(p + 1):
        for b in range(p + 1):
            cols = np.array([index[k] for k in key(base + np.array([a, b])).tolist()])
            er.append(np.arange(len(rows)))
            ec.append(cols)
            ev.append(scale * wx[:, a] * wy[:, b])
    E = sp.csr_matrix((np.concatenate(ev), (np.concatenate(er), np.concatenate(ec))), shape=(len(rows), na))
    # A = (c + 4/h^2) I - h^-2 N E~ on the active rows
    nr, nc = [], []
    for d in ([1, 0], [-1, 0], [0, 1], [0, -1]):
        nr.append(np.arange(na))
        nc.append(np.array([index[k] for k in key(aij + np.array(d)).tolist()]))
    N = sp.csr_matrix((np.ones(4 * na), (np.concatenate(nr), np.concatenate(nc))), shape=(na, len(rows)))
    A = (c + 4.0 / h ** 2) * sp.identity(na, format="csr") - (N @ E) / h ** 2
    xa = coords(aij)
    cpa, code, theta = closest_point(xa)
    f = 1.0 - theta ** 2
    u = spla.spsolve(A.tocsc(), f)
    inner = code == 0
    err = np.abs(u[inner] - exact_solution(theta[inner])).max()
    return {"h": h, "n_act": na, "n_ghost": len(ghosts), "err_inf": float(err), "u": u, "theta": theta,
            "code": code}
