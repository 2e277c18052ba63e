"""Seeded synthetic inputs for the closest point method (CPM) Schwarz solver.

This module is shared by the oracle, the tests and the benchmark. It holds only
*inputs*: surfaces given by their closest-point map (the representation the
paper assumes as given, Section 2.1), real spherical harmonics, and seeded
right-hand-side generators. It contains none of the solver's arithmetic: no
band construction, extension weights, finite differences, partitioning,
Schwarz local problems or Krylov steps.

Every surface exposes ``cp(x) -> (cp, nrm)`` for an ``(n, 3)`` float64 array of
query points, returning the closest points on the surface and the unit surface
normal at those closest points. Points where the closest point is not unique
(a sphere's centre, a torus' axis or core circle) return NaN, which callers
treat as "farther than any band". Only correctly rounded IEEE operations
(+, -, *, /, sqrt) are used, in a fixed evaluation order, so the value for a
point does not depend on how the query is batched.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.special

__all__ = [
    "Sphere",
    "Torus",
    "real_sph_harm",
    "rhs_sphere_y20",
    "rhs_sphere_random_sh",
    "rhs_torus_bumps",
    "torus_area_uniform_points",
    "wrcb_weights",
    "random_vectors",
    "icosphere",
    "bumpy_icosphere",
    "TriMesh",
    "rhs_surface_bumps",
]


def _norm3(a0, a1, a2):
    return np.sqrt((a0 * a0 + a1 * a1) + a2 * a2)


class Sphere:
    """Sphere of radius ``radius`` centred at ``center``."""

    kind = "sphere"

    def __init__(self, radius: float = 1.0, center=(0.0, 0.0, 0.0)):
        self.radius = float(radius)
        self.center = tuple(float(c) for c in center)

    def cp(self, x):
        x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
        d0 = x[:, 0] - self.center[0]
        d1 = x[:, 1] - self.center[1]
        d2 = x[:, 2] - self.center[2]
        r = _norm3(d0, d1, d2)
        with np.errstate(invalid="ignore", divide="ignore"):
            n0 = d0 / r
            n1 = d1 / r
            n2 = d2 / r
        bad = ~(r > 0.0)
        nrm = np.stack([n0, n1, n2], axis=1)
        nrm[bad] = np.nan
        cp = np.empty_like(nrm)
        cp[:, 0] = self.center[0] + self.radius * nrm[:, 0]
        cp[:, 1] = self.center[1] + self.radius * nrm[:, 1]
        cp[:, 2] = self.center[2] + self.radius * nrm[:, 2]
        return cp, nrm


class Torus:
    """Torus around the z axis: core-circle radius ``R``, tube radius ``r``."""

    kind = "torus"

    def __init__(self, R: float = 1.0, r: float = 0.4):
        self.R = float(R)
        self.r = float(r)

    def cp(self, x):
        x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
        rho = np.sqrt(x[:, 0] * x[:, 0] + x[:, 1] * x[:, 1])
        with np.errstate(invalid="ignore", divide="ignore"):
            c0 = self.R * (x[:, 0] / rho)
            c1 = self.R * (x[:, 1] / rho)
            d0 = x[:, 0] - c0
            d1 = x[:, 1] - c1
            d2 = x[:, 2]
            dl = _norm3(d0, d1, d2)
            n0 = d0 / dl
            n1 = d1 / dl
            n2 = d2 / dl
        nrm = np.stack([n0, n1, n2], axis=1)
        bad = ~((rho > 0.0) & (dl > 0.0))
        nrm[bad] = np.nan
        cp = np.empty_like(nrm)
        cp[:, 0] = c0 + self.r * nrm[:, 0]
        cp[:, 1] = c1 + self.r * nrm[:, 1]
        cp[:, 2] = self.r * nrm[:, 2]
        cp[bad] = np.nan
        return cp, nrm


def real_sph_harm(l: int, m: int, xyz):
    """Orthonormal real spherical harmonic Y_l^m evaluated at unit vectors.

    m > 0 uses sqrt(2)(-1)^m Re Y_l^m, m < 0 uses sqrt(2)(-1)^m Im Y_l^|m|,
    m = 0 the complex harmonic itself (Condon-Shortley phase included by scipy).
    """
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    rr = _norm3(xyz[:, 0], xyz[:, 1], xyz[:, 2])
    theta = np.arccos(np.clip(xyz[:, 2] / rr, -1.0, 1.0))
    phi = np.arctan2(xyz[:, 1], xyz[:, 0])
    y = scipy.special.sph_harm_y(l, abs(m), theta, phi)
    if m == 0:
        return y.real.copy()
    s = math.sqrt(2.0) * (-1.0) ** abs(m)
    return s * (y.real if m > 0 else y.imag)


def rhs_sphere_y20(cp, c: float):
    """f = (c + 6) Y_2^0(CP(x)); on the unit sphere the exact solution is Y_2^0."""
    return (c + 6.0) * real_sph_harm(2, 0, cp)


def rhs_sphere_random_sh(cp, c: float, seed: int, lmax: int = 4):
    """f = sum_{l<=lmax, |m|<=l} (c + l(l+1)) a_lm Y_l^m(CP(x)), a_lm ~ N(0,1).

    Returns (f, u_exact) where u_exact = sum a_lm Y_l^m(CP(x)) is the solution
    of the continuous problem on the unit sphere.
    """
    rng = np.random.default_rng(seed)
    f = np.zeros(len(cp))
    u = np.zeros(len(cp))
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            a = rng.standard_normal()
            y = real_sph_harm(l, m, cp)
            f += (c + l * (l + 1)) * a * y
            u += a * y
    return f, u


def torus_area_uniform_points(n: int, R: float, r: float, rng):
    """n points distributed uniformly by area on the torus (rejection sampling)."""
    out = []
    while len(out) < n:
        u = rng.uniform(0.0, 2.0 * math.pi)
        v = rng.uniform(0.0, 2.0 * math.pi)
        w = rng.uniform(0.0, 1.0)
        if w <= (R + r * math.cos(v)) / (R + r):
            out.append(((R + r * math.cos(v)) * math.cos(u),
                        (R + r * math.cos(v)) * math.sin(u),
                        r * math.sin(v)))
    return np.array(out, dtype=np.float64)


def rhs_torus_bumps(cp, R: float, r: float, seed: int, nbumps: int = 16, sigma: float = 0.2):
    """f = sum_b a_b exp(-|CP(x) - y_b|^2 / (2 sigma^2)), y_b area-uniform, a_b ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    centres = torus_area_uniform_points(nbumps, R, r, rng)
    amps = rng.standard_normal(nbumps)
    cp = np.asarray(cp, dtype=np.float64).reshape(-1, 3)
    f = np.zeros(len(cp))
    for b in range(nbumps):
        d = cp - centres[b]
        f += amps[b] * np.exp(-((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
                              / (2.0 * sigma * sigma))
    return f


def wrcb_weights(n_parts: int, seed: int, lo: float = 0.5, hi: float = 2.0):
    """Target part weights for weighted coordinate bisection, w_j ~ U[lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=n_parts).astype(np.float64)


def random_vectors(n: int, k: int, seed: int):
    """k seeded N(0,1) vectors of length n, shape (k, n)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((k, n))


# ---------------------------------------------------------------------------
# Triangulated surfaces
# ---------------------------------------------------------------------------

def icosphere(level: int):
    """Unit icosphere: the icosahedron with every triangle split into four,
    `level` times, vertices pushed to the unit sphere. 20 * 4**level faces."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / math.sqrt(1.0 + t * t) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
             (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
             (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        mid = {}

        def midpoint(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                mid[key] = len(verts) - 1
            return mid[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.array(verts), np.array(faces, dtype=np.int64)


def bumpy_icosphere(level: int = 5, amplitude: float = 0.05, lmax: int = 6, seed: int = 4, far: float = 0.25):
    """Icosphere radially perturbed by a seeded spherical-harmonic field
    B = sum_{l<=lmax,|m|<=l} a_lm Y_l^m, a_lm ~ N(0,1), scaled so max|B| = 1 over
    the vertices: r = 1 + amplitude * B(x/|x|)."""
    verts, faces = icosphere(level)
    rng = np.random.default_rng(seed)
    field = np.zeros(len(verts))
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            field += rng.standard_normal() * real_sph_harm(l, m, verts)
    field /= np.abs(field).max()
    return TriMesh(verts * (1.0 + amplitude * field)[:, None], faces, far=far)


def _closest_on_triangles(p, a, b, c):
    """Closest points to p on triangles (a, b, c) (all (..., 3)), by the Voronoi
    region of p with respect to the triangle's vertices and edges (the published
    point-triangle method of C. Ericson, Real-Time Collision Detection, 2005,
    Section 5.1.5, whose names d1..d6 and va, vb, vc it keeps)."""
    ab = b - a
    ac = c - a
    ap = p - a
    def dot(u, w):
        return (u[..., 0] * w[..., 0] + u[..., 1] * w[..., 1]) + u[..., 2] * w[..., 2]

    d1 = dot(ab, ap)
    d2 = dot(ac, ap)
    bp = p - b
    d3 = dot(ab, bp)
    d4 = dot(ac, bp)
    cp_ = p - c
    d5 = dot(ab, cp_)
    d6 = dot(ac, cp_)
    va = d3 * d6 - d5 * d4
    vb = d5 * d2 - d1 * d6
    vc = d1 * d4 - d3 * d2
    with np.errstate(invalid="ignore", divide="ignore"):
        denom = 1.0 / (va + vb + vc)
        v = vb * denom
        w = vc * denom
    out = a + ab * v[..., None] + ac * w[..., None]  # interior (face region)
    # edge regions
    with np.errstate(invalid="ignore", divide="ignore"):
        t_ab = d1 / (d1 - d3)
        t_ac = d2 / (d2 - d6)
        t_bc = (d4 - d3) / ((d4 - d3) + (d5 - d6))
    e_bc = (va <= 0) & ((d4 - d3) >= 0) & ((d5 - d6) >= 0)
    out = np.where(e_bc[..., None], b + (c - b) * t_bc[..., None], out)
    e_ac = (vb <= 0) & (d2 >= 0) & (d6 <= 0)
    out = np.where(e_ac[..., None], a + ac * t_ac[..., None], out)
    e_ab = (vc <= 0) & (d1 >= 0) & (d3 <= 0)
    out = np.where(e_ab[..., None], a + ab * t_ab[..., None], out)
    # vertex regions
    out = np.where(((d6 >= 0) & (d5 <= d6))[..., None], c, out)
    out = np.where(((d3 >= 0) & (d4 <= d3))[..., None], b, out)
    out = np.where(((d1 <= 0) & (d2 <= 0))[..., None], a, out)
    return out


class TriMesh:
    """Closed triangulated surface with an exact closest-point map.

    cp() returns the closest point on the mesh and the unit normal of the face
    it lies on (lowest face index on ties). Candidates are the faces incident
    to every vertex within d_ub + e_max of the query (d_ub: distance to the
    faces around the nearest vertex, e_max: longest edge): every vertex of the
    closest face lies within e_max of the closest point y and |x - y| <= d_ub,
    so that face is among them. Points with d0 - e_max > far (d0: distance to
    the nearest vertex; such points are farther than `far` from the mesh)
    return NaN, i.e. outside every band; `far` must exceed the distance of every
    band node from the surface. Results are memoized per query batch (identical
    batches recur when two band builders sweep the same grid).
    """

    kind = "trimesh"

    def __init__(self, verts, faces, far: float = 0.25):
        import scipy.spatial

        self.verts = np.ascontiguousarray(verts, dtype=np.float64)
        self.faces = np.ascontiguousarray(faces, dtype=np.int64)
        a, b, c = (self.verts[self.faces[:, q]] for q in range(3))
        n = np.cross(b - a, c - a)
        self.fnrm = n / np.linalg.norm(n, axis=1)[:, None]
        self.emax = float(max(np.linalg.norm(b - a, axis=1).max(), np.linalg.norm(c - b, axis=1).max(),
                              np.linalg.norm(a - c, axis=1).max()))
        self.far = float(far)
        self.tree = scipy.spatial.cKDTree(self.verts)
        nv = len(self.verts)
        valence = np.bincount(self.faces.ravel(), minlength=nv)
        self.vf = np.full((nv + 1, int(valence.max())), -1, dtype=np.int64)  # row nv: no faces
        fill = np.zeros(nv, dtype=np.int64)
        for f, tri in enumerate(self.faces):
            for v in tri:
                self.vf[v, fill[v]] = f
                fill[v] += 1
        self._memo = {}

    def _pairs_closest(self, xs, own, fac):
        y = np.empty((len(fac), 3))
        for q0 in range(0, len(fac), 1 << 20):
            sl = slice(q0, q0 + (1 << 20))
            tri = self.faces[fac[sl]]
            y[sl] = _closest_on_triangles(xs[own[sl]], self.verts[tri[:, 0]], self.verts[tri[:, 1]],
                                          self.verts[tri[:, 2]])
        dd = y - xs[own]
        return y, (dd[:, 0] * dd[:, 0] + dd[:, 1] * dd[:, 1]) + dd[:, 2] * dd[:, 2]

    def _exact(self, xs, v0):
        """Closest points and faces for queries xs with nearest vertices v0."""
        nq = len(xs)
        # Upper bound: the distance to the faces around the nearest vertex.
        F0 = self.vf[v0]
        own0 = np.broadcast_to(np.arange(nq)[:, None], F0.shape)[F0 >= 0]
        _, d2 = self._pairs_closest(xs, own0, F0[F0 >= 0])
        dub = np.sqrt(np.minimum.reduceat(d2, np.searchsorted(own0, np.arange(nq))))
        # Exact: every face with a vertex within dub + e_max.
        lists = self.tree.query_ball_point(xs, dub * (1.0 + 1e-12) + self.emax)
        cnt = np.fromiter((len(q) for q in lists), dtype=np.int64, count=nq)
        vflat = np.fromiter((v for q in lists for v in q), dtype=np.int64, count=int(cnt.sum()))
        F = self.vf[vflat]
        ok = F >= 0
        own = np.broadcast_to(np.repeat(np.arange(nq), cnt)[:, None], F.shape)[ok]
        pair = np.unique(own * len(self.faces) + F[ok])  # sorted by query, then face
        own = pair // len(self.faces)
        fac = pair % len(self.faces)
        y, d2 = self._pairs_closest(xs, own, fac)
        start = np.searchsorted(own, np.arange(nq))
        best = np.minimum.reduceat(d2, start)
        first = np.flatnonzero(d2 == best[own])
        first = first[np.searchsorted(own[first], np.arange(nq))]  # lowest face index on ties
        return y[first], fac[first]

    def cp(self, x):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, 3))
        key = x.tobytes()
        if key in self._memo:
            cp, nrm = self._memo[key]
            return cp.copy(), nrm.copy()
        n = len(x)
        cp = np.full((n, 3), np.nan)
        nrm = np.full((n, 3), np.nan)
        d0, v0 = self.tree.query(x, distance_upper_bound=self.far + self.emax)
        near = np.flatnonzero(np.isfinite(d0) & (d0 - self.emax <= self.far))
        if len(near):
            c, f = self._exact(x[near], v0[near])
            cp[near] = c
            nrm[near] = self.fnrm[f]
        if sum(v[0].nbytes for v in self._memo.values()) > (1 << 30):
            self._memo.clear()
        self._memo[key] = (cp, nrm)
        return cp.copy(), nrm.copy()


def rhs_surface_bumps(cp, seed: int, nbumps: int = 16, sigma: float = 0.2, radius: float = 1.0):
    """f = sum_b a_b exp(-|CP(x) - y_b|^2 / (2 sigma^2)) with bump centres y_b
    uniform on the sphere of the given radius and a_b ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((nbumps, 3))
    centres = radius * g / np.linalg.norm(g, axis=1)[:, None]
    amps = rng.standard_normal(nbumps)
    cp = np.asarray(cp, dtype=np.float64).reshape(-1, 3)
    f = np.zeros(len(cp))
    for q in range(nbumps):
        d = cp - centres[q]
        f += amps[q] * np.exp(-((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]) / (2 * sigma * sigma))
    return f
