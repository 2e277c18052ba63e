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
