"""The triangulated-surface input: mesh topology and the exact closest-point
map, checked against brute force over every triangle and against cases with a
known answer."""

import numpy as np
import pytest

import cpm_inputs as ci


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_icosphere_is_a_closed_triangulated_sphere(level):
    v, f = ci.icosphere(level)
    assert len(f) == 20 * 4 ** level
    np.testing.assert_allclose(np.linalg.norm(v, axis=1), 1.0, rtol=0, atol=1e-15)
    e = np.sort(np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]]), axis=1)
    edges, mult = np.unique(e, axis=0, return_counts=True)
    assert (mult == 2).all()  # every edge shared by exactly two faces
    assert len(v) - len(edges) + len(f) == 2  # Euler characteristic of the sphere
    n = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    assert (np.einsum("ij,ij->i", n, v[f].mean(axis=1)) > 0).all()  # outward orientation


def test_bumpy_icosphere_radius_range():
    m = ci.bumpy_icosphere(level=3, amplitude=0.05, lmax=6, seed=4)
    r = np.linalg.norm(m.verts, axis=1)
    assert r.min() >= 0.95 - 1e-12 and r.max() <= 1.05 + 1e-12
    assert np.isclose(np.abs(r - 1).max(), 0.05)  # the field is scaled to unit maximum


def test_closest_point_on_one_triangle():
    a, b, c = np.array([0.0, 0, 0]), np.array([1.0, 0, 0]), np.array([0.0, 1, 0])
    pts = np.array([[0.2, 0.3, 0.7], [-1, -1, 0.5], [2, -0.5, 0], [0.9, 0.9, -1], [-0.5, 0.4, 0.1],
                    [0.3, -2.0, 0.2], [0, 3, 0]])
    want = np.array([[0.2, 0.3, 0], [0, 0, 0], [1, 0, 0], [0.5, 0.5, 0], [0, 0.4, 0], [0.3, 0, 0],
                     [0, 1, 0]])
    A, B, Cc = (np.broadcast_to(q, pts.shape) for q in (a, b, c))
    np.testing.assert_allclose(ci._closest_on_triangles(pts, A, B, Cc), want, atol=1e-15)


def test_trimesh_cp_matches_brute_force():
    m = ci.bumpy_icosphere(level=3, far=0.6)
    rng = np.random.default_rng(0)
    x = rng.standard_normal((300, 3))
    x *= rng.uniform(0.5, 1.5, (300, 1)) / np.linalg.norm(x, axis=1)[:, None]
    cp, nrm = m.cp(x)
    a, b, c = (m.verts[m.faces[:, q]] for q in range(3))
    for i in range(len(x)):
        y = ci._closest_on_triangles(np.broadcast_to(x[i], a.shape), a, b, c)
        d = np.linalg.norm(y - x[i], axis=1)
        k = int(np.argmin(d))
        if d[k] > m.far + m.emax:
            assert np.isnan(cp[i]).all()
            continue
        if np.isnan(cp[i, 0]):  # only points provably farther than `far`
            assert d[k] > m.far
            continue
        np.testing.assert_allclose(cp[i], y[k], rtol=0, atol=1e-14)
        assert abs(np.linalg.norm(cp[i] - x[i]) - d[k]) <= 1e-14
        # reported normal: unit normal of a face attaining the minimum
        ties = np.flatnonzero(d <= d[k] + 1e-14)
        assert any(np.allclose(nrm[i], m.fnrm[t], atol=1e-14) for t in ties)
    # memoized batches return equal, independent copies
    cp2, _ = m.cp(x)
    np.testing.assert_array_equal(cp2, cp)
    cp2[:] = 0
    np.testing.assert_array_equal(m.cp(x)[0], cp)


def test_trimesh_cp_of_surface_points_is_identity():
    m = ci.bumpy_icosphere(level=3, far=0.6)
    rng = np.random.default_rng(1)
    f = rng.integers(0, len(m.faces), 200)
    w = rng.dirichlet([1, 1, 1], 200)
    y = np.einsum("ik,ikj->ij", w, m.verts[m.faces[f]])
    cp, nrm = m.cp(y)
    np.testing.assert_allclose(cp, y, rtol=0, atol=1e-14)
    # off the surface along the face normal, inside the local feature size
    z = y + 1e-3 * m.fnrm[f]
    cpz, _ = m.cp(z)
    np.testing.assert_allclose(cpz, y, rtol=0, atol=1e-12)
