"""Pins of the oracle's Schwarz node sets, local operators and preconditioner
(paper Sections 2.2, 4 and 5)."""

import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg
import scipy.sparse.linalg as spla

import cpm_inputs as ci
import oracle
from oracle import schwarz


@pytest.fixture(scope="module")
def tiny():
    b = oracle.build_band(ci.Sphere(), 0.2, 3, [-2.0] * 3, [2.0] * 3)
    part = oracle.rcb_partition(b, 6)
    return b, part


def _graph(b):
    na = b.n_act
    r, c = np.nonzero(b.nbr < na)
    return sp.csr_matrix((np.ones(len(r)), (r, b.nbr[r, c])), shape=(na, na))


@pytest.mark.parametrize("no", [1, 2, 3])
def test_overlap_is_graph_distance(tiny, no):
    b, part = tiny
    dec = schwarz.decompose(b, part, no, "ORAS", alpha=2.0)
    G = _graph(b)
    for j, sd in enumerate(dec.subs):
        d = csg.shortest_path(G, unweighted=True, indices=sd.tilde).min(axis=0)
        np.testing.assert_array_equal(sd.sigma, np.flatnonzero(d <= no))
        np.testing.assert_array_equal(sd.final, np.flatnonzero(d == no))


def test_ghost_and_boundary_sets_brute_force(tiny):
    b, part = tiny
    dec = schwarz.decompose(b, part, 2, "RAS")
    na = b.n_act
    for sd in dec.subs[:3]:
        sig = set(sd.sigma.tolist())
        ghost, bnd = set(), set()
        for x in sd.sigma:
            for nb in b.nbr[x]:
                if nb >= na:
                    ghost.add(int(nb))
                elif nb not in sig:
                    bnd.add(int(nb))
        for x in list(sig) + list(ghost):
            for k in b.cols[x]:
                if k not in sig:
                    bnd.add(int(k))
        assert sorted(ghost) == sd.ghost.tolist()
        assert sorted(bnd) == sd.bnd.tolist()


def test_cross_points_brute_force(tiny):
    b, part = tiny
    cross = schwarz.cross_points(b, part)
    na = b.n_act
    for x in range(na):
        others = {int(part[nb]) for nb in b.nbr[x] if nb < na} - {int(part[x])}
        assert cross[x] == (len(others) >= 2)
    assert cross.any()


def test_oras_geometry_brute_force(tiny):
    b, part = tiny
    no = 2
    dec = schwarz.decompose(b, part, no, "ORAS", alpha=3.0, alpha_cross=30.0)
    cross = np.flatnonzero(schwarz.cross_points(b, part))
    for sd in dec.subs[:2]:
        for q, bnode in enumerate(sd.bnd):
            xb = b.xyz[bnode]
            best, arg = math.inf, -1
            for x in sd.final:  # ascending band index: first minimum wins
                d = xb - b.cp[x]
                d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
                if d2 < best:
                    best, arg = d2, x
            assert sd.xstar[q] == arg
            dvec = xb - b.cp[arg]
            n = b.nrm[arg]
            tang = dvec - np.dot(dvec, n) * n
            assert abs(sd.s[q] - np.linalg.norm(tang)) <= 1e-14
            near = any(((b.ijk[bnode] - b.ijk[x]) ** 2).sum() <= (2 * no) ** 2 for x in cross)
            assert sd.alpha[q] == (30.0 if near else 3.0)


@pytest.mark.parametrize("kind", ["RAS", "ORAS"])
def test_single_subdomain_is_global_operator(tiny, kind):
    b, _ = tiny
    c = 1.3
    dec = schwarz.decompose(b, np.zeros(b.n_act, dtype=np.int64), 2, kind, alpha=2.0)
    assert len(dec.subs[0].bnd) == 0
    Aj = schwarz.local_matrix(b, dec, 0, c)
    A = oracle.stabilized_operator(b, c).toarray()
    np.testing.assert_allclose(Aj, A, rtol=1e-13, atol=1e-9)


def test_local_rows_against_global_rows(tiny):
    b, part = tiny
    c = 1.0
    A = oracle.stabilized_operator(b, c).toarray()
    dec = schwarz.decompose(b, part, 2, "ORAS", alpha=2.5)
    sig_ = c + 6.0 / b.h ** 2
    for j in range(2):
        sd = dec.subs[j]
        Aj = schwarz.local_matrix(b, dec, j, c)
        m = len(sd.sigma)
        inside = set(sd.sigma.tolist()) | set(sd.ghost.tolist())
        unk = np.concatenate([sd.sigma, sd.bnd])
        rest = np.setdiff1d(np.arange(b.n_act), unk)
        checked = 0
        for r, x in enumerate(sd.sigma):
            if all(int(nb) in inside for nb in b.nbr[x]):
                # no FD neighbour in B_j: the row is the global row, whose support lies
                # in [Sigma_j ; B_j]
                np.testing.assert_allclose(Aj[r], A[x, unk], atol=1e-9)
                assert not A[x, rest].any()
                checked += 1
        assert checked > 0
        # B rows: (c + 6/h^2) e_b - (6/h^2) E[x*]/(1 + alpha s); E rows sum to one
        rs = Aj[m:].sum(axis=1)
        want = sig_ - (6.0 / b.h ** 2) / (1 + sd.alpha * sd.s)
        np.testing.assert_allclose(rs, want, rtol=1e-9, atol=1e-9)


def test_oras_large_alpha_tends_to_ras():
    # off-centre sphere: no boundary node has d exactly parallel to the normal
    b = oracle.build_band(ci.Sphere(1.0, (0.013, 0.027, 0.031)), 0.2, 3, [-2.0] * 3, [2.0] * 3)
    part = oracle.octant_partition(b)
    c = 1.0
    v = np.random.default_rng(5).standard_normal(b.n_act)
    ras = schwarz.Preconditioner(b, schwarz.decompose(b, part, 2, "RAS"), c).apply(v)
    dec = schwarz.decompose(b, part, 2, "ORAS", alpha=1e15)
    assert min(sd.s.min() for sd in dec.subs) > 1e-6
    oras = schwarz.Preconditioner(b, dec, c).apply(v)
    np.testing.assert_allclose(oras, ras, rtol=1e-7, atol=1e-7 * np.abs(ras).max())


def test_zero_conormal_rows_are_extension_rows(tiny):
    b, part = tiny
    dec = schwarz.decompose(b, part, 2, "ORAS", alpha=4.0)
    dec.subs[0].s = np.zeros_like(dec.subs[0].s)
    sd = dec.subs[0]
    Aj = schwarz.local_matrix(b, dec, 0, 1.0)
    E = oracle.extension_matrix(b).toarray()
    m = len(sd.sigma)
    sig_ = 1.0 + 6.0 / b.h ** 2
    unk = np.concatenate([sd.sigma, sd.bnd])
    for q in range(0, len(sd.bnd), 7):
        row = -(6.0 / b.h ** 2) * E[sd.xstar[q], unk]
        row[m + q] += sig_
        np.testing.assert_allclose(Aj[m + q], row, atol=1e-9)


@pytest.mark.parametrize("kind", ["RAS", "ORAS"])
def test_preconditioned_gmres_reaches_global_solution(kind):
    # Section 6.1 (Figure 7): the DD solution converges to the global discrete solution
    b = oracle.build_band(ci.Sphere(), 0.1, 3, [-2.0] * 3, [2.0] * 3)
    c = 1.0
    A = oracle.stabilized_operator(b, c)
    f = ci.rhs_sphere_y20(b.cp[: b.n_act], c)
    u_ref = np.linalg.solve(A.toarray(), f)
    dec = schwarz.decompose(b, oracle.octant_partition(b), 2, kind, alpha=1 / np.sqrt(0.1))
    M = schwarz.Preconditioner(b, dec, c)
    u, info = oracle.fgmres(lambda v: A @ v, f, M.apply, tol=1e-12)
    assert info["converged"] and info["iters"] < 40
    np.testing.assert_allclose(u, u_ref, rtol=0, atol=1e-9 * np.abs(u_ref).max())
    # one subdomain: M = A^{-1}, one iteration
    dec1 = schwarz.decompose(b, np.zeros(b.n_act, dtype=np.int64), 1, kind, alpha=3.0)
    u1, info1 = oracle.fgmres(lambda v: A @ v, f, schwarz.Preconditioner(b, dec1, c).apply, tol=1e-12)
    assert info1["iters"] == 1
    np.testing.assert_allclose(u1, u_ref, rtol=0, atol=1e-10 * np.abs(u_ref).max())


def test_oras_beats_ras_iterations():
    # qualitative trend of Tables 2-7: ORAS needs fewer iterations than RAS
    b = oracle.build_band(ci.Sphere(), 0.05, 3, [-2.0] * 3, [2.0] * 3)
    c = 1.0
    A = oracle.stabilized_operator(b, c)
    f = ci.rhs_sphere_y20(b.cp[: b.n_act], c)
    part = oracle.rcb_partition(b, 8)
    its = {}
    for kind in ("RAS", "ORAS"):
        dec = schwarz.decompose(b, part, 2, kind, alpha=1 / np.sqrt(0.05))
        M = schwarz.Preconditioner(b, dec, c)
        _, info = oracle.fgmres(lambda v: A @ v, f, M.apply, tol=1e-8)
        its[kind] = info["iters"]
    assert its["ORAS"] < its["RAS"], its


def test_transmission_node_on_the_surface_keeps_local_matrix_regular():
    # Overlap 1 on the h = 0.1 sphere: B nodes at (+-1, 0, 0) lie on the surface and their
    # subsurface closest point is the node itself (d = 0, Kronecker extension row).
    # eq. localOP leaves c u_b = 0 there; the local matrix stays regular.
    b = oracle.build_band(ci.Sphere(), 0.1, 3, [-2.0] * 3, [2.0] * 3)
    part = oracle.rcb_partition(b, 8)
    dec = schwarz.decompose(b, part, 1, "ORAS", alpha=3.0, alpha_cross=30.0)
    found = 0
    for j, sd in enumerate(dec.subs):
        deg = np.flatnonzero((sd.s == 0) & np.all(b.xyz[sd.bnd] == b.cp[sd.xstar], axis=1))
        if len(deg) == 0:
            continue
        found += 1
        Aj = schwarz.local_matrix(b, dec, j, 1.0)
        m = len(sd.sigma)
        for q in deg:
            row = Aj[m + q]
            assert row[m + q] == pytest.approx(1.0) and np.count_nonzero(row) == 1
        assert np.linalg.cond(Aj) < 1e8
    assert found >= 1


def test_stationary_solver_trends_and_fixed_point():
    # Section 2.2: u <- u + M^{-1}(f - A u) converges to A^{-1} f; with one subdomain in
    # one step; ORAS converges in fewer steps than RAS and GMRES in fewer than either
    # (the "Solver" vs "Preconditioner" rows of Tables 2-7)
    b = oracle.build_band(ci.Sphere(), 0.1, 3, [-2.0] * 3, [2.0] * 3)
    c = 1.0
    A = oracle.stabilized_operator(b, c)
    f = ci.rhs_sphere_y20(b.cp[: b.n_act], c)
    u_ref = np.linalg.solve(A.toarray(), f)
    dec1 = schwarz.decompose(b, np.zeros(b.n_act, dtype=np.int64), 1, "RAS")
    u1, i1 = oracle.stationary(lambda x: A @ x, f, schwarz.Preconditioner(b, dec1, c).apply, tol=1e-12)
    assert i1["iters"] == 1 and np.abs(u1 - u_ref).max() < 1e-10 * np.abs(u_ref).max()
    part = oracle.octant_partition(b)
    its = {}
    for kind in ("RAS", "ORAS"):
        dec = schwarz.decompose(b, part, 2, kind, alpha=1 / np.sqrt(0.1), alpha_cross=10.0)
        M = schwarz.Preconditioner(b, dec, c)
        u, info = oracle.stationary(lambda x: A @ x, f, M.apply, tol=1e-10, max_iter=2000)
        assert info["converged"]
        np.testing.assert_allclose(u, u_ref, rtol=0, atol=1e-8 * np.abs(u_ref).max())
        _, ginfo = oracle.fgmres(lambda x: A @ x, f, M.apply, tol=1e-10)
        assert ginfo["iters"] < info["iters"]
        its[kind] = info["iters"]
    assert its["ORAS"] < its["RAS"], its
