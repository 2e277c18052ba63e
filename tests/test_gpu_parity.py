"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs. Floating-point bars:
* operator apply: 1e-12 relative (same sums, different order);
* FP64 local solves / M^{-1} v: 1e-9 relative (cond(A_j) * eps with margin);
* FP32 local solves: 2e-3 relative (cond(A_j) ~ 1e3 times float eps, margin);
* final solution: 1e-8 relative to the direct solution (both at tol 1e-12).
"""

import json
import os
import sys

import numpy as np
import pytest

import cpm_inputs as ci
import oracle
from oracle import schwarz
import paper_1909_08734_amd as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("prec,kb", [(P.FP64, 32), (P.FP64, 13), (P.FP64, 128), (P.FP64, 77),
                                     (P.FP32, 32), (P.FP32, 7), (P.FP32, 128), (P.FP32, 100)])
def test_matrix_core_tile(prec, kb):
    say("tile selftest", prec, kb)
    rng = np.random.default_rng(kb)
    a = rng.standard_normal((64, kb))
    b = rng.standard_normal((kb, 64))
    c = rng.standard_normal((64, 64))
    if prec == P.FP32:
        a, b, c = (x.astype(np.float32).astype(np.float64) for x in (a, b, c))
    got = P.selftest_tile(a, b, c, prec)
    want = c - a @ b
    assert rel(got, want) < (1e-14 if prec == P.FP64 else 2e-5)


SURF = {"sphere": (ci.Sphere(), 0.1), "torus": (ci.Torus(1.0, 0.4), 0.05),
        "offsphere": (ci.Sphere(1.0, (0.013, 0.027, 0.031)), 0.08),
        "trimesh": (ci.bumpy_icosphere(level=3, far=0.6), 0.1)}


@pytest.mark.parametrize("name,p", [("sphere", 3), ("torus", 3), ("offsphere", 2), ("trimesh", 3)])
def test_operator_apply(name, p):
    say("operator", name, p)
    surf, h = SURF[name]
    b = oracle.build_band(surf, h, p, [-2.0] * 3, [2.0] * 3)
    c = 0.7
    A = oracle.stabilized_operator(b, c)
    ctx = P.Context(0)
    ctx.build_band(surf, h, p)
    ctx.build_operator(c)
    x = np.random.default_rng(1).standard_normal(b.n_act)
    ys = []
    for kernel in (0, 1, 2):  # compact rows, LDS-staged groups, full rows
        ctx.set_operator_kernel(kernel)
        assert ctx.operator_kernel() == kernel
        y = torch.zeros(b.n_act, dtype=torch.float64, device="cuda")
        ctx.apply_operator(dev(x), y)
        ys.append(y.cpu().numpy())
        assert rel(ys[-1], A @ x) < 1e-12
    np.testing.assert_array_equal(ys[1], ys[0])  # same sums in the same order
    np.testing.assert_array_equal(ys[2], ys[0])
    ctx.close()


def _setup(name, p, method, n, no, kind, alpha, alpha_cross, c=1.0):
    surf, h = SURF[name]
    b = oracle.build_band(surf, h, p, [-2.0] * 3, [2.0] * 3)
    base = method.split("+")[0]
    if base == "octant":
        part, code = oracle.octant_partition(b), P.PART_OCTANT
    elif base == "rcb":
        part, code = oracle.rcb_partition(b, n), P.PART_RCB
    else:
        part, code = oracle.graph_partition(b, n), P.PART_GRAPH
    if method.endswith("+align"):
        part, code = oracle.align_interfaces(b, part, p + 1), code | P.PART_ALIGN
    dec = schwarz.decompose(b, part, no, kind, alpha=alpha, alpha_cross=alpha_cross)
    ctx = P.Context(0)
    ctx.build_band(surf, h, p)
    ctx.build_operator(c)
    ctx.partition(code, n, None, no, getattr(P, kind), alpha, alpha_cross)
    return b, dec, ctx


PRECOND_CASES = [
    ("sphere", 3, "octant", 8, 2, "RAS", 0.0, 0.0),
    ("sphere", 3, "rcb", 7, 2, "ORAS", 3.16, 0.0),
    ("torus", 3, "rcb", 16, 3, "ORAS", 4.47, 20.0),
    ("offsphere", 2, "rcb", 5, 1, "ORAS", 2.0, 0.0),
    ("trimesh", 3, "rcb", 8, 2, "ORAS", 3.16, 10.0),
    ("torus", 3, "graph+align", 12, 2, "ORAS", 4.47, 20.0),
    # many small subdomains: |Sigma~_j| of 94-95 rows (a ragged last 8-row tile of W_j),
    # |Sigma_j| of 166-232, one 128-column chunk and a ragged one (FP64) or inside the
    # ragged chunk only (FP32)
    ("sphere", 3, "rcb", 96, 1, "ORAS", 3.16, 0.0),
]


@pytest.mark.parametrize("case", range(len(PRECOND_CASES)),
                         ids=[f"{c[0]}-{c[2]}{c[3]}-{c[5]}" for c in PRECOND_CASES])
@pytest.mark.parametrize("prec", [P.FP64, P.FP32], ids=["fp64", "fp32"])
def test_preconditioner_apply(case, prec):
    args = PRECOND_CASES[case]
    say("precond", args, prec)
    b, dec, ctx = _setup(*args)
    c = 1.0
    ctx.factor(prec)
    # restricted local solution operator of one subdomain against the oracle's local matrix
    j = len(dec.subs) // 2
    sd = dec.subs[j]
    Aj = schwarz.local_matrix(b, dec, j, c)
    inv = np.linalg.inv(Aj)
    pos = np.searchsorted(sd.sigma, sd.tilde)
    W_ref = inv[np.ix_(pos, np.arange(len(sd.sigma)))]
    W = ctx.factor_export(j)
    tol = 1e-9 if prec == P.FP64 else 2e-3
    assert rel(W, W_ref) < tol
    # whole preconditioner on a random vector
    M = schwarz.Preconditioner(b, dec, c)
    v = np.random.default_rng(3).standard_normal(b.n_act)
    z = torch.zeros(b.n_act, dtype=torch.float64, device="cuda")
    ctx.apply_precond(dev(v), z)
    assert rel(z.cpu().numpy(), M.apply(v)) < tol
    ctx.close()


@pytest.mark.parametrize("alpha,prec,tol", [(1e-3, P.FP64, 1e-8), (3.0, P.FP64, 1e-8), (3.0, P.FP32, 2e-2)],
                         ids=["alpha1e-3-fp64", "alpha3-fp64", "alpha3-fp32"])
def test_heavily_pivoting_local_solves_match_oracle(alpha, prec, tol):
    """Torus h = 0.05 in 8 RCB parts (about 8,500 local unknowns), ORAS: the LU
    interchanges hundreds of rows per subdomain (a weak Robin weight alpha
    makes the transmission rows compete with the diagonal), so the rows the
    elimination skips as structurally zero must stay zero under partial
    pivoting (Section 5, LU of the local problems). W_j and M^{-1} v on two
    sampled subdomains against the oracle's dense inverses; cond(A_j) is
    4.5e4 (alpha = 3) and 1.1e6 (alpha = 1e-3), hence the bars."""
    import scipy.linalg as sl
    say("heavy pivoting", alpha, prec)
    b, dec_all, ctx = _setup("torus", 3, "rcb", 8, 2, "ORAS", alpha, 0.0)
    sample = [0, 5]
    dec = schwarz.decompose(b, oracle.rcb_partition(b, 8), 2, "ORAS", alpha=alpha, only=set(sample))
    ctx.factor(prec)
    for j in sample:
        sd = dec.subs[j]
        Aj = schwarz.local_matrix(b, dec, j, 1.0)
        Aj = Aj.toarray() if hasattr(Aj, "toarray") else np.asarray(Aj)
        order = ctx.subdomain(j)["order"]
        _, piv = sl.lu_factor(Aj[np.ix_(order, order)], check_finite=False)
        assert np.count_nonzero(piv != np.arange(len(order))) > 200  # the case pivots heavily
        inv = np.linalg.inv(Aj)
        pos = np.searchsorted(sd.sigma, sd.tilde)
        W_ref = inv[np.ix_(pos, np.arange(len(sd.sigma)))]
        assert rel(ctx.factor_export(j), W_ref) < tol
    M = schwarz.Preconditioner(b, dec, 1.0, subs=sample)
    v = np.random.default_rng(5).standard_normal(b.n_act)
    z_ref = M.apply(v)
    z = torch.zeros(b.n_act, dtype=torch.float64, device="cuda")
    ctx.apply_precond(dev(v), z)
    rows = np.concatenate([dec.subs[j].tilde for j in sample])
    assert rel(z.cpu().numpy()[rows], z_ref[rows]) < tol
    ctx.close()


@pytest.fixture(scope="module")
def direct_cfg1():
    surf, h = SURF["sphere"]
    b = oracle.build_band(surf, h, 3, [-2.0] * 3, [2.0] * 3)
    A = oracle.stabilized_operator(b, 1.0)
    f = ci.rhs_sphere_y20(b.cp[: b.n_act], 1.0)
    return b, A, f, np.linalg.solve(A.toarray(), f)


@pytest.mark.parametrize("kind,prec", [("RAS", P.FP64), ("ORAS", P.FP64), ("ORAS", P.FP32)])
def test_solve_matches_direct_solution(direct_cfg1, kind, prec):
    say("solve cfg1", kind, prec)
    b, A, f, u_ref = direct_cfg1
    ctx = P.Context(0)
    ctx.build_band(ci.Sphere(), 0.1, 3)
    ctx.build_operator(1.0)
    ctx.partition(P.PART_OCTANT, 8, None, 2, getattr(P, kind), 1 / np.sqrt(0.1), 0.0)
    ctx.factor(prec)
    u, info, rc = ctx.solve(f, tol=1e-12, max_iter=500, restart=30)
    assert rc == P.OK and info[0]["relres_true"] <= 1e-12
    assert np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref) < 1e-8
    # the oracle's own preconditioned FGMRES takes about as many iterations
    dec = schwarz.decompose(b, oracle.octant_partition(b), 2, kind, alpha=1 / np.sqrt(0.1))
    _, oinfo = oracle.fgmres(lambda x: A @ x, f, schwarz.Preconditioner(b, dec, 1.0).apply, tol=1e-12)
    slack = 2 if prec == P.FP64 else 8
    assert abs(info[0]["iters"] - oinfo["iters"]) <= slack, (info, oinfo["iters"])
    # device-pointer entry point gives the same answer
    fu = dev(np.stack([f, 2 * f]))
    uu = torch.zeros_like(fu)
    infos, rc = ctx.solve_device(fu, uu, tol=1e-12, max_iter=500, restart=30)
    got = uu.cpu().numpy()
    np.testing.assert_allclose(got[0], u, rtol=0, atol=1e-13 * np.abs(u).max())
    np.testing.assert_allclose(got[1], 2 * u, rtol=0, atol=1e-12 * np.abs(u).max())
    ctx.close()


@pytest.mark.parametrize("kind", ["RAS", "ORAS"])
def test_left_preconditioned_solve_follows_oracle(direct_cfg1, kind):
    """The paper's formulation: GMRES on M^{-1} A u = M^{-1} f stopping on a 10^6
    reduction of the preconditioned residual, against the oracle's gmres_left
    with the oracle's Schwarz preconditioner; at tol 1e-12 both reach the
    direct solution."""
    say("left-preconditioned solve", kind)
    b, A, f, u_ref = direct_cfg1
    alpha = 1 / np.sqrt(0.1)
    ctx = P.Context(0)
    ctx.build_band(ci.Sphere(), 0.1, 3)
    ctx.build_operator(1.0)
    ctx.partition(P.PART_OCTANT, 8, None, 2, getattr(P, kind), alpha, 0.0)
    ctx.factor(P.FP64)
    dec = schwarz.decompose(b, oracle.octant_partition(b), 2, kind, alpha=alpha)
    M = schwarz.Preconditioner(b, dec, 1.0)
    for tol, slack in ((1e-6, 2), (1e-12, 3)):
        fd = dev(f)
        u = torch.zeros_like(fd)
        info, rc = ctx.solve_left(fd, u, tol=tol, max_iter=500, restart=30)
        x, oinfo = oracle.gmres_left(lambda v: A @ v, f, M.apply, tol=tol, restart=30, max_iter=500)
        say("  tol", tol, "gpu", info["iters"], info["relres_est"], info["relres_true"], "oracle", oinfo["iters"],
            oinfo["relres"], oinfo["relres_true"])
        assert rc == P.OK and info["relres_est"] <= tol
        assert abs(info["iters"] - oinfo["iters"]) <= slack
        ug = u.cpu().numpy()
        assert info["relres_true"] == pytest.approx(np.linalg.norm(f - A @ ug) / np.linalg.norm(f), rel=1e-6)
        err = np.linalg.norm(ug - u_ref) / np.linalg.norm(u_ref)
        assert err < (1e-4 if tol == 1e-6 else 1e-8), err
    info, rc = ctx.solve_left(dev(np.zeros_like(f)), torch.zeros(b.n_act, dtype=torch.float64, device="cuda"))
    assert rc == P.OK and info["iters"] == 0
    ctx.close()


def test_restarted_solve_follows_oracle(direct_cfg1):
    # short restart cycles: the restart path (update, true residual, new basis) is exercised
    say("restarted solve")
    b, A, f, u_ref = direct_cfg1
    ctx = P.Context(0)
    ctx.build_band(ci.Sphere(), 0.1, 3)
    ctx.build_operator(1.0)
    ctx.partition(P.PART_RCB, 8, None, 1, P.ORAS, 3.0, 30.0)
    ctx.factor(P.FP64)
    u, info, rc = ctx.solve(f, tol=1e-12, max_iter=400, restart=5)
    assert rc == P.OK and info[0]["cycles"] > 2
    assert np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref) < 1e-8
    dec = schwarz.decompose(b, oracle.rcb_partition(b, 8), 1, "ORAS", alpha=3.0, alpha_cross=30.0)
    _, oinfo = oracle.fgmres(lambda x: A @ x, f, schwarz.Preconditioner(b, dec, 1.0).apply, tol=1e-12,
                             restart=5, max_iter=400)
    assert abs(info[0]["iters"] - oinfo["iters"]) <= 3, (info, oinfo["iters"])
    ctx.close()


def test_solve_edge_cases(direct_cfg1):
    say("edge cases")
    b, A, f, u_ref = direct_cfg1
    ctx = P.Context(0)
    ctx.build_band(ci.Sphere(), 0.1, 3)
    ctx.build_operator(1.0)
    # one subdomain: M = A^{-1}, GMRES converges in one iteration
    ctx.partition(P.PART_RCB, 1, None, 1, P.RAS)
    ctx.factor(P.FP64)
    u, info, rc = ctx.solve(f, tol=1e-12)
    assert info[0]["iters"] == 1 and np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref) < 1e-10
    ctx.partition(P.PART_RCB, 5, None, 2, P.ORAS, 3.0, 30.0)
    with pytest.raises(P.CpmError) as e:
        ctx.solve(f)  # new partition: factor again first
    assert e.value.code == P.ESTATE
    ctx.factor(P.FP64)
    u, info, rc = ctx.solve(np.zeros_like(f))
    assert rc == P.OK and info[0]["iters"] == 0 and not u.any()
    bad = f.copy()
    bad[17] = np.nan
    with pytest.raises(P.CpmError) as e:
        ctx.solve(bad)
    assert e.value.code == P.EINVAL
    u, info, rc = ctx.solve(f, tol=1e-15, max_iter=3, restart=2)
    assert rc == P.ENOTCONV and info[0]["iters"] == 3 and info[0]["cycles"] == 2
    for bad_args in ({"tol": 0.0}, {"max_iter": 0}, {"restart": 65}):
        with pytest.raises(P.CpmError) as e:
            ctx.solve(f, **bad_args)
        assert e.value.code == P.EINVAL
    ctx.close()


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sphere_h0025_seed1_solution.npz")


def golden_solution():
    """u = A^{-1} f of the benchmark problem (seed 1), written by the oracle's
    sparse direct solve (tests/golden/make_sphere_h0025_solution.py)."""
    with np.load(GOLDEN, allow_pickle=False) as z:
        return z["u"], z["lin"], json.loads(str(z["meta"]))


@pytest.mark.parametrize("alpha_pow,cross", [(1.0, False), (0.5, True)])
def test_sphere_h0025_rcb64_oras_sampled(alpha_pow, cross):
    """The benchmark configuration: unit sphere h = 0.025, 64 RCB parts, N_O = 3,
    ORAS with alpha = h^{-1} or alpha = h^{-1/2} with the cross-point weight
    alpha_x = h^{-1}. Three subdomains are checked against the oracle's dense
    local solves; the full solve, with FP64 and with FP32 factors, at a true
    relative residual of 1e-12 is compared element by element with the
    oracle's direct solution (Section 6.1: the Schwarz-preconditioned solve
    reproduces the direct one): within 1e-8 relative."""
    h = 0.025
    alpha = h ** -alpha_pow
    ax = 1.0 / h if cross else 0.0
    say("sphere h=0.025 oracle set-up", alpha, ax)
    b = oracle.build_band(ci.Sphere(), h, 3, [-2.0] * 3, [2.0] * 3)
    A = oracle.stabilized_operator(b, 1.0)
    dec = schwarz.decompose(b, oracle.rcb_partition(b, 64), 3, "ORAS", alpha=alpha, alpha_cross=ax)
    sample = [0, 37, 63]
    M = schwarz.Preconditioner(b, dec, 1.0, subs=sample)
    v = np.random.default_rng(11).standard_normal(b.n_act)
    z_ref = M.apply(v)
    rows = np.concatenate([dec.subs[j].tilde for j in sample])
    f, _ = ci.rhs_sphere_random_sh(b.cp[: b.n_act], 1.0, seed=1)
    u_ref, lin_ref, meta = golden_solution()
    assert meta["n_act"] == b.n_act and meta["seed"] == 1
    np.testing.assert_array_equal(lin_ref, b.lin[: b.n_act])
    assert max(meta["relres_history"]) < 1e-12
    ctx = P.Context(0)
    ctx.build_band(ci.Sphere(), h, 3)
    np.testing.assert_array_equal(ctx.band_arrays(3)["lin"][: b.n_act], lin_ref)
    ctx.build_operator(1.0)
    ctx.partition(P.PART_RCB, 64, None, 3, P.ORAS, alpha, ax)
    for prec, tol in ((P.FP64, 1e-9), (P.FP32, 2e-3)):
        say("sphere h=0.025 factor", prec)
        ctx.factor(prec)
        z = torch.zeros(b.n_act, dtype=torch.float64, device="cuda")
        ctx.apply_precond(dev(v), z)
        assert rel(z.cpu().numpy()[rows], z_ref[rows]) < tol
        say("sphere h=0.025 solve", prec)
        u, info, rc = ctx.solve(f, tol=1e-12, max_iter=1000, restart=30)
        assert rc == P.OK
        assert np.linalg.norm(f - A @ u) / np.linalg.norm(f) <= 1.05e-12
        err = rel(u, u_ref)
        say("sphere h=0.025 max relative error vs the oracle's direct solution", prec, err, info[0]["iters"])
        assert err <= 1e-8
    ctx.close()


@pytest.mark.parametrize("kind", ["RAS", "ORAS"])
def test_stationary_solver_follows_oracle(direct_cfg1, kind):
    say("stationary", kind)
    b, A, f, u_ref = direct_cfg1
    alpha, ax = 1 / np.sqrt(0.1), 10.0
    ctx = P.Context(0)
    ctx.build_band(ci.Sphere(), 0.1, 3)
    ctx.build_operator(1.0)
    ctx.partition(P.PART_OCTANT, 8, None, 2, getattr(P, kind), alpha, ax)
    ctx.factor(P.FP64)
    u = torch.zeros(b.n_act, dtype=torch.float64, device="cuda")
    info, rc = ctx.solve_stationary(dev(f), u, tol=1e-10, max_iter=2000)
    assert rc == P.OK and info["relres_true"] <= 1e-10
    dec = schwarz.decompose(b, oracle.octant_partition(b), 2, kind, alpha=alpha, alpha_cross=ax)
    uo, oinfo = oracle.stationary(lambda x: A @ x, f, schwarz.Preconditioner(b, dec, 1.0).apply, tol=1e-10,
                                  max_iter=2000)
    assert abs(info["iters"] - oinfo["iters"]) <= 1, (info, oinfo["iters"])
    got = u.cpu().numpy()
    assert np.abs(got - u_ref).max() <= 1e-8 * np.abs(u_ref).max()
    # a capped run reports ENOTCONV with the residual reached
    info2, rc2 = ctx.solve_stationary(dev(f), u, tol=1e-14, max_iter=3)
    assert rc2 == P.ENOTCONV and info2["iters"] == 3
    ctx.close()


@pytest.mark.parametrize("prec", [P.FP64, P.FP32], ids=["fp64", "fp32"])
def test_grouped_factorisation_is_identical(prec):
    """Factoring the subdomains in workspace-bounded groups gives bit-identical
    local solution operators and preconditioner applies."""
    say("grouped factor", prec)
    surf, h = SURF["torus"]
    ctxs = []
    for limit in (0, 1):  # default (one group) / 1 byte (one subdomain per group)
        ctx = P.Context(0)
        ctx.build_band(surf, h, 3)
        ctx.build_operator(0.8)
        ctx.partition(P.PART_RCB, 11, None, 3, P.ORAS, 4.47, 20.0)
        ctx.set_factor_workspace(limit)
        ctx.factor(prec)
        ctxs.append(ctx)
    assert ctxs[0].factor_groups() == 1 and ctxs[1].factor_groups() == 11
    for j in (0, 4, 10):
        np.testing.assert_array_equal(ctxs[1].factor_export(j), ctxs[0].factor_export(j))
    na = ctxs[0].band_sizes()[0]
    v = dev(np.random.default_rng(5).standard_normal(na))
    zs = []
    for ctx in ctxs:
        z = torch.zeros(na, dtype=torch.float64, device="cuda")
        ctx.apply_precond(v, z)
        zs.append(z.cpu().numpy())
    np.testing.assert_array_equal(zs[0], zs[1])
    r1, p1 = ctxs[1].footprint_estimate(prec, 30)
    r0, p0 = ctxs[0].footprint_estimate(prec, 30)
    assert r1 == r0 and p1 < p0
    for ctx in ctxs:
        ctx.close()


@pytest.mark.parametrize("prec", [P.FP64, P.FP32], ids=["fp64", "fp32"])
def test_factor_tiles_are_identical_and_autotune_caches_the_faster(prec):
    """Both trailing-update tiles give the same W_j bit for bit; the autotuner
    keeps the faster and later factorisations (any context) use it."""
    say("factor tiles", prec)
    b, dec, ctx = _setup("torus", 3, "rcb", 16, 3, "ORAS", 4.47, 20.0)
    js = (0, 7, 15)
    got = {}
    # the bordered LU's update work with no tile skipped (outer blocks of 128,
    # left-looking 32-wide panels inside)
    dense = 0
    for j in range(16):
        s = ctx.subdomain(j)
        m, t = len(s["sigma"]), len(s["tilde"])
        nj = m + len(s["bnd"])
        rows_j, cols_j = nj + t, nj + m
        for k0 in range(0, nj, 128):
            k1 = min(k0 + 128, nj)
            for k in range(k0 + 32, k1, 32):
                dense += 2 * (k - k0) * (rows_j - k) * min(32, nj - k)
            dense += 2 * (k1 - k0) * (rows_j - k1) * (cols_j - k1)
    for rows in (64, 128):
        ctx.set_factor_tile(rows)
        ctx.factor(prec)
        assert ctx.factor_tile() == rows
        got[rows] = [ctx.factor_export(j) for j in js]
        fl = ctx.factor_flops()
        say("  tile", rows, "matrix-core flops", fl, "of dense", dense)
        assert 0 < fl < 0.7 * dense  # exactly-zero tiles are skipped
    for a, c in zip(got[64], got[128]):
        np.testing.assert_array_equal(a, c)
    ctx.set_factor_tile(0)
    best, ms = ctx.autotune_factor(prec)
    say("  autotune", best, ms)
    assert best in (64, 128) and ctx.factor_tile() == best and min(ms) > 0
    for a, j in zip(got[64], js):
        np.testing.assert_array_equal(ctx.factor_export(j), a)
    other = P.Context(0)
    other.build_band(SURF["torus"][0], SURF["torus"][1], 3)
    other.build_operator(1.0)
    other.partition(P.PART_RCB, 16, None, 3, P.ORAS, 4.47, 20.0)
    other.factor(prec)
    assert other.factor_tile() == best
    np.testing.assert_array_equal(other.factor_export(0), got[64][0])
    with pytest.raises(P.CpmError) as e:
        ctx.set_factor_tile(32)
    assert e.value.code == P.EINVAL
    other.close()
    ctx.close()


@pytest.mark.parametrize("chunk", [8, 264, 1024])
def test_chunked_preconditioner_apply(chunk):
    """The chunked apply (v|Sigma_j staged a chunk at a time) against the oracle
    and the unchunked apply, with chunk widths that leave ragged last chunks."""
    say("chunked precond", chunk)
    b, dec, ctx = _setup("torus", 3, "rcb", 16, 3, "ORAS", 4.47, 20.0)
    ctx.factor(P.FP64)
    assert ctx.precond_chunk() == 0
    na = b.n_act
    v = np.random.default_rng(8).standard_normal(na)
    z0 = torch.zeros(na, dtype=torch.float64, device="cuda")
    ctx.apply_precond(dev(v), z0)
    ctx.set_precond_chunk(chunk)
    ctx.factor(P.FP64)
    assert ctx.precond_chunk() == chunk
    z1 = torch.zeros(na, dtype=torch.float64, device="cuda")
    ctx.apply_precond(dev(v), z1)
    assert rel(z1.cpu().numpy(), z0.cpu().numpy()) < 1e-13
    M = schwarz.Preconditioner(b, dec, 1.0)
    assert rel(z1.cpu().numpy(), M.apply(v)) < 1e-9
    with pytest.raises(P.CpmError):
        ctx.set_precond_chunk(12)
    ctx.close()


def test_one_large_subdomain_uses_chunked_apply_and_is_a_direct_solve():
    """One subdomain of 35k nodes (v|Sigma does not fit in LDS): the chunked
    apply is chosen by itself, and with M^{-1} = A^{-1} FGMRES stops after one
    iteration (up to rounding)."""
    h, c = 0.05, 1.0
    say("one large subdomain")
    b = oracle.build_band(ci.Sphere(), h, 3, [-2.0] * 3, [2.0] * 3)
    assert b.n_act > 20480
    A = oracle.stabilized_operator(b, c)
    ctx = P.Context(0)
    ctx.build_band(ci.Sphere(), h, 3)
    ctx.build_operator(c)
    ctx.partition(P.PART_RCB, 1, None, 2, P.RAS, 0.0, 0.0)
    ctx.factor(P.FP64)
    assert ctx.precond_chunk() > 0
    f = ci.rhs_sphere_random_sh(b.cp[: b.n_act], c, seed=4)[0]
    u, info, rc = ctx.solve(f, tol=1e-10, max_iter=20, restart=30)
    assert rc == P.OK and info[0]["iters"] <= 2, info
    assert np.linalg.norm(f - A @ u) / np.linalg.norm(f) <= 1.05e-10
    # the tilings and their autotuner are for the unchunked apply only
    with pytest.raises(P.CpmError) as e1:
        ctx.set_precond_tiling(1)
    with pytest.raises(P.CpmError) as e2:
        ctx.autotune_precond(reps=1)
    assert e1.value.code == P.ESTATE and e2.value.code == P.ESTATE
    ctx.close()


@pytest.mark.parametrize("prec", [P.FP64, P.FP32], ids=["fp64", "fp32"])
def test_precond_tilings_are_identical_and_autotune_keeps_results(prec):
    """Every tiling of the apply gives the same bits; the autotuner picks one
    of them and the solve is unchanged."""
    b, dec, ctx = _setup("sphere", 3, "rcb", 7, 2, "ORAS", 3.16, 0.0)
    ctx.factor(prec)
    na = b.n_act
    v = dev(np.random.default_rng(9).standard_normal(na))
    ref = None
    for t in range(P.PRECOND_TILINGS):
        ctx.set_precond_tiling(t)
        assert ctx.precond_tiling() == t
        z = torch.zeros(na, dtype=torch.float64, device="cuda")
        ctx.apply_precond(v, z)
        if ref is None:
            ref = z.cpu().numpy()
        else:
            np.testing.assert_array_equal(z.cpu().numpy(), ref)
    with pytest.raises(P.CpmError):
        ctx.set_precond_tiling(P.PRECOND_TILINGS)
    f = ci.rhs_sphere_y20(b.cp[: b.n_act], 1.0)
    ctx.set_precond_tiling(0)
    u0, i0, _ = ctx.solve(f, tol=1e-10, max_iter=300)
    ctx.set_timing(True)
    ctx.apply_precond(v, z)
    before = [ctx.kernel_time(w) for w in (P.TIMER_PRECOND, P.TIMER_EXTEND, P.TIMER_STENCIL)]
    best, ms = ctx.autotune_precond(reps=2)
    say("tiling times (ms)", ms, "best", best)
    assert 0 <= best < P.PRECOND_TILINGS and ctx.precond_tiling() == best and all(x > 0 for x in ms)
    # the caller's kernel timers are left as they were
    assert [ctx.kernel_time(w) for w in (P.TIMER_PRECOND, P.TIMER_EXTEND, P.TIMER_STENCIL)] == before
    assert before[0][1] == 1
    ctx.set_timing(False)
    u1, i1, _ = ctx.solve(f, tol=1e-10, max_iter=300)
    np.testing.assert_array_equal(u1, u0)
    assert i1[0]["iters"] == i0[0]["iters"]
    ctx.close()


def test_graph_replayed_iterations_equal_eager_launches():
    """FGMRES iterations captured as HIP graphs and replayed give the eager
    results bit for bit, replay after replay, with eager work in between, after
    a restart-length change and after a new factorisation."""
    b, dec, ctx = _setup("sphere", 3, "rcb", 7, 2, "ORAS", 3.16, 10.0)
    na = b.n_act
    F = [ci.rhs_sphere_random_sh(b.cp[:na], 1.0, seed=40 + q)[0] for q in range(2)]

    def run(f, restart):
        fd = dev(f)
        u = torch.zeros(na, dtype=torch.float64, device="cuda")
        info, rc = ctx.solve_device(fd, u, tol=1e-10, max_iter=400, restart=restart)
        return u.cpu().numpy(), info[0]["iters"]

    side = torch.cuda.Stream()  # graphs are not captured on the null stream
    with torch.cuda.stream(side):
        for prec in (P.FP64, P.FP32):
            ctx.factor(prec)
            ctx.set_graphs(False)
            eager = {(q, m): run(F[q], m) for q in range(2) for m in (30, 5)}
            ctx.set_graphs(True)
            for rep in range(3):
                for (q, m), (u_e, it_e) in eager.items():
                    u_g, it_g = run(F[q], m)
                    np.testing.assert_array_equal(u_g, u_e)
                    assert it_g == it_e
                # eager work between replays
                z = torch.zeros(na, dtype=torch.float64, device="cuda")
                ctx.apply_precond(dev(F[0]), z)
                ctx.apply_operator(z, z.clone())
                torch.cuda.synchronize()
    ctx.close()
