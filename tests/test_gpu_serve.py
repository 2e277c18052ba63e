"""GPU tests of the entry points the request loop uses (implicit steps, context
cloning, footprint estimate) and of the loop itself: every result is the same
alone and in the concurrent mix, under a memory budget that forces evictions,
and each step meets the tolerance against the oracle's operator."""

import sys

import numpy as np
import pytest

import cpm_inputs as ci
import oracle
import paper_1909_08734_amd as P
from paper_1909_08734_amd import serve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def _sphere_ctx(c=1.0, prec=P.FP64, h=0.1):
    ctx = P.Context(0)
    ctx.build_band(ci.Sphere(), h, 3)
    ctx.build_operator(c)
    ctx.partition(P.PART_RCB, 8, None, 2, P.ORAS, h ** -0.5, 1.0 / h)
    ctx.factor(prec)
    return ctx


def test_solve_steps_each_step_meets_tolerance():
    c = 2.0
    b = oracle.build_band(ci.Sphere(), 0.1, 3, [-2.0] * 3, [2.0] * 3)
    A = oracle.stabilized_operator(b, c)
    ctx = _sphere_ctx(c)
    f = ci.rhs_surface_bumps(b.cp[: b.n_act], seed=9)
    fd = torch.from_numpy(f).cuda()
    u = torch.zeros((4, b.n_act), dtype=torch.float64, device="cuda")
    info, rc = ctx.solve_steps(fd, u, c, tol=1e-10, max_iter=500)
    assert rc == P.OK and len(info) == 4
    U = u.cpu().numpy()
    rhs = f
    for k in range(4):
        assert np.linalg.norm(rhs - A @ U[k]) / np.linalg.norm(rhs) <= 1.05e-10, k
        assert info[k]["relres_true"] <= 1e-10
        rhs = c * U[k]
    # the steps decay like a backward Euler heat flow: each is smaller than the last
    assert all(np.linalg.norm(U[k + 1]) < np.linalg.norm(U[k]) for k in range(3))
    # step 0 equals a plain solve
    u0 = torch.zeros(b.n_act, dtype=torch.float64, device="cuda")
    ctx.solve_device(fd, u0, tol=1e-10, max_iter=500)
    np.testing.assert_array_equal(u0.cpu().numpy(), U[0])
    with pytest.raises(P.CpmError):
        ctx.solve_steps(fd, u, float("nan"))
    ctx.close()


def test_clone_factors_equal_fresh_factors_and_estimate_bounds_footprint():
    base = _sphere_ctx(1.0, P.FP32)
    cl = base.clone(0)
    cl.factor(P.FP32)
    for j in (0, 5):
        np.testing.assert_array_equal(cl.factor_export(j), base.factor_export(j))
    cl.build_operator(3.0)
    cl.factor(P.FP32)
    fresh = _sphere_ctx(3.0, P.FP32)
    for j in (0, 5):
        np.testing.assert_array_equal(cl.factor_export(j), fresh.factor_export(j))
    # estimate vs what the context actually holds after a solve (Krylov space allocated)
    na = base.band_sizes()[0]
    f = torch.ones(na, dtype=torch.float64, device="cuda")
    u = torch.zeros_like(f)
    fresh.solve_device(f, u, tol=1e-6, max_iter=200, restart=30)
    res, peak = fresh.footprint_estimate(P.FP32, 30)
    held = fresh.footprint_bytes()
    assert held <= res <= 1.01 * held, (held, res)
    assert peak > res
    for x in (base, cl, fresh):
        x.close()


SURFACES = {
    "sphere": (ci.Sphere(), lambda cp, seed: ci.rhs_surface_bumps(cp, seed)),
    "torus": (ci.Torus(1.0, 0.4), lambda cp, seed: ci.rhs_torus_bumps(cp, 1.0, 0.4, seed)),
    "bumpy": (ci.bumpy_icosphere(level=3, far=0.6), lambda cp, seed: ci.rhs_surface_bumps(cp, seed)),
}


def _requests():
    return serve.poisson_requests(24, 40.0, sorted(SURFACES), [0.08, 0.05], seed=6, steps=(1, 6))


def _serve(reqs, slots, budget=None, realtime=True):
    srv = serve.Server(SURFACES, slots=slots, budget_bytes=budget, keep_solutions=True, c_levels=4)
    try:
        out = srv.run(reqs, realtime=realtime)
        stats = serve.summary(out, srv.makespan)
        stats.update(evictions=srv.evictions, factors=srv.n_factor, peak_used=srv.peak_used)
        return out, stats
    finally:
        srv.close()


def test_serving_mix_equals_alone_and_meets_tolerance():
    reqs = _requests()
    say("mix", len(reqs), "requests")
    mix, st = _serve(reqs, slots=4)
    say("mix stats", st)
    assert st["hit_rate"] > 0
    # concurrency happened: some requests ran at overlapping times
    iv = sorted((r.start, r.finish) for r in mix)
    assert any(iv[q + 1][0] < iv[q][1] for q in range(len(iv) - 1))
    say("alone")
    alone, st1 = _serve(reqs, slots=1, realtime=False)
    say("alone stats", st1)
    for a, m in zip(alone, mix):
        assert a.rid == m.rid and a.c == m.c and a.c_factor == m.c_factor
        assert m.u.shape == (reqs[m.rid].nsteps, a.u.shape[1])
        np.testing.assert_array_equal(m.u, a.u)  # same kernels, same order: bit-identical
        assert max(m.relres) <= 1e-8
    # a memory budget that fits about two factorisations forces evictions and waiting
    peaks = []
    for name, (surf, _) in SURFACES.items():
        for h in (0.08, 0.05):
            ctx = P.Context(-1)
            ctx.build_band(surf, h, 3)
            na = ctx.band_sizes()[0]
            ctx.build_operator(1.0)
            ctx.partition(P.PART_RCB, max(1, round(na / 2200)), None, 3, P.ORAS, h ** -0.5, 1 / h)
            peaks.append(ctx.footprint_estimate(P.FP32, 30)[1] + 7 * na * 8)
            ctx.close()
    budget = int(2.2 * max(peaks))
    tight, st2 = _serve(reqs, slots=4, budget=budget)
    say("tight stats", st2, "budget", budget)
    assert st2["evictions"] > 0 and st2["peak_used"] <= budget
    for a, t in zip(alone, tight):
        np.testing.assert_array_equal(t.u, a.u)
    # each implicit step solves A u_k = c u_{k-1} to the tolerance with the
    # request's own c (oracle operator), though its factors are those of the
    # nearest quantised level: the request with the most steps and the one
    # whose c is farthest from its level
    far = max(mix, key=lambda x: abs(np.log(x.c / x.c_factor)))
    assert abs(np.log(far.c / far.c_factor)) > 0.1
    for r in {max(mix, key=lambda x: len(x.iters)).rid: None, far.rid: None}:
        r = mix[r]
        q = reqs[r.rid]
        assert r.c == q.c
        surf, rhs = SURFACES[q.surface]
        b = oracle.build_band(surf, q.h, 3, [-2.0] * 3, [2.0] * 3)
        A = oracle.stabilized_operator(b, q.c)
        f = rhs(b.cp[: b.n_act], q.seed)
        for k in range(q.nsteps):
            assert np.linalg.norm(f - A @ r.u[k]) / np.linalg.norm(f) <= 1.05e-8, (r.rid, k)
            f = q.c * r.u[k]
