"""Lockstep batches of right-hand sides: several solves share each pass over
the factors, and every right-hand side follows the single-solve sequence, so a
batched solve equals separate solves bit for bit (solutions, iteration counts,
statuses), including zero right-hand sides, restarts and max_iter stops."""

import sys

import numpy as np
import pytest

import cpm_inputs as ci
import oracle
import paper_1909_08734_amd as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def _ctx(h, n_sub, prec, kind=P.ORAS):
    ctx = P.Context(0)
    ctx.build_band(ci.Sphere(), h, 3)
    ctx.build_operator(1.0)
    ctx.partition(P.PART_RCB, n_sub, None, 2, kind, h ** -0.5, 1.0 / h)
    ctx.factor(prec)
    return ctx


def _rhs(cp, n):
    F = [ci.rhs_sphere_random_sh(cp, 1.0, seed=20 + q)[0] for q in range(n)]
    F[1] = ci.rhs_sphere_y20(cp, 1.0)  # a smooth one that converges sooner
    if n > 3:
        F[3] = np.zeros_like(F[3])     # a zero right-hand side
    return np.stack(F)


def _single(ctx, F, **kw):
    U, infos = [], []
    for q in range(F.shape[0]):
        f = torch.from_numpy(F[q]).cuda()
        u = torch.zeros_like(f)
        info, rc = ctx.solve_device(f, u, **kw)
        U.append(u.cpu().numpy())
        infos.append((info[0]["iters"], info[0]["status"], info[0]["cycles"]))
    return np.stack(U), infos


@pytest.mark.parametrize("prec", [P.FP64, P.FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("restart,max_iter", [(30, 500), (4, 500), (30, 6)], ids=["plain", "restarts", "max_iter"])
def test_batched_solve_equals_separate_solves(prec, restart, max_iter):
    say("batch", prec, restart, max_iter)
    ctx = _ctx(0.1, 8, prec)
    na = ctx.band_sizes()[0]
    cp = ctx.band_arrays(3)["cp"][:na]
    F = _rhs(cp, 7)  # a batch of 4, one of 2 and a single one
    kw = dict(tol=1e-10, max_iter=max_iter, restart=restart)
    U1, info1 = _single(ctx, F, **kw)
    Fd = torch.from_numpy(F).cuda()
    Ud = torch.zeros_like(Fd)
    info, rc = ctx.solve_device(Fd, Ud, **kw)
    np.testing.assert_array_equal(Ud.cpu().numpy(), U1)
    assert [(i["iters"], i["status"], i["cycles"]) for i in info] == info1
    assert info1[3][0] == 0 and np.all(U1[3] == 0)
    if max_iter == 6:
        assert rc == P.ENOTCONV and all(i[1] == P.ENOTCONV for q, i in enumerate(info1) if q != 3)
    else:
        assert rc == P.OK and info1[1][0] < info1[0][0]
    ctx.close()


def test_batched_solve_at_benchmark_size_meets_tolerance():
    """Four right-hand sides on the h = 0.025 sphere (64 parts, FP32 factors):
    bit-identical to separate solves, each within tolerance of the oracle's
    operator, and faster than four separate solves."""
    import time
    h = 0.025
    ctx = _ctx(h, 64, P.FP32)
    na = ctx.band_sizes()[0]
    cp = ctx.band_arrays(3)["cp"][:na]
    F = np.stack([ci.rhs_sphere_random_sh(cp, 1.0, seed=30 + q)[0] for q in range(4)])
    kw = dict(tol=1e-8, max_iter=1000, restart=30)
    _single(ctx, F[:1], **kw)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    U1, info1 = _single(ctx, F, **kw)
    t_single = time.perf_counter() - t0
    Fd = torch.from_numpy(F).cuda()
    Ud = torch.zeros_like(Fd)
    ctx.solve_device(Fd, Ud, **kw)  # warm-up (batch workspace)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info, rc = ctx.solve_device(Fd, Ud, **kw)
    t_batch = time.perf_counter() - t0
    say(f"4 separate solves {t_single * 1e3:.1f} ms, one batch {t_batch * 1e3:.1f} ms, iters", info1)
    np.testing.assert_array_equal(Ud.cpu().numpy(), U1)
    b = oracle.build_band(ci.Sphere(), h, 3, [-2.0] * 3, [2.0] * 3)
    A = oracle.stabilized_operator(b, 1.0)
    for q in range(4):
        assert np.linalg.norm(F[q] - A @ U1[q]) / np.linalg.norm(F[q]) <= 1.05e-8
    assert t_batch < 0.7 * t_single
    ctx.close()


@pytest.mark.parametrize("prec", [P.FP64, P.FP32], ids=["fp64", "fp32"])
def test_every_multi_tiling_equals_separate_solves(prec):
    """Each tiling of the batched apply (rows per wave, chunks in flight, and
    the double-buffered forms) gives the separate solves' bits. At h = 0.05
    with 5 parts every W_j has many full 16-byte-per-lane chunks, and both the
    chunk counts and the counts of pairs of chunks are odd for some subdomains
    and even for others, so the double-buffered loops (groups of one and of
    two chunks) run every ending."""
    ctx = _ctx(0.05, 5, prec)
    cw = 128 if prec == P.FP64 else 256
    nfull = [((len(ctx.subdomain(j)["sigma"]) + 7) // 8 * 8) // cw for j in range(5)]
    say("multi tilings", prec, "full chunks per subdomain", nfull)
    assert min(nfull) >= 4
    assert {n % 2 for n in nfull} == {0, 1} and {n // 2 % 2 for n in nfull} == {0, 1}
    na = ctx.band_sizes()[0]
    cp = ctx.band_arrays(3)["cp"][:na]
    F = _rhs(cp, 7)
    kw = dict(tol=1e-10, max_iter=500, restart=30)
    U1, info1 = _single(ctx, F, **kw)
    Fd = torch.from_numpy(F).cuda()
    for t in range(P.MULTI_TILINGS):
        ctx.set_multi_tiling(t)
        Ud = torch.zeros_like(Fd)
        info, rc = ctx.solve_device(Fd, Ud, **kw)
        say("  tiling", t, "rc", rc)
        np.testing.assert_array_equal(Ud.cpu().numpy(), U1)
        assert [(i["iters"], i["status"], i["cycles"]) for i in info] == info1
    best, ms = ctx.autotune_multi(reps=2)
    say("  autotune", best, ["%.3f" % m for m in ms])
    assert 0 <= best < P.MULTI_TILINGS and ctx.multi_tiling() == best
    assert len(ms) == P.MULTI_TILINGS and all(m > 0 for m in ms)
    ctx.close()
