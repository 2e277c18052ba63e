"""The C ABI's contract on the GPU: work ordered on the caller's stream with no
device-wide synchronisation, per-phase solve times, a new operator constant
with the factors kept (serving's cached preconditioners), and a failed band
set-up that leaves the previous state usable."""

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


H = 0.1


@pytest.fixture(scope="module")
def cfg1():
    b = oracle.build_band(ci.Sphere(), H, 3, [-2.0] * 3, [2.0] * 3)
    f = ci.rhs_sphere_y20(b.cp[: b.n_act], 1.0)
    return b, f


def _ctx(c=1.0, prec=P.FP64):
    ctx = P.Context(0)
    ctx.build_band(ci.Sphere(), H, 3)
    ctx.build_operator(c)
    ctx.partition(P.PART_OCTANT, 8, None, 2, P.ORAS, H ** -0.5, 0.0)
    ctx.factor(prec)
    return ctx


def test_solve_on_a_caller_stream_equals_the_default_path(cfg1):
    """The context queues its work on torch's current stream: a right-hand side
    that torch produces on a side stream right before the call (behind a chain
    of large products) is read only after it is written, without any device
    synchronisation, and the result equals the default-stream solve bit for bit."""
    b, f = cfg1
    say("caller stream")
    ctx = _ctx()
    fd = torch.from_numpy(f).cuda()
    u0 = torch.zeros_like(fd)
    info0, rc0 = ctx.solve_device(fd, u0, tol=1e-12, max_iter=500, restart=30)
    assert rc0 == P.OK
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        big = torch.randn(4096, 4096, dtype=torch.float64, device="cuda")
        for _ in range(4):
            big = (big @ big) * 1e-4
        f2 = torch.zeros_like(fd)
        f2.copy_(fd + 0.0 * big[0, 0])  # written last, behind the products
        u1 = torch.full_like(fd, float("nan"))
        info1, rc1 = ctx.solve_device(f2, u1, tol=1e-12, max_iter=500, restart=30)
        got = u1.cpu().numpy()
    assert rc1 == P.OK and info1[0]["iters"] == info0[0]["iters"]
    np.testing.assert_array_equal(got, u0.cpu().numpy())
    # batches and host vectors on the side stream too
    with torch.cuda.stream(side):
        F = torch.stack([fd, 2 * fd])
        U = torch.zeros_like(F)
        infos, rc = ctx.solve_device(F, U, tol=1e-12, max_iter=500, restart=30)
        uh, _, rch = ctx.solve(f, tol=1e-12, max_iter=500, restart=30)
        Ug = U.cpu().numpy()
    assert rc == P.OK and rch == P.OK
    np.testing.assert_array_equal(Ug[0], got)
    np.testing.assert_array_equal(uh, got)
    ctx.close()


def test_phase_times_with_kernel_timing(cfg1):
    b, f = cfg1
    ctx = _ctx()
    fd = torch.from_numpy(f).cuda()
    u = torch.zeros_like(fd)
    info, _ = ctx.solve_device(fd, u, tol=1e-12, max_iter=500, restart=30)
    assert all(v == 0.0 for v in info[0]["phase_ms"].values())  # timing off
    ctx.set_timing(True)
    info, _ = ctx.solve_device(fd, u, tol=1e-12, max_iter=500, restart=30)
    ph = info[0]["phase_ms"]
    say("phases", ph, "wall", info[0]["ms"])
    assert set(ph) == set(P.PHASES) and all(v > 0 for v in ph.values())
    assert sum(ph.values()) <= 1.05 * info[0]["ms"] + 0.05  # kernels of one stream within the wall time
    pre_ms, pre_n = ctx.kernel_time(P.TIMER_PRECOND)
    # one iteration per cycle may be queued ahead and discarded
    assert info[0]["iters"] <= pre_n <= info[0]["iters"] + info[0]["cycles"]
    assert abs(pre_ms - ph["precond"]) < 1e-9
    kr_ms, kr_n = ctx.kernel_time(P.TIMER_KRYLOV)
    assert kr_n > 0 and abs(kr_ms - ph["orthogonalisation"]) < 1e-9
    ctx.set_timing(False)
    ctx.close()


def test_new_operator_constant_keeps_the_factors(cfg1):
    """Factors made for c_f = 1 precondition the operator of c = 2.7 (eq.
    algRAS with the local operators of c_f): FGMRES still reaches the direct
    solution of (2.7 - Delta_S^h) u = f."""
    b, f = cfg1
    c = 2.7
    A = oracle.stabilized_operator(b, c)
    u_ref = np.linalg.solve(A.toarray(), f)
    ctx = _ctx(1.0)
    assert ctx.factor_c() == 1.0
    ctx.set_operator_c(c)
    assert ctx.factor_c() == 1.0  # still factored for c_f
    u, info, rc = ctx.solve(f, tol=1e-12, max_iter=500, restart=30)
    assert rc == P.OK
    assert np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref) < 1e-8
    # the same answer as factors made for c itself, with at most a few more iterations
    fresh = _ctx(c)
    uf, infof, _ = fresh.solve(f, tol=1e-12, max_iter=500, restart=30)
    assert np.linalg.norm(uf - u_ref) / np.linalg.norm(u_ref) < 1e-8
    say("iterations with factors of c_f / of c", info[0]["iters"], infof[0]["iters"])
    assert info[0]["iters"] <= infof[0]["iters"] + 5
    ctx.factor(P.FP64)
    assert ctx.factor_c() == c
    with pytest.raises(P.CpmError) as e:
        ctx.set_operator_c(-1.0)
    assert e.value.code == P.EINVAL
    ctx.close()
    fresh.close()


def test_failed_band_build_keeps_the_previous_state(cfg1):
    b, f = cfg1
    ctx = _ctx()
    u0, _, _ = ctx.solve(f, tol=1e-12, max_iter=500, restart=30)

    class Broken:
        def cp(self, x):
            raise RuntimeError("no closest point")

    with pytest.raises(P.CpmError) as e:
        ctx.build_band(Broken(), H, 3)
    assert e.value.code == P.ECALLBACK
    with pytest.raises(P.CpmError) as e:  # band leaves a box that is too small
        ctx.build_band(ci.Sphere(), H, 3, lo=(-1.1,) * 3, hi=(1.1,) * 3)
    assert e.value.code == P.EINVAL
    assert ctx.band_sizes()[:2] == (b.n_act, b.n_ghost)
    u1, info, rc = ctx.solve(f, tol=1e-12, max_iter=500, restart=30)  # still factored
    assert rc == P.OK
    np.testing.assert_array_equal(u1, u0)
    ctx.close()
