"""Host logic of the request loop and of the entry points it uses (no GPU):
c quantisation, the arrival generator, latency statistics, the memory ledger,
context cloning and the footprint estimate."""

import math

import numpy as np
import pytest

import cpm_inputs as ci
import paper_1909_08734_amd as P
from paper_1909_08734_amd import serve


def make_server(**kw):
    kw.setdefault("budget_bytes", 1000)
    return serve.Server({}, **kw)


def test_quantise_to_log_levels():
    s = make_server(c_range=(0.1, 10.0), c_levels=16)
    assert len(s.c_grid) == 16
    np.testing.assert_allclose(s.c_grid[[0, -1]], [0.1, 10.0])
    np.testing.assert_allclose(np.diff(np.log(s.c_grid)), math.log(100) / 15)
    for c in [0.1, 0.13, 1.0, 3.3, 9.99, 10.0]:
        q = s.quantise(c)
        assert q in s.c_grid
        assert abs(math.log(q / c)) <= math.log(100) / 30 + 1e-12  # nearest level in log distance
    assert s.quantise(s.c_grid[5]) == s.c_grid[5]


def test_poisson_requests_reproducible_and_in_range():
    a = serve.poisson_requests(500, 20.0, ["sphere", "torus"], [0.05, 0.025], seed=6)
    b = serve.poisson_requests(500, 20.0, ["sphere", "torus"], [0.05, 0.025], seed=6)
    assert [vars(r) for r in a] == [vars(r) for r in b]
    t = np.array([r.arrival for r in a])
    assert (np.diff(t) > 0).all()
    assert abs(len(a) / t[-1] - 20.0) < 3.0  # mean rate
    assert all(0.1 <= r.c <= 10.0 for r in a)
    assert {r.nsteps for r in a} <= set(range(1, 33)) and min(r.nsteps for r in a) == 1
    assert {r.surface for r in a} == {"sphere", "torus"} and {r.h for r in a} == {0.05, 0.025}


def test_summary_percentiles():
    res = []
    for i in range(100):
        r = serve.Result(i, ("s", 0.1, 1.0), 1.0, 1.0, arrival=0.0, start=0.0, finish=(i + 1) / 1000.0)
        r.iters = [10, 12]
        r.relres = [1e-9, 5e-9]
        r.hit = i % 4 != 0
        res.append(r)
    s = serve.summary(res, makespan=2.0)
    assert s["solves"] == 200 and s["solves_per_s"] == 100.0
    assert s["p50_ms"] == pytest.approx(50.5) and s["p99_ms"] == pytest.approx(99.01)
    assert s["hit_rate"] == 0.75 and s["worst_relres"] == 5e-9


class _FakeCtx:
    def __init__(self):
        self.closed = False

    def close(self):
        self.closed = True


def test_ledger_evicts_least_recently_used_idle_entries():
    s = make_server(budget_bytes=100)
    for k, (nb, last, busy) in {"a": (30, 3.0, False), "b": (30, 1.0, False), "c": (30, 2.0, True)}.items():
        e = serve._Entry(_FakeCtx(), nb)
        e.last_used, e.busy = last, busy
        s._cache[k] = e
        s.used += nb
    s._active = 1  # another request runs ("c" is busy)
    with s._lock:
        assert s._try_reserve(35)  # 90 + 35 > 100: evict "b" (oldest idle) only
    assert set(s._cache) == {"a", "c"} and s.used == 95 and s.evictions == 1
    with s._lock:
        with pytest.raises(MemoryError):
            s._try_reserve(101)
        assert not s._try_reserve(50, keep="a")  # must wait: "a" is kept, "c" busy
        assert set(s._cache) == {"a", "c"}
        s._release(35)
    assert s.used == 60 and s.peak_used == 95
    s._active = 0  # nothing else runs: waiting could never end
    with s._lock:
        with pytest.raises(MemoryError):
            s._try_reserve(50, keep="a")


class _FakeBase:
    """Host set-up stand-in: every factorisation reserves `peak`, keeps `resident`."""

    def __init__(self, resident, peak):
        self.fp = (resident, peak)

    def footprint_estimate(self, prec, restart):
        return self.fp


class _HostServer(serve.Server):
    """The request loop with the device work replaced by short sleeps, to test
    the scheduling and the memory ledger on the host."""

    def __init__(self, resident, peak, na, **kw):
        super().__init__({"s": (None, lambda cp, seed: np.zeros(len(cp)))}, **kw)
        self.fake = (_FakeBase(resident, peak), np.zeros((na, 3)), na)
        self.max_used = 0

    def _base(self, surface, h):
        return self.fake

    def _new_stream(self):
        return None

    def _make_factors(self, base, c_level):
        with self._lock:
            self.max_used = max(self.max_used, self.used)
            assert self.used <= self.budget
        import time
        time.sleep(0.01)
        return _FakeCtx()

    def _solve(self, ctx, req, res, f, na, stream):
        import time
        with self._lock:
            self.max_used = max(self.max_used, self.used)
            assert self.used <= self.budget
        time.sleep(0.002)
        res.iters = [1] * req.nsteps
        res.relres = [0.0] * req.nsteps


def test_admission_without_deadlock_under_a_tight_budget():
    """Four slots, a budget just above one factorisation's peak plus the vectors
    of one request: factorisations happen one at a time, cached factors are
    evicted for new ones, and every request finishes."""
    import threading
    na = 1000
    resident, peak = 4000, 10000
    vec = 33 * na * 8  # the largest request: 32 steps + the right-hand side
    s = _HostServer(resident, peak, na, slots=4, budget_bytes=peak + vec + 100, c_levels=4)
    reqs = serve.poisson_requests(40, 0.0, ["s"], [0.1], seed=3)
    out = {}
    th = threading.Thread(target=lambda: out.setdefault("r", s.run(reqs, realtime=False)), daemon=True)
    th.start()
    th.join(60)
    assert not th.is_alive(), "request loop did not finish"
    res = out["r"]
    by_id = sorted(reqs, key=lambda r: r.rid)
    assert len(res) == 40 and all(len(r.iters) == q.nsteps for r, q in zip(res, by_id))
    assert s.max_used <= s.budget and s._active == 0
    assert s.used == sum(e.resident for e in s._cache.values())  # only cached factors stay
    assert all(r.c_factor in s.c_grid and r.c == q.c for r, q in zip(res, by_id))
    assert s.n_factor >= len({s.key(r) for r in reqs})


def test_admission_fails_loudly_when_a_request_can_never_fit():
    na = 1000
    s = _HostServer(4000, 10000, na, slots=2, budget_bytes=5000)
    reqs = serve.poisson_requests(3, 0.0, ["s"], [0.1], seed=3)
    with pytest.raises(RuntimeError, match="MemoryError"):
        s.run(reqs, realtime=False)


def test_clone_and_footprint_estimate_host_only():
    ctx = P.Context(-1)
    with pytest.raises(P.CpmError):
        ctx.footprint_estimate()
    ctx.build_band(ci.Sphere(), 0.1, 3)
    ctx.build_operator(1.0)
    with pytest.raises(P.CpmError):
        ctx.footprint_estimate()  # before the partition
    ctx.partition(P.PART_RCB, 8, None, 2, P.ORAS, 3.0, 30.0)
    r32, p32 = ctx.footprint_estimate(P.FP32, 30)
    r64, p64 = ctx.footprint_estimate(P.FP64, 30)
    r0, _ = ctx.footprint_estimate(P.FP32, 0)
    assert p32 > r32 > r0 > 0 and p64 > r64 > r32
    # the W arena dominates: FP64 adds about its FP32 size again
    n = sum(len(ctx.subdomain(j)["tilde"]) * len(ctx.subdomain(j)["sigma"]) for j in range(8))
    assert 4 * n <= r64 - r32 <= 4 * n * 1.05
    cl = ctx.clone(-1)
    for k in ("lin", "cp", "nbr", "wts"):
        np.testing.assert_array_equal(cl.band_arrays()[k], ctx.band_arrays()[k])
    n0, part0, cross0 = ctx.partition_info()
    n1, part1, cross1 = cl.partition_info()
    assert n0 == n1
    np.testing.assert_array_equal(part0, part1)
    np.testing.assert_array_equal(cross0, cross1)
    assert cl.footprint_estimate(P.FP32, 30) == (r32, p32)
    # a smaller factor workspace lowers the peak, not what stays resident
    cl.set_factor_workspace(1)
    r1, p1 = cl.footprint_estimate(P.FP32, 30)
    assert r1 == r32 and r32 < p1 < p32
    cl.set_factor_workspace(0)
    assert cl.footprint_estimate(P.FP32, 30) == (r32, p32)
    cl.build_operator(2.5)  # a new c keeps the partition
    assert cl.partition_info()[0] == 8
    cl.close()
    empty = P.Context(-1)
    with pytest.raises(P.CpmError):
        empty.clone(-1)
    ctx.close()
    empty.close()


def test_one_level_is_the_middle_of_the_range():
    s = make_server(c_range=(0.1, 10.0), c_levels=1)
    np.testing.assert_allclose(s.c_grid, [1.0])
    assert s.quantise(0.1) == s.quantise(9.9) == s.c_grid[0]
    s3 = make_server(c_range=(0.1, 10.0), c_levels=3)
    np.testing.assert_allclose(s3.c_grid, [0.1, 1.0, 10.0])
    g = s3.c_grid
    assert s3.quantise(0.3) == g[0] and s3.quantise(0.4) == g[1] and s3.quantise(3.0) == g[1] and s3.quantise(4.0) == g[2]
