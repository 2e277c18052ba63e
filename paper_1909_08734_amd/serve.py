"""Request loop for many closest point method solves on one GPU.

Requests name a surface, a grid spacing h, a value of c and a number of
sequential right-hand sides (implicit steps u^{n+1} = A^{-1}(c u^n)). The
server

* batches continuously: `slots` worker threads each drive one request at a
  time on its own context (own HIP stream), so requests that arrive while
  others run start as soon as a slot and device memory are free, and their
  kernels overlap on the device;
* keeps factorisations resident: one context per (surface, h, c level) holds
  its restricted local solution operators until evicted (least recently used
  first, never while in use); c is quantised to `c_levels` log-spaced levels
  to pick the factors, so that repeated requests hit the cache, while the
  operator and the implicit-step scale use the request's own c
  (cpm_set_operator_c): the cached factors of the nearest level act as the
  preconditioner and FGMRES stops on the true residual of the requested system;
* admits work by device memory: a request's vectors, plus the peak footprint
  of a factorisation (cpm_footprint_estimate) when its factors must be made,
  are reserved in one step against the budget, evicting idle cached factors;
  otherwise the request waits without holding anything, and fails with
  MemoryError when nothing else runs that could free memory;
* shares host set-up: the band and partition of a (surface, h) are built once
  on a host-only context and cloned onto the device for each c level;
* records per-request arrival, start, finish, iteration counts and cache hits,
  from which `summary()` gives p50/p99 latency and solves/s.

Every computation runs in libcpm; this module only schedules calls to it.
"""

from __future__ import annotations

import math
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import binding as B


@dataclass
class Request:
    rid: int
    surface: str
    h: float
    c: float
    nsteps: int
    seed: int
    arrival: float = 0.0  # seconds after the server's start


@dataclass
class Result:
    rid: int
    key: tuple
    c: float          # the request's c (operator and step scale)
    c_factor: float   # the quantised level whose factors precondition it
    arrival: float
    start: float = math.nan
    finish: float = math.nan
    hit: bool = False
    iters: list = field(default_factory=list)
    relres: list = field(default_factory=list)
    status: int = 0
    error: str = ""
    u: np.ndarray | None = None

    @property
    def latency(self):
        return self.finish - self.arrival


class _Entry:
    def __init__(self, ctx, resident):
        self.ctx = ctx
        self.resident = resident
        self.busy = False
        self.last_used = 0.0


class Server:
    """Continuous-batching solve server on one device (see the module docstring).

    surfaces: name -> (surface, rhs) with rhs(cp_actives, seed) -> f, and surface
    either an object with .cp(x) or a callable h -> such an object (e.g. a mesh
    whose closest-point search radius depends on the band width).
    """

    def __init__(self, surfaces, device=0, slots=4, budget_bytes=None, prec=B.FP32, restart=30, tol=1e-8,
                 max_iter=3000, degree=3, overlap=3, nodes_per_sub=2200, c_range=(0.1, 10.0), c_levels=16,
                 keep_solutions=False):
        import torch

        self.torch = torch
        self.surfaces = dict(surfaces)
        self.device = int(device)
        self.slots = int(slots)
        self.prec, self.restart, self.tol, self.max_iter = prec, int(restart), float(tol), int(max_iter)
        self.degree, self.overlap, self.nodes_per_sub = int(degree), int(overlap), int(nodes_per_sub)
        lo, hi = c_range
        # log-spaced levels over the range (one level: its geometric middle)
        if int(c_levels) == 1:
            self.c_grid = np.array([math.sqrt(lo * hi)])
        else:
            self.c_grid = np.exp(np.linspace(math.log(lo), math.log(hi), int(c_levels)))
        self.keep = bool(keep_solutions)
        if budget_bytes is None:
            # the library keeps released factorisation work buffers for reuse
            # outside this ledger: give that cache a tenth of the free memory
            # (at most 64 GiB) and the ledger what is left of 85%
            free, _ = torch.cuda.mem_get_info(self.device)
            cache = min(64 << 30, int(0.10 * free))
            B.set_workspace_cache(cache)
            budget_bytes = int(0.85 * free) - cache
        self.budget = int(budget_bytes)
        self.used = 0
        self.peak_used = 0
        self._lock = threading.Condition()
        self._bases = {}          # (surface, h) -> (host ctx, cp of actives, n_act)
        self._base_locks = {}
        self._cache = {}          # key -> _Entry
        self._building = set()    # keys being factored
        self._claimed = set()     # keys of requests taken by a slot
        self._active = 0          # requests holding a reservation
        self.evictions = 0
        self.factor_s = 0.0
        self.n_factor = 0

    # ---- keys and host set-up --------------------------------------------------------
    def quantise(self, c):
        """Nearest of the log-spaced c levels (in log distance)."""
        k = int(np.argmin(np.abs(np.log(self.c_grid) - math.log(c))))
        return float(self.c_grid[k])

    def key(self, req):
        return (req.surface, float(req.h), self.quantise(req.c))

    def _base(self, surface, h):
        k = (surface, float(h))
        with self._lock:
            lk = self._base_locks.setdefault(k, threading.Lock())
        with lk:
            if k not in self._bases:
                surf, _ = self.surfaces[surface]
                if not hasattr(surf, "cp"):
                    surf = surf(h)
                ctx = B.Context(-1)
                ctx.build_band(surf, h, self.degree)
                na = ctx.band_sizes()[0]
                cp = ctx.band_arrays(self.degree)["cp"][:na].copy()
                ctx.build_operator(1.0)
                n_sub = max(1, int(round(na / self.nodes_per_sub)))
                ctx.partition(B.PART_RCB, n_sub, None, self.overlap, B.ORAS, h ** -0.5, 1.0 / h)
                self._bases[k] = (ctx, cp, na)
            return self._bases[k]

    # ---- device memory ledger -----------------------------------------------------------
    def _try_reserve(self, nbytes, keep=None):
        """Reserve nbytes if they fit, evicting idle cached factors (least
        recently used first, never `keep`). Caller holds the lock. Returns False
        when they do not fit yet; raises MemoryError when they never can (more
        than the budget, or no other request running that could free memory)."""
        if nbytes > self.budget:
            raise MemoryError(f"request needs {nbytes} bytes, budget {self.budget}")
        while self.used + nbytes > self.budget:
            idle = [(e.last_used, k) for k, e in self._cache.items() if not e.busy and k != keep]
            if not idle:
                break
            _, k = min(idle)
            e = self._cache.pop(k)
            e.ctx.close()
            self.used -= e.resident
            self.evictions += 1
        if self.used + nbytes > self.budget:
            if self._active == 0:
                raise MemoryError(f"request needs {nbytes} bytes; {self.used} of {self.budget} are held by "
                                  "factors that cannot be evicted and no other request is running")
            return False
        self.used += nbytes
        self.peak_used = max(self.peak_used, self.used)
        return True

    def _release(self, nbytes):
        self.used -= nbytes
        self._lock.notify_all()

    # ---- device work (separate methods so the scheduling can be tested on the host) ---------
    def _make_factors(self, base, c_level):
        """A device context with the factors of (base's band and partition, c_level)."""
        ctx = base.clone(self.device)
        try:
            ctx.build_operator(c_level)
            ctx.factor(self.prec)
        except Exception:
            ctx.close()
            raise
        return ctx

    def _solve(self, ctx, req, res, f, na, stream):
        """The request's implicit steps on torch stream `stream` (the context follows it)."""
        torch = self.torch
        with torch.cuda.stream(stream):
            f_dev = torch.from_numpy(f).to(f"cuda:{self.device}", non_blocking=False)
            u_dev = torch.empty((req.nsteps, na), dtype=torch.float64, device=f"cuda:{self.device}")
            ctx.set_operator_c(req.c)
            info, rc = ctx.solve_steps(f_dev, u_dev, req.c, tol=self.tol, max_iter=self.max_iter,
                                       restart=self.restart)
            res.iters = [q["iters"] for q in info]
            res.relres = [q["relres_true"] for q in info]
            res.status = rc
            if self.keep:
                res.u = u_dev.cpu().numpy()
            del f_dev, u_dev

    # ---- one request ----------------------------------------------------------------------
    def _admit(self, req, res, vec_bytes):
        """Take the request's cached factors, or the right to make them, and reserve
        its memory in the same step (vectors; plus the factorisation's peak when
        making them). Returns (entry or None, peak, resident)."""
        k = res.key
        base, _, _ = self._base(req.surface, req.h)
        resident, peak = base.footprint_estimate(self.prec, self.restart)
        with self._lock:
            while True:
                e = self._cache.get(k)
                if e is not None and not e.busy:
                    if self._try_reserve(vec_bytes, keep=k):
                        e.busy = True
                        res.hit = True
                        self._active += 1
                        return e, 0, 0
                elif e is None and k not in self._building:
                    if self._try_reserve(peak + vec_bytes):
                        self._building.add(k)
                        self._active += 1
                        return None, peak, resident
                self._lock.wait(0.05)

    def _factor(self, req, res, peak, resident):
        """Make and cache the factors of res.key (peak bytes reserved by _admit)."""
        k = res.key
        try:
            base, _, _ = self._base(req.surface, req.h)
            t0 = time.perf_counter()
            try:
                ctx = self._make_factors(base, k[2])
            except Exception:
                with self._lock:
                    self._release(peak)
                raise
            dt = time.perf_counter() - t0
            e = _Entry(ctx, resident)
            e.busy = True
            with self._lock:
                self.factor_s += dt
                self.n_factor += 1
                self._release(peak - resident)
                self._cache[k] = e
            return e
        finally:
            with self._lock:
                self._building.discard(k)
                self._lock.notify_all()

    def _run(self, req, res, stream):
        _, cp, na = self._base(req.surface, req.h)
        _, rhs = self.surfaces[req.surface]
        f = np.ascontiguousarray(rhs(cp, req.seed), dtype=np.float64)
        vec_bytes = (req.nsteps + 1) * na * 8
        e, peak, resident = self._admit(req, res, vec_bytes)
        try:
            if e is None:
                e = self._factor(req, res, peak, resident)
            try:
                self._solve(e.ctx, req, res, f, na, stream)
            finally:
                with self._lock:
                    e.busy = False
                    e.last_used = time.perf_counter()
                    self._lock.notify_all()
        finally:
            with self._lock:
                self._release(vec_bytes)
                self._active -= 1

    # ---- the loop ----------------------------------------------------------------------------
    def run(self, requests, realtime=True, progress=None):
        """Serve `requests` (arrival times in seconds from now). With realtime=False
        every request is available at once. `progress(done, total)`, if given, is
        called after each request. Returns a list of Result (request order)."""
        torch = self.torch
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        results = {r.rid: Result(r.rid, self.key(r), r.c, self.key(r)[2], r.arrival if realtime else 0.0)
                   for r in reqs}
        pending = []
        state = {"next": 0, "done": 0, "error": None}
        t_start = time.perf_counter()
        self._t0 = t_start

        def now():
            return time.perf_counter() - t_start

        def pick():
            # earliest-arrived request whose factors no other slot is using
            for q, r in enumerate(pending):
                if results[r.rid].key not in self._claimed:
                    self._claimed.add(results[r.rid].key)
                    return pending.pop(q)
            return None

        def worker(wid):
            stream = self._new_stream()
            while True:
                with self._lock:
                    while True:
                        if state["error"] is not None:
                            return
                        r = pick()
                        if r is not None:
                            break
                        if state["next"] >= len(reqs) and not pending:
                            return
                        self._lock.wait(0.01)
                res = results[r.rid]
                res.start = now()
                try:
                    self._run(r, res, stream)
                except Exception as exc:  # recorded; the loop stops admitting new work
                    res.error = f"{type(exc).__name__}: {exc}"
                    with self._lock:
                        state["error"] = res.error
                        self._lock.notify_all()
                res.finish = now()
                with self._lock:
                    self._claimed.discard(res.key)
                    state["done"] += 1
                    done = state["done"]
                    self._lock.notify_all()
                if progress is not None:
                    progress(done, len(reqs))

        threads = [threading.Thread(target=worker, args=(w,), daemon=True) for w in range(self.slots)]
        for t in threads:
            t.start()
        # arrivals
        for i, r in enumerate(reqs):
            if realtime:
                delay = r.arrival - now()
                if delay > 0:
                    time.sleep(delay)
            if state["error"] is not None:
                break
            with self._lock:
                pending.append(r)
                state["next"] = i + 1
                self._lock.notify_all()
        for t in threads:
            t.join()
        self.makespan = now()
        if state["error"] is not None:
            raise RuntimeError(f"serving stopped: {state['error']}")
        return [results[r.rid] for r in sorted(requests, key=lambda r: r.rid)]

    def _new_stream(self):
        return self.torch.cuda.Stream(device=self.device)

    def close(self):
        with self._lock:
            for e in self._cache.values():
                e.ctx.close()
            self._cache.clear()
            self.used = 0
            for ctx, _, _ in self._bases.values():
                ctx.close()
            self._bases.clear()


def summary(results, makespan):
    """Latency percentiles (ms, arrival to last right-hand side) and throughput."""
    lat = np.array([r.latency for r in results]) * 1e3
    solves = sum(len(r.iters) for r in results)
    return {
        "requests": len(results),
        "solves": int(solves),
        "solves_per_s": solves / makespan if makespan > 0 else math.nan,
        "requests_per_s": len(results) / makespan if makespan > 0 else math.nan,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "max_ms": float(lat.max()),
        "hit_rate": float(np.mean([r.hit for r in results])),
        "mean_iters": float(np.mean([np.mean(r.iters) for r in results if r.iters])),
        "worst_relres": float(max(max(r.relres) for r in results if r.relres)),
        "makespan_s": makespan,
    }


def poisson_requests(n, rate, surfaces, hs, seed, c_range=(0.1, 10.0), steps=(1, 32), c_sigma=1.0):
    """n requests with exponential inter-arrival times (rate per second), surfaces
    and h uniform, c log-normal (median sqrt(lo hi)) truncated to c_range by
    redrawing, steps uniform on the inclusive range, RHS seeds from the stream."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n)) if rate > 0 else np.zeros(n)
    lo, hi = c_range
    mu = 0.5 * (math.log(lo) + math.log(hi))
    out = []
    for i in range(n):
        while True:
            c = float(math.exp(rng.normal(mu, c_sigma)))
            if lo <= c <= hi:
                break
        out.append(Request(rid=i, surface=surfaces[int(rng.integers(len(surfaces)))],
                           h=float(hs[int(rng.integers(len(hs)))]), c=c,
                           nsteps=int(rng.integers(steps[0], steps[1] + 1)), seed=int(rng.integers(1 << 31)),
                           arrival=float(t[i])))
    return out
