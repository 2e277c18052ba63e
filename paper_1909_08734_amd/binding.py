"""ctypes binding of the C ABI in include/cpm.h (argument marshalling only).

Every computation runs in the shared library ``libcpm.so`` built for gfx950;
importing this module fails loudly when the library has not been built.
PyTorch is used only to hand device buffers (``torch.Tensor`` on a HIP
device) and its current HIP stream to the library: a device context queues
its work on torch's current stream of its device (``cpm_set_stream``), after
whatever torch queued there before, so no device-wide synchronisation is
needed around the calls.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpm.so")

OK, ENOTCONV, EINVAL, ESTATE, ENOMEM, ESINGULAR, EDEVICE, ECALLBACK = 0, 1, -1, -2, -3, -4, -5, -6
RAS, ORAS = 0, 1
FP64, FP32 = 0, 1
PART_OCTANT, PART_RCB, PART_GRAPH = 0, 1, 2
PART_ALIGN = 16
PRECOND_TILINGS = 8  # CPM_PRECOND_TILINGS
MULTI_TILINGS = 8  # CPM_MULTI_TILINGS
TIMER_PRECOND, TIMER_EXTEND, TIMER_STENCIL, TIMER_LU_GEMM, TIMER_KRYLOV, TIMER_UPDATE = 0, 1, 2, 3, 4, 5
PHASES = ("precond", "operator", "orthogonalisation", "update")  # cpm_solve_info.phase_ms

_NAMES = {OK: "OK", ENOTCONV: "ENOTCONV", EINVAL: "EINVAL", ESTATE: "ESTATE", ENOMEM: "ENOMEM",
          ESINGULAR: "ESINGULAR", EDEVICE: "EDEVICE", ECALLBACK: "ECALLBACK"}

CP_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double),
                    C.POINTER(C.c_double))


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("cycles", C.c_int32), ("status", C.c_int32),
                ("reserved", C.c_int32), ("relres_true", C.c_double), ("relres_est", C.c_double),
                ("ms", C.c_double), ("phase_ms", C.c_double * 4)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("reserved", "phase_ms")}
        d["phase_ms"] = dict(zip(PHASES, list(self.phase_ms)))
        return d


class CpmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

_SIGS = {
    "cpm_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int]),
    "cpm_destroy": (None, [C.c_void_p]),
    "cpm_clone": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_void_p)]),
    "cpm_set_stream": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "cpm_set_operator_c": (C.c_int, [C.c_void_p, C.c_double]),
    "cpm_factor_c": (C.c_double, [C.c_void_p]),
    "cpm_last_error": (C.c_char_p, [C.c_void_p]),
    "cpm_build_band": (C.c_int, [C.c_void_p, CP_FN, C.c_void_p, C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.c_double, C.c_int, C.c_double]),
    "cpm_build_operator": (C.c_int, [C.c_void_p, C.c_double]),
    "cpm_partition": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_double), C.c_int, C.c_int,
                                C.c_double, C.c_double]),
    "cpm_factor": (C.c_int, [C.c_void_p, C.c_int]),
    "cpm_set_factor_workspace": (C.c_int, [C.c_void_p, C.c_size_t]),
    "cpm_factor_groups": (C.c_int, [C.c_void_p]),
    "cpm_set_precond_chunk": (C.c_int, [C.c_void_p, C.c_int]),
    "cpm_precond_chunk": (C.c_int, [C.c_void_p]),
    "cpm_set_precond_tiling": (C.c_int, [C.c_void_p, C.c_int]),
    "cpm_precond_tiling": (C.c_int, [C.c_void_p]),
    "cpm_autotune_precond": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "cpm_set_graphs": (C.c_int, [C.c_void_p, C.c_int]),
    "cpm_set_operator_kernel": (C.c_int, [C.c_void_p, C.c_int]),
    "cpm_set_factor_tile": (C.c_int, [C.c_void_p, C.c_int]),
    "cpm_factor_tile": (C.c_int, [C.c_void_p]),
    "cpm_autotune_factor": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "cpm_set_multi_tiling": (C.c_int, [C.c_void_p, C.c_int]),
    "cpm_multi_tiling": (C.c_int, [C.c_void_p]),
    "cpm_autotune_multi": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "cpm_operator_kernel": (C.c_int, [C.c_void_p]),
    "cpm_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_double, C.c_int, C.c_int,
                            C.POINTER(SolveInfo)]),
    "cpm_solve_device": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_double, C.c_int,
                                   C.c_int, C.POINTER(SolveInfo)]),
    "cpm_solve_steps": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_double, C.c_double,
                                  C.c_int, C.c_int, C.POINTER(SolveInfo)]),
    "cpm_solve_left": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int, C.c_int,
                                 C.POINTER(SolveInfo)]),
    "cpm_solve_stationary": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int,
                                       C.POINTER(SolveInfo)]),
    "cpm_apply_operator": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "cpm_apply_precond": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "cpm_apply_operator_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "cpm_band_sizes": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                 C.POINTER(C.c_int64)]),
    "cpm_band_arrays": (C.c_int, [C.c_void_p] + [C.c_void_p] * 6),
    "cpm_partition_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.c_void_p, C.c_void_p]),
    "cpm_subdomain_sizes": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int64)]),
    "cpm_subdomain_sets": (C.c_int, [C.c_void_p, C.c_int] + [C.c_void_p] * 8),
    "cpm_factor_flops": (C.c_int, [C.c_void_p, C.c_void_p]),
    "cpm_subdomain_order": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "cpm_factor_export": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "cpm_footprint_bytes": (C.c_size_t, [C.c_void_p]),
    "cpm_footprint_estimate": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_size_t),
                                         C.POINTER(C.c_size_t)]),
    "cpm_set_timing": (C.c_int, [C.c_void_p, C.c_int]),
    "cpm_kernel_time": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "cpm_selftest_tile": (C.c_int, [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "cpm_set_workspace_cache": (C.c_int, [C.c_size_t, C.POINTER(C.c_size_t)]),
    "cpm_workspace_cache": (C.c_int, [C.c_int, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t),
                                      C.POINTER(C.c_size_t)]),
}

EXPORTED = tuple(_SIGS)


def lib():
    """Load libcpm.so (raises if it has not been built).

    torch is imported first when it is installed: its bundled HIP runtime has
    the same soname as the one libcpm.so was linked against, so the library
    then binds to that runtime and the process holds one HIP runtime (whose
    streams the library can use). Loaded the other way round, the process
    would hold two, and torch's could not open the device."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1909_08734_amd.build`")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _dev_ptr(t, dtype="float64"):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("expected a torch tensor on a HIP device")
    if str(t.dtype) != f"torch.{dtype}" or not t.is_contiguous():
        raise TypeError(f"expected a contiguous {dtype} tensor")
    return C.c_void_p(t.data_ptr())


def selftest_tile(a, b, c, prec=FP64, device=0):
    """c - a @ b on one 64x64 matrix-core tile of the LU trailing update (returns new c)."""
    kb = a.shape[1]
    A = np.zeros((64, 128))
    A[:, :kb] = a
    B = np.zeros((128, 64))
    B[:kb] = b
    Cm = np.ascontiguousarray(c, dtype=np.float64).copy()
    rc = lib().cpm_selftest_tile(device, prec, _ptr(A), _ptr(B), _ptr(Cm), kb)
    if rc != 0:
        raise CpmError(rc, "selftest_tile failed")
    return Cm


def set_workspace_cache(nbytes):
    """Most idle bytes of large work buffers kept for reuse per device (0: none);
    returns the idle bytes held on all devices before the call."""
    before = C.c_size_t()
    lib().cpm_set_workspace_cache(int(nbytes), C.byref(before))
    return before.value


def workspace_cache(device=0):
    """(cap, idle bytes, cached bytes in use) of the work-buffer cache on `device`."""
    cap, idle, used = C.c_size_t(), C.c_size_t(), C.c_size_t()
    rc = lib().cpm_workspace_cache(int(device), C.byref(cap), C.byref(idle), C.byref(used))
    if rc != 0:
        raise CpmError(rc, "workspace_cache failed")
    return cap.value, idle.value, used.value


class Context:
    """One solver context (owns device memory and a HIP stream)."""

    def __init__(self, device: int = 0, _handle=None):
        self._L = lib()
        if _handle is None:
            h = C.c_void_p()
            rc = self._L.cpm_create(C.byref(h), int(device))
            if rc != 0:
                raise CpmError(rc, f"cpm_create(device={device}) failed")
            _handle = h
        self._h = _handle
        self._cb = None
        self.device = int(device)
        self._stream = None  # the HIP stream last handed to the library

    def _bind_stream(self):
        """Queue the context's device work on torch's current stream of its device."""
        if self.device < 0:
            return
        import torch
        s = int(torch.cuda.current_stream(self.device).cuda_stream)
        if s != self._stream:
            self._check(self._L.cpm_set_stream(self._h, 1, C.c_void_p(s)), "set_stream")
            self._stream = s

    def clone(self, device=0):
        """New context on `device` with a copy of this one's band, c and partition."""
        h = C.c_void_p()
        rc = self._L.cpm_clone(self._h, int(device), C.byref(h))
        if rc != 0:
            raise CpmError(rc, f"cpm_clone(device={device}) failed")
        return Context(device, _handle=h)

    def close(self):
        if getattr(self, "_h", None):
            self._L.cpm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc, what):
        if rc < 0:
            msg = self._L.cpm_last_error(self._h)
            raise CpmError(rc, f"{what}: {msg.decode() if msg else ''}")
        return rc

    # ---- the five calls of the method -------------------------------------------
    def build_band(self, surface, h, degree=3, lo=(-2.0, -2.0, -2.0), hi=(2.0, 2.0, 2.0),
                   band_factor=0.0):
        def cb(user, n, x, cp, nrm):
            try:
                X = np.ctypeslib.as_array(x, shape=(n, 3))
                c, nr = surface.cp(X)
                np.ctypeslib.as_array(cp, shape=(n, 3))[:] = c
                np.ctypeslib.as_array(nrm, shape=(n, 3))[:] = nr
                return 0
            except Exception:  # reported as ECALLBACK
                return 1
        self._cb = CP_FN(cb)
        lo_a = (C.c_double * 3)(*lo)
        hi_a = (C.c_double * 3)(*hi)
        self._check(self._L.cpm_build_band(self._h, self._cb, None, lo_a, hi_a, float(h), int(degree),
                                           float(band_factor)), "build_band")

    def build_operator(self, c):
        self._check(self._L.cpm_build_operator(self._h, float(c)), "build_operator")

    def set_operator_c(self, c):
        """Change c in the operator, keeping the factors (made for factor_c())."""
        self._check(self._L.cpm_set_operator_c(self._h, float(c)), "set_operator_c")

    def factor_c(self):
        return float(self._L.cpm_factor_c(self._h))

    def partition(self, method=PART_RCB, n_sub=8, weights=None, overlap=2, kind=RAS, alpha=0.0,
                  alpha_cross=0.0):
        w = None
        if weights is not None:
            w = np.ascontiguousarray(weights, dtype=np.float64)
            wp = w.ctypes.data_as(C.POINTER(C.c_double))
        else:
            wp = None
        self._check(self._L.cpm_partition(self._h, int(method), int(n_sub), wp, int(overlap), int(kind),
                                          float(alpha), float(alpha_cross)), "partition")

    def factor(self, prec=FP64):
        self._bind_stream()
        self._check(self._L.cpm_factor(self._h, int(prec)), "factor")

    def set_factor_workspace(self, nbytes=0):
        """Bound the factorisation's work arrays per group of subdomains (0: default)."""
        self._check(self._L.cpm_set_factor_workspace(self._h, int(nbytes)), "set_factor_workspace")

    def factor_groups(self):
        return int(self._L.cpm_factor_groups(self._h))

    def set_precond_chunk(self, columns=0):
        """Force the chunked preconditioner apply with `columns` per pass (0: automatic)."""
        self._check(self._L.cpm_set_precond_chunk(self._h, int(columns)), "set_precond_chunk")

    def precond_chunk(self):
        return int(self._L.cpm_precond_chunk(self._h))

    def set_precond_tiling(self, tiling):
        self._bind_stream()
        self._check(self._L.cpm_set_precond_tiling(self._h, int(tiling)), "set_precond_tiling")

    def precond_tiling(self):
        return int(self._L.cpm_precond_tiling(self._h))

    def set_factor_tile(self, rows=0):
        """Rows of the LU trailing-update tile (64, 128; 0: the tuned one)."""
        self._check(self._L.cpm_set_factor_tile(self._h, int(rows)), "set_factor_tile")

    def factor_tile(self):
        return int(self._L.cpm_factor_tile(self._h))

    def factor_flops(self):
        """Matrix-core flops of the resident factorisation's updates (tiles
        computed; exactly-zero tiles are skipped)."""
        f = C.c_double()
        self._check(self._L.cpm_factor_flops(self._h, C.byref(f)), "factor_flops")
        return f.value

    def autotune_factor(self, prec=FP64):
        """Factor with each trailing-update tile, keep (and cache) the faster.
        Returns (rows, [ms with 64, ms with 128])."""
        best = C.c_int()
        ms = (C.c_double * 2)()
        self._bind_stream()
        self._check(self._L.cpm_autotune_factor(self._h, int(prec), C.byref(best), ms), "autotune_factor")
        return best.value, list(ms)

    def set_multi_tiling(self, tiling):
        self._check(self._L.cpm_set_multi_tiling(self._h, int(tiling)), "set_multi_tiling")

    def multi_tiling(self):
        return int(self._L.cpm_multi_tiling(self._h))

    def autotune_multi(self, reps=3):
        """Time the batched-apply tilings on the resident factors and keep the fastest.
        Returns (best tiling, [ms per tiling])."""
        best = C.c_int()
        ms = (C.c_double * MULTI_TILINGS)()
        self._bind_stream()
        self._check(self._L.cpm_autotune_multi(self._h, int(reps), C.byref(best), ms), "autotune_multi")
        return best.value, list(ms)

    def set_operator_kernel(self, kernel):
        """Extension kernel of the operator apply: 0 gathers, 1 LDS-staged groups."""
        self._check(self._L.cpm_set_operator_kernel(self._h, int(kernel)), "set_operator_kernel")

    def operator_kernel(self):
        return int(self._L.cpm_operator_kernel(self._h))

    def set_graphs(self, on=True):
        """Replay captured FGMRES iterations (HIP graphs) or launch kernels one by one."""
        self._check(self._L.cpm_set_graphs(self._h, 1 if on else 0), "set_graphs")

    def autotune_precond(self, reps=3):
        """Time the apply tilings on the resident factors and keep the fastest.
        Returns (best tiling, [ms per tiling])."""
        best = C.c_int()
        ms = (C.c_double * PRECOND_TILINGS)()
        self._bind_stream()
        self._check(self._L.cpm_autotune_precond(self._h, int(reps), C.byref(best), ms), "autotune_precond")
        return best.value, list(ms)

    def solve(self, f, tol=1e-8, max_iter=1000, restart=30):
        """Host arrays: f (N_A,) or (nrhs, N_A). Returns (u, [info dicts])."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        nrhs = 1 if f.ndim == 1 else f.shape[0]
        u = np.zeros_like(f)
        info = (SolveInfo * max(nrhs, 1))()
        self._bind_stream()
        rc = self._check(self._L.cpm_solve(self._h, _ptr(f), _ptr(u), nrhs, float(tol), int(max_iter),
                                           int(restart), info), "solve")
        return u, [info[q].as_dict() for q in range(nrhs)], rc

    def solve_device(self, f, u, tol=1e-8, max_iter=1000, restart=30):
        """torch float64 HIP tensors f, u of N_A x nrhs (column-major = (nrhs, N_A) row-major),
        used on torch's current stream."""
        nrhs = 1 if f.dim() == 1 else f.shape[0]
        info = (SolveInfo * max(nrhs, 1))()
        self._bind_stream()
        rc = self._check(self._L.cpm_solve_device(self._h, _dev_ptr(f), _dev_ptr(u), nrhs, float(tol),
                                                  int(max_iter), int(restart), info), "solve_device")
        return [info[q].as_dict() for q in range(nrhs)], rc

    def solve_steps(self, f, u, scale, tol=1e-8, max_iter=1000, restart=30):
        """Implicit steps: u[0] = A^{-1} f, u[k] = A^{-1}(scale u[k-1]); torch float64 HIP
        tensors f (N_A) and u (nsteps, N_A)."""
        if u.dim() != 2 or u.shape[1] != f.shape[0]:
            raise ValueError("u must be (nsteps, N_A)")
        nsteps = u.shape[0]
        info = (SolveInfo * max(nsteps, 1))()
        self._bind_stream()
        rc = self._check(self._L.cpm_solve_steps(self._h, _dev_ptr(f), _dev_ptr(u), nsteps, float(scale),
                                                 float(tol), int(max_iter), int(restart), info), "solve_steps")
        return [info[q].as_dict() for q in range(nsteps)], rc

    def solve_left(self, f, u, tol=1e-6, max_iter=1000, restart=30):
        """The paper's left-preconditioned GMRES on torch float64 HIP tensors f, u (N_A),
        stopping when the preconditioned residual has fallen by 1/tol."""
        info = SolveInfo()
        self._bind_stream()
        rc = self._check(self._L.cpm_solve_left(self._h, _dev_ptr(f), _dev_ptr(u), float(tol), int(max_iter),
                                                int(restart), C.byref(info)), "solve_left")
        return info.as_dict(), rc

    def solve_stationary(self, f, u, tol=1e-8, max_iter=1000):
        """(O)RAS as a stationary solver on torch float64 HIP tensors f, u (N_A)."""
        info = SolveInfo()
        self._bind_stream()
        rc = self._check(self._L.cpm_solve_stationary(self._h, _dev_ptr(f), _dev_ptr(u), float(tol),
                                                      int(max_iter), C.byref(info)), "solve_stationary")
        return info.as_dict(), rc

    def apply_operator(self, x, y):
        self._bind_stream()
        self._check(self._L.cpm_apply_operator(self._h, _dev_ptr(x), _dev_ptr(y)), "apply_operator")

    def apply_operator_noalloc(self, x, y):
        """y = A x with the library's static extension scratch (no allocation)."""
        self._bind_stream()
        self._check(self._L.cpm_apply_operator_noalloc(self._h, _dev_ptr(x), _dev_ptr(y)), "apply_operator_noalloc")

    def apply_precond(self, v, z):
        self._bind_stream()
        self._check(self._L.cpm_apply_precond(self._h, _dev_ptr(v), _dev_ptr(z)), "apply_precond")

    # ---- queries --------------------------------------------------------------------
    def band_sizes(self):
        na, ng = C.c_int64(), C.c_int64()
        shape = (C.c_int64 * 3)()
        self._check(self._L.cpm_band_sizes(self._h, C.byref(na), C.byref(ng), shape), "band_sizes")
        return na.value, ng.value, tuple(shape)

    def band_arrays(self, degree=3):
        na, ng, _ = self.band_sizes()
        nt = na + ng
        lin = np.empty(nt, dtype=np.int64)
        cp = np.empty((nt, 3))
        nrm = np.empty((nt, 3))
        nbr = np.empty((na, 6), dtype=np.int32)
        base = np.empty((nt, 3), dtype=np.int32)
        wts = np.empty((nt, 3, degree + 1))
        self._check(self._L.cpm_band_arrays(self._h, _ptr(lin), _ptr(cp), _ptr(nrm), _ptr(nbr), _ptr(base),
                                            _ptr(wts)), "band_arrays")
        return {"lin": lin, "cp": cp, "nrm": nrm, "nbr": nbr, "base": base, "wts": wts}

    def partition_info(self):
        na, _, _ = self.band_sizes()
        n = C.c_int()
        part = np.empty(na, dtype=np.int32)
        cross = np.empty(na, dtype=np.uint8)
        self._check(self._L.cpm_partition_info(self._h, C.byref(n), _ptr(part), _ptr(cross)), "partition_info")
        return n.value, part, cross.astype(bool)

    def subdomain(self, j):
        sz = (C.c_int64 * 5)()
        self._check(self._L.cpm_subdomain_sizes(self._h, int(j), sz), "subdomain_sizes")
        nt, ns, nf, ng, nb = list(sz)
        out = {"tilde": np.empty(nt, np.int32), "sigma": np.empty(ns, np.int32), "final": np.empty(nf, np.int32),
               "ghost": np.empty(ng, np.int32), "bnd": np.empty(nb, np.int32), "xstar": np.empty(nb, np.int32),
               "s": np.empty(nb), "alpha": np.empty(nb)}
        self._check(self._L.cpm_subdomain_sets(self._h, int(j), *[_ptr(out[k]) for k in
                                                                   ("tilde", "sigma", "final", "ghost", "bnd",
                                                                    "xstar", "s", "alpha")]), "subdomain_sets")
        nu = C.c_int64(0)
        self._check(self._L.cpm_subdomain_order(self._h, int(j), C.byref(nu), None), "subdomain_order")
        out["order"] = np.empty(nu.value, np.int32)
        self._check(self._L.cpm_subdomain_order(self._h, int(j), None, _ptr(out["order"])), "subdomain_order")
        return out

    def factor_export(self, j):
        s = self.subdomain(j)
        w = np.empty((len(s["tilde"]), len(s["sigma"])))
        self._bind_stream()
        self._check(self._L.cpm_factor_export(self._h, int(j), _ptr(w)), "factor_export")
        return w

    def footprint_bytes(self):
        return int(self._L.cpm_footprint_bytes(self._h))

    def footprint_estimate(self, prec=FP32, restart=30):
        """(resident, peak) device bytes of a factorisation in `prec`, before making it."""
        res, peak = C.c_size_t(), C.c_size_t()
        self._check(self._L.cpm_footprint_estimate(self._h, int(prec), int(restart), C.byref(res),
                                                   C.byref(peak)), "footprint_estimate")
        return int(res.value), int(peak.value)

    def set_timing(self, on=True):
        self._check(self._L.cpm_set_timing(self._h, 1 if on else 0), "set_timing")

    def kernel_time(self, which):
        ms, n = C.c_double(), C.c_int64()
        self._check(self._L.cpm_kernel_time(self._h, int(which), C.byref(ms), C.byref(n)), "kernel_time")
        return ms.value, n.value
