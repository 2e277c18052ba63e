"""The C-ABI library loads, exports every declared symbol, and its host-side
set-up (band, partitions, Schwarz node sets) equals the oracle bit for bit.
No device calls: contexts are host-only (device = -1)."""

import ctypes
import os
import re

import numpy as np
import pytest

import cpm_inputs as ci
import oracle
from oracle import schwarz
import paper_1909_08734_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "cpm.h")).read()
    return sorted(set(re.findall(r"\b(cpm_[a-z_]+)\s*\(", text)) - {"cpm_cp_fn"})


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(P.binding.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(P.EXPORTED) == names


def test_one_hip_runtime_in_the_process():
    """Loading the library binds it to torch's HIP runtime (same soname), so a
    fresh process that loads the library before touching torch holds one HIP
    runtime, not two (two cannot both open the device)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_1909_08734_amd as P\n"
            "P.lib()\n"
            "maps = open('/proc/self/maps').read()\n"
            "print(sorted(set(l.split()[-1] for l in maps.splitlines() if 'libamdhip64' in l)))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    libs = eval(out.stdout.strip().splitlines()[-1])
    assert len(libs) == 1, libs


def test_binding_constants_match_header():
    """Every #define and enum value of the header is mirrored by the binding."""
    text = open(os.path.join(ROOT, "include", "cpm.h")).read()
    defines = dict(re.findall(r"#define\s+CPM_([A-Z_]+)\s+(-?\d+)", text))
    enums = dict(re.findall(r"\bCPM_([A-Z0-9_]+)\s*=\s*(-?\d+)", text))
    values = {**enums, **defines}
    assert int(values["PRECOND_TILINGS"]) == P.PRECOND_TILINGS
    assert int(values["MULTI_TILINGS"]) == P.MULTI_TILINGS
    for name in ("OK", "ENOTCONV", "EINVAL", "ESTATE", "ENOMEM", "ESINGULAR", "EDEVICE", "RAS", "ORAS", "FP64",
                 "FP32", "PART_OCTANT", "PART_RCB", "PART_GRAPH", "PART_ALIGN"):
        assert int(values[name]) == getattr(P, name), name
    assert int(values["N_TIMERS"]) == P.TIMER_UPDATE + 1
    # the solve record: 4 int32, 3 doubles, then the phase times
    assert ctypes.sizeof(P.SolveInfo) == 16 + 3 * 8 + 4 * 8 and len(P.PHASES) == 4


def test_failed_band_build_keeps_state_and_operator_constant_host_only():
    """A failed cpm_build_band leaves band, operator and partition as they were;
    cpm_set_operator_c changes c without leaving the partitioned state."""
    ctx = P.Context(-1)
    ctx.build_band(ci.Sphere(), 0.1, 3)
    ctx.build_operator(1.0)
    ctx.partition(P.PART_RCB, 8, None, 2, P.ORAS, 3.0, 30.0)
    lin = ctx.band_arrays(3)["lin"].copy()

    class Broken:
        def cp(self, x):
            raise RuntimeError("no closest point")

    with pytest.raises(P.CpmError) as e:
        ctx.build_band(Broken(), 0.1, 3)
    assert e.value.code == P.ECALLBACK
    with pytest.raises(P.CpmError) as e:
        ctx.build_band(ci.Sphere(), 0.1, 3, lo=(-1.1,) * 3, hi=(1.1,) * 3)
    assert e.value.code == P.EINVAL
    np.testing.assert_array_equal(ctx.band_arrays(3)["lin"], lin)
    assert ctx.partition_info()[0] == 8
    ctx.footprint_estimate(P.FP32, 30)  # still partitioned
    with pytest.raises(P.CpmError) as e:  # the batched apply's plan needs factors
        ctx.set_multi_tiling(1)
    assert e.value.code == P.ESTATE
    ctx.set_operator_c(2.0)
    assert ctx.partition_info()[0] == 8 and ctx.factor_c() == 0.0
    for bad in (0.0, -1.0, float("nan")):
        with pytest.raises(P.CpmError) as e:
            ctx.set_operator_c(bad)
        assert e.value.code == P.EINVAL
    L = P.lib()
    assert L.cpm_set_stream(ctx._h, 1, None) == P.EDEVICE  # host-only context
    ctx.close()
    fresh = P.Context(-1)
    with pytest.raises(P.CpmError) as e:
        fresh.set_operator_c(1.0)
    assert e.value.code == P.ESTATE
    fresh.close()


CASES = [
    (ci.Sphere(), 0.1, 3, "rcb", 8, 2),
    (ci.Sphere(), 0.1, 3, "octant", 8, 2),
    (ci.Torus(1.0, 0.4), 0.05, 3, "rcb", 12, 3),
    (ci.Sphere(1.0, (0.013, 0.027, 0.031)), 0.08, 2, "wrcb", 6, 1),
    (ci.bumpy_icosphere(level=3, far=0.6), 0.1, 3, "rcb", 8, 2),
    (ci.Torus(1.0, 0.4), 0.05, 3, "graph", 12, 3),
    (ci.Sphere(), 0.1, 2, "graph+align", 7, 2),
    (ci.Torus(1.0, 0.4), 0.05, 3, "rcb+align", 16, 2),
    (ci.Sphere(1.0, (0.013, 0.027, 0.031)), 0.08, 3, "wgraph+align", 6, 1),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("kind", ["RAS", "ORAS"])
def test_host_setup_matches_oracle(case, kind):
    surf, h, p, method, n, no = CASES[case]
    b = oracle.build_band(surf, h, p, [-2.0] * 3, [2.0] * 3)
    ctx = P.Context(-1)
    ctx.build_band(surf, h, p)
    na, ng, shape = ctx.band_sizes()
    assert (na, ng) == (b.n_act, b.n_ghost) and shape == b.shape
    arr = ctx.band_arrays(p)
    np.testing.assert_array_equal(arr["lin"], b.lin)
    np.testing.assert_array_equal(arr["nbr"], b.nbr)
    np.testing.assert_array_equal(arr["base"], b.base)
    np.testing.assert_array_equal(arr["cp"], b.cp)
    np.testing.assert_allclose(arr["wts"], b.wts, rtol=0, atol=1e-15)
    ctx.build_operator(1.0)
    weights = ci.wrcb_weights(n, seed=2) if method.startswith("w") else None
    base = method.split("+")[0].lstrip("w")
    if base == "octant":
        opart = oracle.octant_partition(b)
        code = P.PART_OCTANT
    elif base == "rcb":
        opart = oracle.rcb_partition(b, n, weights=weights)
        code = P.PART_RCB
    else:
        opart = oracle.graph_partition(b, n, weights=weights)
        code = P.PART_GRAPH
    if method.endswith("+align"):
        opart = oracle.align_interfaces(b, opart, p + 1)
        code |= P.PART_ALIGN
    ctx.partition(code, n, weights, no, getattr(P, kind), 3.0, 30.0)
    nsub, part, cross = ctx.partition_info()
    dec = schwarz.decompose(b, opart, no, kind, alpha=3.0, alpha_cross=30.0)
    assert nsub == len(dec.subs)
    np.testing.assert_array_equal(part, opart)
    np.testing.assert_array_equal(cross, dec.cross)
    for j in range(nsub):
        s = ctx.subdomain(j)
        o = dec.subs[j]
        for k in ("tilde", "sigma", "final", "ghost", "bnd"):
            np.testing.assert_array_equal(s[k], getattr(o, k), err_msg=f"{k} of part {j}")
        n_unk = len(o.sigma) + (len(o.bnd) if kind == "ORAS" else 0)
        np.testing.assert_array_equal(np.sort(s["order"]), np.arange(n_unk))
        if kind == "ORAS":
            np.testing.assert_array_equal(s["xstar"], o.xstar)
            np.testing.assert_array_equal(s["alpha"], o.alpha)
            np.testing.assert_allclose(s["s"], o.s, rtol=0, atol=1e-15)


def _cm_violations(S, order):
    """Checks that reversing `order` gives a Cuthill-McKee order of the
    symmetric pattern S (no diagonal): breadth-first, each component started
    at a remaining node of least degree (lowest index on ties), the nodes
    found from one parent in increasing degree (then index). Returns a list
    of violations (empty if none)."""
    n = S.shape[0]
    deg = np.diff(S.indptr)
    cm = np.asarray(order[::-1])
    pos = np.empty(n, np.int64)
    pos[cm] = np.arange(n)
    bad = []
    last_parent = -1
    prev = None  # (parent, degree, index) of the previous node
    for i, v in enumerate(cm):
        nb = S.indices[S.indptr[v]:S.indptr[v + 1]]
        earlier = pos[nb][pos[nb] < i]
        if earlier.size == 0:  # a component start
            rest = cm[i:]
            best = rest[np.lexsort((rest, deg[rest]))[0]]
            if best != v:
                bad.append(("start", i, int(v), int(best)))
            last_parent = -1
            prev = None
            continue
        par = int(earlier.min())
        if par < last_parent:
            bad.append(("parent order", i))
        if prev is not None and prev[0] == par and (prev[1], prev[2]) > (deg[v], v):
            bad.append(("degree order", i))
        last_parent = par
        prev = (par, deg[v], v)
    return bad


def _envelope(S, order):
    inv = np.empty(len(order), np.int64)
    inv[order] = np.arange(len(order))
    C = S.tocoo()
    first = np.arange(len(order))
    np.minimum.at(first, inv[C.row], inv[C.col])
    return int((np.arange(len(order)) - first).sum())


@pytest.mark.parametrize("case", [0, 2, 4])
@pytest.mark.parametrize("kind", ["RAS", "ORAS"])
def test_elimination_order_is_rcm_of_the_oracle_pattern(case, kind):
    """The factorisation's elimination order (Section 5, LU of the local
    problems) is reverse Cuthill-McKee on the pattern of the oracle's A_j
    (eq. localOP, with the Robin rows of eq. robfo for ORAS), and its
    envelope is no wider than that of band order (about half for ORAS)."""
    import scipy.sparse as sps
    surf, h, p, method, n, no = CASES[case]
    b = oracle.build_band(surf, h, p, [-2.0] * 3, [2.0] * 3)
    ctx = P.Context(-1)
    ctx.build_band(surf, h, p)
    ctx.build_operator(1.0)
    ctx.partition(P.PART_RCB, n, None, no, getattr(P, kind), 3.0, 30.0)
    dec = schwarz.decompose(b, oracle.rcb_partition(b, n), no, kind, alpha=3.0, alpha_cross=30.0, only={0, n - 1})
    for j in (0, n - 1):
        A = sps.csr_matrix(schwarz.local_matrix(b, dec, j, 1.0))
        S = ((abs(A) + abs(A).T) != 0).astype(np.int8).tolil()
        S.setdiag(0)
        S = S.tocsr()
        S.eliminate_zeros()
        S.sort_indices()
        order = ctx.subdomain(j)["order"]
        assert np.array_equal(np.sort(order), np.arange(S.shape[0]))
        assert _cm_violations(S, order) == []
        # ORAS puts the B_j unknowns after Sigma_j in band order, far from the
        # Sigma_j rows that reference them: there the order halves the envelope
        bound = 0.7 if kind == "ORAS" else 1.0
        assert _envelope(S, order) <= bound * _envelope(S, np.arange(S.shape[0]))
    ctx.close()


def test_cm_check_catches_a_wrong_order():
    """The Cuthill-McKee check fails for band order and for a swapped pair."""
    import scipy.sparse as sps
    surf, h, p, method, n, no = CASES[0]
    b = oracle.build_band(surf, h, p, [-2.0] * 3, [2.0] * 3)
    ctx = P.Context(-1)
    ctx.build_band(surf, h, p)
    ctx.build_operator(1.0)
    ctx.partition(P.PART_RCB, n, None, no, P.ORAS, 3.0, 30.0)
    dec = schwarz.decompose(b, oracle.rcb_partition(b, n), no, "ORAS", alpha=3.0, alpha_cross=30.0, only={0})
    A = sps.csr_matrix(schwarz.local_matrix(b, dec, 0, 1.0))
    S = ((abs(A) + abs(A).T) != 0).astype(np.int8).tolil()
    S.setdiag(0)
    S = S.tocsr()
    S.eliminate_zeros()
    S.sort_indices()
    order = ctx.subdomain(0)["order"].copy()
    assert _cm_violations(S, np.arange(S.shape[0])) != []
    order[[5, 400]] = order[[400, 5]]
    assert _cm_violations(S, order) != []
    ctx.close()


def test_state_machine_and_argument_errors():
    ctx = P.Context(-1)
    with pytest.raises(P.CpmError) as e:
        ctx.build_operator(1.0)
    assert e.value.code == P.ESTATE
    with pytest.raises(P.CpmError) as e:
        ctx.build_band(ci.Sphere(), 0.1, 4)
    assert e.value.code == P.EINVAL
    with pytest.raises(P.CpmError) as e:
        ctx.build_band(ci.Sphere(), 0.1, 3, lo=(-1.2,) * 3, hi=(1.2,) * 3)  # ghosts leave the box
    assert e.value.code == P.EINVAL

    class Broken:
        def cp(self, x):
            raise RuntimeError("no")
    with pytest.raises(P.CpmError) as e:
        ctx.build_band(Broken(), 0.1, 3)
    assert e.value.code == P.ECALLBACK
    ctx.build_band(ci.Sphere(), 0.2, 3)
    with pytest.raises(P.CpmError) as e:
        ctx.partition(P.PART_RCB, 4, None, 2, P.RAS)
    assert e.value.code == P.ESTATE
    for bad_c in (0.0, -1.0, float("nan")):
        with pytest.raises(P.CpmError) as e:
            ctx.build_operator(bad_c)
        assert e.value.code == P.EINVAL
    ctx.build_operator(1.0)
    with pytest.raises(P.CpmError) as e:
        ctx.partition(P.PART_OCTANT, 4, None, 2, P.RAS)
    assert e.value.code == P.EINVAL
    with pytest.raises(P.CpmError) as e:
        ctx.partition(P.PART_RCB, 4, None, 0, P.ORAS, 2.0)  # ORAS needs overlap >= 1
    assert e.value.code == P.EINVAL
    with pytest.raises(P.CpmError) as e:
        ctx.partition(P.PART_RCB, 4, None, 2, P.ORAS, 0.0)  # and alpha > 0
    assert e.value.code == P.EINVAL
    with pytest.raises(P.CpmError) as e:
        ctx.factor(P.FP64)
    assert e.value.code == P.ESTATE
    ctx.partition(P.PART_RCB, 4, None, 2, P.ORAS, 2.0)
    with pytest.raises(P.CpmError) as e:
        ctx.factor(P.FP64)  # host-only context
    assert e.value.code == P.EDEVICE
