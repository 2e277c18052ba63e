"""GPU parity at the large configurations: sampled subdomains against the
oracle's dense local solves, full solves checked by the oracle's residual.

Torus R = 1, r = 0.4, h = 0.0125 (about 700k band nodes), c = 0.5, 256
weighted-RCB subdomains (target weights U[0.5, 2], seed 2), overlap 3, ORAS
with alpha = h^{-1/2} and the cross-point weight h^{-1}; FP32 and FP64
factors, FP64 GMRES; f = 16 seeded Gaussian bumps (sigma 0.2) on the surface.
"""

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


H, C, N_SUB, NO = 0.0125, 0.5, 256, 3
ALPHA, AX = H ** -0.5, 1.0 / H


@pytest.fixture(scope="module")
def torus_oracle():
    surf = ci.Torus(1.0, 0.4)
    say("torus oracle band")
    b = oracle.build_band(surf, H, 3, [-2.0] * 3, [2.0] * 3)
    w = ci.wrcb_weights(N_SUB, seed=2)
    part = oracle.rcb_partition(b, N_SUB, weights=w)
    sizes = np.bincount(part, minlength=N_SUB)
    assert sizes.max() > 3 * sizes.min()  # genuinely uneven subdomains
    sample = [int(np.argmin(sizes)), int(np.argsort(sizes)[N_SUB // 2]), int(np.argmax(sizes))]
    dec = schwarz.decompose(b, part, NO, "ORAS", alpha=ALPHA, alpha_cross=AX, only=set(sample))
    say("torus oracle local solves", sample, [dec.subs[j].local_size("ORAS") for j in sample])
    M = schwarz.Preconditioner(b, dec, C, subs=sample)
    v = np.random.default_rng(7).standard_normal(b.n_act)
    z_ref = M.apply(v)
    rows = np.concatenate([dec.subs[j].tilde for j in sample])
    A = oracle.stabilized_operator(b, C)
    return surf, b, w, part, sample, dec, v, z_ref, rows, A


@pytest.mark.parametrize("prec", [P.FP32, P.FP64], ids=["fp32", "fp64"])
def test_torus_h00125_wrcb256_uneven(torus_oracle, prec):
    surf, b, w, part, sample, dec, v, z_ref, rows, A = torus_oracle
    h, c, n_sub, no, alpha, ax = H, C, N_SUB, NO, ALPHA, AX
    say("torus library set-up")
    ctx = P.Context(0)
    ctx.build_band(surf, h, 3)
    assert ctx.band_sizes()[:2] == (b.n_act, b.n_ghost)
    ctx.build_operator(c)
    ctx.partition(P.PART_RCB, n_sub, w, no, P.ORAS, alpha, ax)
    _, lpart, _ = ctx.partition_info()
    np.testing.assert_array_equal(lpart, part)
    for j in sample:
        s = ctx.subdomain(j)
        np.testing.assert_array_equal(s["bnd"], dec.subs[j].bnd)
        np.testing.assert_array_equal(s["xstar"], dec.subs[j].xstar)
    say("torus factor", prec)
    ctx.factor(prec)
    z = torch.zeros(b.n_act, dtype=torch.float64, device="cuda")
    ctx.apply_precond(torch.from_numpy(v).cuda(), z)
    zz = z.cpu().numpy()[rows]
    bar = 2e-3 if prec == P.FP32 else 1e-9
    assert np.abs(zz - z_ref[rows]).max() / np.abs(z_ref[rows]).max() < bar
    say("torus solve")
    f = ci.rhs_torus_bumps(b.cp[: b.n_act], 1.0, 0.4, seed=3)
    u, info, rc = ctx.solve(f, tol=1e-8, max_iter=600, restart=60)  # GMRES(30) can stagnate at this size
    say("torus solve info", info)
    assert rc == P.OK
    assert np.linalg.norm(f - A @ u) / np.linalg.norm(f) <= 1.05e-8
    ctx.close()
