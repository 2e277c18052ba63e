"""GPU parity at the large configurations: sampled subdomains against the
oracle's dense local solves, full solves checked by the oracle's residual.

Torus R = 1, r = 0.4, h = 0.0125 (about 700k band nodes), c = 0.5, 256
weighted-RCB subdomains (target weights U[0.5, 2], seed 2), overlap 3, ORAS
with alpha = h^{-1/2} and the cross-point weight h^{-1}; FP32 factors with
FP64 GMRES; f = 16 seeded Gaussian bumps (sigma 0.2) on the surface.
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


def test_torus_h00125_wrcb256_uneven_fp32():
    h, c, n_sub, no = 0.0125, 0.5, 256, 3
    alpha, ax = h ** -0.5, 1.0 / h
    surf = ci.Torus(1.0, 0.4)
    say("torus oracle band")
    b = oracle.build_band(surf, h, 3, [-2.0] * 3, [2.0] * 3)
    w = ci.wrcb_weights(n_sub, seed=2)
    part = oracle.rcb_partition(b, n_sub, weights=w)
    sizes = np.bincount(part, minlength=n_sub)
    assert sizes.max() > 3 * sizes.min()  # genuinely uneven subdomains
    sample = [int(np.argmin(sizes)), int(np.argsort(sizes)[n_sub // 2]), int(np.argmax(sizes))]
    dec = schwarz.decompose(b, part, no, "ORAS", alpha=alpha, alpha_cross=ax, only=set(sample))
    say("torus oracle local solves", sample, [dec.subs[j].local_size("ORAS") for j in sample])
    M = schwarz.Preconditioner(b, dec, c, subs=sample)
    v = np.random.default_rng(7).standard_normal(b.n_act)
    z_ref = M.apply(v)
    rows = np.concatenate([dec.subs[j].tilde for j in sample])

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
    say("torus factor fp32")
    ctx.factor(P.FP32)
    z = torch.zeros(b.n_act, dtype=torch.float64, device="cuda")
    ctx.apply_precond(torch.from_numpy(v).cuda(), z)
    zz = z.cpu().numpy()[rows]
    assert np.abs(zz - z_ref[rows]).max() / np.abs(z_ref[rows]).max() < 2e-3
    say("torus solve")
    f = ci.rhs_torus_bumps(b.cp[: b.n_act], 1.0, 0.4, seed=3)
    u, info, rc = ctx.solve(f, tol=1e-8, max_iter=600, restart=30)
    say("torus solve info", info)
    assert rc == P.OK
    A = oracle.stabilized_operator(b, c)
    assert np.linalg.norm(f - A @ u) / np.linalg.norm(f) <= 1.05e-8
    ctx.close()
