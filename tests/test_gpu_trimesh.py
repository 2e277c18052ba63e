"""GPU parity on a triangulated surface: sampled subdomains against the oracle's
dense local solves, full solves checked by the oracle's residual.

Icosphere with 20480 triangles, radially perturbed by seeded spherical-harmonic
bumps (l <= 6, amplitude 0.05); closest points by exact search over nearby
triangles. h = 0.02, tricubic extension, c = 1, f = 16 seeded Gaussian bumps
(sigma 0.2) evaluated at the closest points, 128 coordinate-bisection
subdomains, overlap 3, ORAS with alpha = h^{-1/2} and the cross-point weight
h^{-1} (the modified transmission condition where several subdomains meet),
FP64 and FP32 subdomain factors with FP64 GMRES(30).
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

H, C, N_SUB, NO = 0.02, 1.0, 128, 3
ALPHA, AX = H ** -0.5, 1.0 / H


def say(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def setup():
    surf = ci.bumpy_icosphere(level=5, amplitude=0.05, lmax=6, seed=4, far=0.12)
    assert len(surf.faces) == 20480
    say("trimesh oracle band")
    b = oracle.build_band(surf, H, 3, [-2.0] * 3, [2.0] * 3)
    # every band node lies inside the distance up to which cp is defined
    dmax = float(np.sqrt(((b.xyz - b.cp) ** 2).sum(axis=1)).max())
    assert dmax < surf.far - H, dmax
    part = oracle.rcb_partition(b, N_SUB)
    sizes = np.bincount(part, minlength=N_SUB)
    sample = [int(np.argmin(sizes)), int(np.argsort(sizes)[N_SUB // 2]), int(np.argmax(sizes))]
    dec = schwarz.decompose(b, part, NO, "ORAS", alpha=ALPHA, alpha_cross=AX, only=set(sample))
    # the modified condition is exercised in every sampled subdomain
    for j in sample:
        s = dec.subs[j]
        assert np.any(s.alpha > ALPHA), j
    say("trimesh oracle local solves", sample, [dec.subs[j].local_size("ORAS") for j in sample])
    M = schwarz.Preconditioner(b, dec, C, subs=sample)
    v = np.random.default_rng(11).standard_normal(b.n_act)
    z_ref = M.apply(v)
    rows = np.concatenate([dec.subs[j].tilde for j in sample])
    f = ci.rhs_surface_bumps(b.cp[: b.n_act], seed=5)
    A = oracle.stabilized_operator(b, C)

    say("trimesh library set-up")
    ctx = P.Context(0)
    ctx.build_band(surf, H, 3)
    assert ctx.band_sizes()[:2] == (b.n_act, b.n_ghost)
    np.testing.assert_array_equal(ctx.band_arrays()["lin"], b.lin)
    ctx.build_operator(C)
    ctx.partition(P.PART_RCB, N_SUB, None, NO, P.ORAS, ALPHA, AX)
    _, lpart, _ = ctx.partition_info()
    np.testing.assert_array_equal(lpart, part)
    for j in sample:
        s = ctx.subdomain(j)
        np.testing.assert_array_equal(s["bnd"], dec.subs[j].bnd)
        np.testing.assert_array_equal(s["xstar"], dec.subs[j].xstar)
    yield dict(b=b, ctx=ctx, v=v, z_ref=z_ref, rows=rows, f=f, A=A, sol={})
    ctx.close()


@pytest.mark.parametrize("prec,tol", [(P.FP64, 1e-9), (P.FP32, 2e-3)], ids=["fp64", "fp32"])
def test_trimesh_h002_rcb128_oras_cross(setup, prec, tol):
    s = setup
    b, ctx = s["b"], s["ctx"]
    say("trimesh factor", "fp64" if prec == P.FP64 else "fp32")
    ctx.factor(prec)
    z = torch.zeros(b.n_act, dtype=torch.float64, device="cuda")
    ctx.apply_precond(torch.from_numpy(s["v"]).cuda(), z)
    rows = s["rows"]
    zz = z.cpu().numpy()[rows]
    assert np.abs(zz - s["z_ref"][rows]).max() / np.abs(s["z_ref"][rows]).max() < tol
    say("trimesh solve")
    u, info, rc = ctx.solve(s["f"], tol=1e-8, max_iter=600, restart=30)
    say("trimesh solve info", info)
    assert rc == P.OK
    f = s["f"]
    assert np.linalg.norm(f - s["A"] @ u) / np.linalg.norm(f) <= 1.05e-8
    s["sol"][prec] = u
    if len(s["sol"]) == 2:
        u64, u32 = s["sol"][P.FP64], s["sol"][P.FP32]
        # both solve the same FP64 system to 1e-8 relative residual
        assert np.linalg.norm(u32 - u64) / np.linalg.norm(u64) < 1e-6
