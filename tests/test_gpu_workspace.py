"""The cache of large work buffers (cpm_set_workspace_cache): factorisations
that reuse a cached buffer give the same factors, bit for bit, as with the
cache off, and the cache holds and releases what it reports.

Unit sphere h = 0.025, 64 RCB subdomains, overlap 3, ORAS alpha = 1/h, FP32
factors (bordered matrices of about 13 GB, well above the cache threshold).
"""

import sys

import numpy as np
import pytest

import cpm_inputs as ci
import paper_1909_08734_amd as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEFAULT_CAP = 64 << 30


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def test_cached_work_buffers_give_identical_factors():
    h = 0.025
    ctx = P.Context(0)
    try:
        ctx.build_band(ci.Sphere(), h, 3)
        ctx.build_operator(1.0)
        ctx.partition(P.PART_RCB, 64, None, 3, P.ORAS, 1.0 / h, 0.0)
        P.set_workspace_cache(DEFAULT_CAP)
        say("factor with the cache on")
        ctx.factor(P.FP32)
        cap, idle, used = P.workspace_cache(0)
        assert cap == DEFAULT_CAP
        assert idle >= 64 << 20  # the bordered matrices went back to the cache
        assert used > 0  # the W arena is a cached buffer in use
        w_ref = [ctx.factor_export(j) for j in (0, 31, 63)]
        say("factor again (buffers from the cache)")
        ctx.factor(P.FP32)
        _, idle2, used2 = P.workspace_cache(0)
        assert idle2 == idle and used2 == used  # the same buffers were taken and returned
        for j, w in zip((0, 31, 63), w_ref):
            np.testing.assert_array_equal(ctx.factor_export(j), w)
        say("cache off")
        before = P.set_workspace_cache(0)
        assert before >= idle
        assert P.workspace_cache(0)[1] == 0
        ctx.factor(P.FP32)
        assert P.workspace_cache(0)[1] == 0
        for j, w in zip((0, 31, 63), w_ref):
            np.testing.assert_array_equal(ctx.factor_export(j), w)
        # a solve on factors in a cached W arena
        na = ctx.band_sizes()[0]
        f = np.random.default_rng(5).standard_normal(na)
        P.set_workspace_cache(DEFAULT_CAP)
        ctx.factor(P.FP32)
        u, info, rc = ctx.solve(f, tol=1e-8, max_iter=500, restart=30)
        assert rc == P.OK and info[0]["relres_true"] <= 1.05e-8
    finally:
        ctx.close()
        P.set_workspace_cache(DEFAULT_CAP)
