"""The no-allocation operator apply (cpm_apply_operator_noalloc, through the C
ABI) against cpm_apply_operator: bit-identical results on two calls in a row,
the second on a smaller band, each from a fresh context."""

import sys

import numpy as np
import pytest

import cpm_inputs as ci
import paper_1909_08734_amd as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_noalloc_operator_apply_equals_the_allocating_one():
    outs = []
    for h in (0.05, 0.1):  # the second call on a smaller input
        print("noalloc apply, sphere h =", h, flush=True, file=sys.stderr)
        ctx = P.Context(0)
        ctx.build_band(ci.Sphere(), h, 3)
        ctx.build_operator(1.3)
        na = ctx.band_sizes()[0]
        x = torch.from_numpy(np.random.default_rng(int(1 / h)).standard_normal(na)).cuda()
        y_ref = torch.zeros_like(x)
        ctx.apply_operator(x, y_ref)
        y = torch.full_like(x, float("nan"))
        ctx.apply_operator_noalloc(x, y)
        a, b = y.cpu().numpy(), y_ref.cpu().numpy()
        np.testing.assert_array_equal(a, b)
        outs.append(na)
        ctx.close()
    assert outs[1] < outs[0]
