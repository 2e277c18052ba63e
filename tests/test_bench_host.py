"""Host-side checks of the benchmark's bookkeeping (no device): the multi-GPU
refusal, the counter-summary lookup per apply tiling and the algorithmic byte
and flop counts on a small problem, recomputed here from their definitions."""

import json
import os
import subprocess
import sys

import numpy as np
import pytest

import cpm_inputs as ci
import paper_1909_08734_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in (r.stdout + r.stderr)


def test_counter_summary_lookup_by_tiling(tmp_path, monkeypatch):
    src = bench.kernel_source_hash()
    assert len(src) == 16 and src == bench.kernel_source_hash()
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"kernel_source_hash": src, "hbm_bytes_per_launch_by_tiling": [10.0 * (t + 1) for t in range(8)]}
    (prof / "precond_fp64_sphere_h0025_rcb64_pmc.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.pmc_traffic("fp64", src, 0) == 10.0
    assert bench.pmc_traffic("fp64", src, 7) == 80.0
    assert bench.pmc_traffic("fp64", src, 8) is None       # no such tiling
    assert bench.pmc_traffic("fp64", src, None) is None    # chunked apply: no tiling
    assert bench.pmc_traffic("fp64", "0" * 16, 0) is None  # counters of other source
    assert bench.pmc_traffic("fp32", src, 0) is None       # no summary


def _small_ctx():
    ctx = P.Context(-1)
    ctx.build_band(ci.Sphere(), 0.1, 3)
    ctx.build_operator(1.0)
    ctx.partition(P.PART_RCB, 6, None, 2, P.ORAS, 3.0, 0.0)
    return ctx


def test_algorithmic_counts_from_their_definitions():
    ctx = _small_ctx()
    subs = [ctx.subdomain(j) for j in range(6)]
    m = np.array([len(s["sigma"]) for s in subs])
    t = np.array([len(s["tilde"]) for s in subs])
    n = m + np.array([len(s["bnd"]) for s in subs])
    # W_j streamed once (8 bytes per FP64 entry), v|Sigma_j gathered, z|Sigma~_j
    # written with their index lists
    want = int(8 * (t * m).sum() + 12 * m.sum() + 12 * t.sum())
    got, _ = bench.precond_bytes(ctx, 6, 8)
    assert got == want
    # blocked LU update flops with no block skipped: left-looking catch-up of
    # every 32-wide panel inside a 128-wide outer block, then one trailing
    # update per outer block
    flops = 0
    for nj, tj, mj in zip(n, t, m):
        rows, cols = nj + tj, nj + mj
        for k0 in range(0, nj, 128):
            k1 = min(k0 + 128, nj)
            for k in range(k0 + 32, k1, 32):
                flops += 2 * (k - k0) * (rows - k) * min(32, nj - k)
            flops += 2 * (k1 - k0) * (rows - k1) * (cols - k1)
    assert bench.lu_flops(ctx, 6, True) == flops
    ctx.close()
