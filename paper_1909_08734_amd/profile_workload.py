"""Drive the benchmark workload for hardware-counter runs.

Builds the h = 0.025 unit-sphere problem (64 RCB subdomains, overlap 3, ORAS
alpha = 1/h), factors the local operators in the requested precision, runs a
few preconditioner applies (and operator applies) with each apply tiling in
turn, tiling 0 first, then one plain device copy of known size (used to
calibrate the memory counters). Meant to run under ``rocprofv3 --pmc ...``.
"""

from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    import torch

    import cpm_inputs as ci
    import paper_1909_08734_amd as P

    ap = argparse.ArgumentParser()
    ap.add_argument("--prec", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--applies", type=int, default=3)
    ap.add_argument("--copy-mib", type=int, default=1024)
    a = ap.parse_args()
    h = 0.025
    ctx = P.Context(0)
    ctx.build_band(ci.Sphere(), h, 3)
    ctx.build_operator(1.0)
    ctx.partition(P.PART_RCB, 64, None, 3, P.ORAS, 1.0 / h, 0.0)
    ctx.factor(P.FP64 if a.prec == "fp64" else P.FP32)
    na, _, _ = ctx.band_sizes()
    v = torch.randn(na, dtype=torch.float64, device="cuda")
    z = torch.zeros_like(v)
    for t in range(P.PRECOND_TILINGS):
        ctx.set_precond_tiling(t)
        for _ in range(a.applies):
            ctx.apply_precond(v, z)
            ctx.apply_operator(z, v)
    n = a.copy_mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"profile workload done: {a.prec}, {a.applies} applies x {P.PRECOND_TILINGS} tilings, "
          f"copy {a.copy_mib} MiB", flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
