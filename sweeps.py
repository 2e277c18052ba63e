"""Parameter sweeps of the paper's Section 6 on one MI355X: iterations to
convergence of (O)RAS as a stationary solver and as a GMRES preconditioner.

Settings follow Section 6: tri-quadratic extension (p = 2) with the tube radius
2.6067 h (which reproduces the paper's band sizes, e.g. N_A = 654,630 for the
unit sphere at h = 1/100), torus R = 2/3, r = 1/3, convergence when the
residual 2-norm has dropped by 10^6. The preconditioner count is the paper's
formulation: GMRES(30) on M^{-1} A u = M^{-1} f stopping when the
preconditioned residual has dropped by 10^6 (cpm_solve_left); the count of
right-preconditioned FGMRES(30) to a true relative residual of 10^-6 is
reported beside it. The stationary solver stops on the true residual.
Differences: recursive coordinate bisection (or the graph bisection,
optionally with the interface alignment of Section 3.2: --partition) instead
of METIS, seeded synthetic right-hand sides (the paper does not state its
own), c = 1, FP64 local factors.

  table7   subdomain count N_S in {32, 64, 96}, N_O = 4, alpha = 4, alpha_x = 40 (Table 7)
  table5   overlap N_O in {4, 8, 12} at N_S = 32 with the cross-point weight (Table 5)
           and without it (Table 6)
  table2   two subdomains, N_O = 4, alpha swept (Tables 2, 3) at grid spacings coarse
           enough for dense local solves of half the surface

Each result is printed as one JSON line as soon as it is known.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BAND_FACTOR = 2.6067
METHOD = "rcb"  # partitioner: rcb or graph, optionally +align
DEGREE = 2
TOL = 1e-6


def surfaces():
    import cpm_inputs as ci
    return {
        "sphere": (ci.Sphere(), lambda cp, seed: ci.rhs_sphere_random_sh(cp, 1.0, seed=seed)[0]),
        "torus": (ci.Torus(2.0 / 3.0, 1.0 / 3.0),
                  lambda cp, seed: ci.rhs_torus_bumps(cp, 2.0 / 3.0, 1.0 / 3.0, seed=seed)),
    }


def emit(rec):
    print(json.dumps(rec), flush=True)


class Problem:
    def __init__(self, name, h, seed=11):
        import torch
        import paper_1909_08734_amd as P
        self.P, self.torch = P, torch
        surf, rhs = surfaces()[name]
        self.name, self.h = name, h
        self.ctx = P.Context(0)
        t0 = time.time()
        self.ctx.build_band(surf, h, DEGREE, band_factor=BAND_FACTOR)
        self.ctx.build_operator(1.0)
        self.na = self.ctx.band_sizes()[0]
        cp = self.ctx.band_arrays(DEGREE)["cp"][: self.na]
        self.f = torch.from_numpy(np.ascontiguousarray(rhs(cp, seed))).cuda()
        self.band_s = time.time() - t0

    def run(self, n_sub, overlap, kind, alpha=0.0, alpha_x=0.0, prec=None, max_stat=4000, max_gmres=2000):
        P, torch = self.P, self.torch
        prec = P.FP64 if prec is None else prec
        t0 = time.time()
        code = {"rcb": P.PART_RCB, "graph": P.PART_GRAPH}[METHOD.split("+")[0]]
        if METHOD.endswith("+align"):
            code |= P.PART_ALIGN
        self.ctx.partition(code, n_sub, None, overlap, P.ORAS if kind == "ORAS" else P.RAS, alpha, alpha_x)
        self.ctx.factor(prec)
        factor_s = time.time() - t0
        u = torch.zeros_like(self.f)
        torch.cuda.synchronize()
        info_s, rc_s = self.ctx.solve_stationary(self.f, u, tol=TOL, max_iter=max_stat)
        u.zero_()
        info_l, rc_l = self.ctx.solve_left(self.f, u, tol=TOL, max_iter=max_gmres, restart=30)
        u.zero_()
        info_g, rc_g = self.ctx.solve_device(self.f, u, tol=TOL, max_iter=max_gmres, restart=30)
        info_g = info_g[0]
        return {"surface": self.name, "h": self.h, "N_A": self.na, "N_S": n_sub, "N_O": overlap, "kind": kind,
                "alpha": alpha, "alpha_cross": alpha_x, "prec": "fp64" if prec == P.FP64 else "fp32",
                "solver_iters": info_s["iters"] if rc_s == P.OK else None,
                "solver_relres": info_s["relres_true"],
                "precond_iters": info_l["iters"] if rc_l == P.OK else None,
                "precond_relres_true": info_l["relres_true"],
                "fgmres_iters": info_g["iters"] if rc_g == P.OK else None,
                "fgmres_relres": info_g["relres_true"], "factor_s": round(factor_s, 2),
                "groups": self.ctx.factor_groups(), "chunk": self.ctx.precond_chunk(), "partition": METHOD}

    def close(self):
        self.ctx.close()


def table7(args):
    for name in args.surfaces:
        pb = Problem(name, args.h)
        emit({"problem": name, "h": args.h, "N_A": pb.na, "band_s": round(pb.band_s, 1)})
        for n_sub in args.n_sub:
            for kind in ("RAS", "ORAS"):
                emit(pb.run(n_sub, 4, kind, 4.0 if kind == "ORAS" else 0.0, 40.0 if kind == "ORAS" else 0.0))
        pb.close()


def table5(args):
    for name in args.surfaces:
        pb = Problem(name, args.h)
        emit({"problem": name, "h": args.h, "N_A": pb.na, "band_s": round(pb.band_s, 1)})
        a, ax = {"sphere": (2.0, 40.0), "torus": (4.0, 20.0)}[name]
        for no in args.overlaps:
            emit(pb.run(32, no, "RAS"))
            emit(pb.run(32, no, "ORAS", a, ax))
            emit(pb.run(32, no, "ORAS", a, 0.0))
        pb.close()


def table2(args):
    alphas = [0.25, 0.5, 0.75, 1.0, 1.5, 2.0, 4.0, 8.0, 16.0]
    for name in args.surfaces:
        for h in args.hs:
            pb = Problem(name, h)
            emit({"problem": name, "h": h, "N_A": pb.na, "band_s": round(pb.band_s, 1)})
            for a in alphas:
                emit(pb.run(2, 4, "ORAS", a, 0.0))
            emit(pb.run(2, 4, "RAS"))
            pb.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("table", choices=["table7", "table5", "table2"])
    ap.add_argument("--surfaces", nargs="+", default=["sphere", "torus"])
    ap.add_argument("--h", type=float, default=0.01)
    ap.add_argument("--hs", type=float, nargs="+", default=[1 / 15, 1 / 20])
    ap.add_argument("--n-sub", type=int, nargs="+", default=[32, 64, 96])
    ap.add_argument("--overlaps", type=int, nargs="+", default=[4, 8, 12])
    ap.add_argument("--partition", default="rcb", choices=["rcb", "rcb+align", "graph", "graph+align"])
    args = ap.parse_args()
    global METHOD
    METHOD = args.partition
    {"table7": table7, "table5": table5, "table2": table2}[args.table](args)


if __name__ == "__main__":
    main()
