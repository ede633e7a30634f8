"""SIMP inverse homogenization of a periodic cell (App. F.3): the optimisation loop.

Sequencing only: every step runs in libgmt -- the density cell's hierarchy and
Galerkin operators (gmt_build_density_hierarchy), the load and the GMG-PCG solve
of the six cell problems, C_H (gmt_homogenize), the objective on the compliance
S = C_H^-1 and its gradient (gmt_simp_objective), the analytic sensitivities
(gmt_simp_sensitivity), the sensitivity filter (gmt_simp_filter) and the
Optimality-Criteria step with move limits (gmt_simp_oc).

    python -m paper_2604_26518_amd.simp --N 32 --objective bulk --volfrac 0.3 --iters 40
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import binding as B


def initial_density(N: int, volfrac: float, seed: int = 0):
    """volfrac on average, lower in a central soft sphere (a uniform field is a stationary point
    of the isotropic targets), with a small seeded perturbation."""
    rng = np.random.default_rng(seed)
    c = (np.arange(N) + 0.5) / N - 0.5
    r2 = c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2
    rho = np.where(r2 < 0.3 ** 2, 0.5, 1.0) * (1.0 + 0.1 * (rng.random((N, N, N)) - 0.5))
    rho *= volfrac / rho.mean()
    return np.clip(rho, 1e-3, 1.0)


def optimize(rho0, objective="bulk", volfrac=0.3, iters=40, p=3.0, rho_min=1e-4, rmin=1.8, move=0.2,
             tol=1e-5, precision="f32", levels=None, log=None):
    """Runs the loop from rho0 (N^3 array); returns (rho, history)."""
    N = rho0.shape[0]
    levels = levels or B.default_levels(N)
    rho = torch.as_tensor(np.ascontiguousarray(rho0, dtype=np.float64), device="cuda").reshape(-1)
    hist = []
    u = None
    for it in range(iters):
        t0 = time.perf_counter()
        H = B.Hierarchy(None, levels, "elastic", density=rho.reshape(N, N, N), p=p, rho_min=rho_min)
        f = H.load_vector()
        u, rep = H.solve(f, tol=tol, precision=precision, max_iter=3000)
        CH = H.homogenize(u)
        J, G = B.simp_objective(CH, objective)
        dJ, _ = H.simp_sensitivity(u, G=G)
        H.close()
        dc = B.simp_filter(rho, dJ, rmin)
        rho_new, lam = B.simp_oc(rho, dc, volfrac, move=move, rho_lo=1e-3)
        change = float((rho_new - rho).abs().max())
        rho = rho_new
        torch.cuda.synchronize()
        rec = {"iter": it, "J": J, "C11": float(CH[0, 0]), "C44": float(CH[3, 3]), "iterations": rep["iterations"],
               "vol": float(rho.mean()), "change": change, "ms": (time.perf_counter() - t0) * 1e3}
        hist.append(rec)
        if log:
            log(rec)
        if it >= 10 and change < 1e-3:
            break
    return rho.reshape(N, N, N), hist


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=32)
    ap.add_argument("--objective", default="bulk", choices=list(B.SIMP_OBJECTIVES))
    ap.add_argument("--volfrac", type=float, default=0.3)
    ap.add_argument("--iters", type=int, default=40)
    ap.add_argument("--rmin", type=float, default=1.8)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    rho0 = initial_density(args.N, args.volfrac, args.seed)
    _, hist = optimize(rho0, args.objective, args.volfrac, args.iters, rmin=args.rmin,
                       log=lambda r: print(json.dumps(r), flush=True))
    ms = [h["ms"] for h in hist[1:]] or [hist[0]["ms"]]
    print(f"# {len(hist)} iterations, median {np.median(ms):.1f} ms/iteration, J {hist[0]['J']:.4g} -> "
          f"{hist[-1]['J']:.4g}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
