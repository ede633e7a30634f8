"""Smoother and schedule study on synthetic cells (the smoother and schedule comparisons of
Sec. 6.3): for each smoother (Chebyshev, weighted Jacobi, 8-colour Gauss-Seidel, SOR) and
cycle schedule (V, W, F) one cycle from zero and from the network's prediction (FP32, its
relative residual in FP64) and its time, and, for the symmetric cycles, GMG-PCG to the
tolerance (mixed precision) with its iterations and time.

    python -m paper_2604_26518_amd.cycle_study --N 128 --cells 4

One JSON line per (cell, smoother, schedule); a summary line of medians at the end.
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import binding as B
from .learned import channels_for, injection, load_weights

SMOOTHERS = {"chebyshev": {}, "jacobi": {}, "gs": {"omega": 1.0}, "sor": {"omega": 1.2}}


def timed(fn, reps=1):
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t) / reps * 1e3


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--cells", type=int, default=4)
    ap.add_argument("--seed0", type=int, default=1000)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--weights", default="", help="network for the one-cycle-from-prediction column")
    args = ap.parse_args(argv)
    from gmt_inputs.lattices import workload_cell
    cells = [(s,) + workload_cell(args.N, s) for s in range(args.seed0, args.seed0 + args.cells)]
    torch.cuda.set_device(0)
    params, info = (load_weights(args.weights) if args.weights else (None, None))
    L = B.default_levels(args.N)
    recs = []
    for seed, fam, vf, vox in cells:
        H = B.Hierarchy(vox, L, "elastic")
        if params is not None:
            H.nn_setup(channels_for(min(info["levels"], L)), attention=info.get("attention", False))
            preds = H.nn_forward(params)
        f64 = H.load_vector()
        f32 = f64.to(torch.float32)
        rel = lambda u: float(np.max(H.relative_residual(f64, u.to(torch.float64))))  # noqa: E731
        for sm, kw in SMOOTHERS.items():
            name = "gs" if sm in ("gs", "sor") else sm
            om = [kw["omega"]] * L if "omega" in kw else None
            for sch in ("V", "W", "F"):
                u0 = torch.zeros_like(f32)
                H.vcycle(f32, u0, smoother=name, omega=om, schedule=sch)  # warm-up (colours, autotuning)
                u0.zero_()
                _, ms = timed(lambda: H.vcycle(f32, u0, smoother=name, omega=om, schedule=sch))
                rec = {"seed": seed, "family": fam, "vf": round(vf, 3), "n_n": H.n_n(1), "smoother": sm,
                       "schedule": sch, "cycle_ms": round(ms, 3), "one_cycle_from_zero": rel(u0)}
                if params is not None:
                    u1 = preds[0].clone()
                    H.vcycle(f32, u1, e_init=injection(H, preds), smoother=name, omega=om, schedule=sch)
                    rec["one_cycle_from_network"] = rel(u1)
                if sch != "F":  # the F-cycle is not symmetric: no PCG preconditioner
                    H.solve(f64, tol=args.tol, precision="f32", max_iter=3000, smoother=name, omega=om,
                            schedule=sch, raise_on_noconv=False)  # warm-up (graph capture)
                    (u, rep), ms = timed(lambda: H.solve(f64, tol=args.tol, precision="f32", max_iter=3000,
                                                         smoother=name, omega=om, schedule=sch,
                                                         raise_on_noconv=False))
                    rec.update(pcg_iterations=rep["iterations"], pcg_ms=round(ms, 2),
                               pcg_converged=bool(rep["converged"]))
                recs.append(rec)
                print(json.dumps(rec), flush=True)
        H.close()
    summ = {}
    for sm in SMOOTHERS:
        for sch in ("V", "W", "F"):
            rs = [r for r in recs if r["smoother"] == sm and r["schedule"] == sch]
            s = {"one_cycle_from_zero": float(np.median([r["one_cycle_from_zero"] for r in rs])),
                 "cycle_ms": float(np.median([r["cycle_ms"] for r in rs]))}
            if params is not None:
                s["one_cycle_from_network"] = float(np.median([r["one_cycle_from_network"] for r in rs]))
            if sch != "F":
                s["pcg_iterations"] = float(np.median([r["pcg_iterations"] for r in rs]))
                s["pcg_ms"] = float(np.median([r["pcg_ms"] for r in rs]))
            summ[f"{sm}/{sch}"] = s
    print("# " + json.dumps({"cells": len(cells), "N": args.N, "median": summ}), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
