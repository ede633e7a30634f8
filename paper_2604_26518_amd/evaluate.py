"""Learned initializer vs plain GMG-PCG on held-out cells.

    python -m paper_2604_26518_amd.evaluate --weights unet128.npz --cells 32

Per cell (same hierarchy, same load vector, same FP64 stopping test):
  plain    zero-init mixed-precision GMG-PCG to tol
  learned  network forward -> one Alg. 2 V-cycle from u_hat / e_hat -> FP64
           residual check -> warm-started GMG-PCG only if above tol (fallback)
and the one-cycle ablations: zero init, u_hat only (no coarse injection),
u_hat + e_hat.  Times are wall-clock with the stream synchronized on both
sides; C_H of both paths is compared with an FP64 solve to 1e-9.
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


def _sync_time(fn):
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t


def one_cycle_residual(H, f32, u0, e=None):
    u = u0.clone()
    H.vcycle(f32, u, e_init=e)
    return u


def compare(H: B.Hierarchy, params, tol=1e-5, max_iter=3000, reference=True):
    f64 = H.load_vector()
    f32 = f64.to(torch.float32)
    rec = {"n_n": H.n_n(1)}
    # plain GMG-PCG from zero
    (u_plain, rep), t = _sync_time(lambda: H.solve(f64, tol=tol, precision="f32", max_iter=max_iter))
    rec.update(plain_s=t, plain_its=rep["iterations"], plain_conv=bool(rep["converged"]))

    # learned: forward, one V-cycle, FP64 check, fallback
    def learned():
        preds = H.nn_forward(params)
        u = preds[0]
        H.vcycle(f32, u, e_init=injection(H, preds))
        return H.solve(f64, u=u.to(torch.float64), tol=tol, precision="f32", max_iter=max_iter)

    (u_learn, rep_l), t = _sync_time(learned)
    rec.update(learned_s=t, learned_its=rep_l["iterations"], learned_conv=bool(rep_l["converged"]),
               fallback=rep_l["iterations"] > 0, rel_after_vcycle=float(max(rep_l["rel_res_init"])))
    # network time alone
    _, t = _sync_time(lambda: H.nn_forward(params))
    rec["net_s"] = t
    # one-cycle ablations (FP64 residual of the V-cycle result)
    zero = torch.zeros_like(f32)
    preds = H.nn_forward(params)
    rel = lambda u: float(np.max(H.relative_residual(f64, u.to(torch.float64))))  # noqa: E731
    rec["abl_zero_init"] = rel(one_cycle_residual(H, f32, zero))
    rec["abl_u_only"] = rel(one_cycle_residual(H, f32, preds[0]))
    rec["abl_u_and_e"] = rel(one_cycle_residual(H, f32, preds[0], injection(H, preds)))
    rec["abl_net_no_cycle"] = rel(preds[0])
    if reference:
        u_ref, _ = H.solve(f64, tol=1e-9, precision="f64", max_iter=max_iter)
        C_ref = H.homogenize(u_ref)
        nref = np.linalg.norm(C_ref)
        rec["CH_err_plain"] = float(np.linalg.norm(H.homogenize(u_plain) - C_ref) / nref)
        rec["CH_err_learned"] = float(np.linalg.norm(H.homogenize(u_learn) - C_ref) / nref)
    return rec


def summarize(recs):
    a = lambda k: np.array([r[k] for r in recs], dtype=float)  # noqa: E731
    s = {
        "cells": len(recs),
        "plain_ms_per_cell": float(a("plain_s").mean() * 1e3),
        "learned_ms_per_cell": float(a("learned_s").mean() * 1e3),
        "gain_plain_over_learned": float(a("plain_s").sum() / a("learned_s").sum()),
        "net_ms_per_cell": float(a("net_s").mean() * 1e3),
        "plain_iterations_mean": float(a("plain_its").mean()),
        "learned_fallback_iterations_mean": float(a("learned_its").mean()),
        "fallback_rate": float(a("fallback").mean()),
        "rel_after_vcycle_median": float(np.median(a("rel_after_vcycle"))),
        "rel_after_vcycle_p90": float(np.percentile(a("rel_after_vcycle"), 90)),
        "ablation_median": {k: float(np.median(a(k))) for k in ("abl_zero_init", "abl_u_only", "abl_u_and_e",
                                                                "abl_net_no_cycle")},
    }
    ref = [r for r in recs if "CH_err_learned" in r]
    if ref:
        s["CH_err_cells"] = len(ref)
        s["CH_err_plain_max"] = float(max(r["CH_err_plain"] for r in ref))
        s["CH_err_learned_max"] = float(max(r["CH_err_learned"] for r in ref))
    return s


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--weights", required=True)
    ap.add_argument("--cells", type=int, default=32)
    ap.add_argument("--seed0", type=int, default=900000)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    params, info = load_weights(args.weights)
    N, levels = info["N"], info["levels"]
    from gmt_inputs.lattices import workload_cell
    recs = []
    for k in range(args.cells):
        seed = args.seed0 + k
        fam, vf, vox = workload_cell(N, seed)
        H = B.Hierarchy(vox, levels, "elastic")
        H.nn_setup(channels_for(levels), attention=info.get("attention", False))
        if k == 0:  # warm-up of every kernel on the first cell
            compare(H, params, args.tol, reference=False)
        r = compare(H, params, args.tol)
        r.update(seed=seed, family=fam, vf=vf)
        recs.append(r)
        H.close()
        print(json.dumps({k2: (round(v, 6) if isinstance(v, float) else v) for k2, v in r.items()}), flush=True)
    s = summarize(recs)
    print("# " + json.dumps(s), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump({"summary": s, "cells": recs, "weights_info": info}, fh, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:])
