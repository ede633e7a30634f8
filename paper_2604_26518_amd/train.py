"""Trains the learned initializer on seeded synthetic cells (label-free physics loss).

    python -m paper_2604_26518_amd.train --N 128 --cells 256 --steps 3000 --out weights.pt

Every step: network forward (gmt_nn_forward) -> one Alg. 2 V-cycle from its
predictions + the log-residual loss and its adjoint (gmt_vcycle_loss) ->
backward (gmt_nn_backward) -> global-norm clipping -> AdamW (gmt_nn_adamw) ->
EMA.  The saved file holds the FP32 master weights, the EMA weights (used for
inference) and the configuration.
"""

from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np
import torch

from . import binding as B
from .learned import Trainer, channels_for, learned_solve


def _gen(args):
    seed, N = args
    from gmt_inputs.lattices import workload_cell
    return workload_cell(N, seed)


def make_cells(N, seeds, procs=16):
    procs = max(1, min(procs, os.cpu_count() or 1))
    with mp.get_context("fork").Pool(procs) as pool:
        return pool.map(_gen, [(s, N) for s in seeds])


def build(vox, levels, physics="elastic"):
    H = B.Hierarchy(vox, levels, physics)
    H.nn_setup(channels_for(levels))
    return H


def evaluate(params, hs, inject=True):
    """Post-V-cycle relative residual (max over cases) of the learned init on hierarchies hs."""
    out = []
    for H in hs:
        preds = H.nn_forward(params)
        if not inject:
            preds = preds[:1]
        _, _, rel, _, _ = H.vcycle_loss(preds, want_grad=False)
        out.append(float(np.max(rel)))
    return np.array(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--levels", type=int, default=0)
    ap.add_argument("--cells", type=int, default=256)
    ap.add_argument("--cache", type=int, default=96, help="hierarchies kept on the GPU")
    ap.add_argument("--held-out", type=int, default=16)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed0", type=int, default=10000)
    ap.add_argument("--test-seed0", type=int, default=20000)
    ap.add_argument("--out", default="weights.pt")
    ap.add_argument("--log", default="")
    ap.add_argument("--time-budget", type=float, default=0.0, help="stop after this many seconds")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    levels = args.levels or B.default_levels(args.N)
    t0 = time.time()
    cells = make_cells(args.N, range(args.seed0, args.seed0 + args.cells))
    test = make_cells(args.N, range(args.test_seed0, args.test_seed0 + args.held_out))
    print(f"# {len(cells)} train + {len(test)} held-out cells at {args.N}^3 in {time.time() - t0:.1f} s, "
          f"levels {levels}", flush=True)
    n_params = B.nn_param_count(levels, channels_for(levels))
    tr = Trainer(n_params, levels, lr=args.lr)
    cache = {}
    hs_test = [build(v, levels) for (_, _, v) in test]
    base = evaluate(tr.params, hs_test)
    log = []
    print(f"# params {n_params}; held-out post-V-cycle residual at init: median {np.median(base):.3e}", flush=True)
    t_start = time.time()
    rng = np.random.default_rng(0)
    order = rng.permutation(len(cells))
    for k in range(args.steps):
        idx = int(order[k % len(cells)])
        H = cache.get(idx)
        if H is None:
            H = build(cells[idx][2], levels)
            if len(cache) < args.cache:
                cache[idx] = H
        loss, rn, rel = tr.train_cell(H, args.steps)
        if idx not in cache:
            H.close()
        if not math.isfinite(loss):
            raise RuntimeError(f"non-finite loss at step {k}")
        log.append({"step": k, "loss": loss, "rel": rel, "family": cells[idx][0]})
        if (k + 1) % 100 == 0 or k == args.steps - 1:
            recent = np.array([x["rel"] for x in log[-100:]])
            msg = (f"step {k + 1}/{args.steps} lr {tr.lr_at(tr.step, args.steps):.2e} loss "
                   f"{np.mean([x['loss'] for x in log[-100:]]):.3f} train rel median {np.median(recent):.3e} "
                   f"({time.time() - t_start:.0f} s)")
            if (k + 1) % 500 == 0 or k == args.steps - 1:
                ev = evaluate(tr.ema, hs_test)
                msg += f" | held-out EMA median {np.median(ev):.3e} max {ev.max():.3e}"
            print(msg, flush=True)
        if args.time_budget and time.time() - t_start > args.time_budget:
            print(f"# time budget reached after {k + 1} steps", flush=True)
            break
    ev = evaluate(tr.ema, hs_test)
    ev_noinj = evaluate(tr.ema, hs_test, inject=False)
    torch.save({"params": tr.params.cpu(), "ema": tr.ema.cpu(), "levels": levels, "N": args.N,
                "channels": channels_for(levels), "head": 32, "steps": tr.step}, args.out)
    summary = {"held_out_init_median": float(np.median(base)), "held_out_median": float(np.median(ev)),
               "held_out_max": float(ev.max()), "held_out_no_injection_median": float(np.median(ev_noinj)),
               "steps": tr.step, "seconds": time.time() - t_start}
    print("# " + json.dumps(summary), flush=True)
    if args.log:
        with open(args.log, "w") as fh:
            json.dump({"summary": summary, "log": log}, fh)
    for H in list(cache.values()) + hs_test:
        H.close()


if __name__ == "__main__":
    main(sys.argv[1:])
