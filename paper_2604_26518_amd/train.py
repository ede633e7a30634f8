"""Trains the learned initializer on seeded synthetic cells (label-free physics loss).

    python -m paper_2604_26518_amd.train --N 128 --cells 1024 --time-budget 900 --ckpt run.pt

Every step, on one cell: network forward (gmt_nn_forward) -> one Alg. 2
V-cycle from its predictions + the log-residual loss and its adjoint
(gmt_vcycle_loss) -> backward (gmt_nn_backward) -> global-norm clipping ->
AdamW (gmt_nn_adamw) -> EMA (gmt_nn_ema).  Cells come from the mixed lattice
families (family = seed mod 5, VF ~ U(0.15, 0.5)); hierarchies are kept on
the GPU up to a memory budget and rebuilt otherwise.  The checkpoint holds
the FP32 master weights, the AdamW moments, the EMA weights and the step, so
a run can be resumed; --export writes the EMA weights as BF16 for inference.
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
from .learned import Trainer, channels_for, save_weights


def _gen(args):
    """One workload cell, its voxels bit-packed (8x less host memory for thousands of cells)."""
    seed, N = args
    from gmt_inputs.lattices import workload_cell
    fam, vf, vox = workload_cell(N, seed)
    return seed, fam, vf, np.packbits(vox.ravel())


def voxels(cell, N):
    return np.unpackbits(cell[3])[: N ** 3].reshape(N, N, N)


def make_cells(N, seeds, procs=16):
    """Generates cells in worker processes.  Call it before anything touches the GPU: the
    workers are forked, and a process that has initialised HIP must not fork.  The pool is
    closed and joined (not terminated), so every worker exits on its own."""
    procs = max(1, min(procs, os.cpu_count() or 1))
    pool = mp.get_context("fork").Pool(procs)
    try:
        seeds = list(seeds)
        return pool.map(_gen, [(s, N) for s in seeds], chunksize=max(1, min(4, len(seeds) // procs)))
    finally:
        pool.close()
        pool.join()


def build(vox, levels, physics="elastic", attention=False, net_levels=0):
    H = B.Hierarchy(vox, levels, physics)
    H.nn_setup(channels_for(net_levels or levels), attention=attention)
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


def evaluate_zero(hs):
    """Post-V-cycle relative residual from a zero initial guess (the method without the network)."""
    out = []
    for H in hs:
        u0 = H.vec(1, torch.float32).zero_()
        _, _, rel, _, _ = H.vcycle_loss([u0], want_grad=False)
        out.append(float(np.max(rel)))
    return np.array(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--levels", type=int, default=0)
    ap.add_argument("--net-levels", type=int, default=0,
                    help="network on the finest levels only (default: every level of the hierarchy)")
    ap.add_argument("--cells", type=int, default=1024)
    ap.add_argument("--held-out", type=int, default=16)
    ap.add_argument("--steps", type=int, default=20000, help="length of the cosine schedule")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lam", type=float, default=0.0,
                    help="gauge penalty on the per-component mean of u^1 (predictions are centred already)")
    ap.add_argument("--seed0", type=int, default=100000)
    ap.add_argument("--test-seed0", type=int, default=900000)
    ap.add_argument("--init", default="", help="start from these exported (BF16) weights")
    ap.add_argument("--warmup-steps", type=int, default=300)
    ap.add_argument("--ema", type=float, default=0.999, help="decay of the weights' moving average")
    ap.add_argument("--supervised", type=float, default=0.0,
                    help="weight of the supervised term on u_hat^1 against each cell's plain-solver solution")
    ap.add_argument("--target-tol", type=float, default=1e-6, help="tolerance of the target solves")
    ap.add_argument("--attention", action="store_true", help="an attention block per level (Sec. 4.2-4.3)")
    ap.add_argument("--ckpt", default="unet.pt")
    ap.add_argument("--resume", action="store_true")
    ap.add_argument("--export", default="", help="write the EMA weights (BF16) to this .npz at the end")
    ap.add_argument("--log", default="")
    ap.add_argument("--time-budget", type=float, default=0.0, help="stop after this many seconds of training")
    ap.add_argument("--cache-gb", type=float, default=120.0, help="GPU memory for cached hierarchies")
    ap.add_argument("--eval-every", type=int, default=1000)
    ap.add_argument("--steps-per-cell", type=int, default=1,
                    help="consecutive steps on one drawn cell (amortises the build of large uncached cells)")
    args = ap.parse_args(argv)
    levels = args.levels or B.default_levels(args.N)
    nl = args.net_levels or levels
    t0 = time.time()
    # all cells are generated (forked workers) before the first GPU call
    cells = make_cells(args.N, range(args.seed0, args.seed0 + args.cells))
    test = make_cells(args.N, range(args.test_seed0, args.test_seed0 + args.held_out))
    torch.cuda.set_device(0)
    print(f"# {len(cells)} train + {len(test)} held-out cells at {args.N}^3 in {time.time() - t0:.1f} s, "
          f"levels {levels}", flush=True)
    att = args.attention
    n_params = B.nn_param_count(nl, channels_for(nl), attention=att)
    tr = Trainer(n_params, nl, lr=args.lr, lam=args.lam, warmup=args.warmup_steps, attention=att, ema=args.ema)
    if args.init:
        from .learned import load_weights
        w, winfo = load_weights(args.init)
        n_conv = B.nn_param_count(nl, channels_for(nl))
        if w.numel() == n_params:
            tr.params.copy_(w)
        elif att and w.numel() == n_conv:
            # a convolutional network: the attention projections follow its parameters and keep
            # their initialisation (small output projections: every block starts near the identity)
            tr.params[:n_conv].copy_(w)
        else:
            raise ValueError(f"{args.init} holds {w.numel()} parameters, the network has {n_params}")
        tr.ema.copy_(tr.params)
        print(f"# initialised from {args.init} ({winfo.get('step')} steps)", flush=True)
    if args.resume and os.path.exists(args.ckpt):
        tr.load(args.ckpt)
        print(f"# resumed {args.ckpt} at step {tr.step}", flush=True)
    hs_test = [build(voxels(c, args.N), levels, attention=att, net_levels=nl) for c in test]
    base0 = evaluate(tr.ema, hs_test)
    zero = evaluate_zero(hs_test)
    print(f"# params {n_params}; held-out post-V-cycle residual: zero init median {np.median(zero):.3e}, "
          f"network (EMA weights) at start median {np.median(base0):.3e}", flush=True)
    cache = {}
    budget = args.cache_gb * 2**30
    log = []
    t_start = time.time()
    t_last = t_start
    rng = np.random.default_rng(tr.step)
    k = 0
    H, idx, fresh, target = None, -1, False, None
    targets = {}
    while tr.step < args.steps:
        if k % args.steps_per_cell == 0:
            if fresh and idx not in cache:
                H.close()
            idx = int(rng.integers(len(cells)))
            H = cache.get(idx)
            fresh = H is None
            if fresh:
                H = build(voxels(cells[idx], args.N), levels, attention=att, net_levels=nl)
                target = None
                if args.supervised > 0:
                    # the plain solver's solution of this cell (mixed precision, FP32 copy)
                    u64, _ = H.solve(H.load_vector(), tol=args.target_tol, precision="f32", max_iter=3000,
                                     raise_on_noconv=False)
                    target = u64.to(torch.float32)
                    del u64
                if torch.cuda.memory_allocated() < budget:
                    cache[idx] = H
                    targets[idx] = target
            else:
                target = targets.get(idx)
        loss, rn, rel = tr.train_cell(H, args.steps, target=target, alpha=args.supervised)
        if not math.isfinite(loss):
            raise RuntimeError(f"non-finite loss at step {tr.step}")
        log.append({"step": tr.step, "loss": loss, "rel": rel, "family": cells[idx][1]})
        k += 1
        now = time.time()
        if now - t_last > 20 or tr.step % args.eval_every == 0:
            t_last = now
            recent = log[-200:]
            msg = (f"step {tr.step} lr {tr.lr_at(tr.step, args.steps):.2e} loss "
                   f"{np.mean([x['loss'] for x in recent]):.3f} train rel median "
                   f"{np.median([x['rel'] for x in recent]):.3e} ({(now - t_start) / k * 1e3:.0f} ms/step, "
                   f"{len(cache)} cached, {torch.cuda.memory_allocated() / 2**30:.0f} GiB)")
            if tr.step % args.eval_every == 0:
                ev = evaluate(tr.ema, hs_test)
                msg += f" | held-out EMA median {np.median(ev):.3e} max {ev.max():.3e}"
                tr.save(args.ckpt)
            print(msg, flush=True)
        if args.time_budget and now - t_start > args.time_budget:
            print(f"# time budget reached at step {tr.step}", flush=True)
            break
    if fresh and idx not in cache:
        H.close()
    tr.save(args.ckpt)
    ev = evaluate(tr.ema, hs_test)
    ev_noinj = evaluate(tr.ema, hs_test, inject=False)
    summary = {"held_out_zero_init_median": float(np.median(zero)),
               "held_out_start_median": float(np.median(base0)), "held_out_median": float(np.median(ev)),
               "held_out_max": float(ev.max()), "held_out_no_injection_median": float(np.median(ev_noinj)),
               "step": tr.step, "seconds": time.time() - t_start, "ms_per_step": (time.time() - t_start) / max(k, 1) * 1e3}
    print("# " + json.dumps(summary), flush=True)
    if args.export:
        meta = {"step": tr.step, "train_cells": args.cells, "train_seed0": args.seed0,
                "held_out_seed0": args.test_seed0, "steps_per_cell": args.steps_per_cell, "lr": args.lr,
                "ema": args.ema, "supervised": args.supervised, **summary}
        if args.init:
            meta["init"] = os.path.basename(args.init)
        save_weights(args.export, tr.ema, nl, args.N, "elastic", meta=meta, attention=att)
        print(f"# exported EMA weights to {args.export}", flush=True)
    if args.log:
        with open(args.log, "w") as fh:
            json.dump({"summary": summary, "log": log}, fh)
    for H in list(cache.values()) + hs_test:
        H.close()


if __name__ == "__main__":
    main(sys.argv[1:])
