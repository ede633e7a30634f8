"""Timing of the learned initializer's network on one cell (forward and backward, with
and without attention blocks, and every level's window-attention kernel).

    python -m paper_2604_26518_amd.nn_timing --family gyroid --N 512 --seed 30001 --vf 0.25 --net-levels 6

Weights are seeded random (timing does not depend on training); one JSON line per
configuration.  Run it under rocprofv3 for per-kernel statistics.
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import torch

from . import binding as B
from .learned import channels_for, init_params

ATTN_FLOP_PER_SCORE = 35  # the 8-term q.k dot and p v update (2 x 16), exp, offset, sum


def scores_of(n, W, heads):
    """Query-key pairs of one level: full windows of W tokens plus the partial last one."""
    return heads * ((n // W) * W * W + (n % W) ** 2)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--family", default="gyroid")
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--vf", type=float, default=0.3)
    ap.add_argument("--levels", type=int, default=0, help="hierarchy levels (default for N)")
    ap.add_argument("--net-levels", type=int, default=0, help="network levels (default: all)")
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)
    from gmt_inputs.lattices import cell
    vox = cell(args.family, args.N, args.seed, args.vf)
    torch.cuda.set_device(0)
    L = args.levels or B.default_levels(args.N)
    nl = args.net_levels or L
    chs = channels_for(nl)
    H = B.Hierarchy(vox, L, "elastic")
    for att in (False, True):
        H.nn_setup(chs, attention=att)
        params = init_params(H.n_params, nl, attention=att, seed=1)
        grad = torch.zeros_like(params)
        outs = H.nn_forward(params)
        gouts = [torch.randn_like(o) for o in outs]
        H.nn_backward(gouts, grad)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.reps):
            H.nn_forward(params)
        torch.cuda.synchronize()
        tf = (time.perf_counter() - t) / args.reps
        t = time.perf_counter()
        for _ in range(args.reps):
            H.nn_backward(gouts, grad)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t) / args.reps
        rec = {"cell": f"{args.family} {args.N}^3 seed {args.seed} VF {args.vf}", "attention": att,
               "nodes": [H.n_n(l) for l in range(1, nl + 1)], "forward_ms": round(tf * 1e3, 3),
               "backward_ms": round(tb * 1e3, 3)}
        if att:
            H.nn_forward(params)
            lv = []
            for l in range(nl):
                n, W, heads = H.n_n(l + 1), min(256 << l, 1024), chs[l] // 8
                ms = H.nn_time_attention(l + 1, args.reps)
                sc = scores_of(n, W, heads)
                lv.append({"level": l + 1, "window": W, "heads": heads, "scores": sc, "kernel_ms": round(ms, 3),
                           "tflops": round(sc * ATTN_FLOP_PER_SCORE / (ms * 1e-3) / 1e12, 2)})
            rec["attention_levels"] = lv
        print(json.dumps(rec), flush=True)
    H.close()


if __name__ == "__main__":
    main(sys.argv[1:])
