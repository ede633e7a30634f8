"""Benchmark of the periodic GMG homogenization path on one MI355X.

Workload (one "step"): a batch of 64 elasticity cells at 128^3 from the mixed
lattice families (gyroid / Schwarz-P / diamond sheets, periodic truss,
spinodal; family = seed mod 5, VF ~ U(0.15, 0.5), seeds 1000..1063).  Every
cell goes through the whole path: sparse hierarchy + Galerkin operators +
coarse factor, load vector, mixed-precision GMG-PCG (FP32 bulk, FP64
refinement) to relative residual 1e-5 -- all cells in one batched call
(gmt_solve_batch) -- and the FP64 C_H reduction.

Prints one JSON line: metric, value (ms per cell, whole path), ms_per_step, the
batch config, solve-only time, DOF-solves/s, PCG iteration counts; "roofline" for
the level-1 Chebyshev sweep (372 algorithmic bytes per node over its duration,
timed with HIP events on the launch stream, against 8 TB/s; "traffic" is the
counter-measured HBM bytes per sweep of the cell and variant it was measured on,
else null); "learned" (plain vs learned initializer on the same cells) when the
weights exist; "cpu_baseline" (the CPU oracle on a 64^3 sample, scaled by nodes).
"""

from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms to 1e-5 rel. residual per cell + DOF/s: learned-init+1 V-cycle vs plain GMG"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per active node of one fine-level Chebyshev sweep, FP32 elastic:
# read u 72 + f 72 + D^-1 12 + d 72, write u' 72 + d 72
CHEB_BYTES_PER_NODE = 372
COPY_BYTES = 512 << 20
# HBM bytes of one level-1 Chebyshev sweep on the first bench cell (seed 1000, 128^3), from the
# FETCH_SIZE / write-request counters of the interior + boundary kernels, each scaled by what the
# counter reports for a copy of known size (profiles/level1_chebyshev_sweep_gyroid128_hbm_traffic.txt).
# It describes the kernels as they were profiled; re-profile after changing them.
# Keyed by (cell seed, level-1 sweep variant), so that a figure is reported only for the kernels
# it was measured on.
SWEEP_TRAFFIC_BYTES = {(1000, 7): 482_315_397}
# level-1 sweep variants (the autotuner's choice) and the kernels each launches
SWEEP_KERNELS = {
    0: "k_apply_interior_nc + k_apply_boundary_st",
    1: "k_apply_interior + k_apply_boundary",
    2: "k_apply_interior_nc + k_apply_boundary_nc",
    3: "k_apply_interior_run + k_apply_boundary",
    5: "k_apply_interior + k_apply_boundary_cls",
    6: "k_apply_interior_nc + k_apply_boundary_cls",
    7: "k_apply_interior<PRE=1> + k_apply_boundary_cls<PRE=1>",
}
WEIGHTS = os.path.join(ROOT, "paper_2604_26518_amd", "weights", "unet128_elastic.npz")


def _gen(seed_n):
    seed, N = seed_n
    from gmt_inputs.lattices import workload_cell
    fam, vf, vox = workload_cell(N, seed)
    return seed, fam, vf, vox


def make_cells(N, seeds):
    procs = max(1, min(16, os.cpu_count() or 1))
    with mp.get_context("fork").Pool(procs) as pool:
        return pool.map(_gen, [(s, N) for s in seeds])


UNEVEN_SIZES = (64, 96, 128, 192, 256)


def _gen_uneven(seed):
    from gmt_inputs.lattices import workload_cell
    N = UNEVEN_SIZES[(seed // 5) % 5]  # independent of the family (seed mod 5)
    fam, vf, vox = workload_cell(N, seed)
    return seed, fam, vf, vox, ("elastic" if seed % 2 == 0 else "thermal")


def uneven_batch(args):
    """The uneven batched workload: 256 cells, N uniform over {64, 96, 128, 192, 256}, mixed
    families, even seeds elastic (6 cases) and odd seeds thermal (3 cases), FP32 bulk + FP64
    refinement to 1e-5.  Cells go to gmt_solve_batch in chunks that fit a memory budget."""
    import torch

    from paper_2604_26518_amd import binding as B

    seeds = list(range(2000, 2000 + args.cells))
    procs = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs) as pool:
        cells = pool.map(_gen_uneven, seeds, chunksize=2)
    print(f"# generated {len(cells)} uneven cells in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    budget = args.mem_gb * 2**30

    failed = []

    def run(record):
        order = sorted(range(len(cells)), key=lambda k: -cells[k][3].size)
        t_all = time.perf_counter()
        solve_s, dofs, its, k = 0.0, 0, [], 0
        while k < len(order):
            hs, fs, idx = [], [], []
            while k < len(order) and (not hs or torch.cuda.memory_allocated() < budget):
                seed, fam, vf, vox, phys = cells[order[k]]
                H = B.Hierarchy(vox, B.default_levels(vox.shape[0]), phys)
                hs.append(H)
                fs.append(H.load_vector())
                idx.append(order[k])
                k += 1
            torch.cuda.synchronize()
            ts = time.perf_counter()
            us, reps = B.solve_batch(hs, fs, tol=args.tol, precision="f32", max_iter=args.max_iter,
                                     max_outer=16, n_workers=args.workers, graph=not args.no_graph,
                                     raise_on_noconv=False)
            solve_s += time.perf_counter() - ts
            for H, u, rep, j in zip(hs, us, reps, idx):
                H.homogenize(u)
                if not rep["converged"]:
                    failed.append({"seed": cells[j][0], "N": H.N, "physics": H.physics,
                                   "residual": max(rep["rel_res"]), "iterations": rep["iterations"]})
                dofs += H.n_n(1) * H.c * H.d
                its.append(rep["iterations"])
                if record is not None:
                    record.append({"seed": cells[j][0], "family": cells[j][1], "vf": cells[j][2], "N": H.N,
                                   "physics": H.physics, "its": rep["iterations"], "outer": rep["outer"]})
                H.close()
            del us, fs, hs
            print(f"# {k}/{len(order)} cells done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        return time.perf_counter() - t_all, solve_s, dofs, its

    for w in range(args.warmup):
        run(None)
    record = []
    wall, solve_s, dofs, its = 0.0, 0.0, 0, []
    for _ in range(args.steps):
        a, b, c, d = run(record if not record else None)
        wall, solve_s, dofs, its = wall + a, solve_s + b, dofs + c, its + d
    ncell = args.steps * len(cells)
    out = {"metric": "ms per cell, uneven batched solve to 1e-5 (whole path incl. build and C_H)",
           "value": round(wall / ncell * 1e3, 3), "unit": "ms/cell", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 2), "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{len(cells)} cells, N uniform over {list(UNEVEN_SIZES)}, mixed families, VF "
                                  f"U(0.15,0.5), half elasticity (6 cases) half heat conduction (3 cases), FP32 "
                                  f"bulk + FP64 refinement to {args.tol:g}, gmt_solve_batch in memory-bounded "
                                  f"chunks", "cells": len(cells), "workers": args.workers,
                      "graph": not args.no_graph},
           "ms_per_cell_solve_only": round(solve_s / ncell * 1e3, 3),
           "dof_solves_per_s": round(dofs / wall, 1), "iterations_mean": float(np.mean(its)),
           "iterations_max": int(np.max(its)), "not_converged": failed}
    print(json.dumps(out), flush=True)
    if os.environ.get("GMT_BENCH_CELLS"):
        with open(os.environ["GMT_BENCH_CELLS"], "w") as fh:
            json.dump(record, fh, indent=1)


def cpu_baseline(tol):
    """The CPU FP64 oracle on a bounded sample: one 64^3 workload cell, GMG-PCG to tol + C_H."""
    from gmt_inputs.lattices import workload_cell
    from oracle import solve as osolve

    fam, vf, vox = workload_cell(64, 1000)
    w0, c0 = time.perf_counter(), time.process_time()
    P = osolve.Problem(vox, 5)
    u, its = osolve.pcg(P, tol=tol)
    osolve.homogenize(P, u)
    wall = time.perf_counter() - w0
    cpu = time.process_time() - c0
    return {"wall_s": wall, "threads": max(1, round(cpu / wall)), "n_e": int(P.levels[0].n_e),
            "n_n": int(P.levels[0].n_n), "family": fam, "vf": vf, "iterations": its}


def learned_leg(B, vox_dev, levels, args, cells):
    """The learned path on the same cells: network forward -> one V-cycle -> FP64 check -> warm
    GMG-PCG fallback, against plain zero-init GMG-PCG, solve-only times (hierarchy built outside)."""
    import torch

    from paper_2604_26518_amd.evaluate import compare, summarize
    from paper_2604_26518_amd.learned import channels_for, load_weights

    params, info = load_weights(WEIGHTS)
    if info["levels"] != levels or info["N"] != args.N:
        return {"skipped": f"weights are for N={info['N']} L={info['levels']}"}
    recs = []
    for k, vox in enumerate(vox_dev):
        H = B.Hierarchy(vox, levels, "elastic")
        H.nn_setup(channels_for(levels))
        if k == 0:
            compare(H, params, args.tol, reference=False)  # warm-up
        recs.append(compare(H, params, args.tol, reference=(k < 8)))
        H.close()
    torch.cuda.synchronize()
    s = summarize(recs)
    s["weights"] = {"file": os.path.relpath(WEIGHTS, ROOT), "train_steps": info.get("step")}
    s["note"] = "solve-only ms/cell (hierarchy build excluded) for both paths on the bench cells"
    return s


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cells", type=int, default=64)
    ap.add_argument("--seed0", type=int, default=1000, help="first cell seed (cells seed0 .. seed0 + cells - 1)")
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--max-iter", type=int, default=3000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--workers", type=int, default=4, help="host threads / streams of the batched solve")
    ap.add_argument("--no-graph", action="store_true", help="launch PCG kernel by kernel")
    ap.add_argument("--workload", default="cells128", choices=["cells128", "uneven"],
                    help="cells128: the headline 64-cell 128^3 batch; uneven: 256 cells of mixed size and physics")
    ap.add_argument("--mem-gb", type=float, default=120.0, help="uneven workload: GPU memory per solve chunk")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding the "
              "path over several GPUs is not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2604_26518_amd import binding as B

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "uneven":
        if args.cells == 64:
            args.cells = 256
        torch.cuda.set_device(0)
        uneven_batch(args)
        return
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    t0 = time.perf_counter()
    cells = make_cells(args.N, list(range(args.seed0, args.seed0 + args.cells)))
    gen_s = time.perf_counter() - t0
    vox_dev = [torch.from_numpy(v).to(dev) for (_, _, _, v) in cells]
    torch.cuda.synchronize()
    levels = B.default_levels(args.N)
    print(f"# generated {len(cells)} cells at {args.N}^3 in {gen_s:.1f} s; levels={levels}",
          file=sys.stderr, flush=True)

    def step(record=None):
        """One pass of the path over the batch: hierarchies, loads, one batched mixed-precision
        solve (worker threads x streams, captured-graph PCG blocks), C_H per cell."""
        hs = [B.Hierarchy(vox, levels, "elastic") for vox in vox_dev]
        fs = [H.load_vector() for H in hs]
        torch.cuda.synchronize()
        ts = time.perf_counter()
        us, reps = B.solve_batch(hs, fs, tol=args.tol, precision="f32", max_iter=args.max_iter,
                                 n_workers=args.workers, graph=not args.no_graph, raise_on_noconv=False)
        solve_s = time.perf_counter() - ts
        dofs = 0
        its = []
        for k, (H, u, rep) in enumerate(zip(hs, us, reps)):
            CH = H.homogenize(u)
            if not rep["converged"]:
                raise RuntimeError(f"cell {k} did not converge: {rep}")
            dofs += H.n_n(1) * 3 * 6
            its.append(rep["iterations"])
            if record is not None:
                record.append({"seed": cells[k][0], "family": cells[k][1], "n_n": H.n_n(1),
                               "its": rep["iterations"], "outer": rep["outer"],
                               "res": max(rep["rel_res"]), "C11": float(CH[0, 0])})
        for H in hs:
            H.close()
        del us, fs
        return solve_s, dofs, its

    for w in range(args.warmup):
        step()
        print(f"# warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solve_total = 0.0
    dofs = 0
    its_all = []
    record = []
    for k in range(args.steps):
        s, d, its = step(record if k == 0 else None)
        solve_total += s
        dofs += d
        its_all += its
        print(f"# step {k + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ncell = args.steps * len(vox_dev)
    ms_cell = wall / ncell * 1e3
    ms_cell_solve = solve_total / ncell * 1e3

    # --- dominant kernel: the level-1 Chebyshev sweep (interior + boundary kernels, FP32),
    # timed with HIP events on the launch stream by the library
    H = B.Hierarchy(vox_dev[0], levels, "elastic")
    per_launch_s = H.time_sweep(1, reps=100) / 1e3
    nbytes = CHEB_BYTES_PER_NODE * H.n_n(1)
    achieved = nbytes / per_launch_s / 1e9
    variant = H.level_info(1)["sweep_variant"][0]
    kernel_info = {"n_n": H.n_n(1), "us_per_sweep": round(per_launch_s * 1e6, 2), "variant": variant,
                   "kernels": SWEEP_KERNELS.get(variant, "?") + " (float, 3 DOF, EPI_CHEB)"}
    H.close()
    # plain device copy of known size: what HBM sustains here, and the calibration run for the
    # FETCH_SIZE / WRITE_SIZE counters
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    copy_gbs = 2 * COPY_BYTES * 20 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst

    learned = None
    if os.path.exists(WEIGHTS) and not args.no_learned:
        learned = learned_leg(B, vox_dev, levels, args, cells)

    out = {
        "metric": METRIC,
        "value": round(ms_cell, 3),
        "unit": "ms/cell",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{len(vox_dev)} elasticity cells at {args.N}^3, mixed TPMS-sheet/truss/"
                               f"spinodal families, VF U(0.15,0.5), plain GMG-PCG (FP32 bulk, FP64 "
                               f"refinement) to {args.tol:g}, batched solve, whole path incl. hierarchy "
                               f"build and C_H",
                   "cells": len(vox_dev), "seed0": args.seed0, "N": args.N, "levels": levels, "tol": args.tol,
                   "workers": args.workers, "graph": not args.no_graph},
        "ms_per_cell_solve_only": round(ms_cell_solve, 3),
        "dof_solves_per_s": round(dofs / wall, 1),
        "iterations_mean": float(np.mean(its_all)),
        "iterations_max": int(np.max(its_all)),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": SWEEP_TRAFFIC_BYTES.get((cells[0][0], variant)) if args.N == 128 else None,
                     "kernel": "level-1 Chebyshev sweep", **kernel_info,
                     "copy_GBps": round(copy_gbs, 1)},
    }
    if learned is not None:
        out["learned"] = learned
    if not args.no_cpu_baseline:
        cb = cpu_baseline(args.tol)
        n_n_128 = float(np.mean([r["n_n"] for r in record]))
        scale = n_n_128 / cb["n_n"]
        out["cpu_baseline"] = {"value": round(cb["wall_s"] * 1e3 * scale, 1), "unit": "ms/cell", "cores": cb["threads"],
                               "kind": "oracle",
                               "sample": f"one 64^3 {cb['family']} cell (VF {cb['vf']:.2f}, seed 1000), oracle "
                                         f"GMG-PCG to {args.tol:g} + C_H in {cb['wall_s']:.1f} s, scaled by the "
                                         f"node ratio {scale:.2f} to a mean 128^3 cell"}
    print(json.dumps(out), flush=True)
    if os.environ.get("GMT_BENCH_CELLS"):
        with open(os.environ["GMT_BENCH_CELLS"], "w") as fh:
            json.dump(record, fh, indent=1)


if __name__ == "__main__":
    main()
