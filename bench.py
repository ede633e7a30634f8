"""Benchmark of the periodic GMG homogenization path on one MI355X.

Default workload (one "step" = one cell through the whole path): a single
512^3 gyroid-sheet elasticity cell (seed 30001, VF 0.25, 6 load cases, L = 8
levels) homogenized to relative residual 1e-5 by the learned path --
hierarchy + Galerkin operators + coarse factor, load vector, network feature
tables, BF16 network forward (u_hat^1, e_hat^l), one Alg. 2 V-cycle, FP64
residual check, warm-started mixed-precision GMG-PCG fallback (FP32 bulk, FP64
refinement), FP64 C_H.  The plain path (zero-init GMG-PCG, same kernels) is
timed on the same cell for the comparison the metric names.

Prints one JSON line: metric, value (ms per cell, learned path, whole path),
the plain path's time and the gain, DOF-solves/s, C_H of both paths against an
FP64 solve, "roofline" for the level-1 Chebyshev sweep on this cell (372
algorithmic bytes per node over its duration, timed with HIP events on the
launch stream, against 8 TB/s), "extras" (the 512^3 spinodal, seed 30000, once
per path; the mixed-precision versus all-FP64 batch of 64 cells at 128^3; an
uneven batch of 40 cells of sizes 64^3..256^3, half elastic, half thermal), and
"cpu_baseline" (the CPU FP64 oracle on a bounded sample, scaled to this cell).

Other workloads: --workload cells128 (the 64-cell 128^3 batch, plain path) and
--workload uneven (256 cells of mixed size and physics).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import platform
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
# HBM bytes of one level-1 Chebyshev sweep, from the FETCH_SIZE / WRITE_SIZE counters of its two
# kernels, each scaled by what the counter reports for a copy of known size; keyed by (workload,
# sweep variant, SHA-256 prefix of the kernel source the counters were taken on), so that a changed
# kernel reports null until it is profiled again.
SWEEP_TRAFFIC_BYTES = {
    # profiles/level1_chebyshev_sweep_gyroid512_hbm_traffic.txt
    ("gyroid512_seed30001", 9, "64c7445f942b8902"): (22_693_601 + 5_186_849) * 1024,
}
SWEEP_KERNELS = {
    0: "k_apply_interior_nc + k_apply_boundary_st",
    1: "k_apply_interior + k_apply_boundary",
    2: "k_apply_interior_nc + k_apply_boundary_nc",
    3: "k_apply_interior_run + k_apply_boundary",
    5: "k_apply_interior + k_apply_boundary_cls",
    6: "k_apply_interior_nc + k_apply_boundary_cls",
    7: "k_apply_interior<PRE=1> + k_apply_boundary_cls<PRE=1>",
    8: "k_apply_interior<PRE=1> + k_apply_boundary_all",
    9: "k_apply_interior_stage + k_apply_interior<PRE=1> (unstaged rest) + k_apply_boundary_cls<PRE=1>",
}
# one network per resolution (the 512^3 one fine-tuned at 512^3 from the 128^3 one)
WEIGHTS_BY_N = {N: os.path.join(ROOT, "paper_2604_26518_amd", "weights", f"unet{N}_elastic.npz") for N in (128, 512)}


def weights_for(N):
    return WEIGHTS_BY_N.get(N, WEIGHTS_BY_N[128])
HEADLINE = {"family": "gyroid", "N": 512, "seed": 30001, "vf": 0.25}
SPINODAL = {"family": "spinodal", "N": 512, "seed": 30000, "vf": 0.25}
UNEVEN_SIZES = (64, 96, 128, 192, 256)


def kernel_source_hash() -> str:
    """SHA-256 prefix of the operator-sweep section of the kernel source (the level-1 sweep
    kernels and their epilogues), the code the stored counter figures describe."""
    with open(os.path.join(ROOT, "paper_2604_26518_amd", "csrc", "kernels.hip"), "rb") as fh:
        src = fh.read()
    a = src.index(b"// ---------------------------------------------------------------- operator sweeps")
    b = src.index(b"// ---------------------------------------------------------------- transfers")
    return hashlib.sha256(src[a:b]).hexdigest()[:16]


# --------------------------------------------------------------------------- host-side inputs
# Every input is generated in worker processes forked before the first GPU call (a process that
# has initialised HIP must not fork); pools are closed and joined, never terminated.

def _gen_named(spec):
    from gmt_inputs import cell
    return cell(spec["family"], spec["N"], spec["seed"], spec["vf"])


def _gen(seed_n):
    seed, N = seed_n
    from gmt_inputs.lattices import workload_cell
    fam, vf, vox = workload_cell(N, seed)
    return seed, fam, vf, vox


def _gen_uneven(seed):
    from gmt_inputs.lattices import workload_cell
    N = UNEVEN_SIZES[(seed // 5) % 5]  # independent of the family (seed mod 5)
    fam, vf, vox = workload_cell(N, seed)
    return seed, fam, vf, vox, ("elastic" if seed % 2 == 0 else "thermal")


def _pool(procs=16):
    return mp.get_context("fork").Pool(max(1, min(procs, os.cpu_count() or 1)))


def _finish(pool):
    pool.close()
    pool.join()


def cpu_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline_sample(tol):
    """The CPU FP64 oracle as it stands (numpy, matrix-free GMG-PCG, zero start) on a bounded
    sample of the headline workload: the same gyroid-sheet family, seed and VF at 64^3, solved
    to tol (hierarchy setup and solve timed separately), plus C_H."""
    from gmt_inputs import gyroid_sheet
    from oracle import solve as osolve
    try:
        from threadpoolctl import threadpool_info
        blas = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # noqa: BLE001
        blas = None
    vox = gyroid_sheet(64, HEADLINE["seed"], HEADLINE["vf"])
    w0, c0 = time.perf_counter(), time.process_time()
    P = osolve.Problem(vox, 4)
    w1 = time.perf_counter()
    u, its = osolve.pcg(P, tol=tol)
    w2 = time.perf_counter()
    osolve.homogenize(P, u)
    w3 = time.perf_counter()
    cpu = time.process_time() - c0
    return {"setup_s": w1 - w0, "solve_s": w2 - w1, "ch_s": w3 - w2, "wall_s": w3 - w0,
            "threads": max(1, round(cpu / (w3 - w0))), "blas_threads": blas, "n_n": int(P.levels[0].n_n),
            "iterations": int(its), **cpu_info()}


# --------------------------------------------------------------------------- GPU legs

def _sync():
    import torch
    torch.cuda.synchronize()


def learned_cell(B, vox, levels, params, net_levels, tol, max_iter):
    """Whole learned path on one cell; returns timings (s) and the solve record."""
    from paper_2604_26518_amd.learned import channels_for, learned_solve
    _sync()
    t0 = time.perf_counter()
    H = B.Hierarchy(vox, levels, "elastic")
    H.nn_setup(channels_for(net_levels))
    f = H.load_vector()
    _sync()
    t1 = time.perf_counter()
    u, info = learned_solve(H, params, tol=tol, max_iter=max_iter, f64=f)
    CH = H.homogenize(u)
    _sync()
    t2 = time.perf_counter()
    rec = {"whole_s": t2 - t0, "solve_s": t2 - t1, "n_n": H.n_n(1), "CH": CH, **info}
    return H, u, rec


def plain_cell(B, vox, levels, tol, max_iter):
    _sync()
    t0 = time.perf_counter()
    H = B.Hierarchy(vox, levels, "elastic")
    f = H.load_vector()
    _sync()
    t1 = time.perf_counter()
    u, rep = H.solve(f, tol=tol, precision="f32", max_iter=max_iter)
    CH = H.homogenize(u)
    _sync()
    t2 = time.perf_counter()
    if not rep["converged"]:
        raise RuntimeError(f"plain path did not converge: {rep}")
    rec = {"whole_s": t2 - t0, "solve_s": t2 - t1, "n_n": H.n_n(1), "CH": CH, "iterations": rep["iterations"],
           "rel_res": max(rep["rel_res"])}
    return H, u, rec


def sweep_roofline(B, H, workload):
    import torch
    per_launch_s = H.time_sweep(1, reps=20) / 1e3
    nbytes = CHEB_BYTES_PER_NODE * H.n_n(1)
    achieved = nbytes / per_launch_s / 1e9
    variant = H.level_info(1)["sweep_variant"][0]
    src = kernel_source_hash()
    traffic = SWEEP_TRAFFIC_BYTES.get((workload, variant, src))
    # plain device copy of known size: what HBM sustains here, and the calibration run of the counters
    src_t = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst_t = torch.empty_like(src_t)
    dst_t.copy_(src_t)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        dst_t.copy_(src_t)
    e1.record()
    e1.synchronize()
    copy_gbs = 2 * COPY_BYTES * 20 / (e0.elapsed_time(e1) / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": "level-1 Chebyshev sweep", "n_n": H.n_n(1), "algorithmic_bytes": nbytes,
            "us_per_sweep": round(per_launch_s * 1e6, 2), "variant": variant,
            "kernels": SWEEP_KERNELS.get(variant, "?") + " (float, 3 DOF, EPI_CHEB)", "kernel_source": src,
            "copy_GBps": round(copy_gbs, 1)}


def mixed_vs_fp64(B, cells, levels, tol, max_iter, workers):
    """C_H and time of the mixed-precision batch against the all-FP64 batch on the same cells."""
    import torch
    vox_dev = [torch.from_numpy(v).cuda() for (_, _, _, v) in cells]
    out = {}
    CHs = {}
    for prec in ("f32", "f64"):
        hs = [B.Hierarchy(v, levels, "elastic") for v in vox_dev]
        fs = [H.load_vector() for H in hs]
        _sync()
        t = time.perf_counter()
        us, reps = B.solve_batch(hs, fs, tol=tol, precision=prec, max_iter=max_iter, n_workers=workers,
                                 raise_on_noconv=False)
        _sync()
        dt = time.perf_counter() - t
        CHs[prec] = [H.homogenize(u) for H, u in zip(hs, us)]
        out[prec] = {"ms_per_cell_solve_only": round(dt / len(hs) * 1e3, 2),
                     "iterations_mean": float(np.mean([r["iterations"] for r in reps])),
                     "converged": int(sum(bool(r["converged"]) for r in reps)),
                     "max_rel_res": float(max(max(r["rel_res"]) for r in reps))}
        for H in hs:
            H.close()
        del us, fs
    err = [np.linalg.norm(a - b) / np.linalg.norm(b) for a, b in zip(CHs["f32"], CHs["f64"])]
    out["CH_mixed_vs_fp64_max"] = float(max(err))
    out["speedup_mixed_over_fp64"] = round(out["f64"]["ms_per_cell_solve_only"] /
                                           out["f32"]["ms_per_cell_solve_only"], 3)
    out["workload"] = (f"{len(cells)} elasticity cells at 128^3 (seeds {cells[0][0]}..{cells[-1][0]}, mixed "
                       f"families, VF U(0.15,0.5)), batched GMG-PCG to {tol:g}, mixed (FP32 bulk + FP64 "
                       f"refinement) vs all-FP64")
    return out


def cell512(args):
    import torch

    from paper_2604_26518_amd import binding as B
    from paper_2604_26518_amd.learned import load_weights

    t0 = time.perf_counter()
    pool = _pool()
    jobs = {"gyroid": pool.apply_async(_gen_named, (dict(HEADLINE, N=args.N),))}
    if args.extras:
        jobs["spinodal"] = pool.apply_async(_gen_named, (dict(SPINODAL, N=args.N),))
        jobs["c2"] = pool.map_async(_gen, [(s, 128) for s in range(1000, 1000 + args.c2_cells)])
        jobs["uneven"] = pool.map_async(_gen_uneven, range(2000, 2000 + args.uneven_cells), chunksize=1)
    if not args.no_cpu_baseline:
        jobs["cpu"] = pool.apply_async(cpu_baseline_sample, (args.tol,))
    res = {k: j.get() for k, j in jobs.items()}
    _finish(pool)
    print(f"# inputs generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    levels = B.default_levels(args.N)
    WEIGHTS = weights_for(args.N)
    params, info = load_weights(WEIGHTS)
    net_levels = min(info["levels"], levels)
    vox = torch.from_numpy(res["gyroid"]).cuda()

    def lstep():
        H, u, rec = learned_cell(B, vox, levels, params, net_levels, args.tol, args.max_iter)
        H.close()
        return rec

    def pstep():
        H, u, rec = plain_cell(B, vox, levels, args.tol, args.max_iter)
        H.close()
        return rec

    for w in range(args.warmup):
        lstep()
        pstep()
        print(f"# warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    # timed region: K steps of the learned path
    _sync()
    t = time.perf_counter()
    lrecs = []
    for k in range(args.steps):
        lrecs.append(lstep())
        print(f"# learned step {k + 1}/{args.steps} done", file=sys.stderr, flush=True)
    _sync()
    wall = time.perf_counter() - t
    # the comparison: K steps of the plain path on the same cell
    _sync()
    t = time.perf_counter()
    precs = []
    for k in range(args.steps):
        precs.append(pstep())
    _sync()
    wall_plain = time.perf_counter() - t
    print("# plain steps done", file=sys.stderr, flush=True)

    # C_H of both paths against an FP64 solve to 1e-9 on the same hierarchy
    H = B.Hierarchy(vox, levels, "elastic")
    f = H.load_vector()
    u64, rep64 = H.solve(f, tol=1e-9, precision="f64", max_iter=args.max_iter)
    C_ref = H.homogenize(u64)
    nref = np.linalg.norm(C_ref)
    err_l = float(np.linalg.norm(lrecs[0]["CH"] - C_ref) / nref)
    err_p = float(np.linalg.norm(precs[0]["CH"] - C_ref) / nref)
    del u64
    # network time alone, and the dominant kernel's roofline on this cell
    from paper_2604_26518_amd.learned import channels_for
    H.nn_setup(channels_for(net_levels))
    H.nn_forward(params)
    _sync()
    t = time.perf_counter()
    for _ in range(5):
        H.nn_forward(params)
    _sync()
    net_ms = (time.perf_counter() - t) / 5 * 1e3
    roof = sweep_roofline(B, H, f"gyroid512_seed{HEADLINE['seed']}")
    H.close()

    n_n = lrecs[0]["n_n"]
    ms_l = wall / args.steps * 1e3
    ms_p = wall_plain / args.steps * 1e3
    out = {
        "metric": METRIC,
        "value": round(ms_l, 2),
        "unit": "ms/cell",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_l, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"one {args.N}^3 gyroid-sheet elasticity cell (seed {HEADLINE['seed']}, VF "
                               f"{HEADLINE['vf']}, 6 load cases, L={levels}): learned init (BF16 U-Net on levels "
                               f"1..{net_levels}) + one V-cycle + warm mixed-precision GMG-PCG fallback to "
                               f"{args.tol:g}, whole path incl. hierarchy build, network tables and C_H",
                   "N": args.N, "levels": levels, "net_levels": net_levels, "tol": args.tol,
                   "n_n": n_n, "dof": 18 * n_n},
        "dof_solves_per_s": round(18 * n_n / (ms_l / 1e3), 1),
        "ms_per_cell_solve_only": round(float(np.mean([r["solve_s"] for r in lrecs])) * 1e3, 2),
        "plain": {"ms_per_cell": round(ms_p, 2),
                  "ms_per_cell_solve_only": round(float(np.mean([r["solve_s"] for r in precs])) * 1e3, 2),
                  "iterations": precs[0]["iterations"], "dof_solves_per_s": round(18 * n_n / (ms_p / 1e3), 1)},
        "gain_plain_over_learned": round(ms_p / ms_l, 4),
        "learned": {"rel_after_vcycle": lrecs[0]["rel_after_vcycle"], "fallback": lrecs[0]["fallback"],
                    "fallback_iterations": lrecs[0]["iterations"], "net_ms": round(net_ms, 2),
                    "weights": {"file": os.path.relpath(WEIGHTS, ROOT), "trained_N": info["N"],
                                "trained_levels": info["levels"], "train_steps": info.get("step")}},
        "CH_rel_err_vs_fp64": {"learned": err_l, "plain": err_p, "fp64_tol": 1e-9,
                               "fp64_iterations": rep64["iterations"]},
        "roofline": roof,
    }
    if args.extras:
        sv = torch.from_numpy(res["spinodal"]).cuda()
        Hl, _, rl = learned_cell(B, sv, levels, params, net_levels, args.tol, args.max_iter)
        Hl.close()
        Hp, _, rp = plain_cell(B, sv, levels, args.tol, args.max_iter)
        Hp.close()
        out["extras"] = {"spinodal512": {
            "seed": SPINODAL["seed"], "vf": float(res["spinodal"].mean()), "n_n": rl["n_n"],
            "learned_ms": round(rl["whole_s"] * 1e3, 1), "plain_ms": round(rp["whole_s"] * 1e3, 1),
            "learned_fallback_iterations": rl["iterations"], "plain_iterations": rp["iterations"],
            "rel_after_vcycle": rl["rel_after_vcycle"],
            "CH_learned_vs_plain": float(np.linalg.norm(rl["CH"] - rp["CH"]) / np.linalg.norm(rp["CH"]))}}
        del sv
        print("# spinodal done", file=sys.stderr, flush=True)
        out["extras"]["attention512"] = attention_extra(B, vox, levels, net_levels)
        print("# attention done", file=sys.stderr, flush=True)
        out["extras"]["mixed_vs_fp64_128"] = mixed_vs_fp64(B, res["c2"], B.default_levels(128), args.tol,
                                                           args.max_iter, args.workers)
        print("# mixed vs FP64 batch done", file=sys.stderr, flush=True)
        cells = res["uneven"]
        wall_u, solve_u, dofs_u, its_u, failed_u = run_uneven(B, cells, args.tol, args.max_iter, args.workers,
                                                              True, args.mem_gb)
        out["extras"]["uneven_batch"] = {
            "workload": f"{len(cells)} cells (seeds 2000..{1999 + len(cells)}), N over {list(UNEVEN_SIZES)}, mixed "
                        f"families, even seeds elastic (6 cases), odd seeds thermal (3 cases), one gmt_solve_batch "
                        f"call per memory chunk (captured-graph PCG blocks with device-side convergence flags), "
                        f"FP32 bulk + FP64 refinement to {args.tol:g}, whole path incl. build and C_H",
            "ms_per_cell": round(wall_u / len(cells) * 1e3, 2),
            "ms_per_cell_solve_only": round(solve_u / len(cells) * 1e3, 2),
            "dof_solves_per_s": round(dofs_u / wall_u, 1), "iterations_mean": float(np.mean(its_u)),
            "iterations_max": int(np.max(its_u)), "not_converged": failed_u}
        print("# uneven batch done", file=sys.stderr, flush=True)
    if "cpu" in res:
        cb = res["cpu"]
        scale = n_n / cb["n_n"]
        its512 = precs[0]["iterations"]
        est_s = (cb["setup_s"] + cb["ch_s"]) * scale + cb["solve_s"] / max(cb["iterations"], 1) * its512 * scale
        out["cpu_baseline"] = {
            "value": round(est_s * 1e3, 1), "unit": "ms/cell", "cores": cb["threads"], "kind": "oracle",
            "sample": (f"numpy FP64 oracle GMG-PCG (zero start, tol {args.tol:g}) + C_H on the same gyroid "
                       f"(seed {HEADLINE['seed']}, VF {HEADLINE['vf']}) at 64^3: setup {cb['setup_s']:.1f} s, "
                       f"{cb['iterations']} iterations in {cb['solve_s']:.1f} s, C_H {cb['ch_s']:.1f} s, "
                       f"{cb['n_n']} nodes; scaled per node by {scale:.1f} to the {args.N}^3 cell and per "
                       f"iteration to the {its512} iterations the plain path takes there"),
            "nproc": cb["nproc"], "cpu_model": cb["cpu_model"], "blas_threads": cb["blas_threads"]}
    print(json.dumps(out), flush=True)


def cells128(args):
    """The 64-cell 128^3 batch (plain path): hierarchies, loads, one batched mixed-precision solve
    (worker threads x streams, captured-graph PCG blocks), C_H per cell."""
    import torch

    from paper_2604_26518_amd import binding as B

    t0 = time.perf_counter()
    pool = _pool()
    cells = pool.map(_gen, [(s, args.N) for s in range(args.seed0, args.seed0 + args.cells)])
    _finish(pool)
    gen_s = time.perf_counter() - t0
    torch.cuda.set_device(0)
    vox_dev = [torch.from_numpy(v).cuda() for (_, _, _, v) in cells]
    levels = B.default_levels(args.N)
    print(f"# generated {len(cells)} cells at {args.N}^3 in {gen_s:.1f} s; levels={levels}", file=sys.stderr,
          flush=True)

    def step():
        hs = [B.Hierarchy(vox, levels, "elastic") for vox in vox_dev]
        fs = [H.load_vector() for H in hs]
        _sync()
        ts = time.perf_counter()
        us, reps = B.solve_batch(hs, fs, tol=args.tol, precision="f32", max_iter=args.max_iter,
                                 n_workers=args.workers, graph=not args.no_graph, raise_on_noconv=False)
        solve_s = time.perf_counter() - ts
        dofs, its = 0, []
        for k, (H, u, rep) in enumerate(zip(hs, us, reps)):
            H.homogenize(u)
            if not rep["converged"]:
                raise RuntimeError(f"cell {k} did not converge: {rep}")
            dofs += H.n_n(1) * 18
            its.append(rep["iterations"])
        for H in hs:
            H.close()
        return solve_s, dofs, its

    for w in range(args.warmup):
        step()
    _sync()
    t0 = time.perf_counter()
    solve_total, dofs, its_all = 0.0, 0, []
    for k in range(args.steps):
        s, d, its = step()
        solve_total, dofs, its_all = solve_total + s, dofs + d, its_all + its
        print(f"# step {k + 1}/{args.steps} done", file=sys.stderr, flush=True)
    _sync()
    wall = time.perf_counter() - t0
    ncell = args.steps * len(vox_dev)
    H = B.Hierarchy(vox_dev[0], levels, "elastic")
    roof = sweep_roofline(B, H, f"cell128_seed{args.seed0}")
    H.close()
    out = {"metric": "ms per cell, batched plain GMG-PCG to 1e-5 (whole path incl. build and C_H)",
           "value": round(wall / ncell * 1e3, 3), "unit": "ms/cell", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 2), "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{len(vox_dev)} elasticity cells at {args.N}^3, mixed families, VF U(0.15,0.5), "
                                  f"plain GMG-PCG (FP32 bulk, FP64 refinement) to {args.tol:g}, batched",
                      "cells": len(vox_dev), "seed0": args.seed0, "N": args.N, "levels": levels},
           "ms_per_cell_solve_only": round(solve_total / ncell * 1e3, 3),
           "dof_solves_per_s": round(dofs / wall, 1), "iterations_mean": float(np.mean(its_all)),
           "iterations_max": int(np.max(its_all)), "roofline": roof}
    print(json.dumps(out), flush=True)


# algorithmic FP32 operations per attention score in the forward: the 8-term q.k dot
# and the 8-term p v update (2 x 16), the exponential, the offset subtraction and the
# sum of the probabilities
ATTN_FLOP_PER_SCORE = 35
FP32_PEAK_TFLOPS = 157.3


def attention_extra(B, vox, levels, net_levels, reps=5):
    """The network with an attention block per level on the headline cell (seeded random
    weights: timing only): forward time against the convolutional network's, and every
    level's window-attention kernel timed with HIP events on its launch stream."""
    import torch

    from paper_2604_26518_amd.learned import channels_for, init_params
    H = B.Hierarchy(vox, levels, "elastic")
    chs = channels_for(net_levels)
    H.nn_setup(chs, attention=True)
    params = init_params(H.n_params, net_levels, attention=True, seed=1)
    H.nn_forward(params)
    _sync()
    t = time.perf_counter()
    for _ in range(reps):
        H.nn_forward(params)
    _sync()
    fwd_ms = (time.perf_counter() - t) / reps * 1e3
    per_level = []
    for l in range(net_levels):
        n, W, heads = H.n_n(l + 1), min(256 << l, 1024), chs[l] // 8
        scores = heads * ((n // W) * W * W + (n % W) ** 2)
        ms = H.nn_time_attention(l + 1, reps)
        tf = scores * ATTN_FLOP_PER_SCORE / (ms * 1e-3) / 1e12
        per_level.append({"level": l + 1, "tokens": n, "window": W, "heads": heads, "scores": scores,
                          "kernel_ms": round(ms, 3), "tflops": round(tf, 2)})
    H.close()
    top = per_level[0]
    return {"workload": "headline cell, network with one serialized window-attention block (Ra-RoPE) per level "
                        "on levels 1..%d, seeded random weights" % net_levels,
            "forward_ms": round(fwd_ms, 2), "levels": per_level,
            "attention_ms_total": round(sum(x["kernel_ms"] for x in per_level), 2),
            "roofline": {"kernel": "k_attn_fwd, level 1", "bound": "alu", "achieved": top["tflops"],
                         "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(top["tflops"] / FP32_PEAK_TFLOPS, 4),
                         "flop_per_score": ATTN_FLOP_PER_SCORE}}


def run_uneven(B, cells, tol, max_iter, workers, graph, mem_gb):
    """One pass over uneven cells: hierarchies built in memory-bounded chunks, each chunk one
    gmt_solve_batch call (FP32 bulk + FP64 refinement), C_H per cell.
    Returns (wall_s, solve_s, dof_solves, iterations, not_converged)."""
    import torch
    budget = mem_gb * 2**30
    order = sorted(range(len(cells)), key=lambda k: -cells[k][3].size)
    failed = []
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
        _sync()
        ts = time.perf_counter()
        us, reps = B.solve_batch(hs, fs, tol=tol, precision="f32", max_iter=max_iter, max_outer=16,
                                 n_workers=workers, graph=graph, raise_on_noconv=False)
        solve_s += time.perf_counter() - ts
        for H, u, rep, j in zip(hs, us, reps, idx):
            H.homogenize(u)
            if not rep["converged"]:
                failed.append({"seed": cells[j][0], "N": H.N, "physics": H.physics,
                               "residual": max(rep["rel_res"]), "iterations": rep["iterations"]})
            dofs += H.n_n(1) * H.c * H.d
            its.append(rep["iterations"])
            H.close()
        del us, fs, hs
        print(f"# {k}/{len(order)} uneven cells done", file=sys.stderr, flush=True)
    _sync()
    return time.perf_counter() - t_all, solve_s, dofs, its, failed


def uneven(args):
    """256 cells, N uniform over {64, 96, 128, 192, 256}, mixed families, even seeds elastic (6
    cases) and odd seeds thermal (3 cases), FP32 bulk + FP64 refinement to 1e-5; cells go to
    gmt_solve_batch in chunks that fit a memory budget."""
    import torch

    from paper_2604_26518_amd import binding as B

    seeds = list(range(2000, 2000 + args.cells))
    t0 = time.perf_counter()
    pool = _pool()
    cells = pool.map(_gen_uneven, seeds, chunksize=2)
    _finish(pool)
    print(f"# generated {len(cells)} uneven cells in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    for _ in range(args.warmup):
        run_uneven(B, cells, args.tol, args.max_iter, args.workers, not args.no_graph, args.mem_gb)
    wall, solve_s, dofs, its, failed = 0.0, 0.0, 0, [], []
    for _ in range(args.steps):
        a, b, c, d, e = run_uneven(B, cells, args.tol, args.max_iter, args.workers, not args.no_graph, args.mem_gb)
        wall, solve_s, dofs, its, failed = wall + a, solve_s + b, dofs + c, its + d, failed + e
    ncell = args.steps * len(cells)
    out = {"metric": "ms per cell, uneven batched solve to 1e-5 (whole path incl. build and C_H)",
           "value": round(wall / ncell * 1e3, 3), "unit": "ms/cell", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 2), "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{len(cells)} cells, N uniform over {list(UNEVEN_SIZES)}, mixed families, VF "
                                  f"U(0.15,0.5), half elasticity half heat conduction, FP32 bulk + FP64 "
                                  f"refinement to {args.tol:g}, gmt_solve_batch in memory-bounded chunks",
                      "cells": len(cells), "workers": args.workers, "graph": not args.no_graph},
           "ms_per_cell_solve_only": round(solve_s / ncell * 1e3, 3),
           "dof_solves_per_s": round(dofs / wall, 1), "iterations_mean": float(np.mean(its)),
           "iterations_max": int(np.max(its)), "not_converged": failed}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cell512", choices=["cell512", "cells128", "uneven"],
                    help="cell512: the 512^3 learned-vs-plain headline; cells128: 64 cells at 128^3; uneven: "
                         "256 cells of mixed size and physics")
    ap.add_argument("--N", type=int, default=0, help="cell size (cell512: 512, cells128: 128)")
    ap.add_argument("--cells", type=int, default=0)
    ap.add_argument("--seed0", type=int, default=1000)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--max-iter", type=int, default=3000)
    ap.add_argument("--no-extras", dest="extras", action="store_false",
                    help="cell512: skip the spinodal cell and the mixed-vs-FP64 128^3 batch")
    ap.add_argument("--c2-cells", type=int, default=64)
    ap.add_argument("--uneven-cells", type=int, default=40, help="cell512 extras: cells of the uneven batch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workers", type=int, default=4, help="host threads / streams of the batched solve")
    ap.add_argument("--no-graph", action="store_true", help="launch PCG kernel by kernel")
    ap.add_argument("--mem-gb", type=float, default=120.0, help="uneven workload: GPU memory per solve chunk")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding the "
              "path over several GPUs is not built.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "cell512":
        args.N = args.N or 512
        cell512(args)
    elif args.workload == "cells128":
        args.N = args.N or 128
        args.cells = args.cells or 64
        cells128(args)
    else:
        args.cells = args.cells or 256
        uneven(args)


if __name__ == "__main__":
    main()
