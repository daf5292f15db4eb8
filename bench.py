"""Throughput of the random-walker solve on one MI355X.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--no-cpu-baseline]

Workload (default "blob512"): a 512^3 float32 volume of 32 random ellipsoid
blobs (radii U(10, 60), intensities U(0.5, 0.9)) on background 0.2 with
Gaussian noise sigma 0.08, three labels (two blob classes + background),
1000 seeds per label inside their regions, beta = 150, min-max normalised,
stopped at relative residual 1e-6.  Synthetic and seeded; it stands in for
the paper's cell-volume benchmark (Sec. IV-B, Table III).

One step = one whole solve on inputs already resident in HBM: the device
min-max reduction plus rw_solve in mixed precision (float32 stencil and
vectors, float64 dot products, float64 residual refinement).  The plain
float64 solve of the same volume is timed beside it (two steps after one
warm-up, whatever --steps is), and the same run checks the results: the
oracle's float64 relative residual of both outputs, and mixed against
float64 (max-abs difference, argmax away from ties).  The hierarchical
batched workload (hier1024, see bench_hier) runs after it and is reported in
the same line under "hier1024" (its own steps and warm-up, stated there).

Prints ONE JSON line.  `roofline` is for the dominant kernel (CG pass 2):
algorithmic bytes per launch over its average launch duration from HIP
events recorded around every launch on the library's stream.  `cpu_baseline`
is the C/OpenMP float64 oracle timed on a bounded sample of the same
workload.

Other workloads (`--workload`): hier1024 (hierarchical batched bricks),
stream2048 (bricks streamed through device pools), sphere128grad (float64
forward + adjoint gradient), heart4d (4-D random walker of a volume time
series); each is described in its own function.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("solved voxels/sec at rel. residual 1e-6 (FP32+FP64-dot vs FP64); "
          "% HBM roofline")
HBM_PEAK_GBS = 8000.0
# what roofline.traffic counts: the TCC FETCH_SIZE (scaled by a copy kernel
# of known size) and WRITE_SIZE counters, i.e. bytes that missed the L2;
# misses served by the memory-side cache are included, so it bounds HBM
# bytes from above
TRAFFIC_COUNTS = "L2-miss bytes per launch (FETCH_SIZE x copy factor + WRITE_SIZE)"


def pass_bytes(n_vox, launches, rhs_iterations, s_g, s_m, s_v, which):
    """Algorithmic HBM bytes of the CG passes (per voxel: pass 1 reads g, z,
    p_old and writes p_new: s_g + 3 R s_v; pass 2 reads g, labels, p, x, z and
    writes x, z: s_g + s_m + 5 R s_v; R = labels still iterating)."""
    if which == 1:
        return n_vox * (launches * s_g + 3 * s_v * rhs_iterations)
    return n_vox * (launches * (s_g + s_m) + 5 * s_v * rhs_iterations)


def make_workload(name):
    from synth import blob_case
    if name == "hier1024":
        return blob_case(shape=(1024, 1024, 1024), n_blobs=64, K=3, seeds_per_label=8000,
                         sigma=0.08, bg=0.2, rmin=10.0, rmax=60.0, beta=150.0, seed=3,
                         dtype="u16", name="hier1024")
    if name == "blob512":
        return blob_case(shape=(512, 512, 512), n_blobs=32, K=3, seeds_per_label=1000,
                         sigma=0.08, bg=0.2, rmin=10.0, rmax=60.0, beta=150.0, seed=2,
                         dtype="f32", name="blob512")
    if name == "blob256":
        return blob_case(shape=(256, 256, 256), n_blobs=4, K=3, seeds_per_label=125,
                         sigma=0.08, bg=0.2, rmin=10.0, rmax=60.0, beta=150.0, seed=2,
                         dtype="f32", name="blob256")
    raise SystemExit(f"unknown workload {name}")


def kernel_source_hash():
    """sha256 of the stencil kernel source (the traffic counters are only
    quoted while it is unchanged)."""
    import hashlib
    path = os.path.join(ROOT, "paper_2509_26213_amd", "csrc", "rw_cg_kernels.h")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def tile_key(tile):
    """Canonical text of a stencil tile shape (the stats' tile dict)."""
    key = "vx={vx} by={by} zc={zc} xcd={xcd}".format(**tile)
    by2, zc2 = tile.get("by2", tile["by"]), tile.get("zc2", tile["zc"])
    if by2 in (0, tile["by"]) and zc2 in (0, tile["zc"]):
        return key
    return key + f" pass2 by={by2} zc={zc2}"


def measured_traffic(kernel, workload, tile):
    """Ratio of measured HBM bytes (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled
    by a copy kernel of known size) to algorithmic bytes per launch, from the
    committed summary profiles/<kernel>_<workload>_traffic.md; None when it is
    missing or was taken on another version of the kernel source or with
    another tile shape than this run's."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    if vals.get("tile") != tile_key(tile):
        return None
    try:
        return float(vals["traffic_over_algorithmic"])
    except (KeyError, ValueError):
        return None


def traffic(ratio, alg_bytes_per_launch):
    """HBM bytes per launch: the measured traffic ratio times this run's
    algorithmic bytes per launch (None without a current measurement)."""
    return None if ratio is None else ratio * alg_bytes_per_launch


def copy_calibration():
    """A plain device copy of known size, for scaling the FETCH_SIZE /
    WRITE_SIZE counters: 1 GiB read + 1 GiB written per launch, 5 launches."""
    import torch
    n = 1 << 28
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": 4 * n, "launches": 5}), flush=True)


def cpu_baseline(case, gpu_iters_fp64, n_iter, threads):
    """The float64 C oracle on the same volume: a fixed number of Jacobi-PCG
    iterations of label 2, scaled to a whole solve with the float64 GPU
    solve's per-label iteration counts (the oracle needs the same counts to
    within one).  Returns voxels/s of the oracle."""
    import numpy as np
    from oracle import c_oracle, rw_oracle
    g = rw_oracle.case_g(case)
    t0 = time.perf_counter()
    _, it, st = c_oracle.pcg_fixed_iters(g, case.labels, 2, case.beta, n_iter, nthreads=threads)
    wall = time.perf_counter() - t0
    setup_s, loop_s = c_oracle.last_timing()
    t_iter = loop_s / max(it, 1)
    total_iters = sum(gpu_iters_fp64)
    t_solve = setup_s * len(gpu_iters_fp64) + t_iter * total_iters
    n_vox = int(np.prod(case.shape))
    return dict(value=n_vox / t_solve, unit="voxels/s", cores=threads, cpu_model=cpu_model(),
                kind="oracle",
                sample=(f"{it} float64 Jacobi-PCG iterations of label 2 on the full "
                        f"{case.shape[0]}^3 volume ({wall:.1f} s wall, {t_iter * 1e3:.1f} ms/iter, "
                        f"set-up {setup_s:.1f} s), scaled to the {total_iters} iterations "
                        f"({'+'.join(str(i) for i in gpu_iters_fp64)}) of labels 2..K"),
                seconds_per_solve=t_solve)


def cpu_baseline_hier(case, coarse_iters, bricks, brick_iters, n_iter, threads, n_sample=16):
    """The float64 C oracle on the hierarchical workload: its own level-2
    volume (two 2x2x2 means of the float64 level 0) timed over n_iter
    Jacobi-PCG iterations of label 2 and scaled to the GPU's coarse iteration
    counts, plus n_sample bricks (stratified by size, clipped ones included)
    timed over n_iter iterations each and scaled by the GPU's sum over all
    bricks of voxels x iterations.  Returns voxels/s of the oracle."""
    import numpy as np
    from oracle import c_oracle, rw_oracle
    t_all = time.perf_counter()
    g = rw_oracle.case_g(case)
    g2 = rw_oracle.downsample_mean(rw_oracle.downsample_mean(g))
    l2 = rw_oracle.coarse_seeds(rw_oracle.coarse_seeds(case.labels))
    _, it, _ = c_oracle.pcg_fixed_iters(g2, l2, 2, case.beta, n_iter, nthreads=threads)
    setup_s, loop_s = c_oracle.last_timing()
    t_coarse = setup_s * len(coarse_iters) + loop_s / max(it, 1) * sum(coarse_iters)
    vox = np.array([int(np.prod(s)) for _, s in bricks])
    order = np.argsort(vox, kind="stable")
    pick = order[np.linspace(0, len(order) - 1, n_sample).astype(int)]
    per_vox_iter = []
    for i in pick:
        o, s = bricks[i]
        # Dirichlet data 0.5 on the shell: a nonzero right-hand side, so every
        # sampled brick runs its n_iter iterations (a zero one stops at once)
        shell = np.full(tuple(int(v) + 2 for v in s), 0.5)
        t0 = time.perf_counter()
        _, its, _, _ = c_oracle.solve_box(g, case.labels, 2, case.beta, tol=1e-300,
                                          max_iter=n_iter, box=(tuple(o), tuple(s)), shell=shell,
                                          nthreads=threads)
        per_vox_iter.append((time.perf_counter() - t0) / (vox[i] * max(its, 1)))
    work = sum(int(v) * sum(it) for v, it in zip(vox, brick_iters))
    t_bricks = float(np.mean(per_vox_iter)) * work
    n_vox = int(np.prod(case.labels.shape))
    t_solve = t_coarse + t_bricks
    return dict(value=n_vox / t_solve, unit="voxels/s", cores=threads, cpu_model=cpu_model(),
                kind="oracle",
                sample=(f"level-2 {g2.shape[0]}^3 solve: {it} float64 Jacobi-PCG iterations of "
                        f"label 2 scaled to the GPU's {sum(coarse_iters)}; {n_sample} of "
                        f"{len(bricks)} bricks (by size) x {n_iter} iterations, scaled by the "
                        f"GPU's sum of brick voxels x iterations ({work:.3g}); "
                        f"{time.perf_counter() - t_all:.1f} s wall"),
                seconds_per_solve=t_solve)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="blob512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-hier", action="store_true",
                    help="blob512: leave out the hier1024 sub-object")
    ap.add_argument("--hier-steps", type=int, default=3,
                    help="blob512: timed steps of the hier1024 sub-object")
    ap.add_argument("--cpu-iters", type=int, default=12)
    ap.add_argument("--nt", type=int, default=20,
                    help="heart4d: time steps of the 50x224x224 series (the paper has 200: "
                         "about 10000 mixed CG iterations, a minute per solve)")
    ap.add_argument("--pool", type=int, default=256,
                    help="stream2048: bricks per device pool")
    ap.add_argument("--update-delta", type=float, default=None,
                    help="mixed precision: float64 residual refresh when ||r|| fell by this "
                         "factor (default: the library's, 0.1 whole volumes, 0.01 bricks)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--autotune", action="store_true",
                    help="hier1024: run the library's tile autotuners (level-2 whole solve, "
                         "bricks) before timing")
    ap.add_argument("--tune", action="store_true",
                    help="only run the library's tile autotuners on the blob512 and hier1024 "
                         "workloads (their table goes to librw.tune, or RW_TUNE_FILE)")
    ap.add_argument("--profile-iters", type=int, default=0,
                    help="profiling runs only: cap CG iterations (the JSON line is then not a "
                         "whole solve)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU (a volume sharded over GPUs is not implemented); --gpus must be 1",
                          "n_gpus": args.gpus}))
        raise SystemExit(2)

    import numpy as np
    import torch
    from paper_2509_26213_amd import rw

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.tune:
        return tune_tables(args)
    if args.workload == "hier1024":
        return bench_hier(args)
    if args.workload == "stream2048":
        return bench_stream(args)
    if args.workload == "sphere128grad":
        return bench_grad(args)
    if args.workload == "heart4d":
        return bench_4d(args)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    case = make_workload(args.workload)
    print(f"# workload {case.name} generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    vol = torch.from_numpy(case.vol).to(dev)
    lab = torch.from_numpy(case.labels).to(dev)
    n_vox = int(np.prod(case.shape))
    K = case.K
    ctx = rw.default_context()
    ws = torch.empty(rw.solve_workspace_bytes(case.shape, K, "fp64"), dtype=torch.uint8,
                     device=dev)

    extra = {"max_iter": args.profile_iters} if args.profile_iters else {}

    def step(precision, timing):
        import warnings
        lo, hi = rw.minmax(vol, ctx=ctx)
        with warnings.catch_warnings():
            if args.profile_iters:
                warnings.simplefilter("ignore")
            if precision == "mixed" and args.update_delta is not None:
                extra["update_delta"] = args.update_delta
            return rw.solve(vol, lab, K, case.beta, tol=1e-6, precision=precision, lo=lo, hi=hi,
                            ctx=ctx, workspace=ws, return_stats=True, kernel_timing=timing,
                            **extra)

    def timed(precision, steps, warmup, events=True):
        """Wall time per solve over `steps` graph-replayed solves, then (with
        events) one more solve with every pass bracketed by events (no
        graphs) for the per-kernel rooflines; also the last output."""
        for _ in range(warmup):
            step(precision, False)
        torch.cuda.synchronize()
        stats = []
        t = time.perf_counter()
        for _ in range(steps):
            prob, am, st = step(precision, False)
            stats.append(st)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t) / steps
        if events:
            prob, am, st = step(precision, True)
            stats = [st]
        return sec, stats, (prob, am)

    sec_mixed, st_mixed, out_mixed = timed("mixed", args.steps, args.warmup)
    print(f"# mixed: {sec_mixed * 1e3:.1f} ms/step iters {st_mixed[-1]['iters']} "
          f"refinements {st_mixed[-1]['refinements']}", file=sys.stderr, flush=True)
    out_fp64 = None
    checks = {}
    if not args.no_fp64:
        sec_fp64, st_fp64, res_fp64 = timed("fp64", 2, 1, events=False)
        print(f"# fp64: {sec_fp64 * 1e3:.1f} ms/step iters {st_fp64[-1]['iters']}",
              file=sys.stderr, flush=True)
        s = st_fp64[-1]
        out_fp64 = dict(value=n_vox / sec_fp64, ms_per_step=sec_fp64 * 1e3, steps=2, warmup=1,
                        iters=s["iters"], rel_residual=s["rel_residual"])
        if not args.profile_iters:
            checks = result_checks(case, out_mixed, res_fp64)
            print(f"# checks {checks}", file=sys.stderr, flush=True)
        del res_fp64
    del out_mixed

    # roofline of the dominant kernel (pass 2) over the timed mixed steps
    launches2 = sum(s["pass_launches"][1] for s in st_mixed)
    launches1 = sum(s["pass_launches"][0] for s in st_mixed)
    rhs_it = sum(s["rhs_iterations"] for s in st_mixed)
    ms2 = sum(s["pass_ms"][1] for s in st_mixed)
    ms1 = sum(s["pass_ms"][0] for s in st_mixed)
    bytes2 = pass_bytes(n_vox, launches2, rhs_it, 4, 1, 4, 2)
    bytes1 = pass_bytes(n_vox, launches1, rhs_it, 4, 1, 4, 1)
    ach2 = bytes2 / (ms2 * 1e-3) / 1e9
    ach1 = bytes1 / (ms1 * 1e-3) / 1e9
    s = st_mixed[-1]
    result = {
        "metric": METRIC,
        "value": n_vox / sec_mixed,
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_mixed * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64dot",
        "data": "synthetic",
        "config": {"workload": f"{case.name}: {case.shape[0]}x{case.shape[1]}x{case.shape[2]} "
                               f"float32 blob volume, K={K}, 1000 seeds/label, beta={case.beta}, "
                               "tol 1e-6, mixed precision (FP32 stencil+vectors, FP64 dots, "
                               "FP64 refinement)",
                   "voxels": n_vox, "labels": K, "solved_labels": s["num_solved"]},
        "roofline": {"bound": "hbm", "kernel": "k_pass2", "achieved": ach2,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach2 / HBM_PEAK_GBS,
                     "traffic": traffic(measured_traffic("k_cg_pass2", case.name, s["tile"]),
                                        bytes2 / max(launches2, 1)),
                     "traffic_counts": TRAFFIC_COUNTS,
                     "avg_launch_us": ms2 * 1e3 / max(launches2, 1),
                     "bytes_per_launch": bytes2 / max(launches2, 1)},
        "pass1": {"achieved": ach1, "frac": ach1 / HBM_PEAK_GBS,
                  "avg_launch_us": ms1 * 1e3 / max(launches1, 1)},
        "tile": tile_key(s["tile"]),
        "tile_from_autotuner": s["tile_tuned"],
        "stencil_cg_loop_frac": (bytes1 + bytes2) / ((ms1 + ms2) * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "iters": s["iters"],
        "refinements": s["refinements"],
        "rel_residual": s["rel_residual"],
        "device_ms": s["device_ms"],
        "fp64": out_fp64,
        "mixed_speedup_vs_fp64": (out_fp64["value"] and (n_vox / sec_mixed) / out_fp64["value"])
        if out_fp64 else None,
        "checks": checks,
    }
    if not args.no_cpu_baseline:
        threads = len(os.sched_getaffinity(0))
        gpu_iters = out_fp64["iters"] if out_fp64 else s["iters"]
        try:
            result["cpu_baseline"] = cpu_baseline(case, gpu_iters, args.cpu_iters, threads)
        except Exception as e:  # the baseline never hides the GPU result
            result["cpu_baseline"] = {"error": repr(e)}
    del vol, lab, ws
    torch.cuda.empty_cache()
    if args.workload == "blob512" and not args.no_hier and not args.profile_iters:
        try:
            result["hier1024"] = run_hier(args, args.hier_steps, 1)
        except Exception as e:  # the sub-object never hides the headline
            result["hier1024"] = {"error": repr(e)}
    print(json.dumps(result), flush=True)


def tune_tables(args):
    """Run the library's autotuners on the benchmark workloads: the whole-
    volume tiles of blob512 (mixed), and on hier1024 the level-2 whole-volume
    tiles and the brick tiles.  The library records every winner in its
    table file (librw.tune beside librw.so, or RW_TUNE_FILE)."""
    import torch
    from paper_2509_26213_amd import rw
    dev = torch.device("cuda:0")
    case = make_workload("blob512")
    vol = torch.from_numpy(case.vol).to(dev)
    lab = torch.from_numpy(case.labels).to(dev)
    lo, hi = rw.minmax(vol)
    best = rw.autotune(vol, lab, case.K, case.beta, precision="mixed", lo=lo, hi=hi)
    print(json.dumps({"tuned": "blob512 whole (vx, zc, xcd, by)", "best": list(best)}), flush=True)
    del vol, lab
    torch.cuda.empty_cache()
    args.autotune = True
    out = run_hier(args, 1, 0)
    print(json.dumps({"tuned": "hier1024", "best": out["autotuned"]}), flush=True)


def cpu_model():
    """Model name of the host CPU (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def result_checks(case, out_mixed, out_fp64):
    """Checks of this run's outputs: the oracle's float64 relative residual
    ||b - L_U x|| / ||b|| of each solved label of both outputs (its own
    weights from the volume, its own right-hand side from the seeds), and the
    mixed output against the float64 one (max-abs difference, argmax
    mismatches where the float64 top-two gap is at least 1e-4)."""
    import numpy as np
    import torch
    from oracle import c_oracle, rw_oracle
    p32, a32 = out_mixed
    p64, a64 = out_fp64
    top2 = torch.topk(p64, 2, dim=0).values
    clear = (top2[0] - top2[1]) >= 1e-4
    out = {"max_abs_mixed_vs_fp64": float((p32.double() - p64).abs().max()),
           "argmax_mismatch_away_from_ties": int(((a32 != a64) & clear).sum()),
           "near_ties": int((~clear).sum())}
    del top2, clear
    lo, hi = case.norm_range()
    g = rw_oracle.normalize(case.vol, lo, hi)
    for name, p in (("fp64", p64), ("mixed", p32)):
        res = []
        for s in range(2, case.K + 1):
            x = p[s - 1].double().cpu().numpy()
            res.append(c_oracle.residual(g, case.labels, s, case.beta, x))
        out[f"oracle_rel_residual_{name}"] = res
    out["oracle_residual_bound"] = "1e-6 (tol) for fp64; float32 rounding of the output adds to mixed"
    return out


def bench_hier(args):
    """The hierarchical workload alone (see run_hier), as the JSON line."""
    out = run_hier(args, args.steps, args.warmup)
    line = {"metric": METRIC, "value": out.pop("value"), "unit": "voxels/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": out.pop("ms_per_step"),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32+f64dot", "data": "synthetic"}
    line.update(out)
    print(json.dumps(line), flush=True)


def run_hier(args, steps, warmup):
    """Hierarchical workload (1024^3 u16): levels 1, 2 by device LOD steps,
    the 256^3 level solved whole (mixed), 64^3 bricks on a grid offset
    (48, 20, 40) classified from the upsampled coarse solution, the uncertain
    ones solved in one batched brick solve (mixed), the others filled.  One
    step = the whole pipeline on the resident volume.  Returns the result
    dict (value = volume voxels per second end to end)."""
    import warnings

    import numpy as np
    import torch
    from paper_2509_26213_amd import rw
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    case = make_workload("hier1024")
    print(f"# workload {case.name} generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    K, n_vox = case.K, int(np.prod(case.shape))
    vol = torch.from_numpy(case.vol).to(dev)
    lab = torch.from_numpy(case.labels).to(dev)
    brick, offset = (64, 64, 64), (48, 20, 40)

    def step(timing=False):
        g1, l1 = rw.downsample(vol, lab, out_dtype=torch.float32)
        g2, l2 = rw.downsample(g1, l1, lo=0.0, hi=1.0, out_dtype=torch.float32)
        coarse, _, cst = rw.solve(g2, l2, K, case.beta, tol=1e-6, precision="mixed", lo=0.0,
                                  hi=1.0, argmax=False, return_stats=True)
        cands, active = rw.classify_bricks(coarse, lab, 4, brick, offset)
        act = [b for b, a in zip(cands, active) if a]
        ina = [b for b, a in zip(cands, active) if not a]
        prob = torch.empty((K,) + tuple(vol.shape), dtype=torch.float32, device=dev)
        if ina:
            rw.fill_bricks(coarse, lab, 4, ina, prob)
        t = time.perf_counter()
        extra = {"max_iter": args.profile_iters} if args.profile_iters else {}
        extra["update_delta"] = args.update_delta
        with warnings.catch_warnings():
            if args.profile_iters:
                warnings.simplefilter("ignore")
            _, iters, bst = rw.solve_bricks(vol, lab, K, case.beta, coarse, 4, act,
                                            prob_out=prob, tol=1e-6, precision="mixed",
                                            return_stats=True, kernel_timing=timing, lo=0.0,
                                            hi=65535.0, **extra)
        torch.cuda.synchronize()
        return dict(coarse=cst, bricks=bst, n_active=len(act), n_cand=len(cands),
                    brick_s=time.perf_counter() - t, iters=iters, act=act)

    tuned = None
    if args.autotune:
        # the library's autotuners pick the level-2 tiles and the brick tiles
        # on this workload before anything is timed (not timed themselves)
        g1, l1 = rw.downsample(vol, lab, out_dtype=torch.float32)
        g2, l2 = rw.downsample(g1, l1, lo=0.0, hi=1.0, out_dtype=torch.float32)
        whole = rw.autotune(g2, l2, K, case.beta, precision="mixed", lo=0.0, hi=1.0)
        coarse, _ = rw.solve(g2, l2, K, case.beta, tol=1e-6, precision="mixed", lo=0.0, hi=1.0,
                             argmax=False)
        cands, active = rw.classify_bricks(coarse, lab, 4, brick, offset)
        act = [b for b, a in zip(cands, active) if a]
        bt = rw.autotune_bricks(vol, lab, K, case.beta, coarse, 4, act, precision="mixed",
                                lo=0.0, hi=65535.0)
        tuned = {"level2 (vx, zc, xcd, by)": list(whole), "bricks (by, rpl, zc, xcd)": list(bt)}
        del g1, l1, g2, l2, coarse
        print(f"# autotuned {tuned}", file=sys.stderr, flush=True)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    outs = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t) / steps
    og = outs[-1]
    o = step(timing=True)  # per-pass events (no graphs) for the rooflines
    b = o["bricks"]
    bytes2 = b["box_voxel_iterations"] * (2 + 1) + 5 * 4 * b["rhs_voxel_iterations"]
    bytes1 = b["box_voxel_iterations"] * 2 + 3 * 4 * b["rhs_voxel_iterations"]
    persistent = b.get("brick_blocks", 0) > 0
    if persistent:
        # one launch holds every pass (and the starts, refreshes and folds):
        # its algorithmic pass bytes over its whole duration
        ach2 = ach1 = (bytes1 + bytes2) / (b["loop_ms"] * 1e-3) / 1e9
    else:
        ach2 = bytes2 / (b["pass_ms"][1] * 1e-3) / 1e9
        ach1 = bytes1 / (b["pass_ms"][0] * 1e-3) / 1e9
    act_vox = b["unknowns"]
    its = np.array(o["iters"])
    cpu = None
    if not args.no_cpu_baseline:
        try:
            cpu = cpu_baseline_hier(case, og["coarse"]["iters"], og["act"], og["iters"],
                                    args.cpu_iters, len(os.sched_getaffinity(0)))
        except Exception as e:  # the baseline never hides the GPU result
            cpu = {"error": repr(e)}
    del vol, lab
    torch.cuda.empty_cache()
    return {
        "value": n_vox / sec, "ms_per_step": sec * 1e3, "steps": steps, "warmup": warmup,
        "config": {"workload": "hier1024: 1024^3 uint16 blob volume (64 blobs, 8000 seeds per "
                               "label, K=3, beta 150), level-2 256^3 solved whole, 64^3 bricks on "
                               "offset grid, uncertain bricks solved batched, mixed, tol 1e-6",
                   "voxels": n_vox, "candidate_bricks": o["n_cand"],
                   "active_bricks": o["n_active"]},
        "bricks": {"voxels_per_s": act_vox / (og["bricks"]["device_ms"] * 1e-3),
                   "device_ms": og["bricks"]["device_ms"], "loop_ms": og["bricks"]["loop_ms"],
                   "iters_median": float(np.median(its)) if its.size else 0,
                   "iters_max": int(its.max()) if its.size else 0,
                   "refreshes": b["refinements"]},
        "roofline": ({"bound": "hbm", "kernel": "k_bricks_persistent", "achieved": ach2,
                      "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach2 / HBM_PEAK_GBS,
                      "traffic": None, "avg_launch_us": b["loop_ms"] * 1e3,
                      "bytes_per_launch": bytes1 + bytes2, "blocks": b["brick_blocks"]}
                     if persistent else
                     {"bound": "hbm", "kernel": "k_cg_pass2 (bricks)", "achieved": ach2,
                      "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach2 / HBM_PEAK_GBS,
                      "traffic": traffic(measured_traffic("k_cg_pass2", "hier1024", b["tile"]),
                                         bytes2 / max(b["pass_launches"][1], 1)),
                      "traffic_counts": TRAFFIC_COUNTS,
                      "avg_launch_us": b["pass_ms"][1] * 1e3 / max(b["pass_launches"][1], 1),
                      "bytes_per_launch": bytes2 / max(b["pass_launches"][1], 1)}),
        "pass1": {"achieved": ach1, "frac": ach1 / HBM_PEAK_GBS},
        "tile": tile_key(b["tile"]) + (" persistent" if persistent else ""),
        "tile_from_autotuner": b["tile_tuned"],
        "autotuned": tuned,
        "stencil_cg_loop_frac": (bytes1 + bytes2) / ((b["loop_ms"] if persistent else
                                                      b["pass_ms"][0] + b["pass_ms"][1]) * 1e-3)
        / 1e9 / HBM_PEAK_GBS,
        "coarse": {"iters": og["coarse"]["iters"], "device_ms": og["coarse"]["device_ms"]},
        "cpu_baseline": cpu,
    }


def cpu_baseline_4d(case, gpu_iters, n_iter, threads, nt_sample=2):
    """The oracle's 4-D random walker (assembled sparse Laplacian, Jacobi-PCG
    in float64, the only 4-D oracle) on the first nt_sample time steps of
    the series: assembly and n_iter iterations of label 2 timed, scaled to
    the whole series and the GPU's iteration counts.  Returns voxels/s."""
    import numpy as np
    from oracle import rw_oracle as O
    t_all = time.perf_counter()
    lo, hi = case.norm_range()
    g = O.normalize(case.vol[:nt_sample], lo, hi)
    lab = case.labels[:nt_sample].copy()  # the first time step holds seeds of both labels
    t0 = time.perf_counter()
    sysm = O.DirichletSystem(g, lab, case.beta, 0.0, 2)
    b = sysm.rhs(2)
    t_setup = time.perf_counter() - t0
    dinv = 1.0 / sysm.diag
    t0 = time.perf_counter()
    O.pcg_jacobi(sysm.LU, b, dinv, np.zeros(b.size), 1e-300, n_iter)
    t_iter = (time.perf_counter() - t0) / n_iter
    vox_s = int(np.prod(g.shape))
    n_vox = int(np.prod(case.vol.shape))
    scale = n_vox / vox_s
    t_solve = (t_setup + t_iter * sum(gpu_iters)) * scale
    return dict(value=n_vox / t_solve, unit="voxels/s", cores=threads, cpu_model=cpu_model(),
                kind="oracle",
                sample=(f"assembled 4-D system of the first {nt_sample} time steps "
                        f"({vox_s} voxels): set-up {t_setup:.1f} s, {n_iter} float64 Jacobi-PCG "
                        f"iterations at {t_iter * 1e3:.0f} ms, scaled by voxels to the "
                        f"{case.vol.shape[0]} time steps and to the GPU's {sum(gpu_iters)} "
                        f"iterations; {time.perf_counter() - t_all:.1f} s wall"),
                seconds_per_solve=t_solve)


def bench_4d(args):
    """4-D random walker (Sec. V-B): a synthetic stand-in for the paper's
    cardiac MRI series, 50x224x224 voxels per time step and --nt time steps
    (the paper has 200; 20 by default), an ellipsoid pulsing over time on a noisy
    background, 10 foreground and 10 background seeds in the first time step
    and 4 foreground seeds in the last, as in the paper's experiment.  One
    step = one whole-series solve (min-max reduction + rw_solve4d, mixed
    precision, tol 1e-6) on the resident series; the float64 solve is timed
    once beside it."""
    import numpy as np
    import torch
    from paper_2509_26213_amd import rw
    from synth import timeseries_case
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    case = timeseries_case(shape=(args.nt, 50, 224, 224))
    print(f"# workload heart4d ({args.nt} time steps) generated in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    vol = torch.from_numpy(case.vol).to(dev)
    lab = torch.from_numpy(case.labels).to(dev)
    n_vox = int(np.prod(case.vol.shape))
    ctx = rw.default_context()

    def step(precision, timing=False):
        lo, hi = rw.minmax(vol.view(-1, 224, 224), ctx=ctx)
        return rw.solve4d(vol, lab, 2, case.beta, tol=1e-6, precision=precision, lo=lo, hi=hi,
                          ctx=ctx, return_stats=True, kernel_timing=timing)

    for _ in range(args.warmup):
        step("mixed")
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        prob, am, st = step("mixed")
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t) / args.steps
    print(f"# mixed: {sec * 1e3:.1f} ms/step iters {st['iters']}", file=sys.stderr, flush=True)
    s = step("mixed", True)[2]
    bytes2 = pass_bytes(n_vox, s["pass_launches"][1], s["rhs_iterations"], 4, 1, 4, 2)
    bytes1 = pass_bytes(n_vox, s["pass_launches"][0], s["rhs_iterations"], 4, 1, 4, 1)
    ach2 = bytes2 / (s["pass_ms"][1] * 1e-3) / 1e9
    ach1 = bytes1 / (s["pass_ms"][0] * 1e-3) / 1e9
    # checks of the same run: partition of unity, exact seeds, range
    seeded = lab > 0
    checks = {"max_abs_sum_minus_1": float((prob.double().sum(0) - 1).abs().max()),
              "seeds_exact": bool(((prob[1][seeded] == 1) == (lab[seeded] == 2)).all()),
              "min": float(prob.min()), "max": float(prob.max())}
    del prob, am
    torch.cuda.synchronize()
    t = time.perf_counter()
    p64, _, s64 = step("fp64")
    torch.cuda.synchronize()
    sec64 = time.perf_counter() - t
    del p64
    cpu = None
    if not args.no_cpu_baseline:
        try:
            cpu = cpu_baseline_4d(case, st["iters"], args.cpu_iters,
                                  len(os.sched_getaffinity(0)))
        except Exception as e:  # the baseline never hides the GPU result
            cpu = {"error": repr(e)}
    print(json.dumps({
        "metric": METRIC, "value": n_vox / sec, "unit": "voxels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64dot", "data": "synthetic",
        "config": {"workload": f"heart4d: {args.nt}x50x224x224 float32 pulsing-ellipsoid time "
                               "series, K=2, 10+10 seeds in the first and 4 in the last time "
                               "step, beta 100, 8-connected 4-D grid, mixed, tol 1e-6",
                   "voxels": n_vox},
        "iters": st["iters"], "refinements": st["refinements"],
        "rel_residual": st["rel_residual"],
        "roofline": {"bound": "hbm", "kernel": "k_cg_pass2 (4-D)", "achieved": ach2,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach2 / HBM_PEAK_GBS,
                     "traffic": None,
                     "avg_launch_us": s["pass_ms"][1] * 1e3 / max(s["pass_launches"][1], 1),
                     "bytes_per_launch": bytes2 / max(s["pass_launches"][1], 1)},
        "pass1": {"achieved": ach1, "frac": ach1 / HBM_PEAK_GBS},
        "tile": tile_key(s["tile"]),
        "stencil_cg_loop_frac": (bytes1 + bytes2) / ((s["pass_ms"][0] + s["pass_ms"][1]) * 1e-3)
        / 1e9 / HBM_PEAK_GBS,
        "fp64": {"value": n_vox / sec64, "ms_per_step": sec64 * 1e3, "iters": s64["iters"]},
        "checks": checks,
        "cpu_baseline": cpu,
    }), flush=True)


def bench_grad(args):
    """Differentiable solve (128^3 float32 sphere, sigma 0.1, 500 seeds per
    label, beta 120): one step = the float64 forward solve of the foreground
    label and the adjoint solve + edge-gradient kernel giving dL/dg and
    dL/dbeta of L = sum (x_fg - mask)^2, both at tol 1e-6."""
    import numpy as np
    import torch
    from paper_2509_26213_amd import rw
    from synth import sphere_case
    dev = torch.device("cuda:0")
    c = sphere_case(n=128, radius=40, sigma=0.1, seed_radius=20, corner=16, n_seeds=500,
                    beta=120.0, seed=4)
    lo, hi = c.norm_range()
    g = ((torch.from_numpy(c.vol).to(dev).double() - lo) / (hi - lo)).contiguous()
    lab = torch.from_numpy(c.labels).to(dev)
    mask = torch.from_numpy(c.truth.astype(np.float64)).to(dev)
    n_vox = int(np.prod(c.vol.shape))

    def step():
        t0 = time.perf_counter()
        prob, _, fst = rw.solve(g, lab, 2, c.beta, tol=1e-6, precision="fp64", lo=0.0, hi=1.0,
                                argmax=False, return_stats=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        grad_prob = torch.stack([torch.zeros_like(mask), 2 * (prob[1] - mask)])
        dg, db = rw.solve_backward(g, lab, 2, c.beta, prob, grad_prob, tol=1e-6)
        db = float(db)
        torch.cuda.synchronize()
        return t1 - t0, time.perf_counter() - t1, fst, db

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    outs = [step() for _ in range(args.steps)]
    fwd = float(np.median([o[0] for o in outs]))
    bwd = float(np.median([o[1] for o in outs]))
    print(json.dumps({
        "metric": METRIC, "value": n_vox / (fwd + bwd), "unit": "voxels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": (fwd + bwd) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "sphere128grad: 128^3 float32 sphere (radius 40 at 0.7 on 0.3, "
                               "sigma 0.1), K=2, 500 seeds per label, beta 120, loss "
                               "sum (x_fg - mask)^2, float64 forward + adjoint, tol 1e-6",
                   "voxels": n_vox},
        "forward_ms": fwd * 1e3, "backward_ms": bwd * 1e3,
        "forward_iters": outs[-1][2]["iters"], "dL_dbeta": outs[-1][3],
    }), flush=True)


def bench_stream(args):
    """Out-of-core-shaped workload (2048x2048x1024 uint16, K = 4, 256 blobs
    (the blob density of the hierarchical workload), 4000 seeds per label,
    counter-based noise): the volume is generated in
    host memory (threads over z-slabs, not timed), then one streamed
    hierarchical solve: level 1 built brick by brick from pinned
    double-buffered H2D copies, level 2 (512x512x256) solved whole, 128^3
    bricks classified, the uncertain ones streamed through two device pools
    and solved batched, only uint8 labels back to the host.  `value` is the
    volume's voxels over the device time of the solves (coarse + bricks); the
    end-to-end rate includes PCIe and the host-side staging."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch
    from paper_2509_26213_amd import rw
    from paper_2509_26213_amd.stream import streamed_solve
    from synth.volumes import brickwise_blob_case

    t0 = time.perf_counter()
    case = brickwise_blob_case(shape=(1024, 2048, 2048), n_blobs=256, K=4, seeds_per_label=4000,
                               sigma=0.08, bg=0.2, rmin=10.0, rmax=60.0, beta=150.0, seed=5)
    shape = case.shape
    vol = np.empty(shape, np.uint16)
    lab = np.empty(shape, np.uint8)

    def slab(z):
        v, l, _ = case.brick((z, 0, 0), (4, shape[1], shape[2]))
        vol[z:z + 4] = v
        lab[z:z + 4] = l

    with ThreadPoolExecutor(max_workers=16) as ex:
        for i, _ in enumerate(ex.map(slab, range(0, shape[0], 4))):
            if i % 64 == 63:
                print(f"# generated {4 * (i + 1)} of {shape[0]} planes", file=sys.stderr,
                      flush=True)
    print(f"# workload stream2048 generated in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    n_vox = int(np.prod(shape))
    labels = np.zeros(shape, np.uint8)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, info = streamed_solve(vol, lab, case.K, case.beta, brick=(128, 128, 128), pool=args.pool,
                             tol=1e-6, levels=2, lo=0.0, hi=65535.0, precision="mixed",
                             labels_out=labels, update_delta=args.update_delta)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t
    seeded = lab > 0
    seeds_exact = bool(np.array_equal(labels[seeded], lab[seeded]))
    in_range = bool(labels.min() >= 1 and labels.max() <= case.K)
    brick_dev_ms = sum(b["device_ms"] for b in info["brick_stats"])
    its = np.array([i for b in info["brick_iters"] for i in b]) if info["brick_iters"] else np.zeros(1)
    dev_s = info["coarse_s"] + brick_dev_ms * 1e-3
    print(json.dumps({
        "metric": METRIC, "value": n_vox / dev_s, "unit": "voxels/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": sec * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64dot", "data": "synthetic",
        "config": {"workload": "stream2048: 2048x2048x1024 uint16 blob volume generated brick-wise "
                               "(256 blobs, 4000 seeds per label, K=4, beta 150) in host memory, "
                               "level-2 512x512x256 solved whole, 128^3 bricks streamed through "
                               f"two device pools of {args.pool}, mixed, tol 1e-6, labels out",
                   "voxels": n_vox, "bricks": info["bricks"],
                   "active_bricks": info["active_bricks"]},
        "end_to_end_voxels_per_s_pcie_inclusive": n_vox / sec,
        "seconds": {k: info[k] for k in ("lod_s", "coarse_s", "fill_s", "bricks_s",
                                         "brick_solve_s", "total_s")},
        "brick_device_ms": brick_dev_ms,
        "coarse_iters": info["coarse_iters"],
        "brick_iters_median": float(np.median(its)), "brick_iters_max": int(its.max()),
        "pcie": {"h2d_bytes": info["h2d_bytes"], "d2h_bytes": info["d2h_bytes"]},
        "seeds_on_device": info["seeds"],
        "checks": {"seeds_exact": seeds_exact, "labels_in_range": in_range},
    }), flush=True)


if __name__ == "__main__":
    main()
