"""Benchmark: seconds per DMFT iteration of the nonequilibrium Falicov-Kimball
lattice step at N_c = 1800 (t in [-10, 30], dt = dtau = 0.05, beta = 10,
55 x 55 Gauss-Hermite points, E = 1) on one MI355X.

A step is one DMFT iteration: the lattice step over all 3025 points (build,
batched inversion, rho-weighted reduction, current) plus the impurity update.
Inputs are the physical parameters only (synthetic, resident on the device).

python bench.py [--gpus 1] [--steps K] [--warmup W] [--U 1.0]
                [--mixed] [--converge | --no-converge] [--no-cpu-baseline]
                [--workload c2|c1]
Prints ONE JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 matrix peak
PEAK_FP32_TFLOPS = 157.3    # MI355X dense FP32 matrix peak
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the dominant kernel (the big trailing update,
# fk::k_update<double, 2>, 757-matrix batches of the C2 workload), from the
# rocprofv3 FETCH_SIZE and WRITE_SIZE runs summarized under profiles/, each
# scaled by the same counter's reading for a plain 256 MiB copy (FETCH_SIZE x
# 2.00, WRITE_SIZE x 1.00).  Reported only for that kernel and batch size.
PROFILED_TRAFFIC = {"kernel": "fk::k_update<double, 2>", "batch": 757,
                    "bytes_per_launch": 82.58e9}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w, n_sample=48):
    """The oracle (plain numpy/LAPACK complex128) on the host cores: the time of
    n_sample lattice points (each an N_c x N_c dense solve) and one impurity
    update, scaled to the full 3025-point iteration."""
    import numpy as np
    from oracle import dmft, impurity, lattice
    from paper_0711_0999_amd import inputs
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    p = dmft.Problem(t_min=w.t_min, t_max=w.t_max, dt=w.dt, dtau=w.dtau,
                     beta=w.beta, u=w.U, e_field=w.E, n_eps=w.n_eps,
                     n_ebar=w.n_ebar)
    z, wts, n_t, eps, ebar, rho = p.grid()
    n = len(z)
    sig = inputs.random_sigma(n, seed=11, scale=0.01)
    st = lattice.weighted_sigma(sig, wts)
    ks = inputs.sample_points(len(eps), n_sample, seed=12)
    t0 = time.perf_counter()
    for k in ks:
        lattice.point_green(z, n_t, w.E, 0.0, w.beta, eps[k], ebar[k], st)
    t_pts = time.perf_counter() - t0
    gl = np.eye(n, dtype=np.complex128) * 0.1j
    t0 = time.perf_counter()
    impurity.update(gl + 0.01 * sig, sig, wts, 0.0, w.U, w.w1)
    t_imp = time.perf_counter() - t0
    per_iter = t_pts / len(ks) * len(eps) + t_imp
    return {"value": per_iter, "unit": "s/iteration", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{len(ks)} of {len(eps)} points (N_c={n} dense solves, "
                      f"{t_pts:.1f} s) + 1 impurity update ({t_imp:.1f} s), "
                      "scaled to all points"}


def sweep_bench(args):
    """C4: one multi-instance sweep (every instance's lattice step in shared
    batched launches of uneven matrices, plus all impurity updates), recorded
    once in a hipGraph and replayed; seconds per sweep and the achieved rate of
    the inversions (8 N_c^3 flops per point, summed over the instances)."""
    import torch

    from paper_0711_0999_amd import configs, fkdmft

    inst = configs.c4_instances(count=args.instances)
    flops = sum(8.0 * (round((2 * d["t_max"] + 30) / d["dt"])) ** 3 * d["n_eps"] * d["n_ebar"]
                for d in inst)
    with fkdmft.Batch(inst) as b:
        t0 = time.perf_counter()
        b.iterate(max(args.warmup, 1), tol=0.0, use_graph=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        log(f"bench: warm-up sweep(s) incl. plan and graph recording {t1 - t0:.1f} s")
        b.iterate(args.steps, tol=0.0, use_graph=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        tm = b.timings()
    sec = (t2 - t1) / args.steps
    achieved = flops / sec / 1e12
    n_cs = sorted({int(round((2 * d["t_max"] + 30) / d["dt"])) for d in inst})
    print(json.dumps({
        "metric": "sec per multi-instance sweep (C4)", "value": sec, "unit": "s/sweep",
        "n_gpus": 1, "steps": args.steps, "warmup": max(args.warmup, 1),
        "ms_per_step": sec * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": f"C4: {len(inst)} instances, N_c in {n_cs}, "
                               "n x n points, n = 35..55", "parallelism": "1 GPU"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": None, "kernel": "whole sweep (inversions, 8 N_c^3 per point)"},
        "graph": {"captures": tm["captures"], "capture_ms": tm["capture_ms"]},
    }), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--U", type=float, default=1.0)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c4", "long"])
    ap.add_argument("--instances", type=int, default=32)
    ap.add_argument("--mixed", action="store_true")
    ap.add_argument("--converge", action="store_true")
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-converge", action="store_true")
    ap.add_argument("--tune-bytes", type=float, default=0.0,
                    help="autotuner byte budget (default 48 GiB, 96 GiB for the long contour)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only; --gpus {args.gpus} is not "
              "supported (sharding the k-points across GPUs is not implemented).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0711_0999_amd import configs, fkdmft

    torch.cuda.set_device(0)
    if args.workload == "c4":
        sweep_bench(args)
        return
    stream = torch.cuda.current_stream()
    w = {"c2": lambda: configs.c2(args.U), "c1": lambda: configs.C1,
         "long": lambda: configs.long_contour(args.U)}[args.workload]()
    if args.workload == "long":
        # the long contour is measured per lattice step and impurity update;
        # the mixed and convergence blocks belong to the N_c = 1800 workload
        args.no_mixed = args.no_converge = True
    if not args.tune_bytes:
        args.tune_bytes = (96 if args.workload == "long" else 48) * 2.0 ** 30
    ctx = fkdmft.Context(stream=stream, **w.kwargs())
    tuning = None
    if args.batch:
        ctx.set_batch(args.batch)
    elif not args.no_autotune:
        t0 = time.perf_counter()
        tuning = ctx.autotune(max_bytes=args.tune_bytes)
        tuning["seconds"] = time.perf_counter() - t0
        log(f"bench: autotune picked {tuning}")
    n, npts = ctx.n_c, w.n_eps * w.n_ebar
    prec = fkdmft.FK_MIXED if args.mixed else fkdmft.FK_FP64
    log(f"bench: workload {w.name} N_c={n} points={npts} steps={args.steps} "
        f"warmup={args.warmup}")

    def step():
        ctx.compute_gloc(prec)
        tm = ctx.timings()
        ctx.impurity_update()
        return tm

    for i in range(args.warmup):
        step()
        log(f"bench: warmup {i + 1}/{args.warmup} done")
    ctx.set_kernel_clock(True)      # HIP events around every trailing update
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ms, launches, inv_ms = 0.0, 0, 0.0
    for i in range(args.steps):
        tm = step()
        step_ms += tm["step_kernels_ms"]
        launches += tm["launches"]
        inv_ms += tm["invert_ms"]
        log(f"bench: step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = (t1 - t0) / args.steps
    kc = ctx.kernel_clock()
    ctx.set_kernel_clock(False)
    tm_last = ctx.timings()
    tm_last["impurity_ms"] = ctx.timings()["impurity_ms"]

    # algorithmic flops of one complex inversion: 8 N^3 real flops (the
    # textbook 2 N^3 of a real inversion, four real products per complex one)
    flops_iter = 8.0 * n ** 3 * npts
    inversion_tflops = flops_iter * args.steps / (step_ms * 1e-3) / 1e12
    # dominant kernel: the trailing update of each outer block, timed per launch;
    # its algorithmic flops count 8 real flops per complex multiply-add, while
    # the kernel forms each complex product from three real ones, so its matrix
    # cores execute 3/4 of that count ("mfma_frac")
    achieved = kc["flop"] / (kc["ms"] * 1e-3) / 1e12
    peak = PEAK_FP32_TFLOPS if args.mixed else PEAK_FP64_TFLOPS
    tuned = ctx.get_tuning()
    kname = (f"fk::k_update<{'float' if args.mixed else 'double'}, "
             f"{2 if tuned['tile_rows'] == 64 else 4}>")
    traffic = (PROFILED_TRAFFIC["bytes_per_launch"]
               if (kname == PROFILED_TRAFFIC["kernel"] and w.name.startswith("C2")
                   and tuned["batch"] == PROFILED_TRAFFIC["batch"]) else None)
    out = {
        "metric": ("sec/DMFT iteration at N_c=1800, FP64 vs mixed @1e-8; iters to converge"
                   if args.workload == "c2" else f"sec/DMFT iteration at N_c={n}"),
        "value": sec,
        "unit": "s/iteration",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64" if args.mixed else "c128",
        "data": "synthetic (physical parameters of the workload; Sigma from the iteration)",
        "config": {"workload": f"{w.name}: N_c={n}, {w.n_eps}x{w.n_ebar} GH points, "
                               f"U={w.U}, E={w.E}, beta={w.beta}",
                   "n_c": n, "points": npts, "precision": "mixed" if args.mixed else "fp64",
                   "parallelism": "1 GPU"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                     "kernel": kname,
                     "launches": kc["launches"],
                     "flops_per_launch": kc["flop"] / max(kc["launches"], 1),
                     "avg_launch_ms": kc["ms"] / max(kc["launches"], 1),
                     "mfma_flops_per_launch": 0.75 * kc["flop"] / max(kc["launches"], 1),
                     "mfma_frac": 0.75 * achieved / peak,
                     "whole_inversion_tflops": inversion_tflops,
                     "whole_inversion_frac": inversion_tflops / peak},
        "phases_ms_last_step": {k: round(v, 3) for k, v in tm_last.items()},
        "tuning": tuning if tuning is not None else ctx.get_tuning(),
    }
    if not args.no_mixed and not args.mixed:
        # mixed forms on the same Sigma: complex64 inversion + two or one FP64
        # refinement steps, and complex64 alone (the low-precision phase of
        # the switching loop); error vs the FP64 step from that Sigma
        sig_fixed = ctx.get_sigma()
        ctx.compute_gloc(fkdmft.FK_FP64)
        g64 = ctx.get_gloc()
        j64 = ctx.get_current()[1]
        mixed = {}
        for ir in (2, 1, 0):
            ctx.set_sigma(sig_fixed)
            ctx.set_refinement(ir)
            ctx.compute_gloc(fkdmft.FK_MIXED)      # allocation + warmup
            torch.cuda.synchronize()
            ta = time.perf_counter()
            resid = ctx.compute_gloc(fkdmft.FK_MIXED)
            tmm = ctx.timings()
            ctx.impurity_update()
            torch.cuda.synchronize()
            tb = time.perf_counter()
            g = ctx.get_gloc()
            j = ctx.get_current()[1]
            mixed[f"ir{ir}"] = {
                "sec_per_iter": tb - ta,
                "gloc_max_rel_err_vs_fp64": float(np.max(np.abs(g - g64)) / np.max(np.abs(g64))),
                "current_max_rel_err_vs_fp64": float(np.max(np.abs(j - j64)) / np.max(np.abs(j64))),
                "refine_residual": resid,
                "phases_ms": {k: round(v, 3) for k, v in tmm.items()},
                "fp32_inversion_tflops": 8.0 * n ** 3 * npts / (tmm["step_kernels_ms"] * 1e-3) / 1e12,
            }
            log(f"bench: mixed ir={ir} done")
        out["mixed"] = mixed
    # iterations to delta < 1e-8 from Sigma = 0, FP64 and the precision-switching
    # mixed loop.  The default run uses the same contour with 15 x 15 points
    # (the iteration count is a property of the contour and the model; the
    # quadrature order changes it little); --converge runs the full grid.
    conv_kw = dict(w.kwargs())
    if not args.converge:
        conv_kw.update(n_eps=15, n_ebar=15)
    if not args.no_converge:
        conv = {"points": conv_kw["n_eps"] * conv_kw["n_ebar"], "tol": configs.C2_TOL}
        for name, p2 in (("fp64", fkdmft.FK_FP64), ("mixed_switch", fkdmft.FK_MIXED)):
            ctx2 = fkdmft.Context(stream=stream, **conv_kw)
            if args.converge:
                t_now = ctx.get_tuning()
                ctx2.set_tuning(tile_rows=t_now["tile_rows"], batch=t_now["batch"],
                                lookahead=t_now["lookahead"])
            ctx2.set_refinement(0)
            ctx2.compute_gloc(fkdmft.FK_FP64)     # allocations outside the timing
            ctx2.compute_gloc(fkdmft.FK_MIXED)
            ctx2.set_sigma(np.zeros((ctx2.n_c, ctx2.n_c), np.complex128))
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            r = ctx2.iterate(200, tol=configs.C2_TOL, precision=p2)
            torch.cuda.synchronize()
            dt2 = time.perf_counter() - t2
            conv[name] = {"iters": r["iters"], "complex64_iters": ctx2.low_iterations(),
                          "delta": r["delta"],
                          "converged": r["converged"], "seconds": dt2,
                          "sec_per_iter": dt2 / max(r["iters"], 1)}
            log(f"bench: converge {name}: {r['iters']} iterations in {dt2:.1f} s")
            ctx2.close()
        out["converge"] = conv
    if not args.no_cpu_baseline:
        log("bench: timing the oracle on a sample")
        # a sample of about 10-30 s of host work: 48 points at N_c = 1800,
        # proportionally fewer for larger matrices
        out["cpu_baseline"] = cpu_baseline(w, n_sample=max(2, int(48 * (1800.0 / n) ** 3)))
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
