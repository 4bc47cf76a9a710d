"""Benchmark: seconds per DMFT iteration of the nonequilibrium Falicov-Kimball
lattice step at N_c = 1800 (t in [-10, 30], dt = dtau = 0.05, beta = 10,
55 x 55 Gauss-Hermite points, E = 1) on one MI355X.

A step is one DMFT iteration: the lattice step over all 3025 points (build,
batched inversion, rho-weighted reduction, current) plus the impurity update.
Inputs are the physical parameters only (synthetic, resident on the device).

python bench.py [--gpus 1] [--steps K] [--warmup W] [--U 1.0]
                [--mixed] [--converge | --no-converge] [--no-cpu-baseline]
                [--workload c2|c1|long|c4|c2-converge]
Prints ONE JSON line.

--workload c2-converge [--Us 0.5 1 1.5 2] [--forms fp64 switch warm]
    [--weights W.npz]: the headline loop on the full C2 grid, to
    delta < 1e-8 from Sigma = 0 (fp64: plain FP64; switch: complex64 steps
    then FP64), and from the network's judged proposal on the converged Sigma
    of E - 0.25 (warm: the switching loop started there); seconds, iterations
    and the fraction of the matrix-core peak.
--workload c4 [--tol 1e-8] [--max-sweeps 80]: the 32-instance uneven sweep
    (hipGraph replay) to convergence with retirement.
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

# HBM bytes per launch of the dominant kernel (the trailing update,
# fk::k_update<double, 2>, 757-matrix batches of the C2 workload), from the
# rocprofv3 FETCH_SIZE and WRITE_SIZE runs summarized under profiles/, each
# scaled by the same counter's reading for a plain 256 MiB copy.  Reported only
# for that kernel, batch size and schedule (groups of four outer blocks, K up
# to 512); None until the counters have been taken on the current kernel.
# Measured: FETCH_SIZE 69358020 KiB x 2.00 + WRITE_SIZE 26671992 KiB x 1.00
# per launch.
PROFILED_TRAFFIC = {"kernel": "fk::k_update<double, 2>", "batch": 757,
                    "bytes_per_launch": (2.00 * 69358019.7 + 1.00 * 26671992.2) * 1024}

# Each complex product of the trailing update is formed from three real ones
# (Gauss), so its matrix cores execute 6 of the 8 real flops per complex
# multiply-add that the algorithmic count credits.
EXECUTED_PER_ALGORITHMIC = 0.75


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
    the inversions (8 N_c^3 flops per point, summed over the instances).
    With --tol > 0: every instance from Sigma = 0 until its delta falls below
    tol (then it retires and the graph is re-recorded), at most --max-sweeps."""
    import torch

    from paper_0711_0999_amd import configs, fkdmft

    inst = configs.c4_instances(count=args.instances)
    n_cs_of = [int(round((2 * d["t_max"] + 30) / d["dt"])) for d in inst]
    per_iter = [8.0 * nc ** 3 * d["n_eps"] * d["n_ebar"] for nc, d in zip(n_cs_of, inst)]
    flops = sum(per_iter)
    if args.tol > 0:
        with fkdmft.Batch(inst) as b:
            tune = None
            if args.batch_autotune:
                t0 = time.perf_counter()
                for nc in sorted(set(n_cs_of)):      # one size class per call
                    tune = b.autotune(max_bytes=args.tune_bytes or 48 * 2.0 ** 30,
                                      only_nc=nc)
                    log(f"bench: autotuned N_c = {nc} "
                        f"({time.perf_counter() - t0:.1f} s): "
                        f"{[t for t in tune if t['n_c'] == nc][0]}")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            # one sweep per call (the batch keeps its state, retires converged
            # instances and re-records the graph when the active set changes),
            # so progress shows and a time budget can end the run early
            sweeps = 0
            while sweeps < args.max_sweeps:
                r = b.iterate(1, tol=args.tol, use_graph=True)
                if r["sweeps"] == 0:
                    break
                sweeps += 1
                done = [bool(d < args.tol) for d in r["deltas"]]
                el = time.perf_counter() - t0
                log(f"bench: sweep {sweeps}: {sum(done)}/{len(done)} converged, "
                    f"{el:.0f} s, last {b.timings()['last_sweep_ms']:.0f} ms")
                if all(done) or el > args.time_budget:
                    break
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            tm = b.timings()
            r["sweeps"] = sweeps
        iters = [int(v) for v in r["iters"]]
        done = [bool(d < args.tol) for d in r["deltas"]]
        alg = sum(i * f for i, f in zip(iters, per_iter))
        achieved = alg / sec / 1e12
        print(json.dumps({
            "metric": f"seconds to delta < {args.tol:g} for every instance of the C4 sweep",
            "value": sec, "unit": "s", "n_gpus": 1, "steps": r["sweeps"], "warmup": 0,
            "ms_per_step": sec * 1e3 / max(r["sweeps"], 1), "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
            "config": {"workload": f"C4: {len(inst)} instances (rng 0), N_c in "
                                   f"{sorted(set(n_cs_of))}, n x n points, n = 35..55, "
                                   "from Sigma = 0, retirement, hipGraph replay",
                       "parallelism": "1 GPU"},
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                         "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                         "traffic": None,
                         "kernel": "whole sweeps (lattice inversions, 8 N_c^3 per point; "
                                   "impurity updates and reductions in the time only)"},
            "instances": [dict(U=d["U"], E=d["E"], dt=d["dt"], t_max=d["t_max"], n_c=nc,
                               n=d["n_eps"], iters=i, converged=c, delta=float(dl))
                          for d, nc, i, c, dl in zip(inst, n_cs_of, iters, done, r["deltas"])],
            "converged": sum(done), "sweeps": r["sweeps"],
            "stopped_by": ("all converged" if all(done) else
                           "time budget" if sec > args.time_budget else "sweep cap"),
            "graph": {"captures": tm["captures"], "capture_ms": tm["capture_ms"]},
            "tuning": tune if args.batch_autotune else None,
        }), flush=True)
        return
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


def converge_bench(args):
    """The headline loops on the full C2 grid (55 x 55 points, N_c = 1800) for
    each U: from Sigma = 0 to delta < 1e-8 in FP64 ("fp64") and with the
    precision switch (complex64 steps, then FP64: "switch"), and ("warm", needs
    --weights) from the network's judged proposal on the converged Sigma at
    E - 0.25 in the switching loop, beside the same loop from that previous
    field alone.  Fraction of the matrix-core peak: the time the run's lattice
    steps would take at peak (8 N_c^3 per point: FP64 steps at the FP64 peak,
    complex64 steps at the FP32 peak) over the measured time."""
    import numpy as np
    import torch

    from paper_0711_0999_amd import configs, fkdmft

    stream = torch.cuda.current_stream()
    runs = []
    tol = configs.C2_TOL
    for U in args.Us:
        w = configs.c2(U)
        n = 1800
        F = 8.0 * n ** 3 * w.n_eps * w.n_ebar

        def frac_of(n64, n32, sec):
            ideal = n64 * F / (PEAK_FP64_TFLOPS * 1e12) + n32 * F / (PEAK_FP32_TFLOPS * 1e12)
            return ideal / sec

        def make(E=w.E):
            c = fkdmft.Context(stream=stream, **dict(w.kwargs(), E=E))
            c.set_tuning(tile_rows=64, batch=args.batch or 757, lookahead=0)
            c.set_refinement(0)
            c.compute_gloc(fkdmft.FK_FP64)       # allocations outside the timing
            c.compute_gloc(fkdmft.FK_MIXED)
            c.set_sigma(np.zeros((c.n_c, c.n_c), np.complex128))
            return c

        def timed_loop(c, prec, judged_fallback=None):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if judged_fallback is None:
                r = c.iterate(200, tol=tol, precision=prec)
            else:
                r = c.iterate_judged(judged_fallback, 200, tol=tol, accept=0.5,
                                     precision=prec)
            torch.cuda.synchronize()
            return r, time.perf_counter() - t0

        for form in args.forms:
            if form in ("fp64", "switch"):
                c = make()
                prec = fkdmft.FK_FP64 if form == "fp64" else fkdmft.FK_MIXED
                r, sec = timed_loop(c, prec)
                n32 = c.low_iterations()
                rec = dict(U=U, form=form, start="zero", iters=r["iters"], complex64_iters=n32,
                           seconds=sec, sec_per_iter=sec / max(r["iters"], 1),
                           converged=r["converged"], delta=r["delta"],
                           frac_of_peak=frac_of(r["iters"] - n32, n32, sec))
                c.close()
            else:
                from paper_0711_0999_amd import warmstart
                ws = warmstart.WarmStart.load(args.weights)
                cont = warmstart.EVAL_CONTOUR
                c0 = make(E=w.E - warmstart.FIELD_STEP)
                r0, sec0 = timed_loop(c0, fkdmft.FK_MIXED)
                log(f"bench: U={U} previous field E={w.E - warmstart.FIELD_STEP}: "
                    f"{r0['iters']} iterations in {sec0:.1f} s")
                prev = torch.empty((c0.n_c, c0.n_c), dtype=torch.complex128, device="cuda")
                c0.get_sigma(prev)
                c0.close()
                c = make()
                c.set_sigma(prev)
                rp, secp = timed_loop(c, fkdmft.FK_MIXED)
                n32p = c.low_iterations()
                c.close()
                log(f"bench: U={U} from the previous field: {rp['iters']} iterations "
                    f"in {secp:.1f} s")
                c = make()
                prop_s = ws.propose(c, cont, prev, U, w.E)     # timed inside
                r, sec = timed_loop(c, fkdmft.FK_MIXED, judged_fallback=prev)
                sec += prop_s                  # the proposal counts in the start's time
                n32 = c.low_iterations()
                rec = dict(U=U, form="warm", start="network (judged), switching loop",
                           iters=r["iters"], complex64_iters=n32, seconds=sec,
                           propose_s=prop_s, outcome=r["outcome"],
                           sec_per_iter=sec / max(r["iters"], 1),
                           converged=r["converged"], delta=r["delta"],
                           frac_of_peak=frac_of(r["iters"] - n32, n32, sec),
                           previous_field=dict(iters=rp["iters"], complex64_iters=n32p,
                                               seconds=secp, converged=rp["converged"]),
                           previous_field_solve=dict(E=w.E - warmstart.FIELD_STEP,
                                                     iters=r0["iters"], seconds=sec0))
                c.close()
            runs.append(rec)
            log(f"bench: U={U} {form}: {rec['iters']} iterations in {rec['seconds']:.1f} s "
                f"({rec['complex64_iters']} complex64), frac {rec['frac_of_peak']:.3f}")
    print(json.dumps({
        "metric": "sec/DMFT iteration at N_c=1800, FP64 vs mixed @1e-8; iters to converge",
        "value": None, "unit": "s", "n_gpus": 1, "steps": 0, "warmup": 0,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128/c64", "data": "synthetic",
        "config": {"workload": "C2 full grid: N_c=1800, 55x55 GH points, E=1, beta=10, "
                               f"tol {tol:g}, U in {list(args.Us)}", "parallelism": "1 GPU"},
        "runs": runs}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--U", type=float, default=1.0)
    ap.add_argument("--workload", default="c2",
                    choices=["c1", "c2", "c4", "long", "c2-converge"])
    ap.add_argument("--Us", type=float, nargs="+", default=[0.5, 1.0, 1.5, 2.0])
    ap.add_argument("--forms", nargs="+", default=["fp64", "switch"],
                    choices=["fp64", "switch", "warm"])
    ap.add_argument("--weights", default="")
    ap.add_argument("--tol", type=float, default=0.0)
    ap.add_argument("--max-sweeps", type=int, default=80)
    ap.add_argument("--time-budget", type=float, default=900.0,
                    help="c4 with --tol: stop starting sweeps after this many seconds")
    ap.add_argument("--batch-autotune", action="store_true")
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
    if args.workload == "c2-converge":
        converge_bench(args)
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
    # dominant kernel: the trailing update of each group of outer blocks,
    # timed per launch.  Primary rate: the flops its matrix cores execute
    # (three real products per complex one, 6 real flops per complex
    # multiply-add), which the peak bounds; beside it the algorithmic rate (8
    # per complex multiply-add), which exceeds the peak once the kernel passes
    # 3/4 of it
    if kc["ms"] <= 0 or kc["launches"] == 0:
        raise RuntimeError("the kernel clock recorded no trailing-update launch")
    alg_tflops = kc["flop"] / (kc["ms"] * 1e-3) / 1e12
    achieved = EXECUTED_PER_ALGORITHMIC * alg_tflops
    peak = PEAK_FP32_TFLOPS if args.mixed else PEAK_FP64_TFLOPS
    tuned = ctx.get_tuning()
    kname = (f"fk::k_update<{'float' if args.mixed else 'double'}, "
             f"{2 if tuned['tile_rows'] == 64 else 4}>")
    traffic = (PROFILED_TRAFFIC["bytes_per_launch"]
               if (PROFILED_TRAFFIC and kname == PROFILED_TRAFFIC["kernel"]
                   and w.name.startswith("C2")
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
                     "flops_counted": "executed matrix-core flops (3 real products "
                                      "per complex product)",
                     "launches": kc["launches"],
                     "executed_flops_per_launch":
                         EXECUTED_PER_ALGORITHMIC * kc["flop"] / max(kc["launches"], 1),
                     "algorithmic_flops_per_launch": kc["flop"] / max(kc["launches"], 1),
                     "avg_launch_ms": kc["ms"] / max(kc["launches"], 1),
                     "algorithmic_tflops": alg_tflops,
                     "algorithmic_frac": alg_tflops / peak,
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
        conv = {"grid": f"{conv_kw['n_eps']}x{conv_kw['n_ebar']} points on the C2 contour"
                        + ("" if args.converge else
                           " (reduced grid; full-grid runs: --workload c2-converge)"),
                "points": conv_kw["n_eps"] * conv_kw["n_ebar"], "tol": configs.C2_TOL}
        out["config"]["converge_block_grid"] = conv["grid"]
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
