"""Learned warm start of the self-consistency loop.

A tanh network (4 layers, width 512) proposes the self-energy at a new field E
from the converged one at the previous field E - dE: evaluated pointwise on the
contour pairs (t_i, t_j), it predicts the change Sigma_E - Sigma_{E-dE} from
(U, E, dt), the rank-32 randomized singular values of the previous Sigma and the
pair's own coordinates and previous value.  Being pointwise in (t_i, t_j) it
applies to any step size: trained on N_c = 600 contours, used on N_c = 1800.
The plain iteration judges the proposal (fk_iterate_judged) and falls back to the
previous-field start when it is not better.

Everything computed here is a library call (fk_ws_*, fk_mlp_*, the loop); this
module only arranges device buffers (torch) and host bookkeeping.
"""
import time

import numpy as np

from . import fkdmft

RANK = 32
N_GLOB = 3 + RANK
D_IN = 96                     # >= N_GLOB + fk_ws_features' 60 pair features
WIDTH = 512
DEPTH = 4
D_OUT = 2
OMEGA_SEED = 711_0999
FIELD_STEP = 0.25


def omega(n_c, rank=RANK):
    """The fixed Gaussian test matrix of the range sketch for an N_c contour."""
    return np.random.default_rng(OMEGA_SEED + n_c).standard_normal((n_c, rank))


def sigma_scale(u):
    """Scale that brings Sigma to O(1) across U: Sigma grows like U^2/4 at
    small U (second order in U at half filling)."""
    return 1.0 / (0.25 * u * u + 0.01)


# The previous Sigma enters the feature rows as PREV_GAIN * sigma_scale(U) *
# Sigma_prev: sigma_scale brings it to O(0.1-1) across U, the gain to O(1).
PREV_GAIN = 4.0


def contour_length(cont):
    return 2.0 * (cont["t_max"] - cont["t_min"]) + cont["beta"]


def glob_features(ctx, cont, sigma_prev, u, e):
    """(U, E, dt) and the 32 randomized singular values of the weighted previous
    Sigma, each brought to O(1) (singular values by the contour length, the
    largest value a uniform kernel can have, and by the U scale)."""
    sv = ctx.ws_sketch(sigma_prev, omega(ctx.n_c))
    s = sigma_scale(u)
    g = np.concatenate([[u / 2.5, e / 4.0, cont["dt"] / 0.2],
                        s * sv / contour_length(cont)])
    return g.astype(np.float32)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the warm start needs a GPU (HIP device)")
    return torch


class WarmStart:
    """The network and the target normalization it was trained with."""

    def __init__(self, params=None, t_rms=1.0, seed=0):
        _torch()                      # torch's device first, then the library's
        self.net = fkdmft.MLP(D_IN, WIDTH, DEPTH, D_OUT, params=params, seed=seed)
        self.t_rms = float(t_rms)

    def save(self, path):
        np.savez(path, params=self.net.get_params(), t_rms=self.t_rms,
                 dims=np.array([D_IN, WIDTH, DEPTH, D_OUT, RANK]))

    @classmethod
    def load(cls, path):
        f = np.load(path, allow_pickle=False)
        assert list(f["dims"]) == [D_IN, WIDTH, DEPTH, D_OUT, RANK]
        return cls(params=f["params"], t_rms=float(f["t_rms"]))

    def propose(self, ctx, cont, sigma_prev, u, e, bf16=True, keep_pre_field=False):
        """Sets ctx's Sigma to the proposed start; returns the time it took (s).
        keep_pre_field: pairs of contour points before the field is switched on
        keep the previous field's values (the network's change applies after)."""
        torch = _torch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = ctx.n_c
        g = glob_features(ctx, cont, sigma_prev, u, e)
        x = torch.empty((n * n, D_IN), dtype=torch.float32, device="cuda")
        ctx.ws_features(sigma_prev, g, None, n * n, PREV_GAIN * sigma_scale(u), x, D_IN)
        y = self.net.forward(x, bf16=bf16)
        ctx.ws_apply(sigma_prev, y, sigma_scale(u) / self.t_rms, keep_pre_field)
        torch.cuda.synchronize()
        return time.perf_counter() - t0


def field_sweep_data(cont, us, es, n_eps, n_ebar, tol, rows_per_run, seed=0,
                     max_iter=80, log=None, u_rows=None):
    """Converged Sigma along field sweeps E = es[0], es[1], ... for every U
    (each field started from the previous one's Sigma, the first from zero),
    all U of one field solved together in one fk_batch.  Returns device tensors
    x (pairs * rows_per_run x D_IN) and t (x 2, targets scaled by sigma_scale),
    the pair rows sampled uniformly per (E - dE -> E) pair of converged runs,
    and per-field stats.  A run that does not reach tol in max_iter iterations
    contributes no pair (its sweep continues from its last iterate)."""
    torch = _torch()
    rng = np.random.default_rng(seed)
    n_runs = len(us) * (len(es) - 1)
    x = torch.empty((n_runs * rows_per_run, D_IN), dtype=torch.float32, device="cuda")
    t = torch.empty((n_runs * rows_per_run, D_OUT), dtype=torch.float32, device="cuda")
    prev = None
    prev_ok = [False] * len(us)
    stats = []
    row = 0
    for k, e in enumerate(es):
        inst = [dict(cont, U=float(u), E=float(e), n_eps=n_eps, n_ebar=n_ebar) for u in us]
        t0 = time.perf_counter()
        with fkdmft.Batch(inst) as b:
            n = b.instance(0).n_c
            if prev is not None:
                for i in range(len(us)):
                    b.instance(i).set_sigma(prev[i])
            r = b.iterate(max_iter, tol=tol, use_graph=True)
            ok = [bool(d < tol) for d in r["deltas"]]
            new = []
            for i in range(len(us)):
                s_new = torch.empty((n, n), dtype=torch.complex128, device="cuda")
                b.instance(i).get_sigma(s_new)
                new.append(s_new)
            if prev is not None:
                for i, u in enumerate(us):
                    if not (ok[i] and prev_ok[i]):
                        continue
                    c = b.instance(i)
                    g = glob_features(c, cont, prev[i], u, e)
                    idx = torch.from_numpy(
                        rng.integers(0, n * n, rows_per_run).astype(np.int64)).cuda()
                    xs = x[row:row + rows_per_run]
                    ts = t[row:row + rows_per_run]
                    c.ws_features(prev[i], g, idx, rows_per_run, PREV_GAIN * sigma_scale(u),
                                  xs, D_IN)
                    c.ws_targets(prev[i], new[i], idx, rows_per_run, sigma_scale(u), ts)
                    row += rows_per_run
                    if u_rows is not None:
                        u_rows.append(np.full(rows_per_run, u, dtype=np.float32))
        dt_s = time.perf_counter() - t0
        stats.append(dict(E=float(e), iters=[int(v) for v in r["iters"]],
                          converged=ok, seconds=dt_s))
        if log:
            log(f"field E={e:.3f}: iterations {list(r['iters'])} converged "
                f"{sum(ok)}/{len(ok)} in {dt_s:.1f} s")
        prev = new
        prev_ok = ok
    return x[:row], t[:row], stats


def target_stats(t, u_of_row=None):
    """Percentiles of |t| and, per U range, the RMS of the targets (a host
    summary of the training set)."""
    th = np.abs(t.astype(np.float64)).ravel()
    out = dict(p50=float(np.percentile(th, 50)), p90=float(np.percentile(th, 90)),
               p99=float(np.percentile(th, 99)), p999=float(np.percentile(th, 99.9)),
               max=float(th.max()), rms=float(np.sqrt(np.mean(th ** 2))))
    if u_of_row is not None:
        for lo, hi in ((0.0, 0.75), (0.75, 1.5), (1.5, 2.0), (2.0, 3.0)):
            m = (u_of_row >= lo) & (u_of_row < hi)
            if m.any():
                out[f"rms_U{lo}-{hi}"] = float(np.sqrt(np.mean(t[m].astype(np.float64) ** 2)))
    return out


def train(x, t, steps=(12000, 8000, 4000), lrs=(3e-4, 1e-4, 3e-5), batch=4096,
          seed=0, log=None, clip=8.0):
    """Adam on the sampled pairs (minibatches drawn by the library).  The
    targets are scaled by a robust size (the RMS of those within 20 times the
    median magnitude) and clipped at +-clip of it (host arithmetic on a copy):
    a few pairs with changes far beyond the typical one (the largest U near
    field resonances) otherwise dominate the squared loss."""
    torch = _torch()
    th = t.cpu().numpy().astype(np.float64)
    a = np.abs(th)
    core = a[a <= 20.0 * np.median(a) + 1e-30]
    t_rms = float(np.sqrt(np.mean(core ** 2)))
    tn = torch.from_numpy(np.clip(th / t_rms, -clip, clip).astype(np.float32)).cuda()
    if log:
        log(f"targets: scale {t_rms:.4g}, clipped rows {np.mean(np.abs(th / t_rms) > clip):.2e}")
    ws = WarmStart(t_rms=t_rms, seed=seed)
    hist = []
    for k, (n, lr) in enumerate(zip(steps, lrs)):
        for c0 in range(0, n, 2500):      # chunks, so progress is visible
            h = ws.net.train(x, tn, batch, min(2500, n - c0), lr,
                             seed=seed * 1000 + k * 100 + c0 // 2500)
            hist.append(h)
            if log:
                log(f"train phase {k} (lr {lr:g}) steps {c0}..{c0 + len(h)}: "
                    f"loss {np.mean(h[:50]):.4f} -> {np.mean(h[-50:]):.4f}")
    return ws, np.concatenate(hist)


def _error_regions(ctx, cont, prev, start, fixed):
    """Max error of the previous-field and network starts by region of the
    pair plane: branch pair, and within the real branches whether the pair is
    within two indices of the diagonal, before the field (max(t_i, t_j) <= 0)
    or at the turning point (both within 1 of t_max)."""
    n, nt = ctx.n_c, ctx.n_t
    br = np.array([0] * nt + [1] * nt + [2] * (n - 2 * nt))
    z, _ = ctx.contour_points()
    t = np.where(br < 2, z.real, cont["t_min"])
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ep = np.abs(prev - fixed)
    en = np.abs(start - fixed)
    regions = {}
    names = "ULM"
    for a in range(3):
        for b in range(3):
            m = (br[ii] == a) & (br[jj] == b)
            regions[names[a] + names[b]] = m
    regions["near_diag"] = np.abs(ii - jj) <= 2
    regions["pre_field"] = np.maximum(t[ii], t[jj]) <= 0
    regions["turning"] = (t[ii] > cont["t_max"] - 1) & (t[jj] > cont["t_max"] - 1)
    return {k: [float(ep[m].max()) if m.any() else 0.0,
                float(en[m].max()) if m.any() else 0.0] for k, m in regions.items()}


def compare_starts(ws, cont, u, e, n_eps, n_ebar, tol, max_iter=200, accept=0.5,
                   mixed=True, log=None, also_accept=(),
                   starts=("zero", "equilibrium", "previous", "network", "network_mixed")):
    """Iterations to tol at (U, E) from Sigma = 0, from the equilibrium Sigma
    (E = 0, same contour), from the converged Sigma of E - dE (previous field)
    and from the network's proposal on it (judged, with the previous field as
    fallback), all in FP64, and the network's start in the mixed-precision
    loop.  Also reports the distance of both warm starts
    from the fixed point (max and RMS over pairs) and checks that every run
    reaches the same fixed point."""
    torch = _torch()
    out = dict(U=u, E=e, tol=tol)
    with fkdmft.Context(**cont, U=u, E=e - FIELD_STEP, n_eps=n_eps, n_ebar=n_ebar) as c:
        r = c.iterate(max_iter, tol=tol)
        prev = torch.empty((c.n_c, c.n_c), dtype=torch.complex128, device="cuda")
        c.get_sigma(prev)
        out["prev_field_iters"] = r["iters"]
        out["n_c"] = c.n_c
    # the paper's usual guess: the equilibrium self-energy (E = 0 on the same
    # contour), independent of the field
    if "equilibrium" in starts:
        with fkdmft.Context(**cont, U=u, E=0.0, n_eps=n_eps, n_ebar=n_ebar) as c:
            r = c.iterate(max_iter, tol=tol)
            equil = torch.empty((c.n_c, c.n_c), dtype=torch.complex128, device="cuda")
            c.get_sigma(equil)
            out["equilibrium_solve_iters"] = r["iters"]
    glocs = {}
    starts = ([s for s in starts if s != "network_mixed" or mixed]
              + [f"network_accept{a:g}" for a in also_accept]
              + ([f"network_keep_accept{a:g}" for a in also_accept]
                 if "network_keep" in starts else []))
    assert starts[0] == "zero", "the Sigma = 0 run defines the fixed point"
    fixed = None
    for start in starts:
        with fkdmft.Context(**cont, U=u, E=e, n_eps=n_eps, n_ebar=n_ebar) as c:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if start == "zero":
                r = c.iterate(max_iter, tol=tol)
            elif start == "previous":
                c.set_sigma(prev)
                r = c.iterate(max_iter, tol=tol)
            elif start == "equilibrium":
                c.set_sigma(equil)
                r = c.iterate(max_iter, tol=tol)
            else:
                keep = start.startswith("network_keep")
                out[f"{start}_propose_s"] = ws.propose(c, cont, prev, u, e,
                                                       keep_pre_field=keep)
                if fixed is not None and start == "network_keep":
                    s0 = c.get_sigma()
                    out["start_err_keep"] = [float(np.max(np.abs(s0 - fixed))),
                                             float(np.sqrt(np.mean(np.abs(s0 - fixed) ** 2)))]
                if fixed is not None and start == "network":
                    s0 = c.get_sigma()
                    p0 = prev.cpu().numpy()
                    out["start_err_previous"] = [float(np.max(np.abs(p0 - fixed))),
                                                 float(np.sqrt(np.mean(np.abs(p0 - fixed) ** 2)))]
                    out["start_err_network"] = [float(np.max(np.abs(s0 - fixed))),
                                                float(np.sqrt(np.mean(np.abs(s0 - fixed) ** 2)))]
                    out["start_err_regions"] = _error_regions(c, cont, p0, s0, fixed)
                prec = fkdmft.FK_MIXED if start == "network_mixed" else fkdmft.FK_FP64
                acc = accept
                if "_accept" in start:
                    acc = float(start[start.index("_accept") + len("_accept"):])
                r = c.iterate_judged(prev, max_iter, tol=tol, accept=acc, precision=prec)
                out[f"{start}_outcome"] = r["outcome"]
            torch.cuda.synchronize()
            out[f"{start}_iters"] = r["iters"]
            out[f"{start}_s"] = time.perf_counter() - t0
            out[f"{start}_converged"] = bool(r["converged"])
            glocs[start] = c.get_gloc()
            if start == "zero":
                fixed = c.get_sigma()
    ref = glocs["zero"]
    out["gloc_spread"] = max(float(np.max(np.abs(g - ref))) for g in glocs.values())
    if log:
        log(f"U={u:.3f} E={e:.3f} N_c={out['n_c']}: iterations zero {out['zero_iters']}, "
            f"equilibrium {out.get('equilibrium_iters')}, "
            f"previous {out.get('previous_iters')}, network {out.get('network_iters')} "
            f"(outcome {out.get('network_outcome')})"
            + (f", network+mixed {out.get('network_mixed_iters')}" if mixed else "")
            + "".join(f", accept {a:g}: {out[f'network_accept{a:g}_iters']}"
                      for a in also_accept)
            + (f", kept pre-field {out['network_keep_iters']} "
               f"(outcome {out['network_keep_outcome']})" if "network_keep" in starts else "")
            + "".join(f", kept pre-field accept {a:g}: {out[f'network_keep_accept{a:g}_iters']}"
                      for a in also_accept if "network_keep" in starts)
            + f"; start error max/rms previous {out.get('start_err_previous')}, "
            f"network {out.get('start_err_network')}; spread {out['gloc_spread']:.1e}")
    return out


# ------------------------------------------------------------------ recipes
# Training contour: t in [-10, 30], beta = 10, dtau = 0.05 with dt = 0.2
# (N_c = 600) for most field sweeps and dt = 0.1 (N_c = 1000) for the rest, so
# that the network sees the step size change; evaluation on dt = 0.05
# (N_c = 1800).
TRAIN_CONTOURS = (dict(t_min=-10.0, t_max=30.0, dt=0.2, dtau=0.05, beta=10.0),
                  dict(t_min=-10.0, t_max=30.0, dt=0.1, dtau=0.05, beta=10.0))
EVAL_CONTOUR = dict(t_min=-10.0, t_max=30.0, dt=0.05, dtau=0.05, beta=10.0)
FIELDS = tuple(0.5 + FIELD_STEP * k for k in range(15))        # 0.5 .. 4.0


def unseen_cases(count, seed=2):
    """Evaluation pairs (U, E): U ~ U[0.25, 2.5], E ~ U[0.75, 4] drawn with
    numpy's default_rng(seed), so they are off the training runs' (U, E) (the
    training U are other draws; E lies between the training fields with
    probability one).  E >= 0.75 leaves room for the previous field E - 0.25."""
    rng = np.random.default_rng(seed)
    return [(float(rng.uniform(0.25, 2.5)), float(rng.uniform(0.75, 4.0)))
            for _ in range(count)]


def _main(argv=None):
    import argparse
    import json
    import os
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train", help="generate field sweeps, train, save")
    tr.add_argument("--out", required=True)
    tr.add_argument("--n-u", type=int, nargs=2, default=[100, 34],
                    help="U values per training contour (dt = 0.2, dt = 0.1)")
    tr.add_argument("--u-range", type=float, nargs=2, default=[0.25, 1.9],
                    help="U range on the dt = 0.2 contour (where its loop converges)")
    tr.add_argument("--u-range-fine", type=float, nargs=2, default=[0.25, 2.5],
                    help="U range on the dt = 0.1 contour")
    tr.add_argument("--gh", type=int, default=10)
    tr.add_argument("--tol", type=float, default=1e-6)
    tr.add_argument("--rows", type=int, default=4096)
    tr.add_argument("--steps", type=int, nargs=3, default=[12000, 8000, 4000])
    tr.add_argument("--lrs", type=float, nargs=3, default=[3e-4, 1e-4, 3e-5])
    tr.add_argument("--batch", type=int, default=4096)
    tr.add_argument("--seed", type=int, default=1)
    ev = sub.add_parser("evaluate", help="compare starts on unseen (U, E)")
    ev.add_argument("--weights", required=True)
    ev.add_argument("--out", required=True)
    ev.add_argument("--cases", type=float, nargs="+", default=None,
                    help="U E pairs (default: --n-cases unseen pairs)")
    ev.add_argument("--n-cases", type=int, default=32)
    ev.add_argument("--first-case", type=int, default=0)
    ev.add_argument("--starts", nargs="+",
                    default=["zero", "equilibrium", "previous", "network", "network_mixed"])
    ev.add_argument("--gh", type=int, default=15)
    ev.add_argument("--tol", type=float, default=1e-8)
    ev.add_argument("--also-accept", type=float, nargs="*", default=[])
    a = ap.parse_args(argv)

    def log(*m):
        print(*m, flush=True)

    if a.cmd == "train":
        torch = _torch()
        rng = np.random.default_rng(a.seed)
        xs, ts, stats, u_rows = [], [], [], []
        t0 = time.perf_counter()
        for cont, n_u, ur in zip(TRAIN_CONTOURS, a.n_u, (a.u_range, a.u_range_fine)):
            us = np.sort(rng.uniform(ur[0], ur[1], n_u))
            log(f"contour dt={cont['dt']}: {n_u} values of U")
            x, t, st = field_sweep_data(cont, list(us), list(FIELDS), a.gh, a.gh, a.tol,
                                        a.rows, seed=int(rng.integers(1 << 31)),
                                        max_iter=100, log=log, u_rows=u_rows)
            xs.append(x)
            ts.append(t)
            stats.append(dict(dt=cont["dt"], U=[float(u) for u in us], fields=st))
        x, t = torch.cat(xs), torch.cat(ts)
        gen_s = time.perf_counter() - t0
        log(f"data: {x.shape[0]} rows in {gen_s:.0f} s")
        tstats = target_stats(t.cpu().numpy(), np.repeat(np.concatenate(u_rows), 2)
                              .reshape(-1, 2) if u_rows else None)
        log(f"target statistics: {tstats}")
        t0 = time.perf_counter()
        ws, hist = train(x, t, steps=tuple(a.steps), lrs=tuple(a.lrs), batch=a.batch,
                         seed=a.seed, log=log)
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        ws.save(a.out)
        runs = sum(len(f["iters"]) for s in stats for f in s["fields"])
        pairs = x.shape[0] // a.rows
        with open(os.path.splitext(a.out)[0] + "_train.json", "w") as f:
            json.dump(dict(runs=runs, pairs=pairs, rows=int(x.shape[0]), gen_s=gen_s,
                           train_s=time.perf_counter() - t0, t_rms=ws.t_rms,
                           loss_first=float(np.mean(hist[:100])),
                           loss_last=float(np.mean(hist[-100:])), gh=a.gh, tol=a.tol,
                           target_stats=tstats, lrs=list(a.lrs), steps=list(a.steps),
                           sweeps=stats), f, indent=1)
        log(f"saved {a.out}: {runs} runs, {pairs} pairs")
    else:
        ws = WarmStart.load(a.weights)
        if a.cases:
            cases = list(zip(a.cases[0::2], a.cases[1::2]))
        else:
            cases = unseen_cases(a.n_cases)[a.first_case:]
        res = []
        for u, e in cases:
            res.append(compare_starts(ws, EVAL_CONTOUR, u, e, a.gh, a.gh, a.tol, log=log,
                                      also_accept=tuple(a.also_accept),
                                      starts=tuple(a.starts)))
            with open(a.out, "w") as f:
                json.dump(res, f, indent=1)


if __name__ == "__main__":
    _main()
