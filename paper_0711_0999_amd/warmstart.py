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
D_IN = 64                     # >= N_GLOB + fk_ws_features' 20 pair features
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

    def propose(self, ctx, cont, sigma_prev, u, e, bf16=True):
        """Sets ctx's Sigma to the proposed start; returns the time it took (s)."""
        torch = _torch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = ctx.n_c
        g = glob_features(ctx, cont, sigma_prev, u, e)
        x = torch.empty((n * n, D_IN), dtype=torch.float32, device="cuda")
        ctx.ws_features(sigma_prev, g, None, n * n, sigma_scale(u), x, D_IN)
        y = self.net.forward(x, bf16=bf16)
        ctx.ws_apply(sigma_prev, y, sigma_scale(u) / self.t_rms)
        torch.cuda.synchronize()
        return time.perf_counter() - t0


def field_sweep_data(cont, us, es, n_eps, n_ebar, tol, rows_per_run, seed=0,
                     max_iter=80, log=None):
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
                    c.ws_features(prev[i], g, idx, rows_per_run, sigma_scale(u), xs, D_IN)
                    c.ws_targets(prev[i], new[i], idx, rows_per_run, sigma_scale(u), ts)
                    row += rows_per_run
        dt_s = time.perf_counter() - t0
        stats.append(dict(E=float(e), iters=[int(v) for v in r["iters"]],
                          converged=ok, seconds=dt_s))
        if log:
            log(f"field E={e:.3f}: iterations {list(r['iters'])} converged "
                f"{sum(ok)}/{len(ok)} in {dt_s:.1f} s")
        prev = new
        prev_ok = ok
    return x[:row], t[:row], stats


def train(x, t, steps=(3000, 2000, 1000), lrs=(1e-3, 3e-4, 1e-4), batch=4096,
          seed=0, log=None):
    """Adam on the sampled pairs (minibatches drawn by the library); the targets
    are divided by their RMS first (host arithmetic on a copy)."""
    torch = _torch()
    th = t.cpu().numpy()
    t_rms = float(np.sqrt(np.mean(th.astype(np.float64) ** 2)))
    tn = torch.from_numpy((th / t_rms).astype(np.float32)).cuda()
    ws = WarmStart(t_rms=t_rms, seed=seed)
    hist = []
    for k, (n, lr) in enumerate(zip(steps, lrs)):
        h = ws.net.train(x, tn, batch, n, lr, seed=seed * 1000 + k)
        hist.append(h)
        if log:
            log(f"train phase {k}: lr {lr:g}, loss {h[0]:.4f} -> {np.mean(h[-50:]):.4f}")
    return ws, np.concatenate(hist)


def compare_starts(ws, cont, u, e, n_eps, n_ebar, tol, max_iter=200, accept=0.5,
                   precision=fkdmft.FK_FP64, log=None):
    """Iterations to tol at (U, E) from Sigma = 0, from the converged Sigma of
    E - dE (previous field) and from the network's proposal on it (judged, with
    the previous field as fallback).  Also checks that the three fixed points
    agree."""
    torch = _torch()
    out = dict(U=u, E=e, tol=tol)
    with fkdmft.Context(**cont, U=u, E=e - FIELD_STEP, n_eps=n_eps, n_ebar=n_ebar) as c:
        r = c.iterate(max_iter, tol=tol, precision=precision)
        prev = torch.empty((c.n_c, c.n_c), dtype=torch.complex128, device="cuda")
        c.get_sigma(prev)
        out["prev_field_iters"] = r["iters"]
    glocs = {}
    for start in ("zero", "previous", "network"):
        with fkdmft.Context(**cont, U=u, E=e, n_eps=n_eps, n_ebar=n_ebar) as c:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if start == "zero":
                r = c.iterate(max_iter, tol=tol, precision=precision)
            elif start == "previous":
                c.set_sigma(prev)
                r = c.iterate(max_iter, tol=tol, precision=precision)
            else:
                out["propose_s"] = ws.propose(c, cont, prev, u, e)
                r = c.iterate_judged(prev, max_iter, tol=tol, accept=accept,
                                     precision=precision)
                out["outcome"] = r["outcome"]
            torch.cuda.synchronize()
            out[f"{start}_iters"] = r["iters"]
            out[f"{start}_s"] = time.perf_counter() - t0
            out[f"{start}_converged"] = bool(r["converged"])
            glocs[start] = c.get_gloc()
    ref = glocs["zero"]
    out["gloc_spread"] = max(float(np.max(np.abs(g - ref))) for g in glocs.values())
    if log:
        log(f"U={u:.3f} E={e:.3f}: zero {out['zero_iters']}, previous "
            f"{out['previous_iters']}, network {out['network_iters']} "
            f"(outcome {out['outcome']}), spread {out['gloc_spread']:.1e}")
    return out
