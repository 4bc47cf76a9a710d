"""Extrapolation of the discrete results to zero time step.

The paper extrapolates its dt-dependent results with Lagrange polynomials in
dt (Sec. II, the accuracy discussion of the results).  Here several contours
that differ only in the step h (dt = dtau = h) are solved together in one
multi-instance sweep (uneven N_c in shared batched launches, fk_batch); the
current j(t), the filling n(t), the zeroth moment m0(t) and the equal-time
spectral moments mu0, mu1, mu2 (fk_equal_time_moments, on the coarse times
3..N_t - 4 of the coarsest grid) are read on the coarsest time grid, and their
value at h = 0 is the Lagrange combination sum_k w_k f_k with w_k =
prod_{m != k} h_m / (h_m - h_k) (fk_extrapolate_to_zero).  Every DMFT step
and the combination run in the library; this module arranges the calls.
"""
import numpy as np

from . import fkdmft


def lagrange_weights(hs):
    """w_k with sum_k w_k f(h_k) = p(0) for the polynomial p through the points
    (the combination's weights, from the library: the unit vectors' images)."""
    n = len(hs)
    return fkdmft.extrapolate_to_zero(hs, list(np.eye(n)))


def step_sweep(t_min, t_max, beta, steps, model, tol=1e-10, max_iter=200,
               use_graph=True):
    """Solve the contour t in [t_min, t_max], beta with dt = dtau = h for every h
    in steps (the coarsest first; each a whole multiple of the finest) in one
    fk_batch, to delta < tol.  Returns the coarse times, per-step j, n, m0 and
    mu (complex [3, N_t - 6], at the coarse times t_mu) on that grid, their
    extrapolation to h = 0, and the iteration counts."""
    steps = [float(h) for h in steps]
    h0 = max(steps)
    inst = [dict(t_min=t_min, t_max=t_max, dt=h, dtau=h, beta=beta, **model) for h in steps]
    per = {}
    with fkdmft.Batch(inst) as b:
        r = b.iterate(max_iter, tol=tol, use_graph=use_graph)
        if not np.all(r["deltas"] < tol):
            raise RuntimeError(f"not converged: deltas {r['deltas']}")
        t_coarse = None
        for i, h in enumerate(steps):
            c = b.instance(i)
            t, j, n = c.get_current()
            m0 = c.get_zeroth_moment()
            s = int(round(h0 / h))
            if abs(s * h - h0) > 1e-9 * h0:
                raise ValueError("steps must divide the coarsest step")
            if h == h0:
                t_coarse = t
            nc = int(round((t_max - t_min) / h0))
            mu = c.moments(np.arange(3, nc - 3) * s)
            per[h] = dict(j=j[::s][:nc], n=n[::s][:nc], m0=m0[::s][:nc], mu=mu)
    w = lagrange_weights(steps)
    ext = {q: fkdmft.extrapolate_to_zero(steps, [per[h][q] for h in steps])
           for q in ("j", "n", "m0", "mu")}
    return dict(t=t_coarse, t_mu=t_coarse[3:nc - 3], per_step=per, extrapolated=ext,
                weights=w, iters=[int(v) for v in r["iters"]])
