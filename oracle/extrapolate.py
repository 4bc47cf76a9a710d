"""Extrapolation in the time step to dt -> 0 (oracle; test infrastructure
only).

Sec. II (the accuracy discussion of the results): the discretized quantities
approach their continuum limits polynomially in dt, and the paper extrapolates
results from several dt with Lagrange polynomials (linear, quadratic or cubic in
dt).  Here the value at dt = 0 of the polynomial through the points
(dt_k, f_k) is computed by Neville's recursion."""
import numpy as np


def to_zero(hs, fs):
    """Value at h = 0 of the interpolating polynomial through (hs[k], fs[k]);
    fs[k] may be arrays (same shape), combined elementwise."""
    hs = [float(h) for h in hs]
    p = [np.asarray(f, dtype=np.complex128) for f in fs]
    n = len(hs)
    for m in range(1, n):
        # p[i] <- polynomial through points i .. i+m, evaluated at 0
        p = [((0.0 - hs[i + m]) * p[i] - (0.0 - hs[i]) * p[i + 1]) / (hs[i] - hs[i + m])
             for i in range(n - m)]
    return p[0]


def on_coarse_grid(values, dt, dt_coarse, n_coarse):
    """Samples of a per-time-step array at the coarse grid t_min + i dt_coarse."""
    s = int(round(dt_coarse / dt))
    return np.asarray(values)[::s][:n_coarse]
