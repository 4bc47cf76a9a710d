"""Nonequilibrium density of states and equal-time spectral moments of the local
retarded Green's function (oracle; test infrastructure only).

Sec. II, last paragraph of the formalism (eqs. gr_omega, dos_def): with the
average time T = (t + t')/2 and the relative time t_rel = t - t',

  G^R(T, w) = int dt_rel e^{i w t_rel} G^R(T + t_rel/2, T - t_rel/2),
  rho(T, w) = -Im G^R(T, w) / pi,

and G^R(t, t') = theta(t - t') [G^>(t, t') - G^<(t, t')].  On the contour
matrix G_loc (indices of the real branches: upper i < N_t at t_i = t_min + i dt,
lower p(i) = 2 N_t - i at the same time; p(0) is the first imaginary-branch
point, also at t_min):

  G^>(t_a, t_b) = G_loc[p(a), b],   G^<(t_a, t_b) = G_loc[a, p(b)].

Readings (the paper gives no discretization of eq. gr_omega):
  - T is taken on the time grid, T_i = t_i; then t_rel = 2 d dt, d = 0..D with
    D = min(i, N_t - 1 - i) (both times on the upper-branch grid);
  - the integral over t_rel >= 0 is the trapezoid rule on that window with step
    h = 2 dt: weight 1/2 at d = 0 (the half of the jump of theta at t_rel = 0)
    and at d = D > 0, 1 in between;
  - no damping or window function.
Then the integral of rho(T_i, w) over one period of w (2 pi / h) is exactly
-Im G^R(t_i, t_i), the zeroth moment (pinned).

Moments (Sec. II, moments paragraph): for t_rel > 0,
G^R(T, t_rel) = -i int dw rho(T, w) e^{-i w t_rel}, so at t_rel -> 0+ with
f(s) = G^R(T_i + s/2, T_i - s/2):

  mu0 = i f(0),  mu1 = -f'(0),  mu2 = -i f''(0),

exact values 1, 0 and 1/2 + U^2/4 for the Falicov-Kimball model at half filling
in the symmetric convention.  Reading: the derivatives are the one-sided
second-order differences on the points d = 0..3 (step h = 2 dt),
  f'(0)  = (-3 f0 + 4 f1 - f2) / (2 h),
  f''(0) = (2 f0 - 5 f1 + 4 f2 - f3) / h^2,
which needs 3 <= i <= N_t - 4.
"""
import numpy as np


def retarded_pairs(gloc, n_t, i, d):
    """f_d = G^R(t_{i+d}, t_{i-d}) for the relative offsets d (array)."""
    d = np.asarray(d)
    a = i + d
    b = i - d
    return gloc[2 * n_t - a, b] - gloc[a, 2 * n_t - b]


def wigner_dos(gloc, n_t, dt, t_index, omega):
    """rho(T_i, w) for the time indices t_index (each 0 <= i < N_t) and the
    frequencies omega; returns an array [len(t_index), len(omega)]."""
    omega = np.asarray(omega, dtype=np.float64)
    h = 2.0 * dt
    out = np.zeros((len(t_index), len(omega)))
    for r, i in enumerate(t_index):
        if not 0 <= i < n_t:
            raise ValueError("time index outside the real-time grid")
        dmax = min(i, n_t - 1 - i)
        d = np.arange(dmax + 1)
        f = retarded_pairs(gloc, n_t, i, d)
        c = np.ones(dmax + 1)
        c[0] = 0.5
        if dmax > 0:
            c[-1] = 0.5
        phase = np.exp(1j * np.outer(omega, d * h))
        gr_w = h * (phase @ (c * f))
        out[r] = -gr_w.imag / np.pi
    return out


def moments(gloc, n_t, dt, t_index):
    """(mu0, mu1, mu2) at the time indices t_index (each 3 <= i <= N_t - 4);
    complex arrays of len(t_index) (real in the continuum)."""
    h = 2.0 * dt
    mu = np.zeros((3, len(t_index)), dtype=np.complex128)
    for r, i in enumerate(t_index):
        if not 3 <= i <= n_t - 4:
            raise ValueError("time index too close to the ends of the grid")
        f0, f1, f2, f3 = retarded_pairs(gloc, n_t, i, np.arange(4))
        d1 = (-3.0 * f0 + 4.0 * f1 - f2) / (2.0 * h)
        d2 = (2.0 * f0 - 5.0 * f1 + 4.0 * f2 - f3) / (h * h)
        mu[0, r] = 1j * f0
        mu[1, r] = -d1
        mu[2, r] = -1j * d2
    return mu
