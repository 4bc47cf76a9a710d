"""Discrete Kadanoff-Baym-Keldysh contour (oracle; test infrastructure only).

Follows Sec. II, the discretization paragraphs: eq. (time_discrete) for the
points, eq. (integration_rule)/(integration_weights) for the leftpoint weights,
and the displayed matrix M of the point-split operator [i d/dt + mu] delta_c
with its determinant, eq. (det).

Index convention (0-based, contour order):
  upper real branch   U: j in [0, N_t)        z_j = t_min + j dt          W_j = +dt
  lower real branch   L: j in [N_t, 2 N_t)    z_j = t_max - (j - N_t) dt  W_j = -dt
  imaginary branch    M: j in [2 N_t, N_c)    z_j = t_min - i dtau (j-2N_t) W_j = -i dtau

Reading: eq. (time_discrete) prints "-t_min + (j-1) dt" on the upper branch while
the text says that branch runs from t_min to t_max - dt; the sign is taken as a
misprint and the points start at +t_min.  The imaginary branch step is a
parameter dtau (the paper fixes it at 0.1).
"""
import numpy as np


def _count(span, step, what):
    n = span / step
    m = int(round(n))
    if m <= 0 or abs(n - m) > 1e-9 * max(1.0, abs(n)):
        raise ValueError(f"{what}: {span}/{step} is not a positive integer")
    return m


def sizes(t_min, t_max, dt, dtau, beta):
    """(N_t, N_tau, N_c) with N_c = 2 N_t + N_tau (Sec. II discretization)."""
    n_t = _count(t_max - t_min, dt, "N_t")
    n_tau = _count(beta, dtau, "N_tau")
    return n_t, n_tau, 2 * n_t + n_tau


def points(t_min, t_max, dt, dtau, beta):
    """Contour points z[N_c] (complex) and leftpoint weights W[N_c] (complex).

    eq. (time_discrete) and eq. (integration_weights)."""
    n_t, n_tau, n_c = sizes(t_min, t_max, dt, dtau, beta)
    z = np.zeros(n_c, dtype=np.complex128)
    w = np.zeros(n_c, dtype=np.complex128)
    for j in range(n_c):
        if j < n_t:
            z[j] = t_min + j * dt
            w[j] = dt
        elif j < 2 * n_t:
            z[j] = t_max - (j - n_t) * dt
            w[j] = -dt
        else:
            z[j] = complex(t_min, -dtau * (j - 2 * n_t))
            w[j] = complex(0.0, -dtau)
    return z, w


def branch(n_t, n_c):
    """Branch label per point: 0 = upper real, 1 = lower real, 2 = imaginary."""
    b = np.full(n_c, 2, dtype=np.int64)
    b[:n_t] = 0
    b[n_t:2 * n_t] = 1
    return b


def m_matrix(w, mu):
    """The paper's discrete point-split operator matrix M (Sec. II, display of
    M_jk) such that [i d/dt + mu] delta_c(t_j, t_k) = i W_j^-1 M_jk W_k^-1.

    Unit diagonal; subdiagonal M[j, j-1] = -(1 + i W_j mu); the corner
    M[0, N_c-1] = +(1 + i W_0 mu) carries the antiperiodic boundary condition
    that identifies t_min with t_min - i beta.  Every printed entry of the
    display (upper branch -1 - i dt mu, lower branch -1 + i dt mu, imaginary
    branch -1 - dtau mu, corner 1 + i dt mu) follows from this rule with the
    weights of eq. (integration_weights)."""
    n = len(w)
    m = np.eye(n, dtype=np.complex128)
    for j in range(1, n):
        m[j, j - 1] = -(1.0 + 1j * w[j] * mu)
    m[0, n - 1] = 1.0 + 1j * w[0] * mu
    return m


def shift_operator(w, mu, mu_new):
    """Right-weighted form of [(i d/dt + mu_new) - (i d/dt + mu)] delta_c with the
    point-split delta of the M display: i W^-1 (M(mu_new) - M(mu)).

    Right-weighting (multiplying a discrete kernel by diag(W) on the right)
    turns the paper's discrete operator product, eq. (matrix_multiply), into a
    plain matrix product and its inverse rule, eq. (matrix_inverse_discrete),
    into a plain matrix inverse; the i W^-1 M W^-1 kernel becomes i W^-1 M."""
    return 1j * (m_matrix(w, mu_new) - m_matrix(w, mu)) / w[:, None]
