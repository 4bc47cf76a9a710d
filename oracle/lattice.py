"""Lattice step: the nonequilibrium Hilbert transform (oracle; test
infrastructure only).

eq. (dyson) with the discrete operator product of eq. (matrix_multiply) on both
contour integrals gives, at each (eps, ebar) point k,

    G_k = G0_k + G0_k Sigma_t G_k,     Sigma_t = diag(W) Sigma diag(W),

so G_k = (I - G0_k Sigma_t)^-1 G0_k, and eq. (g_loc) sums the points with the
joint-DOS weights: G_loc = sum_k rho_k G_k.  Here Sigma is the matrix of VALUES
Sigma(z_i, z_j) on the contour.

Reading: the kernel form [I - G0 W Sigma]^-1 G0 with one weight equals this one
when its Sigma is the right-weighted Sigma W; values are exchanged here.

Observables from the same points (Sec. II, eq. current_def and the moments
paragraph):
  G^<(t_i, t_i) = G[i, p(i)], p(i) = 2 N_t - i, i < N_t (i = 0 pairs with the
      first imaginary-branch point, the same physical time t_min);
  j(t_i) = Re[ i sum_k rho_k ebar_k(t_i) G_k[i, p(i)] ]  (e = 1, t* = 1, the
      velocity replaced by -ebar at the shifted momentum);
  n(t_i) = Re[ -i G_loc[i, p(i)] ];
  m0(t_i) = G_loc[p(i), i] - G_loc[i, p(i)] = G^> - G^<, which is -i in the
      continuum (zeroth spectral moment equal to one).
Reading: the normalization of the paper's "scaled current" is not given; the
current here is the unscaled sum above.
"""
import numpy as np

from . import green


def weighted_sigma(sigma, w):
    """Sigma_t = diag(W) Sigma diag(W)  (eq. matrix_multiply on both integrals)."""
    return w[:, None] * sigma * w[None, :]


def point_green(z, n_t, e_field, mu, beta, eps, ebar, sigma_t):
    """G_k = solve(I - G0_k Sigma_t, G0_k) by LU with partial pivoting."""
    g0 = green.g0_matrix(z, n_t, e_field, mu, beta, eps, ebar)
    a = np.eye(len(z), dtype=np.complex128) - g0 @ sigma_t
    return np.linalg.solve(a, g0)


def lattice_step(z, w, n_t, e_field, mu, beta, eps, ebar, rho, sigma,
                 keep_points=None):
    """One lattice step: returns (G_loc, j(t_i), dict of kept G_k).

    eq. (g_loc) as the rho-weighted sum over the given points, and eq.
    (current_def) accumulated from the same G_k."""
    n_c = len(z)
    sigma_t = weighted_sigma(sigma, w)
    gloc = np.zeros((n_c, n_c), dtype=np.complex128)
    cur = np.zeros(n_t, dtype=np.complex128)
    rows = np.arange(n_t)
    cols = 2 * n_t - rows
    kept = {}
    for k in range(len(eps)):
        gk = point_green(z, n_t, e_field, mu, beta, eps[k], ebar[k], sigma_t)
        gloc += rho[k] * gk
        vel = green.band_velocity_factor(z, n_t, e_field, eps[k], ebar[k])
        cur += rho[k] * vel * gk[rows, cols]
        if keep_points is not None and k in keep_points:
            kept[k] = gk
    return gloc, (1j * cur).real, kept


def density(gloc, n_t):
    """n(t_i) = Re[-i G^<_loc(t_i, t_i)], i < N_t."""
    rows = np.arange(n_t)
    return (-1j * gloc[rows, 2 * n_t - rows]).real


def zeroth_moment(gloc, n_t):
    """m0(t_i) = G^>_loc(t_i, t_i) - G^<_loc(t_i, t_i), i < N_t."""
    rows = np.arange(n_t)
    cols = 2 * n_t - rows
    return gloc[cols, rows] - gloc[rows, cols]
