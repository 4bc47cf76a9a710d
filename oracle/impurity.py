"""Falicov-Kimball impurity solution and self-energy update (oracle; test
infrastructure only).

Sec. II: eq. (effective_medium) G0_eff = [G_loc^-1 + Sigma]^-1; eq.
(dynamical_mean_field) lambda = (i d + mu) delta - G0_eff^-1; eq. (g_imp_solve)
G_imp = (1 - w1) [(i d + mu0) delta - lambda]^-1 + w1 [(i d + mu1) delta - lambda]^-1;
and Dyson's equation again, Sigma_new = G0_eff^-1 - G_imp^-1.

Discretization (Sec. II): a kernel A(t_i, t_j) is carried in right-weighted form
A W, in which the operator product of eq. (matrix_multiply) is the matrix product
and the operator inverse of eq. (matrix_inverse_discrete) is the matrix inverse.
The (i d + mu) delta term cancels from the mean field except for the chemical
potential shifts, which are taken point-split as in the paper's M display:
(mu' - mu) delta -> i W^-1 (M(mu') - M(mu)).

Readings:
  * Half filling.  The paper's Hamiltonian carries +U w n - mu n; with w1 = 1/2
    this is half filled at mu = U/2.  The particle-hole symmetric form
    U (w - 1/2) n with mu = 0 is the same Hamiltonian; its shifts are
    mu0 - mu = +U/2 (no f electron) and mu1 - mu = -U/2 (one f electron).
    convention="symmetric" (default) uses these; convention="paper" uses
    mu0 - mu = 0 and mu1 - mu = -U with the caller's mu.
  * The U shift is point-split (the paper reports point splitting works better
    for inverses); it differs from a diagonal shift at O(dt).
"""
import numpy as np

from . import contour


def shifts(u, convention="symmetric"):
    """(mu0 - mu, mu1 - mu) for the empty and occupied f site."""
    if convention == "symmetric":
        return 0.5 * u, -0.5 * u
    if convention == "paper":
        return 0.0, -u
    raise ValueError(convention)


def update(gloc, sigma, w, mu, u, w1, convention="symmetric"):
    """Sigma_new (values on the contour) from G_loc and Sigma (values)."""
    n = len(w)
    g_r = gloc * w[None, :]          # right-weighted G_loc
    s_r = sigma * w[None, :]         # right-weighted Sigma
    g0inv = np.linalg.inv(g_r) + s_r  # right-weighted G0_eff^-1
    d0, d1 = shifts(u, convention)
    a0 = g0inv + contour.shift_operator(w, mu, mu + d0)
    a1 = g0inv + contour.shift_operator(w, mu, mu + d1)
    g_imp = (1.0 - w1) * np.linalg.inv(a0) + w1 * np.linalg.inv(a1)
    s_new_r = g0inv - np.linalg.inv(g_imp)
    assert s_new_r.shape == (n, n)
    return s_new_r / w[None, :]
