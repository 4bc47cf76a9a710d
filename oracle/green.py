"""Noninteracting contour-ordered Green's function of one (eps, ebar) point in the
uniform field (oracle; test infrastructure only).

eq. (g_contour_non_final2): with the field along the diagonal and the vector
potential A(t) = -theta(t) E t (eq. vector_potential, Peierls substitution),

  G0(t, t') = i [f(eps - mu) - theta_c(t, t')] e^{i mu (t - t')}
              exp(-i int_{t'}^{t} dtb { [theta(-tb) + theta(tb) cos(E tb)] eps
                                        - theta(tb) ebar sin(E tb) })

with the time integral running along the contour.  The integral is written as a
difference phi(t) - phi(t') of the antiderivative

  phi(z) = eps * alpha(z) + ebar * gamma(z),
  alpha(z) = sin(E t)/E,  gamma(z) = (cos(E t) - 1)/E     for real t > 0,
  alpha(z) = z,           gamma(z) = 0                      otherwise,

"otherwise" covering t <= 0 on the real branches and the whole imaginary branch
(where the integrand is eps, because the field is off there).  The constant
-eps t_min of the lower limit cancels in the difference.

Readings: theta_c(t, t) = 1 on the diagonal of the sampled matrix (the paper does
not say; this makes the sampled G0 exactly the inverse of the paper's own discrete
operator at eps = ebar = mu = 0, see the pins).  E = 0 means alpha = z, gamma = 0.
"""
import numpy as np


def phase_tables(z, n_t, e_field):
    """alpha_j and gamma_j of the antiderivative above, for every contour point."""
    n_c = len(z)
    alpha = np.array(z, dtype=np.complex128)
    gamma = np.zeros(n_c, dtype=np.complex128)
    if e_field != 0.0:
        for j in range(2 * n_t):
            t = z[j].real
            if t > 0.0:
                alpha[j] = np.sin(e_field * t) / e_field
                gamma[j] = (np.cos(e_field * t) - 1.0) / e_field
    return alpha, gamma


def fermi_pair(x, beta):
    """(f(x), 1 - f(x)) with f(x) = 1/(1 + e^{beta x}); 1 - f computed directly as
    1/(1 + e^{-beta x}) so that it keeps its relative accuracy when tiny."""
    with np.errstate(over="ignore"):
        f = 1.0 / (1.0 + np.exp(beta * x))
        g = 1.0 / (1.0 + np.exp(-beta * x))
    return f, g


def g0_matrix(z, n_t, e_field, mu, beta, eps, ebar):
    """Sampled G0 matrix (N_c x N_c, complex128) of eq. (g_contour_non_final2) at
    one (eps, ebar) point, contour-ordered with theta_c(t_i, t_j) = [i >= j]."""
    alpha, gamma = phase_tables(z, n_t, e_field)
    phi = eps * alpha + ebar * gamma
    # exponent of the point factor: -i phi(z) + i mu z
    expo = -1j * phi + 1j * mu * z
    f, one_minus_f = fermi_pair(eps - mu, beta)
    n_c = len(z)
    i_idx = np.arange(n_c)[:, None]
    j_idx = np.arange(n_c)[None, :]
    later_or_equal = i_idx >= j_idx  # theta_c(t_i, t_j)
    # f - theta_c: f where theta = 0, -(1 - f) where theta = 1
    occ = np.where(later_or_equal, -one_minus_f, f)
    return 1j * occ * np.exp(expo[:, None] - expo[None, :])


def band_velocity_factor(z, n_t, e_field, eps, ebar):
    """ebar at the Peierls-shifted momentum, for the upper-branch times:
    ebar(k + E t) = ebar cos(E t) + eps sin(E t) for t > 0 and ebar otherwise.

    Sec. II, eq. (current_def): the velocity is evaluated at k + theta(t) E t and
    replaced by -ebar for a field along the diagonal; shifting every k_i by E t
    in ebar = -sum sin(k_i)/sqrt(d) gives the rotation above."""
    t = z[:n_t].real
    out = np.full(n_t, ebar, dtype=np.float64)
    pos = t > 0.0
    out[pos] = ebar * np.cos(e_field * t[pos]) + eps * np.sin(e_field * t[pos])
    return out
