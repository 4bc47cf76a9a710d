"""Equilibrium Falicov-Kimball DMFT on the Matsubara axis (oracle; test
infrastructure only).

The standard equilibrium algorithm the paper starts from (Sec. II, the DMFT
loop, here with imaginary frequencies z_n = i w_n, w_n = (2n + 1) pi / beta):

  G(z)       = int rho(e) de / (z + mu - Sigma(z) - e)
             = -i sqrt(pi) w(z + mu - Sigma)      (Gaussian DOS of eq. joint_dos,
                                                   w the Faddeeva function)
  G0^-1(z)   = G(z)^-1 + Sigma(z)                  (eq. effective_medium)
  G_imp(z)   = (1 - w1) / (G0^-1 - d0) + w1 / (G0^-1 - d1)   (eq. g_imp_solve)
  Sigma(z)   = G0^-1(z) - G_imp(z)^-1              (Dyson again)

with the impurity shifts d0 = mu0 - mu, d1 = mu1 - mu of the convention
(symmetric: +U/2, -U/2).  The same scalar equations at z = w + i0 give the
real-axis density of states; at w = 0 and half filling the metallic solution
ends at U = sqrt(2) (the metal-insulator transition quoted in Sec. III: with
G(0) = -i g, G0^-1(0) = i a one finds g = a/(a^2 + U^2/4) = sqrt(pi) w(iy),
y = U^2/(4a), whose a -> 0 expansion has a nonzero root only for U^2 < 2).

G(tau) on [0, beta) from the Matsubara sum with the 1/(i w_n) tail subtracted:
  G(tau) = -1/2 + (2 / beta) sum_{n >= 0} Re[e^{-i w_n tau} (G(i w_n) - 1/(i w_n))],
valid at half filling (G(-i w) = conj G(i w)).  On the contour the imaginary
branch carries G_c(t_min - i tau, t_min - i tau') = i G(tau - tau') for
tau >= tau'.
"""
import numpy as np
from scipy.special import wofz

from . import impurity


def hilbert_gaussian(z):
    """int exp(-e^2)/sqrt(pi) / (z - e) de for Im z > 0."""
    return -1j * np.sqrt(np.pi) * wofz(z)


def solve(u, beta, n_freq, mu=0.0, w1=0.5, convention="symmetric", tol=1e-14,
          max_iter=10000, z=None):
    """Iterate the scalar DMFT equations at the frequencies z (default the
    first n_freq positive Matsubara frequencies i w_n) until the change of
    Sigma relative to max(1, |z|) is below tol.  Returns (z, G, Sigma,
    iterations)."""
    if z is None:
        z = 1j * (2 * np.arange(n_freq) + 1) * np.pi / beta
    d0, d1 = impurity.shifts(u, convention)
    sig = np.zeros_like(z)
    for it in range(1, max_iter + 1):
        g = hilbert_gaussian(z + mu - sig)
        g0inv = 1.0 / g + sig
        gimp = (1.0 - w1) / (g0inv - d0) + w1 / (g0inv - d1)
        new = g0inv - 1.0 / gimp
        if np.max(np.abs(new - sig) / np.maximum(1.0, np.abs(z))) < tol:
            sig = new
            break
        sig = new
    g = hilbert_gaussian(z + mu - sig)
    return z, g, sig, it


def g_tau(beta, g_iw, tau):
    """G(tau) for 0 <= tau < beta at half filling from G(i w_n), n >= 0."""
    n = len(g_iw)
    w = (2 * np.arange(n) + 1) * np.pi / beta
    tau = np.asarray(tau, dtype=np.float64)
    rest = g_iw - 1.0 / (1j * w)
    ph = np.exp(-1j * np.outer(tau, w))
    return -0.5 + (2.0 / beta) * (ph @ rest).real


def dos_at_zero(u, eta=1e-9, max_iter=200000):
    """rho(w = 0) = -Im G(i eta) / pi of the half-filled symmetric model, from
    the same scalar equations at z = i eta (the real-axis limit).  Zero, to
    O(eta), once the metallic solution has ended (U >= sqrt(2))."""
    _, g, _, _ = solve(u, 1.0, 1, z=np.array([1j * eta]), tol=1e-15, max_iter=max_iter)
    return float(-g[0].imag / np.pi)
