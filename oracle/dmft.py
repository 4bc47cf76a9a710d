"""The self-consistency loop (oracle; test infrastructure only).

Sec. II summary paragraph: start from a guess for Sigma, sum the lattice Green's
functions to G_loc, extract the dynamical mean field, solve the impurity, extract
the new Sigma, and repeat until the Green's functions converge pointwise.

One iteration n here is: G_loc(n) = lattice(Sigma(n-1)); delta(n) =
max |G_loc(n) - G_loc(n-1)| (n >= 2); Sigma(n) = impurity(G_loc(n), Sigma(n-1)).
The loop stops after the iteration whose delta falls below tol, or after
max_iter iterations.

Readings: the paper starts from the equilibrium Sigma; the default start here is
Sigma = 0 (a caller may pass any start).  No mixing is described, so the update
is plain substitution.  The convergence norm is the max-abs over all entries of
the change in G_loc (|G| <= 1, so absolute and relative agree in scale).
"""
import dataclasses

import numpy as np

from . import contour, quadrature, lattice, impurity


@dataclasses.dataclass
class Problem:
    t_min: float
    t_max: float
    dt: float
    dtau: float
    beta: float
    u: float
    e_field: float
    mu: float = 0.0
    w1: float = 0.5
    n_eps: int = 10
    n_ebar: int = 10
    convention: str = "symmetric"
    gh_average: bool = False

    def grid(self):
        z, w = contour.points(self.t_min, self.t_max, self.dt, self.dtau,
                              self.beta)
        n_t, _, _ = contour.sizes(self.t_min, self.t_max, self.dt, self.dtau,
                                  self.beta)
        grid = quadrature.averaged_grid if self.gh_average else quadrature.product_grid
        eps, ebar, rho = grid(self.n_eps, self.n_ebar)
        return z, w, n_t, eps, ebar, rho


def lattice_only(p, sigma, keep_points=None):
    z, w, n_t, eps, ebar, rho = p.grid()
    return lattice.lattice_step(z, w, n_t, p.e_field, p.mu, p.beta, eps, ebar,
                                rho, sigma, keep_points)


def run(p, max_iter, tol=0.0, sigma0=None):
    """Iterate; returns a dict with gloc, sigma, current, density, m0, iters,
    deltas (delta history, first entry inf)."""
    z, w, n_t, eps, ebar, rho = p.grid()
    n_c = len(z)
    sigma = (np.zeros((n_c, n_c), dtype=np.complex128) if sigma0 is None
             else np.array(sigma0, dtype=np.complex128))
    prev = None
    deltas = []
    gloc = cur = None
    it = 0
    for it in range(1, max_iter + 1):
        gloc, cur, _ = lattice.lattice_step(z, w, n_t, p.e_field, p.mu, p.beta,
                                            eps, ebar, rho, sigma)
        d = np.inf if prev is None else float(np.max(np.abs(gloc - prev)))
        deltas.append(d)
        sigma = impurity.update(gloc, sigma, w, p.mu, p.u, p.w1, p.convention)
        prev = gloc
        if d < tol:
            break
    return dict(gloc=gloc, sigma=sigma, current=cur,
                density=lattice.density(gloc, n_t),
                m0=lattice.zeroth_moment(gloc, n_t), iters=it, deltas=deltas,
                z=z, w=w, n_t=n_t)
