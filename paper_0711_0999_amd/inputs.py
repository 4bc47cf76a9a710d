"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
legs.  Holds no arithmetic of the method: only random draws and shapes."""
import numpy as np


def random_sigma(n_c, seed, scale=0.05):
    """A dense complex N_c x N_c matrix of self-energy VALUES on the contour,
    entries ~ scale * (N(0,1) + i N(0,1)).  Used where a parity test needs one
    lattice step from a fixed, non-trivial Sigma."""
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal((n_c, n_c)) +
                    1j * rng.standard_normal((n_c, n_c)))


def sample_points(n_points, n_sample, seed):
    """A sorted random subset of quadrature-point indices."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_points, size=min(n_sample, n_points), replace=False))
