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


def random_rows(rows, cols, seed, scale=1.0):
    """Float32 rows ~ scale * N(0, 1) (network inputs and targets in tests)."""
    rng = np.random.default_rng(seed)
    return (scale * rng.standard_normal((rows, cols))).astype(np.float32)


def network_params(shapes, seed, gain=1.0):
    """Float32 parameters packed layer by layer (W_l out x in, then b_l):
    W ~ N(0, gain / in), b ~ 0.1 N(0, 1)."""
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in shapes:
        parts.append((rng.standard_normal(o * i) * np.sqrt(gain / i)))
        parts.append(0.1 * rng.standard_normal(o))
    return np.concatenate(parts).astype(np.float32)


def pair_indices(n_c, rows, seed):
    """Random pair indices p = i * N_c + j (with repeats)."""
    return np.random.default_rng(seed).integers(0, n_c * n_c, rows).astype(np.int64)
