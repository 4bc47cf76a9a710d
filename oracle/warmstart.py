"""Inputs and outputs of the learned warm start (oracle; test infrastructure
only).  Not a passage of the paper: the network that proposes a starting
self-energy is this project's addition to the self-consistency loop of Sec. II;
these functions define, in plain numpy, what its feature rows, training
targets, sketch and update are, so that the device versions can be checked.

Pair p = i * N_c + j of a contour with N_t points per real branch; T = t_max -
t_min; t+ = max(t, 0) on the real branches (the field is on for t > 0, Sec. II)
and 0 on the imaginary branch.  Feature row:
    glob | one-hot branch of i (3) | one-hot branch of j (3) |
    t_i/T, tau_i/beta, t_j/T, tau_j/beta | [i >= j] | [i - j >= 2] |
    (t_i - t_j)/T | max(t_i, t_j, 0)/T |
    sin E t_i+, cos E t_i+, sin E t_j+, cos E t_j+ |
    s Re Sigma_prev(i, j), s Im Sigma_prev(i, j) |
    sin, cos(pi k t_i/T) for k = 1..8 | the same for t_j |
    sin, cos(pi k tau_i/beta) for k = 1, 2 | the same for tau_j | zeros up to d_in
where t is Re z on the real branches (0 on the imaginary one) and tau = -Im z
on the imaginary branch (0 on the real ones).
"""
import numpy as np

N_FEATURES = 60


def branch(n_c, n_t):
    return np.array([0] * n_t + [1] * n_t + [2] * (n_c - 2 * n_t))


def features(z, n_t, t_span, beta, e_field, sigma_prev, glob, idx, scale, d_in):
    n = len(z)
    idx = np.arange(n * n) if idx is None else np.asarray(idx)
    br = branch(n, n_t)
    t = np.where(br < 2, z.real, 0.0)
    tau = np.where(br == 2, -z.imag, 0.0)
    rows = np.zeros((len(idx), d_in))
    ng = len(glob)
    for r, p in enumerate(idx):
        i, j = divmod(int(p), n)
        f = list(glob)
        f += [1.0 if br[i] == q else 0.0 for q in range(3)]
        f += [1.0 if br[j] == q else 0.0 for q in range(3)]
        f += [t[i] / t_span, tau[i] / beta, t[j] / t_span, tau[j] / beta]
        f += [1.0 if i >= j else 0.0, 1.0 if i - j >= 2 else 0.0]
        f += [(t[i] - t[j]) / t_span, max(t[i], t[j], 0.0) / t_span]
        pi, pj = e_field * max(t[i], 0.0), e_field * max(t[j], 0.0)
        f += [np.sin(pi), np.cos(pi), np.sin(pj), np.cos(pj)]
        s = sigma_prev[i, j]
        f += [scale * s.real, scale * s.imag]
        for xv, kmax in ((t[i] / t_span, 8), (t[j] / t_span, 8),
                         (tau[i] / beta, 2), (tau[j] / beta, 2)):
            for k in range(1, kmax + 1):
                f += [np.sin(np.pi * k * xv), np.cos(np.pi * k * xv)]
        assert len(f) == ng + N_FEATURES
        rows[r, :len(f)] = f
    return rows


def targets(sigma_prev, sigma_new, idx, scale):
    n = sigma_prev.shape[0]
    idx = np.arange(n * n) if idx is None else np.asarray(idx)
    d = (sigma_new - sigma_prev).ravel()[idx] * scale
    return np.stack([d.real, d.imag], axis=1)


def apply(sigma_prev, y, scale, pre_field=None):
    """Sigma_prev + y / scale, y holding (Re, Im) rows of all pairs in order.
    pre_field (optional, N_c booleans): the contour points before the field is
    switched on; pairs of two such points keep Sigma_prev."""
    n = sigma_prev.shape[0]
    out = sigma_prev + (y[:, 0] + 1j * y[:, 1]).reshape(n, n) / scale
    if pre_field is not None:
        keep = np.outer(pre_field, pre_field)
        out[keep] = sigma_prev[keep]
    return out


def pre_field_points(z, n_t):
    """Contour points before the field (Sec. II: the vector potential is zero
    up to t = 0): real time <= 0 on the two real branches (the first n_t and
    the next n_t points), and every point of the imaginary branch."""
    z = np.asarray(z)
    idx = np.arange(len(z))
    return np.where(idx < 2 * n_t, z.real <= 1e-12, True)


def randomized_singular_values(a, omega):
    """Rank-r randomized SVD (Halko, Martinsson & Tropp 2011, the basic range
    finder): Y = A Omega, Q = orthonormal basis of the range of Y, B = Q^H A;
    returns the r singular values of B, descending.  They equal the leading
    singular values of A whenever the range of Y holds A's leading singular
    vectors (exactly if rank(A) <= r)."""
    y = a @ omega
    q, _ = np.linalg.qr(y)
    return np.linalg.svd(q.conj().T @ a, compute_uv=False)


def weighted_sketch(sigma, w, omega):
    """Randomized singular values of D Sigma D, D = diag(sqrt|W|): the sketch of
    the contour integral operator with the symmetric square-root weighting,
    which approximates the continuum operator and so does not grow with N_c."""
    d = np.sqrt(np.abs(w))
    return randomized_singular_values(d[:, None] * sigma * d[None, :], omega)
