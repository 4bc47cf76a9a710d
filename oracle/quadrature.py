"""Gauss-Hermite quadrature over the joint band-energy DOS (oracle; test
infrastructure only).

eq. (joint_dos): rho(eps, ebar) = exp(-eps^2 - ebar^2) / pi.  The paper integrates
each Gaussian dimension with Gaussian quadrature (Sec. II, the quadrature
paragraph).  Reading: one n x n product rule per lattice step; the paper's
average of the N and N+1 rules is a flag of the caller, not done here.
"""
import numpy as np


def hermite_rule(n):
    """Nodes x_a and normalized weights w_a (sum w_a = 1) such that
    sum_a w_a g(x_a) ~ int g(x) exp(-x^2) dx / sqrt(pi).

    Golub-Welsch: the nodes are the eigenvalues of the symmetric Jacobi matrix of
    the Hermite recurrence (zero diagonal, off-diagonal sqrt(k/2)), and each
    normalized weight is the squared first component of its unit eigenvector."""
    if n < 1:
        raise ValueError("n must be >= 1")
    k = np.arange(1, n, dtype=np.float64)
    jac = np.diag(np.sqrt(k / 2.0), 1) + np.diag(np.sqrt(k / 2.0), -1)
    x, v = np.linalg.eigh(jac)
    w = v[0, :] ** 2
    # make the rule exactly symmetric (the Hermite weight is even)
    x = 0.5 * (x - x[::-1])
    w = 0.5 * (w + w[::-1])
    return x, w


def product_grid(n_eps, n_ebar):
    """Points k = a * n_ebar + b with eps = x_a, ebar = x_b and
    rho_k = w_a w_b, the quadrature of eq. (joint_dos) over the plane."""
    xa, wa = hermite_rule(n_eps)
    xb, wb = hermite_rule(n_ebar)
    eps = np.repeat(xa, n_ebar)
    ebar = np.tile(xb, n_eps)
    rho = np.repeat(wa, n_ebar) * np.tile(wb, n_eps)
    return eps, ebar, rho


def averaged_grid(n_eps, n_ebar):
    """The average of the n_eps x n_ebar and (n_eps + 1) x (n_ebar + 1) product
    rules (Sec. II, the quadrature paragraph: averaging N and N + 1 points):
    the points of both rules, the first rule's first, weights halved."""
    e1, b1, r1 = product_grid(n_eps, n_ebar)
    e2, b2, r2 = product_grid(n_eps + 1, n_ebar + 1)
    return (np.concatenate([e1, e2]), np.concatenate([b1, b2]),
            0.5 * np.concatenate([r1, r2]))
