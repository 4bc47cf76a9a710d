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


# ------------------------------------------------------- extended precision
_EXT = None


def _ext_library():
    """The C implementation in impurity_ext.c (built next to it with gcc on
    first use when the build step has not done so)."""
    global _EXT
    if _EXT is None:
        import ctypes
        import os
        import subprocess
        here = os.path.dirname(os.path.abspath(__file__))
        lib = os.path.join(here, "_impurity_ext.so")
        if not os.path.exists(lib):
            build_extension()
        _EXT = ctypes.CDLL(lib)
        dp = ctypes.POINTER(ctypes.c_double)
        _EXT.oracle_impurity_update_ld.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_double,
                                                   ctypes.c_double, ctypes.c_double, dp]
        _EXT.oracle_inverse_ld.argtypes = [ctypes.c_int, dp, dp]
    return _EXT


def build_extension():
    """Compile impurity_ext.c into _impurity_ext.so (gcc, OpenMP)."""
    import os
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    src = os.path.join(here, "impurity_ext.c")
    lib = os.path.join(here, "_impurity_ext.so")
    tmp = lib + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src, "-lm"],
                   check=True)
    os.replace(tmp, lib)
    return lib


def _dptr(a):
    import ctypes
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def inverse_extended(a):
    """Inverse by Gauss-Jordan elimination with partial pivoting in long double
    complex (impurity_ext.c), rounded to complex128."""
    a = np.ascontiguousarray(a, dtype=np.complex128)
    out = np.zeros_like(a)
    s = _ext_library().oracle_inverse_ld(a.shape[0], _dptr(a), _dptr(out))
    if s != 0:
        raise np.linalg.LinAlgError(f"extended-precision inverse failed ({s})")
    return out


def update_extended(gloc, sigma, w, mu, u, w1, convention="symmetric"):
    """update() with every step carried out in long double complex (C,
    impurity_ext.c): the same sequence (effective medium, the two shifted
    resolvents, Dyson again), rounded to complex128 only at the end.  The final
    Dyson step subtracts two matrices of order 1/dt to leave one of order Sigma,
    so the complex128 update() loses digits in proportion; at N_c in the
    thousands its own rounding reaches 1e-10 of max|Sigma| (6.9e-10 at N_c =
    1050 against this version), which this version stays far below.  mu
    cancels from the point-split shifts (only mu' - mu enters)."""
    d0, d1 = shifts(u, convention)
    g = np.ascontiguousarray(gloc, dtype=np.complex128)
    s = np.ascontiguousarray(sigma, dtype=np.complex128)
    ww = np.ascontiguousarray(w, dtype=np.complex128)
    out = np.zeros_like(g)
    st = _ext_library().oracle_impurity_update_ld(len(ww), _dptr(g), _dptr(s), _dptr(ww),
                                                  float(d0), float(d1), float(w1), _dptr(out))
    if st != 0:
        raise np.linalg.LinAlgError(f"extended-precision impurity update failed ({st})")
    return out
