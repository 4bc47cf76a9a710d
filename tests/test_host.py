"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point that include/fkdmft.h declares, and its host-only helpers
(Gauss-Hermite rule, contour) agree with independent references."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import contour as ocontour

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "fkdmft.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fk_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(lib.LIB_PATH)
    syms = header_symbols()
    assert len(syms) >= 20
    for name in syms:
        assert hasattr(raw, name), name
    assert set(syms) == set(lib.SIGNATURES)


@pytest.mark.parametrize("n", [1, 2, 7, 10, 35, 55, 101, 150])
def test_gauss_hermite_against_numpy(lib, n):
    x, w = lib.gauss_hermite(n)
    xl, wl = np.polynomial.hermite.hermgauss(n)
    assert np.max(np.abs(x - xl)) < 2e-13 * max(1.0, abs(xl).max())
    assert np.max(np.abs(w - wl / np.sqrt(np.pi))) < 1e-15 + 1e-12 * w.max()
    assert abs(w.sum() - 1.0) < 1e-13


def test_gauss_hermite_rejects_bad_order(lib):
    for n in (0, -3, 151):
        with pytest.raises(lib.FkError):
            lib.gauss_hermite(n)


@pytest.mark.parametrize("args", [(-5.0, 5.0, 0.2, 0.2, 10.0), (-10.0, 30.0, 0.05, 0.05, 10.0),
                                  (-1.0, 2.0, 0.1, 0.1, 1.3)])
def test_contour_matches_oracle(lib, args):
    dims, z, w = lib.contour_build(*args)
    zo, wo = ocontour.points(*args)
    assert dims == ocontour.sizes(*args)
    assert np.max(np.abs(z - zo)) < 1e-12 and np.max(np.abs(w - wo)) < 1e-15


@pytest.mark.parametrize("args", [(-5.0, 5.0, 0.3, 0.2, 10.0), (5.0, -5.0, 0.2, 0.2, 10.0),
                                  (-5.0, 5.0, 0.2, 0.0, 10.0), (-5.0, 5.0, 0.2, 0.3, 10.0)])
def test_contour_rejects_bad_input(lib, args):
    with pytest.raises(lib.FkError) as e:
        lib.contour_build(*args)
    assert e.value.status == lib.FK_EINVAL


def test_status_strings(lib):
    assert lib.status_string(lib.FK_ESINGULAR) == "FK_ESINGULAR"
    assert lib.status_string(12345) == "FK_UNKNOWN"


def test_create_rejects_bad_model(lib):
    with pytest.raises(lib.FkError) as e:
        lib.Context(-5, 5, 0.2, 0.2, 10, 0.5, 1.0, w1=1.5)
    assert e.value.status in (lib.FK_EINVAL, lib.FK_EDEVICE)


def test_create_rejects_averaged_rule_beyond_150_points(lib):
    """The N / N+1 average needs N + 1 <= 150 (the host rule's limit); the
    check runs before any device call."""
    with pytest.raises(lib.FkError) as e:
        lib.Context(-5, 5, 0.2, 0.2, 10, 0.5, 1.0, n_eps=150, n_ebar=10, gh_average=True)
    assert e.value.status == lib.FK_EINVAL


def test_create_rejects_contour_beyond_5120_points(lib):
    """N_c = 2 * 2550 + 22 = 5122 exceeds the inversion's largest matrix
    (5120); the check runs before any device call."""
    with pytest.raises(lib.FkError) as e:
        lib.Context(-5, 250, 0.1, 0.1, 2.2, 0.5, 1.0)
    assert e.value.status == lib.FK_EINVAL


def _gauss_jordan_block(x, cols, candidates):
    """In-place Gauss-Jordan elimination of the columns `cols` of x with partial
    pivoting among `candidates`; returns the pivot rows in pivot order."""
    piv = []
    for c in cols:
        free = [r for r in candidates if r not in piv]
        p = max(free, key=lambda r: abs(x[r, c].real) + abs(x[r, c].imag))
        piv.append(p)
        inv = 1.0 / x[p, c]
        ps = x[p, :] * inv
        ps[c] = inv
        for r in range(x.shape[0]):
            if r != p:
                m = x[r, c]
                x[r, :] -= m * ps
                x[r, c] = -m * inv
        x[p, :] = ps
    return piv


def test_deferred_rows_block_identity():
    """The identity the panel relies on when it leaves out the rows pivoted in
    earlier blocks: after eliminating a block of columns P with pivot rows R,
    every other row r holds X[r, P] = -X0[r, P] X[R, P], and X[R, P] (rows in
    pivot order) is the inverse of X0[R, P].  Checked on a random complex
    matrix, with the blocked inverse assembled this way equal to numpy's."""
    rng = np.random.default_rng(11)
    n, w = 24, 8
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    x = a.copy()
    done = []
    for j0 in range(0, n, w):
        cols = list(range(j0, j0 + w))
        x0 = x.copy()
        cand = [r for r in range(n) if r not in done]
        full = x.copy()
        piv = _gauss_jordan_block(full, cols, cand)
        minv = full[np.ix_(piv, cols)]
        np.testing.assert_allclose(minv, np.linalg.inv(x0[np.ix_(piv, cols)]),
                                   rtol=1e-12, atol=1e-12)
        for r in done:
            np.testing.assert_allclose(full[r, cols], -x0[r, cols] @ minv,
                                       rtol=1e-12, atol=1e-12)
        x = full
        done += piv
    # inv(A)[a][b] = X[piv[a]][rowcol[b]]
    rowcol = np.empty(n, int)
    rowcol[done] = np.arange(n)
    inv = x[np.ix_(done, rowcol)]
    np.testing.assert_allclose(inv, np.linalg.inv(a), rtol=1e-10, atol=1e-12)


def test_spectral_entry_points_reject_null_arguments(lib):
    """fk_wigner_dos and fk_equal_time_moments check their arguments before
    any device call: a NULL context or array, or empty sizes, give FK_EINVAL."""
    L = lib.library()
    ti = (ctypes.c_int * 1)(0)
    om = (ctypes.c_double * 1)(0.0)
    out = (ctypes.c_double * 6)()
    assert L.fk_wigner_dos(None, 1, ti, 1, om, out) == lib.FK_EINVAL
    assert L.fk_equal_time_moments(None, 1, ti, out) == lib.FK_EINVAL
    assert L.fk_get_zeroth_moment(None, out) == lib.FK_EINVAL


@pytest.mark.parametrize("convention,w1", [("symmetric", 0.5), ("paper", 0.5),
                                            ("symmetric", 0.3)])
def test_impurity_update_single_inversion_identity(convention, w1):
    """The library's impurity update needs one inversion instead of four:
    with A_m = G0^-1 + d_m S (the point-split shifts, S[j][j-1] = 1,
    S[0][n-1] = -1) and C = (1 - w1) A_1 + w1 A_0 = G0^-1 + d_c S, one has
    [(1 - w1) A_0^-1 + w1 A_1^-1]^-1 = A_1 C^-1 A_0, hence
    Sigma_new W = -h S + w1 (1 - w1) (d0 - d1)^2 S C^-1 S with
    h = (1 - w1) d0 + w1 d1, and C^-1 = X (I + Y X)^-1 with X = G_loc W,
    Y = Sigma W + d_c S.  Checked against the oracle's update (the paper's
    sequence of inversions) on a random contour matrix."""
    from oracle import contour as oc, impurity
    rng = np.random.default_rng(17)
    z, w = oc.points(-1.0, 1.0, 0.2, 0.2, 1.0)
    n = len(w)
    gloc = 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) \
        + 0.5j * np.eye(n)
    sigma = 0.1 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    u, mu = 1.3, (0.0 if convention == "symmetric" else 0.65)
    ref = impurity.update(gloc, sigma, w, mu, u, w1, convention)
    d0, d1 = impurity.shifts(u, convention)
    s = np.zeros((n, n))
    s[np.arange(1, n), np.arange(0, n - 1)] = 1.0
    s[0, n - 1] = -1.0
    g0inv = np.linalg.inv(gloc * w[None, :]) + sigma * w[None, :]
    dc = (1 - w1) * d1 + w1 * d0
    h = (1 - w1) * d0 + w1 * d1
    cinv = np.linalg.inv(g0inv + dc * s)
    new_r = -h * s + w1 * (1 - w1) * (d0 - d1) ** 2 * (s @ cinv @ s)
    np.testing.assert_allclose(new_r / w[None, :], ref, rtol=1e-10, atol=1e-10)
    # and the single-inversion form the library takes:
    # C^-1 = (X^-1 + Y)^-1 = X (I + Y X)^-1, X = G_loc W, Y = Sigma W + d_c S
    x = gloc * w[None, :]
    y = sigma * w[None, :] + dc * s
    cinv1 = x @ np.linalg.inv(np.eye(n) + y @ x)
    new_r1 = -h * s + w1 * (1 - w1) * (d0 - d1) ** 2 * (s @ cinv1 @ s)
    np.testing.assert_allclose(new_r1 / w[None, :], ref, rtol=1e-10, atol=1e-10)


def test_extrapolate_to_zero_reproduces_polynomials(lib):
    """fk_extrapolate_to_zero (host): through k steps it returns the value at
    step 0 of any polynomial of degree < k exactly, elementwise, for real and
    complex data; invalid steps are refused."""
    hs = [0.2, 0.1, 0.05]
    t = np.linspace(-1.0, 1.0, 7)
    c0, c1, c2 = np.sin(t), np.cos(t) + 0.5j * t, t ** 2 - 1j
    vals = [c0 + c1 * h + c2 * h * h for h in hs]
    got = lib.extrapolate_to_zero(hs, vals)
    assert np.max(np.abs(got - c0)) < 1e-13
    real = lib.extrapolate_to_zero(hs[:2], [np.array([1 + h, 2 - 3 * h]) for h in hs[:2]])
    assert np.allclose(real, [1.0, 2.0], atol=1e-14) and real.dtype == np.float64
    for bad in ([0.1, 0.1], [0.1, -0.2], [0.1, float("nan")]):
        with pytest.raises(lib.FkError):
            lib.extrapolate_to_zero(bad, [np.zeros(3)] * len(bad))


def _gauss_jordan_by_plan(lib, a, nb=128):
    """The blocked in-place Gauss-Jordan inversion in numpy, with the library's
    own schedule (fk_update_plan): per outer block the columns are eliminated
    one by one over all rows (pivot: largest |re| + |im| among rows not yet
    pivoted), the block's pivot rows are copied to the side buffer, and the
    three update phases of the plan are applied as C <- mask(C) + M B.  Rows
    are never swapped: inv(A)[i][j] = X[piv[i]][rowcol[j]]."""
    n = a.shape[0]
    x = a.astype(np.complex128).copy()
    piv = -np.ones(n, dtype=int)
    rowcol = -np.ones(n, dtype=int)
    side = np.zeros((8 * nb, n), dtype=np.complex128)
    nout = (n + nb - 1) // nb
    for s in range(nout):
        j0, w = s * nb, min(nb, n - s * nb)
        cols = slice(j0, j0 + w)
        for c in range(j0, j0 + w):
            key = np.abs(x[:, c].real) + np.abs(x[:, c].imag)
            key[rowcol >= 0] = -1.0
            p = int(np.argmax(key))
            piv[c], rowcol[p] = p, c
            inv = 1.0 / x[p, c]
            q = x[p, cols] * inv
            m = x[:, c].copy()
            x[:, cols] -= np.outer(m, q)
            x[p, cols] = q
            x[:, c] = -m * inv
            x[p, c] = inv
        brow = lib.update_plan(n, s, 0)["brow"]
        side[brow:brow + w] = x[piv[j0:j0 + w]]
        for ph in range(3):
            pl = lib.update_plan(n, s, ph)
            blk = np.arange(n) // nb
            if ph < 2:
                take = (blk >= pl["lo"]) & (blk <= pl["hi"])
            else:
                take = ((blk < pl["lo"]) | (blk > pl["hi"])) & (pl["kw"] > 0)
            if not take.any():
                continue
            m0, kw, b0 = pl["jb"] * nb, pl["kw"], pl["b0"]
            keep = ~((rowcol >= m0) & (rowcol < m0 + kw))
            x[:, take] = x[:, take] * keep[:, None] + x[:, m0:m0 + kw] @ side[b0:b0 + kw][:, take]
    return x[piv][:, rowcol]


@pytest.mark.parametrize("n", [100, 300, 520, 700, 1050, 1800])
def test_update_plan_inverts(lib, n):
    """The library's schedule of the batched inversion (outer blocks of 128
    columns grouped from the last block, delayed trailing updates), applied in
    numpy, gives the inverse: against numpy.linalg.inv for block counts that
    leave every group shape (1, 3, 5, 6, 9 and 15 blocks, ragged last blocks)."""
    rng = np.random.default_rng(n)
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    got = _gauss_jordan_by_plan(lib, a)
    ref = np.linalg.inv(a)
    assert np.max(np.abs(got - ref)) < 1e-9 * np.max(np.abs(ref))


def test_update_plan_groups_and_errors(lib):
    """Groups of up to four blocks counted from the last: at N_c = 1800 (15
    blocks) the trailing updates run after blocks 2, 6, 10 and 14, with K = 384,
    512, 512 and 392; invalid arguments are refused."""
    trail = [(s, lib.update_plan(1800, s, 2)) for s in range(15)]
    done = [(s, p["kw"], p["jb"]) for s, p in trail if p["kw"] > 0]
    assert done == [(2, 384, 0), (6, 512, 3), (10, 512, 7), (14, 392, 11)]
    p = lib.update_plan(1800, 5, 0)      # third block of the group 3 .. 6
    assert (p["jb"], p["kw"], p["b0"], p["lo"], p["hi"], p["brow"]) == (5, 128, 256, 3, 4, 256)
    p = lib.update_plan(1800, 5, 1)      # the next block with the group so far
    assert (p["jb"], p["kw"], p["lo"], p["hi"]) == (3, 384, 6, 6)
    for bad in ((0, 0, 0), (1800, -1, 0), (1800, 0, 3), (6000, 0, 0)):
        with pytest.raises(lib.FkError):
            lib.update_plan(*bad)
