"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the identity it checks and the passage of the paper (Freericks,
arXiv:0711.0999, Sec. II) that fixes it.  None of them re-types the oracle's own
formula: they compare it with closed forms, special cases that reduce to a
textbook or library result, invariants, or a high-precision brute force.
"""
import math

import numpy as np
import pytest

from oracle import contour, green, impurity, lattice, quadrature, dmft


# ----------------------------------------------------------------- quadrature
@pytest.mark.parametrize("n", [1, 2, 5, 10, 35, 55])
def test_gauss_hermite_matches_library(n):
    """Gauss-Hermite rule for the Gaussian DOS of eq. (joint_dos): nodes and
    normalized weights equal numpy's hermgauss (weights / sqrt(pi))."""
    x, w = quadrature.hermite_rule(n)
    xl, wl = np.polynomial.hermite.hermgauss(n)
    assert np.max(np.abs(x - xl)) < 1e-12 * max(1.0, np.max(np.abs(xl)))
    assert np.max(np.abs(w - wl / math.sqrt(math.pi))) < 1e-14
    assert abs(w.sum() - 1.0) < 1e-14


@pytest.mark.parametrize("n", [3, 10, 55])
def test_gauss_hermite_moments_exact(n):
    """Gaussian moments int x^{2m} e^{-x^2} dx / sqrt(pi) = (2m-1)!!/2^m are
    integrated exactly for 2m <= 2n - 1."""
    x, w = quadrature.hermite_rule(n)
    for m in range(0, min(n, 8)):
        exact = float(np.prod(np.arange(1, 2 * m, 2))) / 2.0 ** m
        got = float(np.sum(w * x ** (2 * m)))
        assert abs(got - exact) < 1e-12 * max(1.0, exact)
        assert abs(float(np.sum(w * x ** (2 * m + 1)))) < 1e-12 * max(1.0, exact)


def test_product_grid_weights_sum_to_one():
    eps, ebar, rho = quadrature.product_grid(10, 7)
    assert eps.shape == ebar.shape == rho.shape == (70,)
    assert abs(rho.sum() - 1.0) < 1e-14
    # k = a * n_ebar + b
    x10, _ = quadrature.hermite_rule(10)
    x7, _ = quadrature.hermite_rule(7)
    assert eps[3 * 7 + 5] == x10[3] and ebar[3 * 7 + 5] == x7[5]


# -------------------------------------------------------------------- contour
def test_contour_branch_endpoints():
    """Sec. II: the upper branch runs t_min .. t_max - dt, the lower t_max ..
    t_min + dt, the imaginary one t_min .. t_min - i beta + i dtau."""
    z, w = contour.points(-5.0, 5.0, 0.2, 0.2, 10.0)
    n_t, n_tau, n_c = contour.sizes(-5.0, 5.0, 0.2, 0.2, 10.0)
    assert (n_t, n_tau, n_c) == (50, 50, 150)
    assert z[0] == -5.0 and abs(z[n_t - 1] - 4.8) < 1e-12
    assert z[n_t] == 5.0 and abs(z[2 * n_t - 1] - (-4.8)) < 1e-12
    assert z[2 * n_t] == -5.0 and abs(z[-1] - complex(-5.0, -9.8)) < 1e-12
    # leftpoint rule: the real branches cancel, the imaginary one gives -i beta
    assert abs(w[:2 * n_t].sum()) < 1e-12
    assert abs(w[2 * n_t:].sum() - complex(0, -10.0)) < 1e-12
    with pytest.raises(ValueError):
        contour.sizes(-5.0, 5.0, 0.3, 0.2, 10.0)


@pytest.mark.parametrize("mu", [0.0, 0.3, -0.7])
def test_det_m_partition_function(mu):
    """eq. (det): det M is the partition function of a spinless level.  The
    discrete value is 1 + prod_j (1 + i W_j mu) = 1 + (1 + dt^2 mu^2)^{N_t}
    (1 + dtau mu)^{N_tau} (the printed sign prefactor is taken as a misprint),
    and it tends to 1 + e^{beta mu} as dt, dtau -> 0."""
    t_min, t_max, beta = -5.0, 5.0, 10.0
    errs = []
    for dt in (0.2, 0.1, 0.05):
        z, w = contour.points(t_min, t_max, dt, dt, beta)
        n_t, n_tau, _ = contour.sizes(t_min, t_max, dt, dt, beta)
        det = np.linalg.det(contour.m_matrix(w, mu))
        closed = 1.0 + (1.0 + dt * dt * mu * mu) ** n_t * (1.0 + dt * mu) ** n_tau
        assert abs(det - closed) < 1e-9 * abs(closed)
        errs.append(abs(det - (1.0 + math.exp(beta * mu))) / (1.0 + math.exp(beta * mu)))
    if mu != 0.0:
        assert errs[0] > errs[1] > errs[2]
        assert errs[1] / errs[2] > 1.6   # first order in dt
    else:
        assert max(errs) < 1e-12


def test_shift_operator_is_point_split_identity():
    """i W^-1 (M(mu') - M(mu)) = (mu' - mu) S with S the point-split delta:
    S[j, j-1] = +1 and the antiperiodic corner S[0, N-1] = -1."""
    z, w = contour.points(-1.0, 1.0, 0.2, 0.25, 1.0)
    n = len(w)
    s = np.zeros((n, n), dtype=np.complex128)
    s[np.arange(1, n), np.arange(n - 1)] = 1.0
    s[0, n - 1] = -1.0
    got = contour.shift_operator(w, 0.4, 0.4 - 0.75)
    assert np.max(np.abs(got - (-0.75) * s)) < 1e-14


# ---------------------------------------------------------------- noninteracting
def test_g0_is_inverse_of_paper_operator_at_zero_energy():
    """At eps = ebar = mu = 0 the sampled G0 of eq. (g_contour_non_final2) with
    theta_c(t, t) = 1 is exactly the inverse of the paper's discrete operator
    W [i d/dt] delta W = i M (the M display at mu = 0); theta_c(t, t) = 0 would
    fail this."""
    for (a, b, dt, dtau, beta) in [(-1.0, 1.0, 0.2, 0.2, 1.0), (-5.0, 5.0, 0.2, 0.2, 10.0)]:
        z, w = contour.points(a, b, dt, dtau, beta)
        n_t, _, _ = contour.sizes(a, b, dt, dtau, beta)
        g0 = green.g0_matrix(z, n_t, 1.0, 0.0, beta, 0.0, 0.0)
        ref = np.linalg.inv(1j * contour.m_matrix(w, 0.0))
        assert np.max(np.abs(g0 - ref)) < 1e-12


@pytest.mark.parametrize("eps,ebar,mu,efield", [
    (0.3, -0.8, 0.0, 1.0), (-3.1, 2.2, 0.0, 2.0), (7.5, 0.1, 0.2, 0.5),
    (-9.2, -4.0, 0.0, 4.0), (1.1, 1.7, -0.3, 0.0)])
def test_g0_inverse_is_bidiagonal_plus_corner(eps, ebar, mu, efield):
    """The sampled G0 = i D (f 1 1^T - Theta) D^-1 with D = diag(e^{-i phi + i mu z})
    and Theta the lower triangle including the diagonal.  Sherman-Morrison on
    Theta - f 1 1^T gives the exact sparse inverse
        G0^-1 = i D [I - P + e^{-beta (eps - mu)} e_0 e_{N-1}^T] D^-1
    (P the unit subdiagonal).  A wrong phase sign, occupation or diagonal
    convention in the generator makes the numerical inverse dense."""
    beta = 10.0
    z, w = contour.points(-2.0, 3.0, 0.1, 0.25, beta)
    n_t, _, n_c = contour.sizes(-2.0, 3.0, 0.1, 0.25, beta)
    g0 = green.g0_matrix(z, n_t, efield, mu, beta, eps, ebar)
    inv = np.linalg.inv(g0)
    # closed form built from the antiderivative evaluated independently here
    t = z.real
    alpha = z.copy()
    gamma = np.zeros(n_c, dtype=np.complex128)
    if efield != 0.0:
        on = (np.arange(n_c) < 2 * n_t) & (t > 0)
        alpha[on] = np.sin(efield * t[on]) / efield
        gamma[on] = -2.0 * np.sin(0.5 * efield * t[on]) ** 2 / efield
    ex = -1j * (eps * alpha + ebar * gamma) + 1j * mu * z
    ref = np.zeros((n_c, n_c), dtype=np.complex128)
    ref[np.arange(n_c), np.arange(n_c)] = 1j
    ref[np.arange(1, n_c), np.arange(n_c - 1)] = -1j * np.exp(ex[1:] - ex[:-1])
    ref[0, n_c - 1] = 1j * np.exp(-beta * (eps - mu) + ex[0] - ex[-1])
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(inv - ref)) < 1e-10 * scale
    # |G0| <= 1 entrywise (bounded generator)
    assert np.max(np.abs(g0)) <= 1.0 + 1e-12


def test_u0_bloch_oscillation_closed_form():
    """U = 0 (Sec. III: undamped Bloch oscillations).  With Sigma = 0 the
    lesser function at equal times is i f(eps - mu) at every k, so n(t) =
    sum_a w_a f(x_a - mu) (= 1/2 at mu = 0), and with the velocity at the
    shifted momentum j(t) = -K sin(E t) theta(t), K = sum_a w_a x_a f(x_a - mu),
    exactly at any dt.  The period is 2 pi / E."""
    p = dmft.Problem(t_min=-5.0, t_max=5.0, dt=0.2, dtau=0.2, beta=10.0,
                     u=0.0, e_field=1.0, n_eps=10, n_ebar=10)
    z, w, n_t, eps, ebar, rho = p.grid()
    n_c = len(z)
    gloc, cur, _ = dmft.lattice_only(p, np.zeros((n_c, n_c), dtype=np.complex128))
    x, wa = np.polynomial.hermite.hermgauss(10)
    wa = wa / math.sqrt(math.pi)
    f = 1.0 / (1.0 + np.exp(10.0 * x))
    kin = float(np.sum(wa * x * f))
    assert kin < 0.0
    t = z[:n_t].real
    expect = np.where(t > 0, -kin * np.sin(1.0 * t), 0.0)
    assert np.max(np.abs(cur - expect)) < 1e-13
    assert np.max(np.abs(lattice.density(gloc, n_t) - 0.5)) < 1e-13
    # impurity update returns Sigma = 0 at U = 0
    s_new = impurity.update(gloc, np.zeros_like(gloc), w, 0.0, 0.0, 0.5)
    assert np.max(np.abs(s_new)) < 1e-9


@pytest.mark.parametrize("efield", [0.5, 2.0])
def test_retarded_gaussian_average(efield):
    """First lattice step from Sigma = 0: G^R_loc(t, t') = G^> - G^< =
    -i <exp(-i eps da - i ebar dg)>_rho = -i exp(-(da^2 + dg^2)/4) for t > t',
    the characteristic function of the Gaussian DOS of eq. (joint_dos), with
    da, dg the differences of sin(E t)/E and (cos(E t) - 1)/E (t > 0) or t."""
    p = dmft.Problem(t_min=-2.0, t_max=4.0, dt=0.1, dtau=0.2, beta=4.0, u=0.0,
                     e_field=efield, n_eps=20, n_ebar=20)
    z, w, n_t, eps, ebar, rho = p.grid()
    gl, _, _ = dmft.lattice_only(p, np.zeros((len(z),) * 2, dtype=np.complex128))
    t = z[:n_t].real
    a = np.where(t > 0, np.sin(efield * t) / efield, t)
    g = np.where(t > 0, (np.cos(efield * t) - 1.0) / efield, 0.0)
    worst = 0.0
    for i in range(n_t):
        for j in range(i):
            gr = gl[2 * n_t - i if i else 2 * n_t, j] - gl[i, 2 * n_t - j if j else 2 * n_t]
            ex = -1j * math.exp(-((a[i] - a[j]) ** 2 + (g[i] - g[j]) ** 2) / 4.0)
            worst = max(worst, abs(gr - ex))
    assert worst < 1e-10


# -------------------------------------------------------------------- impurity
def _lattice_gloc(u=1.0, efield=1.0):
    p = dmft.Problem(t_min=-1.0, t_max=1.0, dt=0.2, dtau=0.25, beta=2.0, u=u,
                     e_field=efield, n_eps=4, n_ebar=4)
    z, w, n_t, eps, ebar, rho = p.grid()
    rng = np.random.default_rng(5)
    n = len(z)
    sig = 0.1 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    gl, _, _ = dmft.lattice_only(p, sig)
    return gl, sig, w


IMPURITY_FORMS = [pytest.param("update", id="complex128"),
                  pytest.param("update_extended", id="long-double")]


@pytest.mark.parametrize("form", IMPURITY_FORMS)
def test_impurity_empty_and_full_f_site(form):
    """eq. (g_imp_solve) with <w1> = 0 or 1 is a single level in a static
    potential, so Sigma is that potential whatever G_loc and Sigma were:
    Sigma W = -(mu0 - mu) S for w1 = 0 and -(mu1 - mu) S for w1 = 1 (S the
    point-split delta).  Symmetric convention: -U/2 and +U/2; the paper's
    literal convention: 0 and +U.  Both evaluations of the update: complex128
    and long double."""
    update = getattr(impurity, form)
    gl, sig, w = _lattice_gloc()
    n = len(w)
    s = np.zeros((n, n), dtype=np.complex128)
    s[np.arange(1, n), np.arange(n - 1)] = 1.0
    s[0, n - 1] = -1.0
    u = 1.3
    for w1, conv, expect in [(0.0, "symmetric", -0.5 * u), (1.0, "symmetric", 0.5 * u),
                             (0.0, "paper", 0.0), (1.0, "paper", u)]:
        got = update(gl, sig, w, 0.0, u, w1, conv) * w[None, :]
        assert np.max(np.abs(got - expect * s)) < 1e-9, (w1, conv)


@pytest.mark.parametrize("form", IMPURITY_FORMS)
def test_impurity_u0_returns_zero(form):
    gl, sig, w = _lattice_gloc()
    got = getattr(impurity, form)(gl, sig, w, 0.0, 0.0, 0.5)
    assert np.max(np.abs(got)) < 1e-8


def test_extended_inverse_of_the_sparse_propagator_inverse():
    """The long-double Gauss-Jordan inverse (impurity_ext.c) returns the
    sampled noninteracting G0 from its exact bidiagonal-plus-corner inverse
    i D (I - P + e^{-beta(eps - mu)} e_0 e_{N-1}^T) D^-1 (Sherman-Morrison on
    eq. g_contour_non_final2), and A X = I for a random matrix (to the rounding
    of the complex128 result)."""
    z, w = contour.points(-1.0, 1.5, 0.1, 0.25, 2.0)
    n_t = contour.sizes(-1.0, 1.5, 0.1, 0.25, 2.0)[0]
    eps, ebar, mu, beta = 0.4, -0.7, 0.1, 2.0
    g0 = green.g0_matrix(z, n_t, 1.3, mu, beta, eps, ebar)
    alpha, gamma = green.phase_tables(z, n_t, 1.3)
    d = np.exp(-1j * (eps * alpha + ebar * gamma) + 1j * mu * z)
    n = len(z)
    core = np.eye(n, dtype=np.complex128)
    core[np.arange(1, n), np.arange(n - 1)] = -1.0
    core[0, n - 1] = np.exp(-beta * (eps - mu))
    g0inv = 1j * d[:, None] * core / d[None, :]
    got = impurity.inverse_extended(g0inv)
    assert np.max(np.abs(got - g0)) < 1e-14
    rng = np.random.default_rng(8)
    a = rng.standard_normal((40, 40)) + 1j * rng.standard_normal((40, 40))
    x = impurity.inverse_extended(a)
    assert np.max(np.abs(x @ a - np.eye(40))) < 1e-13


def test_extended_update_agrees_with_complex128_on_a_small_contour():
    """On a small contour the complex128 update loses little to the Dyson
    subtraction, so the long-double evaluation of the same sequence agrees
    with it to the complex128 rounding; both conventions and w1 != 1/2."""
    gl, sig, w = _lattice_gloc()
    for conv, w1 in (("symmetric", 0.5), ("paper", 0.3)):
        a = impurity.update(gl, sig, w, 0.0, 1.1, w1, conv)
        b = impurity.update_extended(gl, sig, w, 0.0, 1.1, w1, conv)
        assert np.max(np.abs(a - b)) / np.max(np.abs(b)) < 1e-12


# ------------------------------------------------------------------- lattice
def test_static_sigma_shifts_chemical_potential():
    """A static potential V enters Dyson's equation as Sigma = V delta, i.e.
    Sigma W = V S point-split; the lattice then describes free electrons at
    mu - V, so n(t) -> sum_a w_a f(x_a - mu + V) with an O(dt) error.  This
    fixes the weighting of both contour integrals in eq. (dyson): a single W
    leaves an O(1/dt) error."""
    v = 0.3
    errs = []
    for dt in (0.2, 0.1, 0.05):
        p = dmft.Problem(t_min=-1.0, t_max=1.0, dt=dt, dtau=dt, beta=2.0,
                         u=0.0, e_field=0.0, n_eps=8, n_ebar=1)
        z, w, n_t, eps, ebar, rho = p.grid()
        n = len(z)
        s = np.zeros((n, n), dtype=np.complex128)
        s[np.arange(1, n), np.arange(n - 1)] = 1.0
        s[0, n - 1] = -1.0
        sigma = v * s / w[None, :]
        gl, _, _ = dmft.lattice_only(p, sigma)
        x, wa = quadrature.hermite_rule(8)
        exact = float(np.sum(wa / (1.0 + np.exp(2.0 * (x + v)))))
        errs.append(np.max(np.abs(lattice.density(gl, n_t) - exact)))
    assert errs[0] < 0.1
    assert errs[0] / errs[1] > 1.6 and errs[1] / errs[2] > 1.6


def test_equilibrium_reduces_to_one_dimension():
    """E = 0 (eq. joint_dos remark): nothing depends on ebar, so the 2-D sum
    equals the 1-D sum over eps and the current vanishes."""
    rng = np.random.default_rng(3)
    base = dict(t_min=-1.0, t_max=1.0, dt=0.2, dtau=0.2, beta=2.0, u=1.0, e_field=0.0, n_eps=6)
    p1 = dmft.Problem(n_ebar=1, **base)
    p5 = dmft.Problem(n_ebar=5, **base)
    n = len(p1.grid()[0])
    sig = 0.2 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    g1, c1, _ = dmft.lattice_only(p1, sig)
    g5, c5, _ = dmft.lattice_only(p5, sig)
    assert np.max(np.abs(g1 - g5)) < 1e-13
    assert np.max(np.abs(c5)) < 1e-13


def test_equilibrium_fixed_point_is_time_translation_invariant():
    """At E = 0 the converged G_loc on the upper branch depends only on
    t - t' (the equilibrium state of the Keldysh boundary problem)."""
    p = dmft.Problem(t_min=-2.0, t_max=2.0, dt=0.2, dtau=0.2, beta=3.0, u=1.0,
                     e_field=0.0, n_eps=6, n_ebar=1)
    r = dmft.run(p, 60, tol=1e-12)
    assert r["deltas"][-1] < 1e-12
    g, n_t = r["gloc"], r["n_t"]
    d = max(abs(g[i + 1, j + 1] - g[i, j]) for i in range(n_t - 1) for j in range(n_t - 1))
    assert d < 1e-11
    assert np.max(np.abs(r["current"])) < 1e-13


def test_lattice_inverse_form_agrees():
    """G_k = (I - G0 Sigma_t)^-1 G0 equals (G0^-1 - Sigma_t)^-1 (operator
    Dyson equation G^-1 = G0^-1 - Sigma with the inverse rule of eq.
    (matrix_inverse_discrete)) and satisfies the right-hand Dyson equation
    G = G0 + G Sigma_t G0 as well."""
    p = dmft.Problem(t_min=-1.0, t_max=2.0, dt=0.1, dtau=0.25, beta=2.0, u=1.0,
                     e_field=1.5, n_eps=3, n_ebar=3)
    z, w, n_t, eps, ebar, rho = p.grid()
    n = len(z)
    rng = np.random.default_rng(11)
    sig = 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    st = lattice.weighted_sigma(sig, w)
    for k in range(len(eps)):
        gk = lattice.point_green(z, n_t, p.e_field, 0.0, p.beta, eps[k], ebar[k], st)
        g0 = green.g0_matrix(z, n_t, p.e_field, 0.0, p.beta, eps[k], ebar[k])
        alt = np.linalg.inv(np.linalg.inv(g0) - st)
        assert np.max(np.abs(gk - alt)) < 1e-11 * np.max(np.abs(gk))
        assert np.max(np.abs(gk - (g0 + gk @ st @ g0))) < 1e-11 * np.max(np.abs(gk))


def test_convergence_order_of_invariants():
    """U > 0 invariants that hold only in the continuum (Sec. III moments
    paragraph and the extrapolation paragraph): n(t) = 1/2 at half filling, the
    zeroth moment G^> - G^< = -i, and j(t < 0) = 0.  Their errors must shrink
    about linearly as dt = dtau halves."""
    res = []
    for dt in (0.2, 0.1, 0.05):
        p = dmft.Problem(t_min=-2.0, t_max=2.0, dt=dt, dtau=dt, beta=4.0, u=1.0,
                         e_field=1.0, n_eps=6, n_ebar=6)
        r = dmft.run(p, 80, tol=1e-10)
        n_t = r["n_t"]
        t = r["z"][:n_t].real
        res.append((np.max(np.abs(r["density"] - 0.5)),
                    np.max(np.abs(r["m0"] + 1j)),
                    np.max(np.abs(r["current"][t < 0]))))
    for q in range(3):
        e = [x[q] for x in res]
        assert e[0] > e[1] > e[2], (q, e)
        assert e[1] / e[2] > 1.5, (q, e)


# ------------------------------------------------------------ brute force
def test_mpmath_brute_force_one_iteration():
    """One full iteration (lattice step + impurity update) on a 12-point contour
    with a 2 x 2 rule, evaluated at 40 digits from the same discrete equations
    with mpmath: bounds the rounding of the complex128 oracle."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    t_min, t_max, dt, dtau, beta = -0.4, 0.4, 0.2, 0.2, 0.8
    u, efield, w1 = 1.0, 1.0, 0.5
    p = dmft.Problem(t_min=t_min, t_max=t_max, dt=dt, dtau=dtau, beta=beta,
                     u=u, e_field=efield, n_eps=2, n_ebar=2)
    z, w, n_t, eps, ebar, rho = p.grid()
    n = len(z)
    rng = np.random.default_rng(2)
    sig0 = 0.2 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    r = dmft.run(p, 1, sigma0=sig0)

    mpc = mp.mpc
    zs = []
    ws = []
    for j in range(n):
        if j < n_t:
            zs.append(mpc(mp.mpf(t_min) + j * mp.mpf(dt))); ws.append(mpc(mp.mpf(dt)))
        elif j < 2 * n_t:
            zs.append(mpc(mp.mpf(t_max) - (j - n_t) * mp.mpf(dt))); ws.append(mpc(-mp.mpf(dt)))
        else:
            zs.append(mpc(mp.mpf(t_min), -(j - 2 * n_t) * mp.mpf(dtau))); ws.append(mpc(0, -mp.mpf(dtau)))
    # 2-point Gauss-Hermite: nodes +-1/sqrt(2), normalized weights 1/2
    nodes = [-1 / mp.sqrt(2), 1 / mp.sqrt(2)]
    wts = [mp.mpf(1) / 2, mp.mpf(1) / 2]
    sig = mp.matrix(n, n)
    for i in range(n):
        for j in range(n):
            sig[i, j] = mpc(float(sig0[i, j].real), float(sig0[i, j].imag))
    sig_t = mp.matrix(n, n)
    for i in range(n):
        for j in range(n):
            sig_t[i, j] = ws[i] * sig[i, j] * ws[j]

    def phi(j, e, eb):
        zz = zs[j]
        if j < 2 * n_t and mp.re(zz) > 0:
            tt = mp.re(zz)
            return e * mp.sin(efield * tt) / efield + eb * (mp.cos(efield * tt) - 1) / efield
        return e * zz

    gl = mp.matrix(n, n)
    for a in range(2):
        for b in range(2):
            e, eb = nodes[a], nodes[b]
            f = 1 / (1 + mp.exp(beta * e))
            g0 = mp.matrix(n, n)
            for i in range(n):
                for j in range(n):
                    occ = f - (1 if i >= j else 0)
                    g0[i, j] = 1j * occ * mp.exp(-1j * (phi(i, e, eb) - phi(j, e, eb)))
            gk = (mp.eye(n) - g0 * sig_t) ** -1 * g0
            gl += wts[a] * wts[b] * gk
    assert max(abs(complex(gl[i, j]) - r["gloc"][i, j]) for i in range(n) for j in range(n)) < 1e-12

    gr = mp.matrix(n, n)
    sr = mp.matrix(n, n)
    shift = mp.matrix(n, n)
    for i in range(n):
        for j in range(n):
            gr[i, j] = gl[i, j] * ws[j]
            sr[i, j] = sig[i, j] * ws[j]
    for j in range(1, n):
        shift[j, j - 1] = 1
    shift[0, n - 1] = -1
    g0inv = gr ** -1 + sr
    gimp = (1 - w1) * (g0inv + (u / 2) * shift) ** -1 + w1 * (g0inv - (u / 2) * shift) ** -1
    snew = g0inv - gimp ** -1
    worst = 0.0
    for i in range(n):
        for j in range(n):
            worst = max(worst, abs(complex(snew[i, j] / ws[j]) - r["sigma"][i, j]))
    assert worst < 1e-10 * max(1.0, float(np.max(np.abs(r["sigma"]))))


def test_c1_reference_delta_history():
    """C1 (t in [-5, 5], dt = dtau = 0.2, beta = 10, U = 0.5, E = 1, 10 x 10
    rule, Sigma = 0): plain substitution contracts; ten iterations bring the
    change of G_loc to ~5e-8."""
    p = dmft.Problem(t_min=-5.0, t_max=5.0, dt=0.2, dtau=0.2, beta=10.0,
                     u=0.5, e_field=1.0, n_eps=10, n_ebar=10)
    r = dmft.run(p, 10)
    d = r["deltas"]
    assert len(d) == 10
    assert all(d[i + 1] < d[i] for i in range(1, 9))
    assert 1e-8 < d[-1] < 1e-7


@pytest.mark.parametrize("form", IMPURITY_FORMS)
def test_impurity_second_order_perturbation(form):
    """Weak coupling of eq. (g_imp_solve): expanding both resolvents in the
    shifts +-U/2 gives the textbook Falicov-Kimball result
        Sigma = U (w1 - 1/2) delta + U^2 w1 (1 - w1) G0_eff + O(U^3),
    with G0_eff = [G_loc^-1 + Sigma]^-1 of eq. (effective_medium) and delta the
    point-split S.  Checks the effective medium (including the +Sigma term) and
    the mixing weights; the remainder must fall as U^3."""
    gl, sig, w = _lattice_gloc()
    n = len(w)
    s = np.zeros((n, n), dtype=np.complex128)
    s[np.arange(1, n), np.arange(n - 1)] = 1.0
    s[0, n - 1] = -1.0
    g_r = gl * w[None, :]
    g0eff_r = np.linalg.inv(np.linalg.inv(g_r) + sig * w[None, :])
    w1 = 0.3
    rem = []
    for u in (0.02, 0.01):
        got = getattr(impurity, form)(gl, sig, w, 0.0, u, w1) * w[None, :]
        pred = u * (w1 - 0.5) * s + u * u * w1 * (1 - w1) * (s @ g0eff_r @ s)
        rem.append(np.max(np.abs(got - pred)))
    assert rem[0] / rem[1] > 6.0, rem


# ----------------------------------------------------------- warm-start net
def test_mlp_backprop_matches_finite_differences():
    """The numpy reference gradient of the warm-start network equals central
    finite differences of its loss (pins the backward pass)."""
    from oracle import mlp
    rng = np.random.default_rng(4)
    shapes = mlp.layer_shapes(7, 9, 4, 2)
    p = 0.4 * rng.standard_normal(mlp.n_params(shapes))
    x = rng.standard_normal((5, 7))
    t = rng.standard_normal((5, 2))
    loss, g = mlp.loss_and_grad(p, shapes, x, t)
    h = 1e-6
    idx = rng.choice(len(p), 40, replace=False)
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (mlp.loss_and_grad(p + e, shapes, x, t)[0] -
              mlp.loss_and_grad(p - e, shapes, x, t)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-7 * max(1.0, abs(fd))


def test_randomized_svd_recovers_low_rank_spectrum():
    """Probing with the top right singular vectors of a matrix, the randomized
    SVD returns exactly its leading singular values (library SVD); with random
    probes of a rank-r matrix it returns all r of them, the rest zero."""
    from oracle import warmstart
    rng = np.random.default_rng(6)
    n, r = 40, 6
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    u, sv_full, vh = np.linalg.svd(a)
    sv = warmstart.randomized_singular_values(a, vh.conj().T[:, :r])
    assert np.max(np.abs(sv - sv_full[:r])) < 1e-10 * sv_full[0]
    lo = (rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))) @ \
        (rng.standard_normal((r, n)) + 1j * rng.standard_normal((r, n)))
    s2 = warmstart.randomized_singular_values(lo, rng.standard_normal((n, r + 3)))
    s_lib = np.linalg.svd(lo, compute_uv=False)
    assert np.max(np.abs(s2[:r] - s_lib[:r])) < 1e-10 * s_lib[0]
    assert np.all(s2[r:] < 1e-10 * s2[0])


def test_bf16_rounding_is_nearest_even():
    """bfloat16 keeps 7 explicit significand bits: values near 1 are 1 + k/128.
    Halfway cases go to the even k; anything above halfway rounds up."""
    from oracle import mlp
    x = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -20,
                  -(1 + 2.0 ** -8), 3.0, 2.0 ** -130], dtype=np.float32)
    want = [1.0, 1.0, 1 + 2.0 ** -6, 1 + 2.0 ** -7, -1.0, 3.0, 2.0 ** -130]
    assert list(mlp.round_bf16(x)) == want


def test_bf16_forward_is_exact_on_bf16_values():
    """With weights and inputs that bfloat16 represents exactly (small dyadic
    values) and a linear network of one layer, the bf16 product equals the
    exact one; on generic values it differs by about 2^-8 relative."""
    from oracle import mlp
    rng = np.random.default_rng(9)
    shapes = mlp.layer_shapes(16, 8, 2, 3)
    p = rng.integers(-8, 9, mlp.n_params(shapes)) / 16.0
    x = rng.integers(-8, 9, (4, 16)) / 8.0
    w, b = mlp.unpack(p, shapes)[0]
    y0 = x @ w.T + b
    y, _ = mlp.forward(p, shapes[:1], x, bf16=True)
    assert np.array_equal(y, y0)
    pg = rng.standard_normal(mlp.n_params(shapes))
    xg = rng.standard_normal((64, 16))
    ya, _ = mlp.forward(pg, shapes, xg)
    yb, _ = mlp.forward(pg, shapes, xg, bf16=True)
    rel = np.max(np.abs(ya - yb)) / np.max(np.abs(ya))
    assert 1e-4 < rel < 3e-2


def test_weighted_sketch_of_constant_kernel_is_contour_length():
    """Sigma = 1 on every pair is rank one: D 1 D = d d^T with d_j = sqrt|W_j|, so
    its one singular value is sum_j |W_j| = 2 (t_max - t_min) + beta for the
    rectangle weights of the contour (Sec. II), at every step size."""
    from oracle import warmstart
    rng = np.random.default_rng(12)
    for dt, dtau in [(0.5, 0.25), (0.1, 0.05), (0.025, 0.1)]:
        z, w = contour.points(-2.0, 3.0, dt, dtau, 1.5)
        n = len(z)
        sv = warmstart.weighted_sketch(np.ones((n, n), complex), w,
                                       rng.standard_normal((n, 4)))
        assert abs(sv[0] - (2 * 5.0 + 1.5)) < 1e-11
        assert np.all(sv[1:] < 1e-10)


def test_weighted_sketch_converges_with_step_size():
    """For the separable kernel Sigma(z, z') = f(z) conj(f(z')) with f = cos(Re z)
    + i Im z the single singular value is the squared L2 norm of f along the
    contour; the rectangle sums approach it at first order in the step."""
    from oracle import warmstart
    t0, t1, beta = -1.0, 2.0, 1.0
    # exact: two real branches of int cos^2 t dt, imaginary branch
    # int_0^beta (cos^2 t0 + tau^2) dtau
    real = (t1 - t0) / 2 + (np.sin(2 * t1) - np.sin(2 * t0)) / 4
    exact = 2 * real + beta * np.cos(t0) ** 2 + beta ** 3 / 3
    errs = []
    for dt in [0.1, 0.05, 0.025]:
        z, w = contour.points(t0, t1, dt, dt, beta)
        f = np.cos(z.real) + 1j * z.imag
        sv = warmstart.weighted_sketch(np.outer(f, f.conj()), w,
                                       np.random.default_rng(1).standard_normal((len(z), 3)))
        errs.append(abs(sv[0] - exact))
    assert errs[0] < 0.2
    assert 1.6 < errs[0] / errs[1] < 2.4 and 1.6 < errs[1] / errs[2] < 2.4


def test_warm_start_feature_rows_by_hand():
    """Feature rows worked by hand on the contour t in [-1, 1], dt = 0.5,
    beta = 1, dtau = 0.5 (points: upper -1, -0.5, 0, 0.5; lower 1, 0.5, 0,
    -0.5; imaginary -1, -1 - 0.5i), E = 2, T = 2."""
    from oracle import warmstart
    z, w = contour.points(-1.0, 1.0, 0.5, 0.5, 1.0)
    n_t = contour.sizes(-1.0, 1.0, 0.5, 0.5, 1.0)[0]
    assert len(z) == 10 and n_t == 4
    sp = np.zeros((10, 10), complex)
    sp[5, 2] = 0.3 - 0.1j
    sp[1, 3] = -0.25j
    rows = warmstart.features(z, n_t, 2.0, 1.0, 2.0, sp, [0.7], [52, 99, 13], 2.0, 64)
    s1, c1 = np.sin(1.0), np.cos(1.0)
    r2 = np.sqrt(0.5)
    # sin, cos (pi k x) for k = 1..8 at x = 1/4, 0, -1/4; k = 1, 2 at x = 0, 1/2
    q = [(r2, r2), (1, 0), (r2, -r2), (0, -1), (-r2, -r2), (-1, 0), (-r2, r2), (0, 1)]
    f_quarter = [v for pair in q for v in pair]
    f_minus = [v for (a, b) in q for v in (-a, b)]
    f_zero8 = [0, 1] * 8
    f_zero2 = [0, 1] * 2
    f_half2 = [1, 0, 0, -1]
    want = np.zeros((3, 64))
    want[0, :61] = ([0.7, 0, 1, 0, 1, 0, 0, 0.25, 0, 0, 0, 1, 1, 0.25, 0.25,
                     s1, c1, 0, 1, 0.6, -0.2] + f_quarter + f_zero8 + f_zero2 + f_zero2)
    want[1, :61] = ([0.7, 0, 0, 1, 0, 0, 1, 0, 0.5, 0, 0.5, 1, 0, 0, 0,
                     0, 1, 0, 1, 0, 0] + f_zero8 + f_zero8 + f_half2 + f_half2)
    want[2, :61] = ([0.7, 1, 0, 0, 1, 0, 0, -0.25, 0, 0.25, 0, 0, 0, -0.5, 0.25,
                     0, 1, s1, c1, 0, -0.5] + f_minus + f_quarter + f_zero2 + f_zero2)
    assert np.max(np.abs(rows - want)) < 1e-15


def test_warm_start_targets_by_hand():
    """Training targets t = scale (Sigma_new - Sigma_prev) at pair p = i N_c + j
    (row-major: pair 1 is (0, 1), pair 2 is (1, 0)), worked by hand on a
    non-symmetric 2 x 2 example, so a transposed pair index, a sign or a
    missing scale fails."""
    from oracle import warmstart
    prev = np.array([[1 + 2j, 0], [3j, -1]])
    new = np.array([[2 + 2j, 1j], [0, -1]])
    t = warmstart.targets(prev, new, None, 2.0)
    want = np.array([[2.0, 0.0], [0.0, 2.0], [0.0, -6.0], [0.0, 0.0]])
    assert np.array_equal(t, want)
    t2 = warmstart.targets(prev, new, [2, 1], 0.5)
    assert np.array_equal(t2, np.array([[0.0, -1.5], [0.0, 0.5]]))


def test_warm_start_apply_by_hand_and_inverts_targets():
    """The update Sigma_prev + y / scale with y the (Re, Im) rows of all pairs
    in row-major order, worked by hand; and applying the targets of a pair of
    matrices to the first reproduces the second (the two are inverse maps)."""
    from oracle import warmstart
    prev = np.array([[1 + 2j, 0], [3j, -1]])
    y = np.array([[2.0, 0.0], [0.0, 2.0], [0.0, -6.0], [4.0, 0.0]])
    got = warmstart.apply(prev, y, 2.0)
    want = np.array([[2 + 2j, 1j], [0, 1]])
    assert np.array_equal(got, want)
    rng = np.random.default_rng(3)
    a = rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5))
    b = rng.standard_normal((5, 5)) + 1j * rng.standard_normal((5, 5))
    back = warmstart.apply(a, warmstart.targets(a, b, None, 8.0), 8.0)
    assert np.max(np.abs(back - b)) < 1e-14


def test_coarse_grid_sampling_hits_the_coarse_times():
    """Samples on the coarse grid t_min + i dt_c of a quantity tabulated at
    t_min + i dt (dt_c = s dt): taking the fine times themselves as the values,
    the samples are exactly the coarse times, so an off-by-one in the stride
    or the start fails; the length is the coarse point count."""
    from oracle import extrapolate
    t_min, dt, n_fine = -2.0, 0.05, 80
    t_fine = t_min + dt * np.arange(n_fine)
    for dt_c, n_c in ((0.2, 20), (0.1, 40), (0.05, 80)):
        got = extrapolate.on_coarse_grid(t_fine, dt, dt_c, n_c)
        assert len(got) == n_c
        assert np.max(np.abs(got - (t_min + dt_c * np.arange(n_c)))) < 1e-12
    # fewer coarse points than the fine array holds: truncated at n_coarse
    assert len(extrapolate.on_coarse_grid(t_fine, dt, 0.2, 7)) == 7


def test_splitmix64_published_sequence():
    """SplitMix64 from state 1234567 gives the sequence of the published
    reference generator (Vigna's splitmix64.c), the state advancing by the
    golden-ratio increment."""
    from oracle import mlp
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    z = 1234567
    got = []
    for _ in range(5):
        got.append(mlp.splitmix64(z))
        z = (z + 0x9E3779B97F4A7C15) % 2 ** 64
    assert got == want
    r = mlp.minibatch_rows(3, 2, 1000, 7)
    assert r.min() == 0 and r.max() == 6 and abs(np.bincount(r).mean() - 1000 / 7) < 1e-9


def test_adam_first_step_moves_every_parameter_by_lr():
    """Adam's bias correction makes the first step -lr * g / (|g| + eps): every
    parameter with |g| >> eps moves by lr against its gradient."""
    from oracle import mlp
    rng = np.random.default_rng(2)
    shapes = mlp.layer_shapes(5, 6, 3, 2)
    p = rng.standard_normal(mlp.n_params(shapes))
    x = rng.standard_normal((9, 5))
    t = rng.standard_normal((9, 2))
    p1, losses = mlp.train(p, shapes, x, t, 9, 1, 1e-3, seed=0)
    r = mlp.minibatch_rows(0, 0, 9, 9)
    _, g = mlp.loss_and_grad(p, shapes, x[r], t[r])
    big = np.abs(g) > 1e-4
    assert np.allclose((p - p1)[big], 1e-3 * np.sign(g[big]), rtol=1e-3, atol=0)


def test_m_matrix_matches_printed_display():
    """The oracle's point-split operator M equals the paper's printed M display
    (Sec. II) entry by entry, written out by hand in tests/golden for N_t = 2,
    N_tau = 3, dt = 0.5, dtau = 0.25, mu = 0.4."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "m_display_small.txt")
    want = np.zeros((7, 7), complex)
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            r, c, re, im = line.split()
            want[int(r), int(c)] = float(re) + 1j * float(im)
    z, w = contour.points(0.0, 1.0, 0.5, 0.25, 0.75)
    assert len(w) == 7
    assert np.max(np.abs(contour.m_matrix(w, 0.4) - want)) < 1e-15


def test_averaged_quadrature_counts_and_moments():
    """The N / N+1 average (Sec. II quadrature paragraph): with N = 54 it has
    the 5941 points the paper quotes (and 20201 with N = 100); weights sum to
    one; both rules integrate eps^2 ebar^2 exp(-eps^2 - ebar^2)/pi = 1/4 and
    eps^4 (3/4) exactly, so their average does too; an odd moment vanishes."""
    for n, count in [(54, 5941), (100, 20201)]:
        e, b, r = quadrature.averaged_grid(n, n)
        assert len(e) == count
    e, b, r = quadrature.averaged_grid(6, 7)
    assert len(e) == 6 * 7 + 7 * 8
    assert abs(r.sum() - 1.0) < 1e-14
    assert abs(np.sum(r * e ** 2 * b ** 2) - 0.25) < 1e-14
    assert abs(np.sum(r * e ** 4) - 0.75) < 1e-13
    assert abs(np.sum(r * e ** 3 * b)) < 1e-14
    # a moment beyond the 6-point rule's exactness (degree 12 > 2*6-1) differs
    # from the exact 10395/64 for one rule but the average is their mean
    e1, b1, r1 = quadrature.product_grid(6, 7)
    e2, b2, r2 = quadrature.product_grid(7, 8)
    m = lambda ee, rr: np.sum(rr * ee ** 12)
    assert abs(np.sum(r * e ** 12) - 0.5 * (m(e1, r1) + m(e2, r2))) < 1e-9


def test_neville_extrapolation_is_exact_for_polynomials():
    """Extrapolation to dt = 0 through k points reproduces any polynomial of
    degree < k exactly (the Lagrange extrapolation of the paper's accuracy
    discussion), and a linear rule from two points cancels the O(dt) term."""
    from oracle import extrapolate
    hs = [0.2, 0.1, 0.05]
    for coeffs in ([3.0], [1.0, -2.0], [0.5, 4.0, -7.0]):
        f = [sum(c * h ** p for p, c in enumerate(coeffs)) for h in hs]
        assert abs(extrapolate.to_zero(hs, f) - coeffs[0]) < 1e-12
    # vector values, elementwise
    f = [np.array([1 + h, 2 - 3 * h]) for h in hs[:2]]
    assert np.allclose(extrapolate.to_zero(hs[:2], f), [1, 2], atol=1e-13)
    # a cubic through three points is not reproduced (degree too high)
    f = [h ** 3 for h in hs]
    assert abs(extrapolate.to_zero(hs, f)) > 1e-4


# ------------------------------------------------- nonequilibrium DOS, moments
def _free_local_green(t_min, t_max, dt, dtau, beta, mu, n_eps):
    """G_loc = sum_k rho_k G0_k at U = 0, E = 0 (Sigma = 0, so G_k = G0_k)."""
    z, w = contour.points(t_min, t_max, dt, dtau, beta)
    n_t = contour.sizes(t_min, t_max, dt, dtau, beta)[0]
    x, wa = quadrature.hermite_rule(n_eps)
    g = np.zeros((len(z), len(z)), dtype=np.complex128)
    for a in range(n_eps):
        g += wa[a] * green.g0_matrix(z, n_t, 0.0, mu, beta, x[a], 0.0)
    return g, n_t


@pytest.mark.parametrize("mu", [0.0, 0.5])
def test_dos_of_free_equilibrium_lattice_is_the_gaussian(mu):
    """Sec. II, eqs. (gr_omega), (dos_def): without interaction and field the
    local G^R(t, t') = -i int rho(e) e^{-i (e - mu)(t - t')} de, so the DOS at any
    average time is the Gaussian DOS of eq. (joint_dos) shifted to w = e - mu:
    rho(T, w) = exp(-(w + mu)^2) / sqrt(pi).  The window (t_rel <= 12,
    exp(-36)) and the trapezoid aliasing (period 2 pi / h = 31) are negligible;
    the 80-point rule integrates e^{-i e t} to ~1e-15 for t <= 12 (40 points
    would leave 4e-5 at t = 12)."""
    from oracle import dos
    g, n_t = _free_local_green(0.0, 12.0, 0.1, 0.1, 1.0, mu, 80)
    w = np.linspace(-3.0, 3.0, 61)
    rho = dos.wigner_dos(g, n_t, 0.1, [60], w)[0]
    assert np.max(np.abs(rho - np.exp(-(w + mu) ** 2) / math.sqrt(math.pi))) < 1e-9


def test_dos_integrates_to_the_zeroth_moment():
    """The w-integral of rho(T, w) over one period of the discrete transform
    (2 pi / h, h = 2 dt) keeps only the t_rel = 0 term: it equals
    -Im G^R(T, T) for any matrix (sum rule of the zeroth moment, Sec. II)."""
    from oracle import dos
    rng = np.random.default_rng(41)
    n_t, n_tau, dt = 20, 4, 0.15
    n_c = 2 * n_t + n_tau
    g = rng.standard_normal((n_c, n_c)) + 1j * rng.standard_normal((n_c, n_c))
    h = 2 * dt
    m = 64                                       # > 2 * max window
    w = -np.pi / h + (2 * np.pi / h) * np.arange(m) / m
    for i in (0, 3, 9, 10, 19):
        rho = dos.wigner_dos(g, n_t, dt, [i], w)[0]
        integral = rho.sum() * (2 * np.pi / h) / m
        m0 = g[2 * n_t - i, i] - g[i, 2 * n_t - i]
        assert abs(integral + m0.imag) < 1e-12


def test_dos_of_one_level_peaks_at_its_energy():
    """A single level: G^R(t, t') = -i e^{-i e0 (t - t')}.  The truncated
    transform is the trapezoid sum of a geometric series; it peaks at w = e0
    (the sign of the exponent of eq. gr_omega) with height (h / pi) D
    (D + 1 window points, end weights 1/2)."""
    from oracle import dos
    n_t, n_tau, dt, e0 = 41, 2, 0.1, 0.8
    n_c = 2 * n_t + n_tau
    t = np.arange(n_t) * dt
    g = np.zeros((n_c, n_c), dtype=np.complex128)
    for a in range(n_t):
        for b in range(n_t):
            g[2 * n_t - a, b] = -1j * np.exp(-1j * e0 * (t[a] - t[b]))
    w = np.linspace(-2.0, 3.0, 501)
    rho = dos.wigner_dos(g, n_t, dt, [20], w)[0]
    assert abs(w[np.argmax(rho)] - e0) < 1e-12
    h, dmax = 2 * dt, 20
    assert abs(rho.max() - h / np.pi * dmax) < 1e-12


def test_moments_exact_for_low_degree_polynomials():
    """Sec. II moments: mu0 = i f(0), mu1 = -f'(0), mu2 = -i f''(0) with
    f(s) = G^R(T + s/2, T - s/2).  The one-sided differences are exact for
    f(s) = c0 + c1 s + c2 s^2 (first derivative) and for cubics (second)."""
    from oracle import dos
    n_t, n_tau, dt = 16, 3, 0.05
    n_c = 2 * n_t + n_tau
    t = np.arange(n_t) * dt
    c0, c1, c2, c3 = 0.3 - 1.1j, -0.7 + 0.2j, 0.45 + 0.9j, -0.35 + 0.6j
    for cubic in (0.0, c3):
        g = np.zeros((n_c, n_c), dtype=np.complex128)
        for a in range(n_t):
            for b in range(a + 1):
                s = t[a] - t[b]
                g[2 * n_t - a, b] = c0 + c1 * s + c2 * s * s + cubic * s ** 3
        mu = dos.moments(g, n_t, dt, [3, 7, n_t - 4])
        assert np.max(np.abs(mu[0] - 1j * c0)) < 1e-13
        assert np.max(np.abs(mu[2] - (-1j) * 2 * c2)) < 1e-9
        if cubic == 0.0:
            assert np.max(np.abs(mu[1] + c1)) < 1e-11


def test_moments_of_free_equilibrium_lattice():
    """Without interaction and field, mu0 = 1, mu1 = <e - mu> = -mu and
    mu2 = <(e - mu)^2> = 1/2 + mu^2 (Gaussian DOS); the differences are
    second-order accurate, error below 1e-3 at h = 0.02."""
    from oracle import dos
    mu_c = 0.3
    g, n_t = _free_local_green(0.0, 0.4, 0.01, 0.1, 1.0, mu_c, 30)
    mu = dos.moments(g, n_t, 0.01, [10, 20])
    assert np.max(np.abs(mu[0] - 1.0)) < 1e-12
    assert np.max(np.abs(mu[1] + mu_c)) < 1e-3
    assert np.max(np.abs(mu[2] - (0.5 + mu_c ** 2))) < 1e-3


# ------------------------------------------ equilibrium Matsubara-axis solver
def test_matsubara_free_g_tau_matches_real_energy_quadrature():
    """U = 0: the Matsubara sum with the 1/(i w_n) tail subtracted equals
    G(tau) = -int rho(e) (1 - f(e)) e^{-e tau} de, evaluated by adaptive
    quadrature over the Gaussian DOS (eq. joint_dos)."""
    from scipy.integrate import quad
    from oracle import matsubara
    beta = 4.0
    _, giw, _, _ = matsubara.solve(0.0, beta, 40000)
    for tau in (0.1, 1.0, 2.0, 3.7):
        f = lambda e: -np.exp(-e * e) / math.sqrt(math.pi) * np.exp(-e * tau) / (1.0 + np.exp(-beta * e))
        ref = quad(f, -12.0, 12.0, epsabs=1e-13, limit=200)[0]
        assert abs(matsubara.g_tau(beta, giw, [tau])[0] - ref) < 1e-8


def test_matsubara_self_energy_tail_is_second_moment():
    """Half filling, symmetric convention: Sigma = U^2/(4 G0^-1) exactly, so
    i w Sigma(i w) -> U^2/4 at large frequency (the U^2/4 of the second
    moment, Sec. II)."""
    from oracle import matsubara
    for u in (0.5, 1.0, 2.0):
        z, _, sig, _ = matsubara.solve(u, 4.0, 3000)
        assert abs((z[-1] * sig[-1]).real - u * u / 4.0) < 1e-4 * max(1.0, u * u)


def test_metal_insulator_transition_at_sqrt_two():
    """Sec. III: the equilibrium model is a metal below U = sqrt(2) and an
    insulator above: rho(0) = 1/sqrt(pi) at U = 0, positive and decreasing
    up to sqrt(2), zero (to the O(eta) of z = i eta) beyond."""
    from oracle import matsubara
    assert abs(matsubara.dos_at_zero(0.0) - 1.0 / math.sqrt(math.pi)) < 1e-8
    vals = [matsubara.dos_at_zero(u) for u in (0.5, 1.0, 1.3, 1.41)]
    assert all(a > b for a, b in zip(vals, vals[1:])) and vals[-1] > 0.01
    for u in (1.42, 1.5, 1.6):
        assert matsubara.dos_at_zero(u) < 1e-5


def test_contour_imaginary_branch_matches_matsubara_solver():
    """The contour oracle at E = 0 (the equilibrium of Sec. II): its
    imaginary-branch block is i G(tau - tau') of the independent Matsubara
    solver, to first order in the step (errors 6e-3, 2.6e-3, 1.2e-3 at
    dtau = 0.2, 0.1, 0.05; U = 1, beta = 4)."""
    from oracle import matsubara
    beta, u = 4.0, 1.0
    _, giw, _, _ = matsubara.solve(u, beta, 40000)
    errs = []
    for dtau in (0.2, 0.1, 0.05):
        p = dmft.Problem(t_min=0.0, t_max=dtau, dt=dtau, dtau=dtau, beta=beta, u=u,
                         e_field=0.0, n_eps=30, n_ebar=1)
        ro = dmft.run(p, 300, tol=1e-13)
        n_t = ro["n_t"]
        k = np.arange(int(round(beta / dtau)))
        g_contour = -1j * ro["gloc"][2 * n_t + k, 2 * n_t]
        errs.append(np.max(np.abs(g_contour - matsubara.g_tau(beta, giw, k * dtau))))
    assert errs[-1] < 2e-3
    assert 0.35 < errs[1] / errs[0] < 0.6 and 0.35 < errs[2] / errs[1] < 0.6


def test_warm_start_pre_field_mask_by_hand():
    """Pairs of contour points before the field (Sec. II: the vector potential
    vanishes up to t = 0) on the contour t in [-1, 1], dt = 0.5, beta = 1,
    dtau = 0.5: upper -1, -0.5, 0, 0.5; lower 1, 0.5, 0, -0.5; imaginary
    -1, -1 - 0.5i.  Before the field: indices 0, 1, 2, 6, 7, 8, 9.  The masked
    proposal keeps Sigma_prev exactly on the pairs of two such points and adds
    y / scale everywhere else."""
    from oracle import warmstart
    z, _ = contour.points(-1.0, 1.0, 0.5, 0.5, 1.0)
    pre = warmstart.pre_field_points(z, 4)
    assert list(np.nonzero(pre)[0]) == [0, 1, 2, 6, 7, 8, 9]
    sp = np.arange(100).reshape(10, 10) * (1 + 0.5j)
    y = np.tile([2.0, -4.0], (100, 1))
    out = warmstart.apply(sp, y, 2.0, pre)
    for i in range(10):
        for j in range(10):
            want = sp[i, j] if (i in (0, 1, 2, 6, 7, 8, 9) and j in (0, 1, 2, 6, 7, 8, 9)) \
                else sp[i, j] + 1 - 2j
            assert out[i, j] == want
    assert np.array_equal(warmstart.apply(sp, y, 2.0), sp + 1 - 2j)
