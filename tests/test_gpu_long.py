"""Long contours: matrices beyond 2048 rows, where the panel switches to its
large shape (ten rows per thread, four columns per register block).

- N_c = 2300 (t in [-5, 50], dt = 0.05, beta = 10, dtau = 0.1; 18 outer blocks,
  the last one 124 columns wide), 2 x 2 points, random Sigma: the whole G_loc
  and j(t) against the oracle's lattice step, in one batch and in batches of
  three (a full batch and a ragged one).
- N_c = 4100 (t in [-5, 195], dt = dtau = 0.1, beta = 10: the paper's long
  runs), 3 x 3 points: two sampled G_k of the last batch against the oracle's
  LAPACK solve from the same Sigma.
- N_c = 5120, the largest contour the library takes (t in [-5, 245],
  dt = dtau = 0.1, beta = 12: 40 full outer blocks and every one of the
  panel's ten row slots per thread in use), 2 x 2 points: one sampled G_k
  against the oracle's LAPACK solve, and the weighted sum G_loc against the
  sum of the four oracle solves at two sampled rows.
- N_c = 4100 with U = 0 and 15 x 15 points: the Bloch current
  j(t) = -K sin(E t) theta(t) and n(t) = 1/2, independently of the oracle.
"""
import math

import numpy as np
import pytest

from oracle import dmft, lattice
from paper_0711_0999_amd import inputs

pytestmark = pytest.mark.gpu

MID = dict(t_min=-5.0, t_max=50.0, dt=0.05, dtau=0.1, beta=10.0)
LONG = dict(t_min=-5.0, t_max=195.0, dt=0.1, dtau=0.1, beta=10.0)
MAXN = dict(t_min=-5.0, t_max=245.0, dt=0.1, dtau=0.1, beta=12.0)


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("batch", [4, 3])
def test_nc_2300_matches_oracle(lib, batch):
    print(f"case: N_c = 2300, 2 x 2 points, batch {batch}", flush=True)
    with lib.Context(**MID, U=1.0, E=1.0, n_eps=2, n_ebar=2) as ctx:
        assert ctx.n_c == 2300
        ctx.set_tuning(tile_rows=64, batch=batch, lookahead=0)
        sig = inputs.random_sigma(ctx.n_c, seed=31, scale=0.02)
        ctx.set_sigma(sig)
        ctx.compute_gloc()
        g = ctx.get_gloc()
        _, j, _ = ctx.get_current()
    p = dmft.Problem(**MID, u=1.0, e_field=1.0, n_eps=2, n_ebar=2)
    z, w, n_t, eps, ebar, rho = p.grid()
    go, jo, _ = lattice.lattice_step(z, w, n_t, 1.0, 0.0, 10.0, eps, ebar, rho, sig)
    assert relerr(g, go) < 1e-10
    assert np.max(np.abs(j - jo)) < 1e-10 * max(1.0, np.max(np.abs(jo)))


def test_nc_4100_sampled_points_match_oracle(lib):
    print("case: N_c = 4100, 3 x 3 points, sampled points", flush=True)
    with lib.Context(**LONG, U=1.0, E=1.0, n_eps=3, n_ebar=3) as ctx:
        assert ctx.n_c == 4100
        ctx.set_tuning(tile_rows=64, batch=9, lookahead=0)
        sig = inputs.random_sigma(ctx.n_c, seed=32, scale=0.01)
        ctx.set_sigma(sig)
        ctx.compute_gloc()
        p = dmft.Problem(**LONG, u=1.0, e_field=1.0, n_eps=3, n_ebar=3)
        z, w, n_t, eps, ebar, rho = p.grid()
        st = lattice.weighted_sigma(sig, w)
        for k in (0, 7):
            print(f"  point {k}: eps {eps[k]:.3f} ebar {ebar[k]:.3f}", flush=True)
            g = ctx.get_point_green(k)
            go = lattice.point_green(z, n_t, 1.0, 0.0, 10.0, eps[k], ebar[k], st)
            assert relerr(g, go) < 1e-10, k


def test_nc_5120_largest_contour(lib):
    print("case: N_c = 5120, 2 x 2 points, batch 4", flush=True)
    with lib.Context(**MAXN, U=1.0, E=1.0, n_eps=2, n_ebar=2) as ctx:
        assert ctx.n_c == 5120
        ctx.set_tuning(tile_rows=64, batch=4, lookahead=0)
        sig = inputs.random_sigma(ctx.n_c, seed=33, scale=0.01)
        ctx.set_sigma(sig)
        ctx.compute_gloc()
        g = ctx.get_gloc()
        gk = ctx.get_point_green(3)
    p = dmft.Problem(**MAXN, u=1.0, e_field=1.0, n_eps=2, n_ebar=2)
    z, w, n_t, eps, ebar, rho = p.grid()
    st = lattice.weighted_sigma(sig, w)
    gsum = np.zeros((2, ctx.n_c), dtype=np.complex128)
    rows = [0, 5119]
    for k in range(4):
        print(f"  point {k}: eps {eps[k]:.3f} ebar {ebar[k]:.3f}", flush=True)
        go = lattice.point_green(z, n_t, 1.0, 0.0, 12.0, eps[k], ebar[k], st)
        if k == 3:
            assert relerr(gk, go) < 1e-10
        gsum += rho[k] * go[rows, :]
    assert relerr(g[rows, :], gsum) < 1e-10


def test_nc_4100_u0_bloch_current(lib):
    print("case: N_c = 4100, U = 0, 15 x 15 points", flush=True)
    with lib.Context(**LONG, U=0.0, E=1.0, n_eps=15, n_ebar=15) as ctx:
        ctx.compute_gloc()
        t, j, n = ctx.get_current()
    x, wa = np.polynomial.hermite.hermgauss(15)
    wa = wa / math.sqrt(math.pi)
    kin = float(np.sum(wa * x / (1.0 + np.exp(10.0 * x))))
    assert np.max(np.abs(j - np.where(t > 0, -kin * np.sin(t), 0.0))) < 1e-10
    assert np.max(np.abs(n - 0.5)) < 1e-10
