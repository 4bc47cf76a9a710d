"""Extrapolation to zero time step (the paper's Lagrange extrapolation in dt,
accuracy discussion of Sec. II) with the three contours solved together in one
multi-instance sweep.  dt = dtau = h in {0.2, 0.1, 0.05} on t in [-2, 2],
beta = 4, U = 1, E = 1, 6 x 6 points.

Parity: the per-step j, n, m0 on the coarse grid and their extrapolations
against the oracle's (its own Neville extrapolation of its own runs), 1e-8.
Accuracy: the O(h) invariants n = 1/2, m0 = -i and j(t < 0) = 0 (the field is
switched on at t = 0) are met an order of magnitude better after extrapolation
than at the finest step."""
import numpy as np
import pytest

from oracle import dmft, lattice
from oracle import extrapolate as oex

pytestmark = pytest.mark.gpu

STEPS = [0.2, 0.1, 0.05]
MODEL = dict(U=1.0, E=1.0, n_eps=6, n_ebar=6)


def test_step_extrapolation_matches_oracle_and_improves_invariants(lib):
    from paper_0711_0999_amd import extrapolate
    print("case: dt -> 0 extrapolation, h = 0.2, 0.1, 0.05 in one batch", flush=True)
    r = extrapolate.step_sweep(-2.0, 2.0, 4.0, STEPS, MODEL, tol=1e-11)
    nc = 20
    ref = {}
    for h in STEPS:
        p = dmft.Problem(t_min=-2.0, t_max=2.0, dt=h, dtau=h, beta=4.0, u=1.0,
                         e_field=1.0, n_eps=6, n_ebar=6)
        ro = dmft.run(p, 200, tol=1e-12)
        n_t = int(round(4.0 / h))
        ref[h] = dict(j=oex.on_coarse_grid(ro["current"], h, 0.2, nc),
                      n=oex.on_coarse_grid(lattice.density(ro["gloc"], n_t), h, 0.2, nc),
                      m0=oex.on_coarse_grid(lattice.zeroth_moment(ro["gloc"], n_t), h, 0.2, nc))
    for q in ("j", "n", "m0"):
        for h in STEPS:
            assert np.max(np.abs(r["per_step"][h][q] - ref[h][q])) < 1e-8, (q, h)
        e_ref = oex.to_zero(STEPS, [ref[h][q] for h in STEPS])
        assert np.max(np.abs(r["extrapolated"][q] - e_ref)) < 1e-7, q
    t = r["t"]
    fine = r["per_step"][0.05]
    ext = r["extrapolated"]
    err = lambda a, b: float(np.max(np.abs(a - b)))
    print(f"max|n - 1/2|: finest {err(fine['n'], 0.5):.2e}, extrapolated {err(ext['n'], 0.5):.2e}; "
          f"max|m0 + i|: {err(fine['m0'], -1j):.2e}, {err(ext['m0'], -1j):.2e}; "
          f"max|j(t<0)|: {err(fine['j'][t < 0], 0):.2e}, {err(ext['j'][t < 0], 0):.2e}",
          flush=True)
    assert err(ext["n"], 0.5) < 0.1 * err(fine["n"], 0.5)
    assert err(ext["m0"], -1j) < 0.2 * err(fine["m0"], -1j)
    assert err(ext["j"][t < 0], 0) < 0.1 * err(fine["j"][t < 0], 0)
