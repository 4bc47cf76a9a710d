"""Equilibrium (E = 0) through the library against the independent
Matsubara-axis solver of the oracle: the imaginary-branch block of the
converged G_loc is i G(tau - tau') to first order in the step (U = 1,
beta = 4, dtau = 0.1 and 0.05, a minimal real-time range), and the second
halving of the step roughly halves the error."""
import numpy as np
import pytest

from oracle import matsubara

pytestmark = pytest.mark.gpu


def test_imaginary_branch_matches_matsubara_solver(lib):
    beta, u = 4.0, 1.0
    _, giw, _, _ = matsubara.solve(u, beta, 40000)
    errs = []
    for dtau in (0.1, 0.05):
        print(f"case: E = 0, U = 1, beta = 4, dtau = {dtau}", flush=True)
        with lib.Context(t_min=0.0, t_max=dtau, dt=dtau, dtau=dtau, beta=beta, U=u,
                         E=0.0, n_eps=30, n_ebar=1) as ctx:
            r = ctx.iterate(300, tol=1e-12)
            assert r["converged"]
            g = ctx.get_gloc()
            n_t = ctx.n_t
        k = np.arange(int(round(beta / dtau)))
        g_contour = -1j * g[2 * n_t + k, 2 * n_t]
        errs.append(np.max(np.abs(g_contour - matsubara.g_tau(beta, giw, k * dtau))))
    assert errs[-1] < 2e-3
    assert 0.35 < errs[1] / errs[0] < 0.6
