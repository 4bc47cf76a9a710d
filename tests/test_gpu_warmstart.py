"""The learned warm start end to end on a small contour family: field sweeps
solved by the plain method (multi-instance batch) give the training pairs, the
network trains on the GPU with its own kernels, and its BF16 proposal starts
the judged loop at a finer step size than it was trained on.

Checked: every start reaches the same fixed point; the judged start never costs
more than the one iteration a rejected proposal wastes; the proposal is closer
to the fixed point than the previous field in RMS.  The iteration counts of the
three starts (Sigma = 0, previous field, network) are printed: they are the
gain this test shows, not a bar."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BASE = dict(t_min=-2.0, t_max=6.0, dtau=0.1, beta=2.0)


def test_warm_start_small_family(lib):
    from paper_0711_0999_amd import warmstart as W
    print("case: warm start, train dt 0.2 / 0.1 (N_c 100 / 180), test dt 0.1 and 0.05",
          flush=True)
    us = list(np.linspace(0.3, 1.5, 12))
    es = list(np.arange(0.5, 3.01, 0.25))
    x1, t1, _ = W.field_sweep_data(dict(BASE, dt=0.2), us[0::2], es, 6, 6, 1e-8, 8192,
                                   max_iter=150)
    x2, t2, _ = W.field_sweep_data(dict(BASE, dt=0.1), us[1::2], es, 6, 6, 1e-8, 8192,
                                   max_iter=150)
    x, t = torch.cat([x1, x2]), torch.cat([t1, t2])
    assert x.shape[0] == 12 * 10 * 8192
    ws, hist = W.train(x, t, steps=(3000, 1500), lrs=(1e-3, 3e-4), batch=4096, seed=1)
    assert np.mean(hist[-100:]) < 0.2 * np.mean(hist[:10])
    for u, e, dt in [(0.8, 1.6, 0.1), (1.25, 2.4, 0.05)]:
        r = W.compare_starts(ws, dict(BASE, dt=dt), u, e, 6, 6, 1e-10, mixed=False)
        print(f"U={u} E={e} dt={dt}: iterations zero {r['zero_iters']}, previous "
              f"{r['previous_iters']}, network {r['network_iters']} "
              f"(outcome {r['network_outcome']}); start error max/rms previous "
              f"{r['start_err_previous']}, network {r['start_err_network']}", flush=True)
        assert r["zero_converged"] and r["previous_converged"] and r["network_converged"]
        assert r["gloc_spread"] < 1e-8
        assert r["network_iters"] <= r["previous_iters"] + 1
        assert r["start_err_network"][1] < r["start_err_previous"][1]
