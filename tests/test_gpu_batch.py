"""Multi-instance sweep (uneven contours and (U, E) in shared batched
launches, hipGraph replay, retirement of converged instances) against
single-instance runs and the oracle."""
import numpy as np
import pytest

from oracle import dmft

pytestmark = pytest.mark.gpu

# three uneven instances: N_c = 73, 150, 200 with different rules, U and E
INSTANCES = [
    dict(t_min=-1.0, t_max=2.0, dt=0.1, dtau=0.1, beta=1.3, U=1.0, E=1.5, n_eps=3, n_ebar=4),
    dict(t_min=-5.0, t_max=5.0, dt=0.2, dtau=0.2, beta=10.0, U=0.5, E=1.0, n_eps=5, n_ebar=5),
    dict(t_min=-2.0, t_max=2.0, dt=0.05, dtau=0.05, beta=2.0, U=2.0, E=3.0, n_eps=4, n_ebar=3),
]


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_batch_matches_single_instances_and_oracle(lib):
    print("case: batch of 3 uneven instances, 4 sweeps, eager", flush=True)
    with lib.Batch(INSTANCES) as b:
        b.set_chunk_bytes(3e6)       # force several chunks per sweep
        r = b.iterate(4, tol=0.0, use_graph=False)
        assert r["sweeps"] == 4 and list(r["iters"]) == [4, 4, 4]
        for i, kw in enumerate(INSTANCES):
            with lib.Context(**kw) as c:
                rs = c.iterate(4, tol=0.0)
                v = b.instance(i)
                assert relerr(v.get_gloc(), c.get_gloc()) < 1e-12
                assert relerr(v.get_sigma(), c.get_sigma()) < 1e-11
                assert relerr(v.get_current()[1], c.get_current()[1]) < 1e-12
                assert abs(r["deltas"][i] - rs["delta"]) < 1e-10 * max(1.0, rs["delta"])
        kw = INSTANCES[0]
        ro = dmft.run(dmft.Problem(t_min=kw["t_min"], t_max=kw["t_max"], dt=kw["dt"],
                                   dtau=kw["dtau"], beta=kw["beta"], u=kw["U"],
                                   e_field=kw["E"], n_eps=kw["n_eps"],
                                   n_ebar=kw["n_ebar"]), 4)
        assert relerr(b.instance(0).get_gloc(), ro["gloc"]) < 1e-10


def test_graph_replays_match_eager_sweeps(lib):
    """Record the sweep once, replay it sweep by sweep with the program's own
    eager work and synchronizations in between; every replay must equal the
    eager sweep from the same state bit for bit."""
    print("case: graph replays vs eager", flush=True)
    with lib.Batch(INSTANCES) as b:
        eager = []
        for _ in range(4):
            b.iterate(1, tol=0.0, use_graph=False)
            eager.append([(b.instance(i).get_gloc(), b.instance(i).get_sigma())
                          for i in range(3)])
        for i in range(3):
            b.instance(i).set_sigma(np.zeros((b.instance(i).n_c,) * 2, np.complex128))
        b.reset()
        for s in range(4):
            b.iterate(1, tol=0.0, use_graph=True)
            for i in range(3):                    # eager work between replays
                g = b.instance(i).get_gloc()
                sg = b.instance(i).get_sigma()
                assert np.array_equal(g, eager[s][i][0]), (s, i)
                assert np.array_equal(sg, eager[s][i][1]), (s, i)
        assert b.timings()["captures"] == 1


def test_retirement_and_recapture(lib):
    """Each instance stops after the iteration whose delta < tol, exactly like
    its single-instance loop; retirements re-record the graph."""
    print("case: retirement", flush=True)
    tol = 1e-8
    with lib.Batch(INSTANCES) as b:
        r = b.iterate(60, tol=tol, use_graph=True)
        for i, kw in enumerate(INSTANCES):
            with lib.Context(**kw) as c:
                rs = c.iterate(60, tol=tol)
                assert rs["converged"]
                assert r["iters"][i] == rs["iters"], (i, r["iters"], rs["iters"])
                assert r["deltas"][i] < tol
                assert relerr(b.instance(i).get_gloc(), c.get_gloc()) < 1e-11
        assert len(set(r["iters"])) > 1
        assert b.timings()["captures"] >= 2


def test_batch_mixing_small_and_long_contours(lib):
    """An uneven batch whose largest matrix exceeds 2048 rows runs every matrix
    with the panel's large shape (ten rows per thread, four columns per
    register block): N_c = 73 and 2300 in one sweep, replayed from the graph,
    against single-instance runs (where the N_c = 73 instance takes the small
    shape) and the oracle."""
    print("case: batch of N_c = 73 and 2300, 2 sweeps, graph", flush=True)
    inst = [INSTANCES[0],
            dict(t_min=-5.0, t_max=50.0, dt=0.05, dtau=0.1, beta=10.0, U=1.0, E=1.0,
                 n_eps=2, n_ebar=2)]
    with lib.Batch(inst) as b:
        r = b.iterate(2, tol=0.0, use_graph=True)
        assert list(r["iters"]) == [2, 2]
        for i, kw in enumerate(inst):
            with lib.Context(**kw) as c:
                c.iterate(2, tol=0.0)
                v = b.instance(i)
                assert relerr(v.get_gloc(), c.get_gloc()) < 1e-10
                assert relerr(v.get_sigma(), c.get_sigma()) < 1e-9
        kw = inst[0]
        ro = dmft.run(dmft.Problem(t_min=kw["t_min"], t_max=kw["t_max"], dt=kw["dt"],
                                   dtau=kw["dtau"], beta=kw["beta"], u=kw["U"],
                                   e_field=kw["E"], n_eps=kw["n_eps"],
                                   n_ebar=kw["n_ebar"]), 2)
        assert relerr(b.instance(0).get_gloc(), ro["gloc"]) < 1e-10
