"""Multi-instance sweep (uneven contours and (U, E) in shared batched
launches, hipGraph replay, retirement of converged instances) against
single-instance runs and the oracle."""
import numpy as np
import pytest

from oracle import dmft, impurity

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


# C4-sized uneven instances (t_min = -10, dtau = dt, beta = 10, as the C4
# sweep): N_c = 500, 1050 and 750, with small rules so the oracle stays quick
C4_SIZED = [
    dict(t_min=-10.0, t_max=10.0, dt=0.1, dtau=0.1, beta=10.0, U=1.3, E=2.2,
         n_eps=5, n_ebar=5),
    dict(t_min=-10.0, t_max=20.0, dt=1.0 / 15.0, dtau=1.0 / 15.0, beta=10.0, U=0.7,
         E=0.9, n_eps=3, n_ebar=3),
    dict(t_min=-10.0, t_max=10.0, dt=1.0 / 15.0, dtau=1.0 / 15.0, beta=10.0, U=2.1,
         E=3.4, n_eps=3, n_ebar=4),
]


def test_c4_sized_batch_every_instance_against_oracle(lib):
    """Two replayed sweeps from Sigma = 0 give each instance a physical Sigma;
    the third sweep (lattice steps of all instances in shared uneven chunks,
    then the batched impurity updates) is checked for every instance against
    the oracle's lattice step and impurity update from that same Sigma:
    G_loc, j(t) and the new Sigma within 1e-10.  The odd (N_c = 1050, 9
    blocks) and even (500, 750: 4 and 6 blocks) block counts follow different
    pairings of the blocks within the same launches."""
    print("case: C4-sized batch, N_c = 500 / 1050 / 750, every instance", flush=True)
    with lib.Batch(C4_SIZED) as b:
        assert [b.instance(i).n_c for i in range(3)] == [500, 1050, 750]
        b.set_chunk_bytes(60e6)      # several chunks, instances split across them
        b.iterate(2, tol=0.0, use_graph=True)
        sig = [b.instance(i).get_sigma() for i in range(3)]
        r = b.iterate(1, tol=0.0, use_graph=True)
        assert list(r["iters"]) == [3, 3, 3]
        for i, kw in enumerate(C4_SIZED):
            v = b.instance(i)
            print(f"  instance {i}: oracle, N_c = {v.n_c}", flush=True)
            p = dmft.Problem(t_min=kw["t_min"], t_max=kw["t_max"], dt=kw["dt"],
                             dtau=kw["dtau"], beta=kw["beta"], u=kw["U"],
                             e_field=kw["E"], n_eps=kw["n_eps"], n_ebar=kw["n_ebar"])
            go, jo, _ = dmft.lattice_only(p, sig[i])
            g = v.get_gloc()
            assert np.max(np.abs(sig[i])) > 0.01
            assert relerr(g, go) < 1e-10, i
            assert relerr(v.get_current()[1], jo) < 1e-10, i
            z, wts = v.contour_points()
            # the oracle's sequence in long double (its complex128 rounding
            # reaches 7e-10 of max|Sigma| at N_c = 1050)
            ref = impurity.update_extended(g, sig[i], wts, 0.0, kw["U"], 0.5)
            assert relerr(v.get_sigma(), ref) < 1e-10, i


def test_batch_zero_pivot_names_instance_and_point(lib):
    """An exactly singular point matrix in one instance of a sweep: FK_ESINGULAR
    naming the instance, the point and the column (the construction of the
    single-context test: 3 x 3 rule, point 4 has eps = ebar = 0, Sigma cancels
    column 5 of its G0^-1 exactly)."""
    print("case: batch with an exactly singular point matrix", flush=True)
    kw = dict(t_min=-2.0, t_max=2.0, dt=0.5, dtau=0.5, beta=2.0, U=1.0, E=1.0,
              n_eps=3, n_ebar=3)
    with lib.Batch([INSTANCES[0], kw]) as b:
        v = b.instance(1)
        s = np.zeros((v.n_c, v.n_c), np.complex128)
        s[5, 5], s[6, 5] = 4j, -4j            # (i, -i) / dt^2 with dt = 0.5
        v.set_sigma(s)
        with pytest.raises(lib.FkError) as err:
            b.iterate(1, tol=0.0, use_graph=False)
        assert err.value.status == lib.FK_ESINGULAR
        assert "instance 1: zero pivot at column 5 of matrix 4" in str(err.value), str(err.value)


def test_batch_autotune_per_size_class(lib):
    """fk_batch_autotune picks a schedule per contour size (tile height,
    matrices per chunk) on each class's own matrices; sweeps with the per-class
    plan (one size class per chunk) give the results of the default plan."""
    print("case: batch autotune per N_c class", flush=True)
    with lib.Batch(INSTANCES) as b, lib.Batch(INSTANCES) as ref:
        one = b.autotune(max_bytes=64 * 2 ** 20, only_nc=150)
        assert [c["n_c"] for c in one] == [150]
        cls = b.autotune(max_bytes=64 * 2 ** 20)
        assert sorted(c["n_c"] for c in cls) == [73, 150, 200]
        assert all(c["tile_rows"] in (64, 128) and c["batch"] >= 1 and c["trials"] >= 2
                   for c in cls)
        b.iterate(2, tol=0.0, use_graph=True)
        ref.iterate(2, tol=0.0, use_graph=True)
        for i in range(3):
            assert relerr(b.instance(i).get_gloc(), ref.instance(i).get_gloc()) < 1e-13
            assert relerr(b.instance(i).get_sigma(), ref.instance(i).get_sigma()) < 1e-12
