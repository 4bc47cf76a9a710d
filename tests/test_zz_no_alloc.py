"""The entry point that allocates nothing, fk_wigner_dos_noalloc (staging in the
library's static device array), against fk_wigner_dos (staging in a per-call
allocation), through the C ABI: two calls in a row, the second smaller, and a
size beyond the static array refused."""
import numpy as np
import pytest

from paper_0711_0999_amd import inputs

pytestmark = pytest.mark.gpu


def test_noalloc_dos_matches_the_allocating_entry_point(lib):
    print("case: fk_wigner_dos_noalloc vs fk_wigner_dos, N_c = 150", flush=True)
    kw = dict(t_min=-5.0, t_max=5.0, dt=0.2, dtau=0.2, beta=10.0, U=0.5, E=1.0,
              n_eps=6, n_ebar=6)
    with lib.Context(**kw) as ctx:
        ctx.set_sigma(inputs.random_sigma(ctx.n_c, seed=41, scale=0.05))
        ctx.compute_gloc()
        ti1 = np.arange(0, ctx.n_t, 2)
        om1 = np.linspace(-4.0, 4.0, 801)
        a1 = ctx.wigner_dos(ti1, om1)
        b1 = ctx.wigner_dos_noalloc(ti1, om1)
        assert b1.shape == (len(ti1), len(om1))
        assert np.array_equal(a1, b1)
        # a smaller second call: the static array still holds the first call's
        # data beyond what this one writes, which must not leak into the result
        ti2 = np.array([7, 30, 45])
        om2 = np.linspace(-2.0, 2.0, 37)
        a2 = ctx.wigner_dos(ti2, om2)
        b2 = ctx.wigner_dos_noalloc(ti2, om2)
        assert np.array_equal(a2, b2)
        assert np.max(np.abs(b2)) > 0.0
        # 700 x 1000 frequencies need 5.6 MB of staging: refused
        with pytest.raises(lib.FkError) as err:
            ctx.wigner_dos_noalloc(np.zeros(700, dtype=np.int32), np.zeros(1000))
        assert err.value.status == lib.FK_EINVAL
        assert "static scratch" in str(err.value)
