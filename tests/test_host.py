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
