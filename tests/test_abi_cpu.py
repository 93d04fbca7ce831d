"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every function include/rexi_swe.h declares, and its host-only entry point
(rexi_coefficients) matches the oracle and rejects bad arguments."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1805_06557_amd import _lib, api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rexi_swe.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\s*\*)\s*([a-z_0-9]+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared_functions()
    assert "rexi_linear_step" in names and "rexi_coefficients" in names
    for name in names:
        assert hasattr(lib, name), name
    # and the binding knows the signature of each of them
    assert set(names) <= set(_lib.SIGNATURES)


@pytest.mark.parametrize("fn,N,p0,y", [(0, 128, 10.0, 30.0), (0, 800, 8.0, 67.9), (1, 64, 6.0, 14.0),
                                        (2, 64, 6.0, 14.0), (0, 2, 1.0, 1.0)])
def test_host_coefficients_match_oracle(fn, N, p0, y):
    from oracle import rexi as orexi
    a, b, r, mu = api.rexi_coefficients(fn, N, p0, y)
    ao, bo, ro, muo = orexi.coefficients(fn, N, p0, y)
    assert r == pytest.approx(ro, rel=1e-15) and mu == pytest.approx(muo, rel=1e-15, abs=1e-15)
    # both are rounded once from extended precision: agree to about an ulp
    np.testing.assert_allclose(a, ao, rtol=4e-16, atol=0)
    assert np.all(np.abs(b - bo) <= 4e-16 * np.abs(bo))


@pytest.mark.parametrize("args", [(7, 128, 10.0, 30.0), (0, 127, 10.0, 30.0), (0, 0, 10.0, 30.0),
                                  (0, 128, -1.0, 30.0), (0, 128, 10.0, 0.0), (0, 128, float("nan"), 3.0)])
def test_host_coefficients_reject_bad_arguments(args):
    with pytest.raises(api.RexiError) as ei:
        api.rexi_coefficients(*args)
    assert ei.value.code == api.REXI_EINVAL
    assert "rexi_coefficients" in str(ei.value)


def test_null_context_and_pointers_are_rejected():
    lib = _lib.load()
    assert lib.swe_destroy(None) == 0
    assert lib.swe_sync(None) == api.REXI_EINVAL
    assert lib.rexi_linear_step(None, None, None, 2, 1.0, None, None, None) == api.REXI_EINVAL
    assert lib.swe_set_fusion(None, 1) == api.REXI_EINVAL
    assert lib.swe_get_fusion(None, None) == api.REXI_EINVAL
    assert b"NULL" in lib.rexi_last_error()
    out = ctypes.c_void_p()
    assert lib.swe_create(0, 0, 0, 1.0, 1.0, 1.0, 0.0, 0, ctypes.byref(out)) == api.REXI_EINVAL
    assert lib.swe_create(31, 31, 64, 1.0, 1.0, 1.0, 0.0, 0, ctypes.byref(out)) == api.REXI_EINVAL
    assert lib.swe_create(31, 0, 0, 1.0, 1.0, 1.0, 0.0, 6, ctypes.byref(out)) == api.REXI_EINVAL
