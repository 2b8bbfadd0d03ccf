"""Host-side checks of the C ABI (CPU only: no kernel is launched).

The library must load, export every function include/odwf.h declares, reject
bad arguments before touching the GPU, and compute the optimal weights on the
host identically (to rounding) to the oracle's independent implementation.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.zolotarev import omega_zolotarev
from paper_1811_08095_amd import odwf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "odwf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(odwf_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = odwf.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(odwf.SYMBOLS)


def test_version_string():
    assert "gfx950" in odwf.version()


@pytest.mark.parametrize("Ns", [4, 8, 16, 32])
def test_zolotarev_weights_match_oracle(Ns):
    w = odwf.zolotarev_omega(Ns, 0.05, 6.2)
    ref = omega_zolotarev(0.05, 6.2, Ns)
    assert np.allclose(w, ref, rtol=1e-12, atol=0)


def test_argument_validation_without_gpu():
    L = odwf.lib()
    h = ctypes.c_void_p()
    bad = (ctypes.c_int * 4)(4, 4, 3, 4)  # odd extent
    assert L.odwf_lattice_create(bad, -1, 0, ctypes.byref(h)) == odwf.EINVAL
    assert b"even" in L.odwf_last_error()
    good = (ctypes.c_int * 4)(4, 4, 4, 4)
    assert L.odwf_lattice_create(good, 0, 0, ctypes.byref(h)) == odwf.EINVAL  # bc_t
    assert L.odwf_lattice_create(None, -1, 0, ctypes.byref(h)) == odwf.EINVAL
    w = np.ones(6)
    assert L.odwf_solver_create(None, 6, 1.3, w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                ctypes.byref(h)) == odwf.EINVAL
    out = np.zeros(3)
    assert L.odwf_zolotarev_omega(3, 0.05, 6.2, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) \
        == odwf.EINVAL
    assert L.odwf_solve(None, 1, None, None, 1, 0, 10, None, None, 0, None, None) == odwf.EINVAL
    assert L.odwf_apply(None, 0, None, 0, 1, None, None, None) == odwf.EINVAL


def test_footprint_scales_with_precision_and_rhs():
    dims = (64, 64, 64, 64)
    f64 = odwf.footprint(dims, 16, 1, odwf.FP64)
    f32 = odwf.footprint(dims, 16, 1, odwf.FP32)
    f16 = odwf.footprint(dims, 16, 1, odwf.FP16S)
    unit = 64 ** 4 // 2 * 16 * 12 * 16  # one FP64 half field
    assert f64 >= 6 * unit and f64 < 6.2 * unit
    assert 4 * unit < f16 < f32 < f64 + unit
    # the full-size mixed solve fits one 288 GB device with room for the caller's field
    assert f32 + 2 * (64 ** 4) * 8 * 18 * 1.5 + 2 * unit < 288e9
    assert odwf.footprint((8, 8, 8, 8), 16, 12, odwf.FP32) > odwf.footprint((8, 8, 8, 8), 16, 1, odwf.FP32)
