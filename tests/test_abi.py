"""CPU checks of the C ABI: the library loads and exports every function that
include/magfft.h declares; host-side argument checks that run before any GPU
call.  No compute calls (there may be no GPU)."""
import ctypes
import os

import pytest

from paper_1801_04869_amd import _lib


def _load():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmagfft.so not built (run __graft_entry__.build())")
    return _lib.lib()


def test_header_declares_the_boundary():
    names = _lib.header_symbols()
    for required in ["mag_create", "mag_destroy", "mag_set_grid", "mag_set_domain", "mag_set_params",
                     "mag_set_solver", "mag_set_field", "mag_rhs", "mag_step", "mag_integrate",
                     "mag_observe", "mag_rhs_vjp", "mag_reset_warm_start", "mag_last_error"]:
        assert required in names
    assert set(names) == set(_lib.SIGNATURES)


def test_library_exports_every_declared_symbol():
    L = _load()
    for name in _lib.header_symbols():
        assert hasattr(L, name), name


def test_create_rejects_bad_arguments_before_touching_the_gpu():
    L = _load()
    h = ctypes.c_void_p()
    assert L.mag_create(None, 3, 0, None) == -1
    assert L.mag_create(ctypes.byref(h), 4, 0, None) == -1
    assert L.mag_create(ctypes.byref(h), 3, 7, None) == -1
    # the final-FP64-evaluation form is a film form
    assert L.mag_create(ctypes.byref(h), 3, 2, None) == -1
    assert not h.value
    assert L.mag_last_error(None) == b"null context"
    assert L.mag_set_grid(None, 16, 16, 16, 1.0, 1.0, 1.0) == -1
    assert L.mag_rhs(None, None, 0.0, None, None) == -1
    assert L.mag_set_derivatives(None, 1, -1.0) == -1
    assert L.mag_prof_kernel_name(0) is not None
    assert L.mag_prof_kernel_name(10 ** 6) is None
    L.mag_destroy(None)


def test_python_constants_match_the_header():
    """Status codes, precisions and field kinds of the binding are the
    enumerators of include/magfft.h."""
    import re
    from paper_1801_04869_amd import api
    txt = open(_lib.HEADER).read()
    enum = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(MAG_[A-Z0-9_]+)\s*=\s*(-?\d+)", txt)}
    pairs = {"OK": "MAG_OK", "NOT_CONVERGED": "MAG_NOT_CONVERGED", "STEP_UNDERFLOW": "MAG_STEP_UNDERFLOW",
             "E_ARG": "MAG_E_ARG", "E_STATE": "MAG_E_STATE", "E_HIP": "MAG_E_HIP", "E_NOMEM": "MAG_E_NOMEM",
             "E_NUMERIC": "MAG_E_NUMERIC", "FP64": "MAG_FP64", "MIXED": "MAG_MIXED",
             "MIXED_FINAL64": "MAG_MIXED_FINAL64", "RAMP": "MAG_FIELD_RAMP", "SINE": "MAG_FIELD_SINE",
             "ROTATE": "MAG_FIELD_ROTATE", "STAGGERED": "MAG_DERIV_STAGGERED", "SPECTRAL": "MAG_DERIV_SPECTRAL"}
    for py, c in pairs.items():
        assert getattr(api, py) == enum[c], (py, c)
