"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/demag.h declares with the binding's signatures, and
rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import pytest

from paper_1204_4302_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "demag.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(demag_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(_lib.SIGNATURES)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_codes_match_header():
    text = open(HEADER).read()
    for code, name in _lib.STATUS.items():
        assert re.search(rf"{name}\s*=\s*{code}\b", text), name


@pytest.mark.parametrize("args", [
    (0, 4, 4, 1e-9, 1e-9, 1e-9),
    (4, -1, 4, 1e-9, 1e-9, 1e-9),
    (4, 4, 4, 0.0, 1e-9, 1e-9),
    (4, 4, 4, 1e-9, float("nan"), 1e-9),
    (4, 4, 4, 1e-9, 1e-9, float("inf")),
    (4, 4, 4, -2e-9, 1e-9, 1e-9),
])
def test_plan_create_rejects_invalid_grid(args):
    lib = _lib.load()
    h = ctypes.c_void_p(123)
    rc = lib.demag_plan_create(ctypes.byref(h), *args, 0, None)
    assert rc == -1
    assert h.value is None
    assert lib.demag_last_error()


def test_plan_create_rejects_unknown_dtype_and_oversize():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.demag_plan_create(ctypes.byref(h), 4, 4, 4, 1e-9, 1e-9, 1e-9, 7, None) == -1
    assert lib.demag_plan_create(ctypes.byref(h), 4097, 4, 4, 1e-9, 1e-9, 1e-9, 0, None) == -4
    assert lib.demag_plan_create(None, 4, 4, 4, 1e-9, 1e-9, 1e-9, 0, None) == -1


def test_null_handles_rejected():
    lib = _lib.load()
    assert lib.demag_field(None, None, 1.0, None, None) == -1
    assert lib.demag_field_adjoint(None, None, 1.0, None, 0, None) == -1
    assert lib.demag_energy(None, None, 1.0, None, None) == -1
    assert lib.demag_plan_destroy(None) == -1
    assert lib.demag_batch_autotune(None, None) == -1
    assert lib.demag_sp_prepare(None, None) == -1
    assert lib.demag_llg_heun(None, None, 1.0, 0.1, 2.2e5, 0.0, 0.0, 0.0, 1e-13, 1, None, None) == -1
    assert lib.demag_llg_heun_static(None, None, 1.0, 0.1, 2.2e5, 0.0, 0.0, 0.0, 1e-13, 1, None) == -1
    assert lib.demag_energy_gradient(None, None, 1.0, None, None, 0, None) == -1
    assert lib.demag_sp_field(None, None, 1.0, None, None) == -1
    assert lib.demag_sp_field_energy(None, None, 1.0, None, None, None) == -1
    assert lib.demag_sp_kernel(None, None) == -1
    assert lib.demag_tg_prepare(None, None) == -1
    assert lib.demag_tg_info(None, None) == -1
    assert lib.demag_tg_lowrank_prepare(None, None) == -1
    assert lib.demag_tg_lowrank_field(None, 0, 1, None, None, 1.0, None, None, None, None) == -1
    assert lib.demag_tg_lowrank_info(None, None) == -1
    assert lib.demag_batch_launch(None, None) == -1
    assert lib.demag_batch_destroy(None) == -1
    assert lib.demag_plan_set_option(None, b"far_cut", 40.0) == -1
    assert b"NULL" in lib.demag_last_error()


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(ImportError):
        _lib.load(str(tmp_path / "nope.so"))
