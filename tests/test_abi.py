"""The C-ABI library loads, exports every symbol include/cpamg.h declares, and
rejects invalid arguments on the host (no GPU needed: NULL contexts never reach HIP)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cpamg.h")
LIB = os.path.join(ROOT, "paper_1111_6091_amd", "libcpamg.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:cp_status|const char\*)\s+(cp_\w+)\s*\(", src, flags=re.M)))


needs_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="libcpamg.so not built")


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for n in ["cp_mttkrp", "cp_als_sweep", "cp_restrict", "cp_prolong", "cp_fas_vcycle",
              "cp_objective", "cp_ctx_create", "cp_ctx_destroy", "cp_last_error", "cp_get_status"]:
        assert n in names


@needs_lib
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s+(cp_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n)


@needs_lib
def test_binding_covers_the_header():
    from paper_1111_6091_amd import _lib
    assert set(declared_functions()) == set(_lib.exported_names())


@needs_lib
def test_null_context_is_rejected_without_touching_the_gpu():
    from paper_1111_6091_amd import _lib
    lib = _lib.load()
    INVALID = _lib.CP_ERR_INVALID
    z = _lib.CpTensor()
    f = _lib.CpFactors()
    assert lib.cp_mttkrp(None, ctypes.byref(z), ctypes.byref(f), 0, None, 0) == INVALID
    assert lib.cp_als_sweep(None, ctypes.byref(z), ctypes.byref(f), None, 1, 0, 10, 1, 0, None) == INVALID
    assert lib.cp_objective(None, ctypes.byref(z), ctypes.byref(f), 1, None, None, 0) == INVALID
    ph = (ctypes.c_void_p * 8)()
    assert lib.cp_restrict(None, ctypes.byref(z), ph, ctypes.byref(z), 0) == INVALID
    assert lib.cp_prolong(None, 4, 2, 1, None, None, None, None) == INVALID
    assert lib.cp_restrict_factor(None, 4, 2, 1, None, None, None) == INVALID
    assert lib.cp_transfer_build(None, 4, None, None) == INVALID
    assert lib.cp_fas_vcycle(None, None, 0, ctypes.byref(f), None, 0) == INVALID
    assert lib.cp_sort(None, None, 3, ctypes.byref(f)) == INVALID
    assert lib.cp_norm2(None, ctypes.byref(z), None) == INVALID
    assert lib.cp_cast_f32(None, None, None, 0) == INVALID
    ms = ctypes.c_double()
    assert lib.cp_time_mttkrp(None, ctypes.byref(z), ctypes.byref(f), 0, 0, 1, ctypes.byref(ms)) == INVALID
    assert lib.cp_profile_enable(None, 1) == INVALID
    assert lib.cp_profile_read(None, None, None) == INVALID
    assert lib.cp_autotune(None, ctypes.byref(z), ctypes.byref(f), 0, 5) == INVALID
    assert lib.cp_plans_import(None, b"") == INVALID
    assert lib.cp_plans_export(None) == b""
    prm = _lib.CpBatchParams(2, 0, 16, 1e-9, 1e-12, 100, 16)
    assert lib.cp_als_batched(None, None, 0, ctypes.byref(prm), None, None) == INVALID
    flags = ctypes.c_int32()
    assert lib.cp_get_status(None, ctypes.byref(flags)) == INVALID
    assert lib.cp_ctx_destroy(None) == INVALID
    assert lib.cp_set_stream(None, None) == INVALID
    assert lib.cp_set_option(None, 1, 0) == INVALID
    assert lib.cp_ctx_create(None, None) == INVALID
    assert lib.cp_last_error(None) == b"invalid context"
