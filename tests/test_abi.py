"""The C ABI: libkrr.so loads and exports every function include/krr.h declares (CPU only),
the Python binding binds each of them, and host-side argument checks work without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "krr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(krr_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_1905_10587_amd as krr
    path = krr.library_path()
    if not os.path.exists(path):
        pytest.fail("libkrr.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(path)


def test_header_declares_the_four_calls():
    names = declared_functions()
    for f in ("krr_build_precond", "krr_kernel_mv", "krr_pcg_solve", "krr_grad"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, f"not exported: {missing}"


def test_binding_covers_header():
    import paper_1905_10587_amd as krr
    assert set(declared_functions()) == set(krr._SIGS)


def test_host_validation_without_gpu(lib):
    lib.krr_last_error.restype = ctypes.c_char_p
    lib.krr_kernel_mv.restype = ctypes.c_int
    lib.krr_kernel_mv.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                  ctypes.c_double, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    # eps <= 0 is rejected before any device work
    st = lib.krr_kernel_mv(None, 10, None, 10, 3, -1.0, None, 1, None, 0, 0, None, None)
    assert st == -1 and b"eps" in lib.krr_last_error()
    st = lib.krr_kernel_mv(None, 10, None, 10, 0, 1.0, None, 1, None, 0, 0, None, None)
    assert st == -1 and b"d must" in lib.krr_last_error()
    lib.krr_version.restype = ctypes.c_int
    assert lib.krr_version() >= 10000


def test_variant_table_roundtrip(lib, tmp_path):
    import paper_1905_10587_amd as krr
    L = krr.load()
    krr._chk(L, L.krr_set_variant(4, 1, 2, 3))
    krr._chk(L, L.krr_set_variant(8, 1, 1, 1))
    a, b = tmp_path / "a.json", tmp_path / "b.json"
    krr._chk(L, L.krr_autotune_save(str(a).encode()))
    krr._chk(L, L.krr_set_variant(4, 1, 2, -1))         # clear, then restore from the file
    krr._chk(L, L.krr_autotune_load(str(a).encode()))
    krr._chk(L, L.krr_autotune_save(str(b).encode()))
    assert a.read_text() == b.read_text()
    assert '"2:4:1": 3' in a.read_text()
    assert L.krr_set_variant(4, 1, 2, 99) == -1          # out of range
