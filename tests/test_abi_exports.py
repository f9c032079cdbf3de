"""The C-ABI library loads and exports every function include/lqtrace.h declares (no GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lqtrace.h")
LIB = os.path.join(ROOT, "paper_1909_12234_amd", "liblqtrace.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lqt_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary_calls():
    names = declared()
    for must in ["lqt_create", "lqt_set_gauge", "lqt_apply", "lqt_solve", "lqt_basis_eig", "lqt_basis_prolongator",
                 "lqt_basis_eigenvalues", "lqt_basis_free", "lqt_precond_set", "lqt_precond_train", "lqt_trace",
                 "lqt_last_error", "lqt_destroy"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build liblqtrace.so first (python -m paper_1909_12234_amd.build)"
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_1909_12234_amd import lqtrace

    assert sorted(lqtrace.exported_symbols()) == declared()


def test_null_arguments_are_rejected_without_a_device():
    L = ctypes.CDLL(LIB)
    L.lqt_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_void_p]
    assert L.lqt_create(None, None, 0.0, 1, None) == -1
    L.lqt_last_error.restype = ctypes.c_char_p
    L.lqt_last_error.argtypes = [ctypes.c_void_p]
    assert L.lqt_last_error(None) == b"null context"
