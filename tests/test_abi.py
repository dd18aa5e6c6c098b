"""CPU-side checks of the C ABI: the library loads and exports every declared symbol."""
import ctypes
import os
import re

import pytest
import torch  # noqa: F401  (loads torch's HIP runtime before the library, as the binding does)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "psweep.h")
SO = os.path.join(ROOT, "paper_1008_3699_amd", "libpsweep.so")


def declared():
    txt = open(HDR).read()
    return sorted(set(re.findall(r"^\s*(?:psw_status|const char \*)\s*\**\s*(psw_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("psw_problem_create", "psw_set_diagonals", "psw_set_relaxation", "psw_set_decomposition",
                 "psw_sweep", "psw_precond_apply", "psw_solve", "psw_batch_solve", "psw_autotune",
                 "psw_server_create", "psw_server_submit", "psw_server_poll", "psw_server_destroy",
                 "psw_status_string"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(SO):
        pytest.fail("libpsweep.so is not built (run __graft_entry__.build())")
    try:
        L = ctypes.CDLL(SO)
    except OSError as e:  # the HIP runtime must be loadable even without a GPU
        pytest.fail(f"cannot load {SO}: {e}")
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings_without_gpu():
    L = ctypes.CDLL(SO)
    L.psw_status_string.restype = ctypes.c_char_p
    assert L.psw_status_string(0) == b"ok"
    assert L.psw_status_string(-6) == b"non-positive ILU pivot"


def test_create_rejects_bad_arguments_without_touching_gpu():
    L = ctypes.CDLL(SO)
    h = ctypes.c_void_p()
    n = (ctypes.c_int64 * 3)(8, 8, 1)
    # stencil must be 2*dim+1; dim 4 and dim 0 invalid
    assert L.psw_problem_create(2, n, 7, ctypes.byref(h)) == -1
    assert L.psw_problem_create(4, n, 9, ctypes.byref(h)) == -1
    assert L.psw_problem_create(1, n, 5, ctypes.byref(h)) == -1
    assert L.psw_problem_create(0, n, 1, ctypes.byref(h)) == -1


def test_server_rejects_bad_arguments_without_touching_gpu():
    L = ctypes.CDLL(SO)
    h = ctypes.c_void_p()
    L.psw_server_create.argtypes = [ctypes.c_size_t, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    assert L.psw_server_create(0, None, ctypes.byref(h)) == -1  # zero budget
    assert L.psw_server_destroy(None) == -1
    done = ctypes.c_int()
    L.psw_server_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p]
    assert L.psw_server_poll(None, 1, 0, ctypes.byref(done), None, None, None) == -1
