"""The C ABI library loads and exports every entry point include/*.h declares
(no compute: this runs without a GPU)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1402_4073_amd", "libtq.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(tq_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def libtq():
    if not os.path.exists(LIB):
        import importlib.util
        spec = importlib.util.spec_from_file_location("tqbuild", os.path.join(ROOT, "paper_1402_4073_amd", "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build_lib()
    import torch  # noqa: F401  (same HIP runtime as the GPU path)
    return ctypes.CDLL(LIB)


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("tq_create", "tq_destroy", "tq_status_string", "tq_ctx_check", "tq_threshold",
                 "tq_symmetric"):
        assert must in names


def test_every_declared_symbol_exported(libtq):
    missing = [n for n in declared_functions() if not hasattr(libtq, n)]
    assert not missing, missing


def test_binding_has_same_names(libtq):
    import paper_1402_4073_amd.binding as b
    for n in declared_functions():
        if n in ("tq_status_string",):
            continue
        assert hasattr(b, n), n


def test_status_strings(libtq):
    libtq.tq_status_string.restype = ctypes.c_char_p
    for s in range(0, -8, -1):
        assert libtq.tq_status_string(s).startswith(b"TQ_")
    assert b"unknown" in libtq.tq_status_string(-99)


def test_create_rejects_without_device(libtq):
    # no GPU in the build container: tq_create must fail cleanly, not crash
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    libtq.tq_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]
    assert libtq.tq_create(ctypes.byref(h), 0) != 0
    assert not h.value


def test_null_context_rejected(libtq):
    libtq.tq_threshold.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64,
                                   ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
    assert libtq.tq_threshold(None, None, 1, 64, 1, None, None) == -1
    assert libtq.tq_destroy(None) == 0
