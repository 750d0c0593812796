"""The C-ABI library loads on the CPU and exports every function include/cm.h declares.

No compute call is made (there may be no GPU here).
"""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cm.h")
LIB = os.path.join(ROOT, "paper_1908_10574_amd", "libcm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s+\**\s*(cm_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("cm_sw_score_batch", "cm_sw_span_batch", "cm_sw_traceback_batch", "cm_clustermerge_run",
                     "cm_clustermerge_extend", "cm_allvsall_count", "cm_kmer_features", "cm_screen_infer",
                     "cm_screen_train_step", "cm_screen_train", "cm_screen_train_steps", "cm_context_create"):
        assert required in names
    assert len(names) >= 29


def test_header_is_plain_c(tmp_path):
    """The boundary header compiles as C99 on its own (no C++ or HIP types)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        import pytest
        pytest.skip("no C compiler")
    src = tmp_path / "use_header.c"
    src.write_text('#include "cm.h"\nint main(void) { return 0; }\n')
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only",
                        "-I", os.path.join(ROOT, "include"), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libcm.so not built (run __graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_without_device():
    lib = ctypes.CDLL(LIB)
    lib.cm_status_str.restype = ctypes.c_char_p
    assert lib.cm_status_str(0) == b"ok"
    assert lib.cm_status_str(-2) == b"input data out of range"
    lib.cm_screen_num_params.restype = ctypes.c_int64
    assert lib.cm_screen_num_params() == 1312257


def test_train_steps_without_device():
    """The step count of a training run is host arithmetic (no device)."""
    lib = ctypes.CDLL(LIB)

    class Cfg(ctypes.Structure):
        _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                    ("shuffle", ctypes.c_int32), ("seed", ctypes.c_uint64), ("drop_last", ctypes.c_int32)]

    lib.cm_screen_train_steps.restype = ctypes.c_int64
    lib.cm_screen_train_steps.argtypes = [ctypes.c_int64, ctypes.POINTER(Cfg)]
    assert lib.cm_screen_train_steps(10000, ctypes.byref(Cfg(3, 4096, 1e-3, 1, 0, 1))) == 6
    assert lib.cm_screen_train_steps(10000, ctypes.byref(Cfg(3, 4096, 1e-3, 1, 0, 0))) == 9
    assert lib.cm_screen_train_steps(10000, ctypes.byref(Cfg(1, 0, 1e-3, 1, 0, 0))) == -1
