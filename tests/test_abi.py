"""The C ABI: header is plain C, and the built library exports every symbol
it declares.  No compute call is made (no GPU needed)."""

import ctypes
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "km.h")
LIB = os.path.join(ROOT, "paper_1805_10638_amd", "libkmaa.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b((?:km|kmeans)_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for need in ("kmeans_g", "kmeans_solve", "km_create", "km_destroy", "km_status_str",
                 "km_last_error", "km_opts_default"):
        assert need in names


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_header_is_plain_c(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "km.h"\nint main(void){ km_opts o; km_opts_default(&o); return (int)sizeof(o) > 0 ? 0 : 1; }\n')
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-fsyntax-only",
                        "-I", os.path.dirname(HEADER), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libkmaa.so not built")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_without_device():
    if not os.path.exists(LIB):
        pytest.skip("libkmaa.so not built")
    lib = ctypes.CDLL(LIB)
    lib.km_status_str.restype = ctypes.c_char_p
    assert lib.km_status_str(0) == b"ok"
    assert b"invalid" in lib.km_status_str(-1)
    assert lib.km_version() >= 10000
