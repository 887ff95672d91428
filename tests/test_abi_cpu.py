"""Host-side checks of the C ABI: the library builds for gfx950, loads, and
exports every entry point that include/nrs.h declares (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nrs.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nrs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpath():
    from paper_2001_06468_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2001_06468_amd import build
        build.build()
    return _lib.LIB_PATH


def test_header_declares_entry_points():
    names = _declared()
    for must in ("nrs_create", "nrs_nearest", "nrs_assemble", "nrs_solve", "nrs_lu_factor",
                 "nrs_lu_solve", "nrs_apply", "nrs_geometry", "nrs_rk4_step"):
        assert must in names


def test_library_exports_every_declared_symbol(libpath):
    lib = ctypes.CDLL(libpath)
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (nrs_[a-z0-9_]+)$", out, flags=re.M))
    assert set(_declared()) <= exported


def test_binding_prototypes_cover_header():
    from paper_2001_06468_amd import _lib
    assert set(_declared()) == set(_lib.PROTOTYPES)


def test_header_compiles_as_c(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "nrs.h"\nint main(void){ nrs_options o = {0}; (void)o; return 0; }\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    "-c", str(src), "-o", str(tmp_path / "t.o")], check=True)


def test_code_object_targets_gfx950(libpath):
    """The offload bundle embedded in the library is built for gfx950."""
    data = open(libpath, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_status_strings_without_gpu(libpath):
    from paper_2001_06468_amd import _lib
    lib = _lib.load(libpath)
    assert lib.nrs_status_string(0) == b"ok"
    assert lib.nrs_status_string(-3) == b"workspace too small"
    assert lib.nrs_version().startswith(b"nrs ")


def test_product_path_fails_loudly_without_library(tmp_path):
    from paper_2001_06468_amd import _lib
    saved = _lib._LIB
    _lib._LIB = None
    try:
        with pytest.raises(ImportError):
            _lib.load(str(tmp_path / "missing.so"))
    finally:
        _lib._LIB = saved
