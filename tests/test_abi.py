"""The C-ABI library loads and exports every entry point include/mls.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "mls.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|mls_status|void)\s*(mls_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ("mls_ctx_create", "mls_ctx_destroy", "mls_build", "mls_interp", "mls_spread", "mls_sync"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1805_01113_amd import mls
    assert os.path.exists(mls.LIB_PATH), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(mls.LIB_PATH)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing
    lib.mls_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.mls_version()


def test_library_was_built_from_these_sources():
    """mls_version() carries the SHA-256 of the sources the library was
    compiled from; it must be that of csrc/ and include/mls.h as they are."""
    from paper_1805_01113_amd import build, mls
    lib = ctypes.CDLL(mls.LIB_PATH)
    lib.mls_version.restype = ctypes.c_char_p
    v = lib.mls_version().decode()
    assert v.endswith("src " + build.source_sha256()), (v, build.source_sha256())


def test_null_arguments_are_rejected_on_the_host():
    """Host-side argument checks return MLS_E_ARG before touching a device."""
    from paper_1805_01113_amd import mls
    lib = ctypes.CDLL(mls.LIB_PATH)
    lib.mls_ctx_create.argtypes = [ctypes.c_void_p] * 4
    assert lib.mls_ctx_create(None, None, None, None) == -1
    lib.mls_build.argtypes = [ctypes.c_void_p, ctypes.c_int64] + [ctypes.c_void_p] * 3 + [ctypes.c_int32] + [ctypes.c_void_p] * 4
    assert lib.mls_build(None, 0, None, None, None, 0, None, None, None, None) == -1
