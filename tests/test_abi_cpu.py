"""CPU checks of the C-ABI boundary: the library loads and exports every function
that include/aslam.h declares, and the binding covers the same set (no compute
calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", fn)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(aslam_[a-z0-9_]+)\s*\(", txt))
    return names


@pytest.fixture(scope="module")
def libaslam():
    from paper_2603_25834_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2603_25834_amd import build
        build.build_library()
    return ctypes.CDLL(_lib.LIB_PATH)


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for must in ("aslam_env_create", "aslam_env_reset", "aslam_env_step", "aslam_env_observe",
                 "aslam_env_destroy", "aslam_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(libaslam):
    for name in sorted(declared_functions()):
        assert hasattr(libaslam, name), f"{name} declared but not exported"


def test_binding_covers_the_header():
    from paper_2603_25834_amd import _lib
    assert set(_lib.SIGNATURES) == declared_functions()


def test_last_error_is_callable_without_gpu(libaslam):
    libaslam.aslam_last_error.restype = ctypes.c_char_p
    assert libaslam.aslam_last_error() is not None
