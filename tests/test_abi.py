"""The C-ABI library loads and exports every entry point include/ffsga.h declares.

Runs without a GPU: loading the library does not touch the device.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1903_10741_amd", "libffsga.so")


def declared_functions():
    names = []
    for name in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not name.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", name)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                            text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ffs_decode", "ga_init", "ga_step", "ga_best", "reschedule", "ffs_prepare"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libffsga.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_the_abi():
    from paper_1903_10741_amd import ffsga
    assert set(ffsga.exported_symbols()) == set(declared_functions())


def test_strerror_is_host_only():
    from paper_1903_10741_amd import ffsga
    assert "power" in ffsga.ffs_strerror(ffsga.FFS_E_INFEASIBLE)
    assert ffsga.ffs_strerror(0) == "ok"
