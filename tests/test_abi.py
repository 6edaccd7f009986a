"""The C-ABI libraries load and export every entry point their headers declare:
include/ffsga.h and include/ffs_surrogate.h for libffsga.so, include/ffs_peaks.h
for libffspeaks.so.

Runs without a GPU: loading a library does not touch the device.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1903_10741_amd", "libffsga.so")
PEAKS_LIB = os.path.join(ROOT, "paper_1903_10741_amd", "libffspeaks.so")
PEAKS_HEADERS = ("ffs_peaks.h",)
FFS_E_INVAL, FFS_E_DEVICE = -1, -4  # include/ffsga.h


def test_every_header_belongs_to_a_library():
    headers = {n for n in os.listdir(os.path.join(ROOT, "include")) if n.endswith(".h")}
    assert headers == {"ffsga.h", "ffs_surrogate.h", *PEAKS_HEADERS}


def declared_functions(peaks=False):
    names = []
    for name in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not name.endswith(".h") or (name in PEAKS_HEADERS) != peaks:
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


def test_peaks_library_exports_its_header():
    if not os.path.exists(PEAKS_LIB):
        pytest.fail("libffspeaks.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(PEAKS_LIB)
    names = declared_functions(peaks=True)
    assert names == ["ffs_peak_mfma_bf16", "ffs_peak_valu_int32"]
    assert all(hasattr(lib, n) for n in names)
    from paper_1903_10741_amd import peaks
    assert set(peaks.exported_symbols()) == set(names)


def test_strerror_is_host_only():
    from paper_1903_10741_amd import ffsga
    assert "power" in ffsga.ffs_strerror(ffsga.FFS_E_INFEASIBLE)
    assert ffsga.ffs_strerror(0) == "ok"


def test_island_group_setter_checks_its_argument():
    """ga_set_island_groups rejects counts outside 0..4 before any device call, and
    1 (every launch on the caller's stream) needs no streams: both run without a
    GPU. The default (0) is restored afterwards; without a device that call can
    only report FFS_E_DEVICE for the streams it could not create."""
    lib = ctypes.CDLL(LIB)
    lib.ga_set_island_groups.argtypes = [ctypes.c_int32]
    lib.ga_set_island_groups.restype = ctypes.c_int
    try:
        assert lib.ga_set_island_groups(-1) == FFS_E_INVAL
        assert lib.ga_set_island_groups(5) == FFS_E_INVAL
        assert lib.ga_set_island_groups(1) == 0
    finally:
        assert lib.ga_set_island_groups(0) in (0, FFS_E_DEVICE)
