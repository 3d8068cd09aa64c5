"""The C-ABI library loads and exports every entry point include/morse.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1511_01157_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "morse.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(morse_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("morse_build_map", "morse_search", "morse_refine", "morse_chi2_grad",
              "morse_autotune", "morse_rayshoot", "morse_normalize_convolve"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = _abi.load()
    for n in declared():
        assert hasattr(lib, n), n
    assert set(declared()) == set(_abi.SIGNATURES)


def test_abi_version_matches_header():
    txt = open(os.path.join(ROOT, "include", "morse.h")).read()
    v = int(re.search(r"#define MORSE_ABI_VERSION (\d+)", txt).group(1))
    assert _abi.load().morse_abi_version() == v


def test_struct_layouts_match_header():
    assert ctypes.sizeof(_abi.Grid2D) == 40
    assert ctypes.sizeof(_abi.MapView) == 48
    assert ctypes.sizeof(_abi.LightCurves) == 48
    assert ctypes.sizeof(_abi.Trajectories) == 72
    assert ctypes.sizeof(_abi.SearchOut) == 64
    assert ctypes.sizeof(_abi.LbfgsOpts) == 32
    assert ctypes.sizeof(_abi.MapStats) == 48


def test_null_arguments_fail_without_device_work():
    lib = _abi.load()
    assert lib.morse_ctx_create(0, None, None) == _abi.MORSE_EINVAL
    assert b"NULL" in lib.morse_last_error(None)
    assert lib.morse_build_map(None, 1.0, 0.1, None, None, 0.0, None, None, None) == _abi.MORSE_EINVAL
    assert lib.morse_search(None, None, 0, None, None, 0, None) == _abi.MORSE_EINVAL
    assert lib.morse_ctx_set_timing(None, 1) == _abi.MORSE_EINVAL
    assert lib.morse_autotune_load(None, b"x.json", None) == _abi.MORSE_EINVAL
    assert lib.morse_ctx_kernel_time(None, 0, None, None, 0) == _abi.MORSE_EINVAL
    assert lib.morse_convolve_stack(None, None, None, None, None, 0, 0.5, 0, None) == _abi.MORSE_EINVAL
    rx, ry = ctypes.c_int32(), ctypes.c_int32()
    assert lib.morse_profile_weights(0.01, 1e-3, 1e-3, 0.5, None, 0, None, None) == _abi.MORSE_EINVAL
    assert lib.morse_profile_weights(0.01, 1e-3, 1e-3, 1.5, None, 0, ctypes.byref(rx), ctypes.byref(ry)) == _abi.MORSE_EINVAL
    assert lib.morse_profile_weights(-1.0, 1e-3, 1e-3, 0.5, None, 0, ctypes.byref(rx), ctypes.byref(ry)) == _abi.MORSE_EINVAL
    assert lib.morse_ctx_destroy(None) == _abi.MORSE_OK
