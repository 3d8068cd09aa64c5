"""Host logic of the library without a device: caustic geometry (Aberth-Ehrlich roots
of the critical-curve quartic, nearest-next-phase joins, bounding boxes) and the
caustic-centred lines, against the oracle (companion-matrix roots of the same quartic)."""
import ctypes

import numpy as np
import pytest

import paper_1511_01157_amd as M
from paper_1511_01157_amd import _abi
from oracle.lines import caustic_components, caustic_lines


@pytest.mark.parametrize("s,q", [(0.6, 1.0), (1.0, 1.0), (2.5, 1.0), (0.8, 5e-3), (0.5, 1e-4),
                                 (2.0, 1e-4), (1.2, 0.3), (1.0, 1e-3)])
def test_caustics_match_oracle(s, q):
    a = M.caustics(s, q, 4096)
    b = caustic_components(s, q, 4096)
    assert a.shape == b.shape
    scale = np.maximum(b[:, 4:5], 1e-12)
    assert np.all(np.abs(a - b) <= 1e-9 * np.maximum(scale, np.abs(b)))


def test_lines_match_oracle_bitwise():
    c = M.caustics(0.8, 5e-3, 2048)
    r = np.linspace(0.0, 4.0, 9)
    phi = np.linspace(0.0, 2 * np.pi, 33)[:-1]
    assert np.array_equal(M.caustic_lines(c, r, phi), caustic_lines(c, r, phi))


def test_caustic_argument_errors():
    lib = _abi.load()
    n = ctypes.c_int32()
    assert lib.morse_caustics(1.0, 0.0, 1024, None, 0, ctypes.byref(n)) == _abi.MORSE_EINVAL
    assert lib.morse_caustics(-1.0, 0.5, 1024, None, 0, ctypes.byref(n)) == _abi.MORSE_EINVAL
    assert lib.morse_caustics(1.0, 0.5, 8, None, 0, ctypes.byref(n)) == _abi.MORSE_EINVAL
    assert lib.morse_caustics(0.6, 1.0, 1024, None, 0, ctypes.byref(n)) == _abi.MORSE_OK and n.value == 3
    out = (ctypes.c_double * 5)()
    assert lib.morse_caustics(0.6, 1.0, 1024, out, 1, ctypes.byref(n)) == _abi.MORSE_ERANGE
    assert lib.morse_caustic_lines(None, 1, None, 1, None, 1, None) == _abi.MORSE_EINVAL
    assert lib.morse_line_filter(None, None, None, 0, 1.0, None, None, None, None, None) == _abi.MORSE_EINVAL
    assert lib.morse_lines_to_trajectories(None, None, None, 0, None, 0, None, 0, None) == _abi.MORSE_EINVAL
