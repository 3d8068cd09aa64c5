"""Host-only argument validation of the library (no device): light-curve arrays, the
CSR offsets and the per-event length cap (events longer than 2^28 points return
MORSE_ERANGE, since the kernels address an event's FP64 arrays with 32-bit byte
offsets).  The check is compiled for the host from the library's own header."""
import os
import subprocess

import pytest

from paper_1511_01157_amd import _abi

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def host_checks(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("hv") / "host_checks")
    subprocess.run(["/opt/rocm/bin/hipcc", "-std=c++17", "--cuda-host-only", "-x", "hip",
                    os.path.join(HERE, "host_checks.cpp"), "-o", exe], check=True,
                   capture_output=True)
    return subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()


def test_event_length_cap(host_checks):
    ok, too_long, too_short, bad_start, cap = (int(v) for v in host_checks)
    assert cap == 1 << 28
    assert ok == _abi.MORSE_OK
    assert too_long == _abi.MORSE_ERANGE
    assert too_short == _abi.MORSE_EINVAL
    assert bad_start == _abi.MORSE_EINVAL


def test_entry_points_share_the_check():
    src = os.path.join(HERE, "..", "paper_1511_01157_amd", "csrc")
    for f in ("api_search.hip", "api_refine.hip"):
        assert "check_lightcurves(ctx, lcs)" in open(os.path.join(src, f)).read(), f
