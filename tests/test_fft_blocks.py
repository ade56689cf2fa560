"""The small DFTs of the FFT passes, built for the host from the same header
(fft_core.h), against numpy's FFT: every supported radix, both directions,
including the prime-factor (coprime) splits and the upper-half-zero DFT used
by the pruned first stage. CPU only (hipcc compiles the host side)."""

import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1010_1456_amd", "csrc")


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    pytest.skip("hipcc not available")


@pytest.fixture(scope="module")
def lines():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "fft_blocks")
        subprocess.run([_hipcc(), "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                        "-I", CSRC, os.path.join(HERE, "fft_blocks_check.cpp"), "-o", exe],
                       check=True, capture_output=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    rows = {}
    for ln in out.splitlines():
        R, inv, uz, k, re, im = ln.split()
        rows.setdefault((int(R), int(inv), int(uz)), {})[int(k)] = complex(float(re), float(im))
    return rows


def test_every_radix_and_direction(lines):
    radices = sorted({k[0] for k in lines})
    assert radices == [2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 14, 16, 18]
    for (R, inv, uz), got in lines.items():
        i = np.arange(R)
        x = np.sin(1.3 * i + 0.2) + 1j * np.cos(0.7 * i * i)
        if uz:
            x[R // 2:] = 0
        ref = np.fft.ifft(x) * R if inv else np.fft.fft(x)
        g = np.array([got[k] for k in range(R)])
        assert np.abs(g - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()), (R, inv, uz)


def test_line_maps_stay_in_bounds():
    """Line selection with fields innermost or field-major, as the z passes
    use them: every pass line, and the clamped line of threads past the last
    one, reads an in-bounds selection entry and addresses an in-bounds line
    (a tail thread once read past the selection table)."""
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "fft_map_check")
        subprocess.run([_hipcc(), "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                        "-I", CSRC, os.path.join(HERE, "fft_map_check.cpp"), "-o", exe],
                       check=True, capture_output=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    rows = [ln.split() for ln in out.splitlines()]
    assert len(rows) == 9
    for name, max_sel, nsel, max_first, max_last, limit in rows:
        assert int(max_sel) == int(nsel) - 1, name
        assert 0 <= int(max_first) and int(max_last) < int(limit), name


def test_fast_division_matches_integer_division():
    """The x pass divides its work number by the field and tile counts with a
    multiply-high and a shift: it equals integer division for every divisor
    and numerator the check program tries (all divisors up to 4096, powers of
    two and their neighbours, random divisors up to 2^31 - 1; numerators at
    multiples of the divisor and their neighbours, and random ones)."""
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "fastdiv_check")
        subprocess.run([_hipcc(), "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                        "-I", CSRC, os.path.join(HERE, "fastdiv_check.cpp"), "-o", exe],
                       check=True, capture_output=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    assert out[0] == "checked" and int(out[1]) > 1_000_000, out
    assert out[2] == "mismatches" and int(out[3]) == 0, out
