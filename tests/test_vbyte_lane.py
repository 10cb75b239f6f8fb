"""The device VByte decoder's per-lane arithmetic, run on the host.

`vdecode_lane` (csrc/vbyte.hpp) is plain integer code compiled for both the
device and the host.  tests/vbyte_lane_check.cpp emulates one wave of it over
2,000 random lists (gaps of 1 byte up to five-byte values near 2^32, streams
starting 0-3 bytes into a word) against an encoder written there from the
format's definition, so a mistake in byte packing, value length, start
detection or the window step fails here without a GPU.
"""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2307_01716_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_vdecode_lane_on_host(tmp_path):
    exe = str(tmp_path / "vbyte_lane_check")
    # host pass only: the check runs on the CPU
    subprocess.check_call([HIPCC, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17", "-I", CSRC,
                           os.path.join(HERE, "vbyte_lane_check.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert " 0 mismatches" in out.stdout
