"""The blend kernels' block culling (csrc/cull.hpp, compiled for the host):
no 4 x 4 block that a splat's cut-off ellipse meets may be skipped, and no
flagged block may lie more than 0.03 px from it, over 400k random splats
(thin, round, rotated, large, on and off the tile).  The check program is
tests/native/cull_check.cpp."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2410_16978_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host compiler")
def test_band_blocks_never_drops_a_reached_block():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "cull_check")
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", CSRC, "-o", exe,
                               os.path.join(HERE, "native", "cull_check.cpp")])
        r = subprocess.run([exe, "400000"], capture_output=True, text=True, timeout=120)
    misses, loose, checked, flagged = (int(x) for x in r.stdout.split()[-4:])
    assert r.returncode == 0, r.stdout
    assert misses == 0 and loose == 0
    assert checked == 400000 * 16 and flagged > 0
