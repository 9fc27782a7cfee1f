"""Host check of the particle position helpers of the HIP library (wrap into
the box, lattice cell of a coordinate): after a numerical failure positions
can be non-finite or far outside the box, and no node index may leave the
lattice.  Compiled for the host with hipcc."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_position_helpers_keep_indices_in_range():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "guards")
        subprocess.check_call([hipcc, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", "-Xclang",
                               "-target-feature", "-Xclang", "-packed-fp32-ops",
                               os.path.join(HERE, "native", "position_guards.cpp"), "-o", exe],
                              stderr=subprocess.DEVNULL)
        out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout
    assert out.stdout.strip().endswith("OK")
