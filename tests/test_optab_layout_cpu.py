"""The generator table that maps a connection (holes, particles) to its pool
operator: every single and every spin-conserving double of a complete pool
gets its own slot inside the table, for several orbital counts.  The layout
functions are host-and-device code; this test compiles them for the host
(no GPU) and walks every operator."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2411_07920_amd", "csrc")


def test_generator_table_slots_are_unique(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "optab_layout")
    subprocess.run([hipcc, "--offload-host-only", "-O1", "-I", CSRC,
                    os.path.join(HERE, "host", "optab_layout.cpp"), "-o", exe],
                   check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    lines = dict(l.split(" ", 1) for l in out.stdout.splitlines())
    assert lines["bad"] == "0"
    # at 26 spatial orbitals the complete pool (301,600 operators) fills the
    # table without collisions
    assert "nsp 26 size 334776 used 301600" in out.stdout
