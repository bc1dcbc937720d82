"""Host check of the derivative-bin kernel's tables, without a GPU.

tests/host/grad_tables_emu.cpp builds the gradient chunk tables with the
library's host code (the gradient's launch shape: 512-row tiles, fewer rows
for small states; one row layout at N = 8 ... 28 and two at N = 34) and
evaluates the bins of two weighted (g, v) pairs from them the way k_grad_bins
reads them: each wave's share of a near chunk's QUAD members by row class with
the per-tile fold, far chunks, and the per-tile PAIR and DIAG outputs.  It
compares with the bins' definitions and checks that all lanes of an in-wave
sum group compute the same bin index and that each QUAD member is visited by
exactly one wave per tile.  The kernel source is compiled with hipcc (device
code included); nothing runs on a GPU.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2002_05725_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_grad_tables_match_bin_definitions(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "grad_tables_emu")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "host", "grad_tables_emu.cpp"),
           os.path.join(CSRC, "terms.cpp"), os.path.join(CSRC, "timing.cpp"), os.path.join(CSRC, "apply_h.hip"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("N=")]
    assert len(lines) == 6
    assert "layouts=2" in lines[-1]
