"""Host check of the apply kernel's chunk tables, without a GPU.

tests/host/apply_tables_emu.cpp builds the tables with the library's host code
(both row layouts, complex128 and complex64 chunk sizes, 8 rows per thread) and
evaluates H psi from them the way k_apply reads them: groups of three QUAD
masks sharing their source rows, single QUAD masks by row class, PAIR masks
(flat and row by row, from their staged row forms) and the diagonal.  It
compares with the direct sum over the term tables, for the full space and for
both fermion-parity sectors, whose tables (M - 1 qubits, implied top qubit) are
first compared with the full H on the sector state embedded in the full space.
The kernel source is compiled with hipcc (device code included); nothing runs
on a GPU.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2002_05725_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_apply_tables_match_direct_quad_sum(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "apply_tables_emu")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "host", "apply_tables_emu.cpp"),
           os.path.join(CSRC, "terms.cpp"), os.path.join(CSRC, "timing.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("N=")]
    assert len(lines) == 17
    assert sum("sector=0" in ln for ln in lines) == 2 and sum("sector=1" in ln for ln in lines) == 3
