"""The level tables built on the host against the way the step kernel reads them.

`tests/host/tables_check.cpp` is compiled with the library's table builder and
checks, for 49 schedules (1137 levels, T from 0 to 5e9): every level's buckets
and reject-all entry fit the LDS staging area where the kernel looks for them;
the band-test form, the one-bracket-read form and the direct-table form of the
acceptance test each equal d <= thr[u] (the Metropolis test of Algorithm 2 on
the 16-bit draw) for costs across the band, beyond it and at the ends of the int32
range; so does the per-draw estimate form (sign of d - glo + G(u) - 1, exact
entry only inside the measured window, G of the device's fp32 form with the
host's log2 in place of the device's), whose int32 sums never wrap for fields
up to the bound the host allows and offsets up to 2^30; the autotuner's timing window stays inside its schedule; and the host
guard of every step-kernel launch (job_range_error) passes every step range
inside a schedule and rejects ranges reaching step S or beyond, negative or
reversed ranges, offset increments above 2^30 and oversized shapes.  Planting
either of two past mistakes (the last bucket's cut clamped to tmax, a window
starting at S/3 for every S) makes it fail.  Host code only: runs on the CPU.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hipcc():
    for c in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return None


def test_level_tables_match_kernel_use(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found")
    csrc = os.path.join(ROOT, "paper_1806_08815_amd", "csrc")
    exe = str(tmp_path / "tables_check")
    cmd = [hipcc, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", csrc,
           os.path.join(ROOT, "tests", "host", "tables_check.cpp"),
           os.path.join(csrc, "da_tables.cpp"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-2000:]
    assert "failures 0" in r.stdout
