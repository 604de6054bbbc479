"""LDS exchange layouts of the FP32 pass kernels, checked on the host.

The layouts are compile-time objects (engine.hpp); a small host program
includes the same header and walks every instantiated schedule: each
exchange must be a permutation of the chunk onto the LDS words and
free of bank conflicts for 16- and 32-lane groups of 8-byte accesses."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which(HIPCC)), reason="hipcc not available")
def test_every_schedule_exchange_is_a_conflict_free_permutation(tmp_path):
    exe = str(tmp_path / "lds_layout_check")
    cmd = [HIPCC, "-std=c++17", "-O1", "-x", "hip", "--offload-arch=gfx950", "--cuda-host-only",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_1505_08019_amd", "csrc"),
           os.path.join(ROOT, "tests", "lds_layout_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok ") and int(out.stdout.split()[1]) > 400, out.stdout


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which(HIPCC)), reason="hipcc not available")
def test_split_form_index_arithmetic(tmp_path):
    """LDS words, digit-reversed positions, step-table reads and the XCD
    chunk order of the MFMA forms, for every shape the forms accept
    (tests/split_layout_check.cpp)."""
    exe = str(tmp_path / "split_layout_check")
    cmd = [HIPCC, "-std=c++17", "-O1", "-x", "hip", "--offload-arch=gfx950", "--cuda-host-only",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_1505_08019_amd", "csrc"),
           os.path.join(ROOT, "tests", "split_layout_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    fields = out.stdout.split()
    assert fields[0] == "ok" and int(fields[1]) > 100 and int(fields[3]) > 10000, out.stdout
