"""bench.py on the host (no GPU): the one-GPU rule, kernel names of a plan
description, and the roofline figure it derives from measured launch times."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_kernel_names_of_a_plan_description():
    desc = ("row(bn=10,j=2,nreg=3,grid=256,threads=512) "
            "col(cb=4,nz=8,s_lo=2,nreg=3,grid=256,threads=512)")
    assert bench.kernel_names(desc) == ["pass_kernel<0,10,2,3,false>", "pass_kernel<1,4,8,3,false>"]
    # a ping-pong variant is the kernel with register-bit code nreg + 8
    desc = ("row(bn=10,j=2,nreg=3,pingpong,grid=256,threads=512) "
            "col(cb=4,nz=8,s_lo=2,nreg=3,grid=256,threads=512)")
    assert bench.kernel_names(desc) == ["pass_kernel<0,10,2,11,false>", "pass_kernel<1,4,8,3,false>"]


def test_roofline_uses_algorithmic_bytes_over_launch_time():
    # 1024^2: 16 MiB per pass; 8 us per launch -> 2097.152 GB/s
    res = {"kernel_share": {"pass_kernel<0,10,2,3,false>": 0.6, "pass_kernel<1,4,8,3,false>": 0.4},
           "kernel_ms": {"pass_kernel<0,10,2,3,false>": 0.008, "pass_kernel<1,4,8,3,false>": 0.006}}
    r = bench.roofline_for(res, 1024, 1024, copy_gbs=6000.0)
    assert r["kernel"] == "pass_kernel<0,10,2,3,false>"
    assert r["alg_bytes_per_launch"] == 16 * 1024 * 1024
    assert abs(r["achieved"] - 2097.2) < 0.05
    assert r["peak"] == 8000.0 and r["unit"] == "GB/s" and r["bound"] == "hbm"
    assert abs(r["frac"] - 2097.152 / 8000.0) < 1e-4
    assert abs(r["frac_of_copy"] - 2097.152 / 6000.0) < 1e-4
