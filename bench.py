#!/usr/bin/env python3
"""Benchmark of the 2D image FFT hot path on one MI355X.

A step is one forward and one inverse 2D FFT (the round trip) of one
1024 x 1024 complex64 image in FP32 through the C ABI, the image of the
paper's worked flop count (introduction).  Inputs are seeded synthetic
"gray images" (uniform integer pixels 0..255), already resident in HBM; 48
distinct input/output buffer sets rotate so that every step reads and writes
HBM rather than the 256 MB Infinity Cache.

Printed: ONE JSON line with
  value        GFLOP/s of the whole step, 5*M*N*log2(M*N) flops per transform
  roofline     for the dominant kernel: algorithmic bytes per launch (one read
               and one write of the image, 16*M*N) / its average launch
               duration, timed with events on the launch stream, against
               8 TB/s; traffic = FETCH_SIZE+WRITE_SIZE per launch from the
               committed rocprofv3 counter summary, or null if the kernel
               sources changed since it was taken
  cpu_baseline the FP64 oracle timed on this host's cores on a bounded sample
  extra        the same measurement at other sizes (context)

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "2D FFT GFLOP/s (5NMlog2NM) & % HBM roofline; serve p50/p99 ms vs plain FP32"


def kernel_source_hash() -> str:
    """Hash of the kernel sources the counter summary was taken with."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1505_08019_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """Per-launch HBM bytes of `kernel` from profiles/traffic.json, or None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


def time_round_trip(F, torch, rows, cols, steps, warmup, nbuf, kinds=("uniform",)):
    """Time `steps` forward+inverse round trips; returns a dict of results."""
    from paper_1505_08019_amd import inputs

    dev = torch.device("cuda:0")
    pf = F.Plan(rows, cols, F.FORWARD)
    pi = F.Plan(rows, cols, F.INVERSE)
    npass = pf.info()[0]
    host = [inputs.uniform_pixels(rows, cols, cfg_seed=2, index=i) for i in range(min(nbuf, 8))]
    xin = [torch.from_numpy(host[i % len(host)]).to(dev) for i in range(nbuf)]
    mid = [torch.empty_like(xin[0]) for _ in range(nbuf)]
    out = [torch.empty_like(xin[0]) for _ in range(nbuf)]
    stream = torch.cuda.current_stream()

    def step(k):
        b = k % nbuf
        pf.exec(xin[b], mid[b], stream)
        pi.exec(mid[b], out[b], stream)

    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    # Timed region: K steps between two events, nothing else on the stream.
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(steps):
        step(k)
    e1.record(stream)
    e1.synchronize()
    ms_step = e0.elapsed_time(e1) / steps

    # Kernel durations: the same steps again with an event between passes.
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps * 2 * npass + 1)]
    j = 0
    for k in range(steps):
        b = k % nbuf
        for plan, src, dst in ((pf, xin[b], mid[b]), (pi, mid[b], out[b])):
            for p in range(npass):
                evs[j].record(stream)
                j += 1
                plan.exec_pass(p, src, dst, stream)
    evs[j].record(stream)
    evs[j].synchronize()
    per_pass = [[] for _ in range(npass)]
    j = 0
    for k in range(steps):
        for _t in range(2):
            for p in range(npass):
                per_pass[p].append(evs[j].elapsed_time(evs[j + 1]))
                j += 1
    # Correctness guard on the timed output (round trip returns the input).
    torch.cuda.synchronize()
    b = (steps - 1) % nbuf
    err = (torch.linalg.vector_norm((out[b] - xin[b]).to(torch.complex128)) /
           torch.linalg.vector_norm(xin[b].to(torch.complex128))).item()
    sched = F.describe_schedule(rows, cols)
    pf.close()
    pi.close()
    del xin, mid, out
    torch.cuda.empty_cache()
    return {"ms_step": ms_step, "per_pass_ms": [sum(v) / len(v) for v in per_pass], "npass": npass,
            "round_trip_rel_l2": err, "schedule": sched}


def kernel_names(sched: str) -> list[str]:
    """Kernel template names of each pass in a schedule description."""
    import re
    names = []
    for m in re.finditer(r"(row|col)\(([^)]*)\)", sched):
        kv = dict(re.findall(r"(\w+)=(\d+)", m.group(2)))
        if m.group(1) == "row":
            names.append("pass_kernel<0,%s,%s>" % (kv["bn"], kv["j"]))
        else:
            names.append("pass_kernel<1,%s,%s>" % (kv["cb"], kv["nz"]))
    return names


def roofline_for(res, rows, cols):
    """Dominant kernel of a round trip: the pass with the largest time."""
    names = kernel_names(res["schedule"])
    totals = {}
    for name, ms in zip(names, res["per_pass_ms"]):
        totals.setdefault(name, []).append(ms)
    dom = max(totals, key=lambda n: sum(totals[n]))
    avg_ms = sum(totals[dom]) / len(totals[dom])
    alg = 16 * rows * cols
    achieved = alg / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": load_traffic(dom),
            "kernel": dom, "alg_bytes_per_launch": alg, "avg_launch_us": round(avg_ms * 1e3, 3)}


def cpu_baseline(rows, cols, seconds):
    """FP64 oracle round trips on all host cores for about `seconds`."""
    import oracle
    from paper_1505_08019_amd import inputs
    from paper_1505_08019_amd.metrics import flops_5nm

    x = inputs.uniform_pixels(rows, cols, cfg_seed=2)
    threads = oracle.max_threads()
    n = 0
    t0 = time.perf_counter()
    while True:
        X = oracle.fft2(x, -1, threads=0)
        oracle.fft2(X, +1, threads=0)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    gflops = 2 * flops_5nm(rows, cols) * n / el / 1e9
    return {"value": round(gflops, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": "%d forward+inverse round trips of one %dx%d uniform-pixel image, FP64 C oracle "
                      "(OpenMP over rows, then columns), %.1f s" % (n, rows, cols, el)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--buffers", type=int, default=48)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only; the transform of one image is not sharded "
              "across GPUs here (--gpus %d, WORLD_SIZE %d requested)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1505_08019_amd import fft2 as F
    from paper_1505_08019_amd.metrics import flops_5nm

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    F.lib()  # fails loudly if the HIP library is missing

    rows = cols = args.size
    res = time_round_trip(F, torch, rows, cols, args.steps, args.warmup, args.buffers)
    if not res["round_trip_rel_l2"] <= 2e-6:
        print("bench.py: round-trip check failed (%.3e)" % res["round_trip_rel_l2"], file=sys.stderr)
        sys.exit(1)
    flops_step = 2 * flops_5nm(rows, cols)
    value = flops_step / (res["ms_step"] * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_step"], 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": "%dx%d complex64 2D FFT, forward then inverse round trip, FP32 radix-2 DIT, "
                               "uniform 0..255 pixels, %d rotating HBM buffer sets" % (rows, cols, args.buffers),
                   "rows": rows, "cols": cols, "schedule": res["schedule"],
                   "round_trip_rel_l2": res["round_trip_rel_l2"]},
        "roofline": roofline_for(res, rows, cols),
    }
    if not args.no_extra:
        extra = {}
        for n, steps in ((4096, 20), (8192, 10)):
            r = time_round_trip(F, torch, n, n, steps, 3, 2)
            extra["%dx%d" % (n, n)] = {
                "ms_per_round_trip": round(r["ms_step"], 4),
                "gflops": round(2 * flops_5nm(n, n) / (r["ms_step"] * 1e-3) / 1e9, 1),
                "hbm_frac_whole_transform": round(2 * 16 * n * n * r["npass"] / (r["ms_step"] * 1e-3) / 1e9 /
                                                  HBM_PEAK_GBS, 4),
                "roofline": roofline_for(r, n, n),
                "round_trip_rel_l2": r["round_trip_rel_l2"],
            }
        line["extra"] = extra
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(rows, cols, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
