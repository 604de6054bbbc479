#!/usr/bin/env python3
"""Benchmark of the 2D image FFT hot path on one MI355X.

A step is one forward and one inverse 2D FFT (the round trip) of one
1024 x 1024 complex64 image in FP32 through the C ABI, the image of the
paper's worked flop count (introduction).  Inputs are seeded synthetic
"gray images" (uniform integer pixels 0..255), already resident in HBM; 48
distinct input/intermediate/output buffer sets (1.15 GB) rotate with one
counter that runs on through the warm-up, the timed steps and the per-pass
loops, so a set is reused only after all 48 have been (4.5x the 256 MB
Infinity Cache): every step reads and writes HBM, whatever --steps is.  The pass schedules come from the
table of autotuned schedules that ships with the library.

Printed: ONE JSON line with
  value        GFLOP/s of the whole step, 5*M*N*log2(M*N) flops per transform
  roofline     for the dominant kernel: algorithmic bytes per launch (one read
               and one write of the image, 16*M*N) / its average launch
               duration, timed with events on the launch stream, against
               8 TB/s; traffic = counter bytes per launch from the committed
               rocprofv3 record (FETCH_SIZE and WRITE_SIZE scaled by the
               reference copy), or null if the kernel sources changed since
  cpu_baseline the FP64 oracle timed on this host's cores on a bounded sample
  extra        context: other sizes, the MFMA precision forms, the ragged
               persistent batch against per-image launches

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1505_08019_amd.prof import COPY_ELEMS, COPY_BYTES, kernel_source_hash, normalise  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "2D FFT GFLOP/s (5NMlog2NM) & % HBM roofline; serve p50/p99 ms vs plain FP32"
PASS_KIND = {"row": 0, "col": 1}


def log(msg: str) -> None:
    """Progress on stderr (the result line goes to stdout)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def load_traffic(kernel: str, record: str = "bench_default_traffic.json"):
    """Per-launch HBM bytes of `kernel` from a counter record under profiles/
    (taken on the workload the record names), or None if there is none or
    the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", record)
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


def kernel_names(desc: str) -> list[str]:
    """Kernel names (as rocprofv3 reports them, normalised) of each pass of a plan description."""
    import re
    names = []
    for m in re.finditer(r"(row|col)\(([^)]*)\)", desc):
        kv = dict(re.findall(r"(\w+)=(\d+)", m.group(2)))
        b1, b2 = (kv["bn"], kv["j"]) if m.group(1) == "row" else (kv["cb"], kv["nz"])
        code = int(kv["nreg"]) + (8 if "pingpong" in m.group(2) else 0)  # ping-pong variants: register bits + 8
        names.append(normalise("pass_kernel<%d, %s, %s, %d, false>" % (PASS_KIND[m.group(1)], b1, b2, code)))
    return names


def copy_reference(torch, reps=10):
    """Bandwidth of a plain streaming copy (float32 multiply by one) of COPY_BYTES.

    It also gives the counter calibration: the same launches appear in the
    FETCH_SIZE / WRITE_SIZE runs of this script."""
    a = torch.ones(COPY_ELEMS, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(2):
        torch.mul(a, 1.0, out=b)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * COPY_BYTES / (ms * 1e-3) / 1e9


def time_round_trip(F, torch, rows, cols, steps, warmup, nbuf, precision=None, per_pass=True):
    """Time `steps` forward+inverse round trips; returns a dict of results."""
    from paper_1505_08019_amd import inputs

    precision = F.PREC_FP32 if precision is None else precision
    dev = torch.device("cuda:0")
    pf = F.Plan(rows, cols, F.FORWARD, precision)
    pi = F.Plan(rows, cols, F.INVERSE, precision)
    npass = pf.info()[0]
    host = [inputs.uniform_pixels(rows, cols, cfg_seed=2, index=i) for i in range(min(nbuf, 8))]
    xin = [torch.from_numpy(host[i % len(host)]).to(dev) for i in range(nbuf)]
    mid = [torch.empty_like(xin[0]) for _ in range(nbuf)]
    out = [torch.empty_like(xin[0]) for _ in range(nbuf)]
    stream = torch.cuda.current_stream()
    rot = [0]  # buffer-set counter, continued across every loop below

    def next_set():
        b = rot[0] % nbuf
        rot[0] += 1
        return b

    def step():
        b = next_set()
        pf.exec(xin[b], mid[b], stream)
        pi.exec(mid[b], out[b], stream)
        return b

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # Timed region: K steps between two events, nothing else on the stream.
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        b = step()
    e1.record(stream)
    e1.synchronize()
    ms_step = e0.elapsed_time(e1) / steps
    # Correctness guard on the timed output (round trip returns the input).
    err = (torch.linalg.vector_norm((out[b] - xin[b]).to(torch.complex128)) /
           torch.linalg.vector_norm(xin[b].to(torch.complex128))).item()

    res = {"ms_step": ms_step, "npass": npass, "round_trip_rel_l2": err,
           "schedule": [pf.describe(), pi.describe()], "buffer_sets": nbuf,
           "buffer_set_bytes": 3 * 8 * rows * cols}
    if per_pass:
        # Average duration of each pass kernel: `steps` back-to-back launches
        # of that pass alone (rotating buffers) between two events on the
        # launch stream, the way a profiler's kernel trace averages them.
        names = kernel_names(pf.describe()) + kernel_names(pi.describe())
        times, share = {}, {}
        t = 0
        for plan, src, dst in ((pf, xin, mid), (pi, mid, out)):
            for p in range(npass):
                e0.record(stream)
                for _ in range(steps):
                    b = next_set()
                    plan.exec_pass(p, src[b], dst[b], stream)
                e1.record(stream)
                e1.synchronize()
                ms = e0.elapsed_time(e1) / steps
                times.setdefault(names[t], []).append(ms)
                share[names[t]] = share.get(names[t], 0.0) + ms
                t += 1
        res["kernel_ms"] = {n: sum(v) / len(v) for n, v in times.items()}
        res["kernel_share"] = share
    pf.close()
    pi.close()
    del xin, mid, out
    torch.cuda.empty_cache()
    return res


def timing_detail(F, torch, rows, cols, nbuf, k=100, repeats=20, replays=20, shots=20):
    """Three more views of the round trip: `repeats` timings of `k`
    back-to-back round trips (median, min, max), a HIP graph of one round
    trip per buffer set replayed `replays` times, and single-shot latency
    (one round trip from an idle stream; GPU time between events and host
    wall time to completion).  Buffer sets rotate as in the timed region."""
    import statistics
    from paper_1505_08019_amd import inputs

    dev = torch.device("cuda:0")
    pf = F.Plan(rows, cols, F.FORWARD)
    pi = F.Plan(rows, cols, F.INVERSE)
    host = [inputs.uniform_pixels(rows, cols, cfg_seed=2, index=i) for i in range(min(nbuf, 8))]
    xin = [torch.from_numpy(host[i % len(host)]).to(dev) for i in range(nbuf)]
    mid = [torch.empty_like(xin[0]) for _ in range(nbuf)]
    out = [torch.empty_like(xin[0]) for _ in range(nbuf)]
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rot = [0]

    def step(st):
        b = rot[0] % nbuf
        rot[0] += 1
        pf.exec(xin[b], mid[b], st)
        pi.exec(mid[b], out[b], st)
        return b

    def check(b):
        return (torch.linalg.vector_norm((out[b] - xin[b]).to(torch.complex128)) /
                torch.linalg.vector_norm(xin[b].to(torch.complex128))).item()

    for _ in range(nbuf):
        step(s)
    torch.cuda.synchronize()
    per = []
    for _ in range(repeats):
        e0.record(s)
        for _ in range(k):
            step(s)
        e1.record(s)
        e1.synchronize()
        per.append(e0.elapsed_time(e1) / k)
    res = {"repeats": {"round_trips_each": k, "repeats": repeats, "median_ms_per_round_trip":
                       round(statistics.median(per), 6), "min_ms": round(min(per), 6), "max_ms": round(max(per), 6)}}

    # Graph: every buffer set once, captured on a side stream, replayed on `s`.
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    rot[0] = 0
    with torch.cuda.graph(g, stream=cap, capture_error_mode="relaxed"):
        for _ in range(nbuf):
            step(cap)
    for y in out:
        y.zero_()
    g.replay()
    torch.cuda.synchronize()
    errs = [check(b) for b in range(nbuf)]
    e0.record(s)
    for _ in range(replays):
        g.replay()
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / (replays * nbuf)
    res["graph"] = {"round_trips_per_replay": nbuf, "replays": replays, "ms_per_round_trip": round(ms, 6),
                    "max_round_trip_rel_l2": max(errs)}
    del g

    # Single shot: the stream drained before each round trip.
    ev, wall = [], []
    for _ in range(shots):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(s)
        b = step(s)
        e1.record(s)
        e1.synchronize()
        wall.append((time.perf_counter() - t0) * 1e6)
        ev.append(e0.elapsed_time(e1) * 1e3)
    res["single_shot"] = {"shots": shots, "median_us_gpu_events": round(statistics.median(ev), 2),
                          "median_us_host_wall": round(statistics.median(wall), 2), "rel_l2": check(b)}
    pf.close()
    pi.close()
    del xin, mid, out
    torch.cuda.empty_cache()
    return res


def roofline_for(res, rows, cols, copy_gbs=None, traffic_record="bench_default_traffic.json"):
    """Dominant kernel of a round trip: the kernel with the largest total time.
    `traffic_record` is the counter record taken on this workload, or None."""
    dom = max(res["kernel_share"], key=res["kernel_share"].get)
    avg_ms = res["kernel_ms"][dom]
    alg = 16 * rows * cols
    achieved = alg / (avg_ms * 1e-3) / 1e9
    r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 4),
         "traffic": load_traffic(dom, traffic_record) if traffic_record else None,
         "kernel": dom, "alg_bytes_per_launch": alg, "avg_launch_us": round(avg_ms * 1e3, 3),
         "kernels_avg_us": {n: round(v * 1e3, 3) for n, v in res["kernel_ms"].items()}}
    if copy_gbs:
        r["copy_gbs"] = round(copy_gbs, 1)
        r["frac_of_copy"] = round(achieved / copy_gbs, 4)
    return r


def precision_forms(F, torch, flops):
    """The MFMA precision forms against FP32 at 1024^2 and 4096^2 (round trips)."""
    out = {}
    for n, steps, nbuf in ((1024, 100, 48), (4096, 20, 4)):
        for name, prec in (("fp32", F.PREC_FP32), ("split_bf16", F.PREC_SPLIT_BF16), ("fp16", F.PREC_FP16)):
            r = time_round_trip(F, torch, n, n, steps, 3, nbuf, precision=prec, per_pass=False)
            out["%dx%d_%s" % (n, n, name)] = {
                "ms_per_round_trip": round(r["ms_step"], 4),
                "gflops_nominal": round(2 * flops(n, n) / (r["ms_step"] * 1e-3) / 1e9, 1),
                "hbm_frac_whole_transform": round(2 * 16 * n * n * r["npass"] / (r["ms_step"] * 1e-3) / 1e9 /
                                                  HBM_PEAK_GBS, 4),
                "round_trip_rel_l2": r["round_trip_rel_l2"]}
    return out


def real_transforms(F, torch, flops):
    """Real-image transforms (R2C forward, C2R inverse, and the 2D DCT-II built
    on them) of uniform-pixel images
    against the complex transform of the same image, with rotating buffer
    sets past the Infinity Cache.  Bytes: the complex transform of the
    rows x cols/2 image read as complex pairs (two passes, 16 B per complex
    value each) plus the split kernel (reads rows x cols/2, writes
    rows x (cols/2+1) complex values): about 24 B per real pixel, against 32
    for the complex transform."""
    out = {}
    for n, steps, nbuf in ((1024, 100, 48), (8192, 10, 2)):
        g = torch.Generator(device="cuda:0")
        g.manual_seed(6)
        xs = [torch.randint(0, 256, (n, n), generator=g, device="cuda:0", dtype=torch.int32).to(torch.float32)
              for _ in range(nbuf)]
        hs = [torch.empty((n, n // 2 + 1), dtype=torch.complex64, device="cuda:0") for _ in range(nbuf)]
        ys = [torch.empty_like(xs[0]) for _ in range(nbuf)]
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        res = {}
        with F.RealPlan(n, n) as pf, F.RealPlan(n, n, F.INVERSE) as pi:
            for label, fn in (("r2c", lambda b: pf.exec(xs[b], hs[b], s)), ("c2r", lambda b: pi.exec(hs[b], ys[b], s))):
                for b in range(min(3, nbuf)):
                    fn(b)
                e0.record(s)
                for k in range(steps):
                    fn((k + 3) % nbuf)
                e1.record(s)
                e1.synchronize()
                ms = e0.elapsed_time(e1) / steps
                alg = 16 * n * n + 4 * n * n + 8 * n * (n // 2 + 1)
                res[label] = {"ms": round(ms, 4), "gflops_nominal_real": round(0.5 * flops(n, n) / (ms * 1e-3) / 1e9, 1),
                              "alg_bytes": alg, "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            b = (steps + 2) % nbuf
            err = (torch.linalg.vector_norm((ys[b] - xs[b]).double()) / torch.linalg.vector_norm(xs[b].double())).item()
            res["round_trip_rel_l2"] = err
        # 2D DCT-II through the real-image transform (reorder, R2C, twiddle post-process)
        with F.DctPlan(n, n) as pd:
            for b in range(min(3, nbuf)):
                pd.exec(xs[b], ys[b], s)
            e0.record(s)
            for k in range(steps):
                pd.exec(xs[(k + 3) % nbuf], ys[(k + 3) % nbuf], s)
            e1.record(s)
            e1.synchronize()
            res["dct2"] = {"ms": round(e0.elapsed_time(e1) / steps, 4)}
        out["%dx%d" % (n, n)] = res
        del xs, hs, ys
        torch.cuda.empty_cache()
    return out


def ragged_batch(F, torch, flops, reps=5):
    """512 ragged images (sides 64..2048, a quarter rectangular) in one persistent
    launch, FP32 and split BF16, against one fft2_exec per image on one stream."""
    from paper_1505_08019_amd import inputs

    shapes = inputs.ragged_shapes()
    points = sum(r * c for r, c in shapes)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(4)
    xs = [torch.randint(0, 256, (r, c), generator=g, device="cuda:0", dtype=torch.int32).to(torch.complex64)
          for r, c in shapes]
    ys = [torch.empty_like(x) for x in xs]
    alg = sum((16 if r * c <= 16384 else 32) * r * c for r, c in shapes)
    nom = sum(flops(r, c) for r, c in shapes)
    s = torch.cuda.current_stream()
    res = {"images": len(shapes), "points": points, "alg_bytes": alg}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            fn()
        e1.record(s)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    plans = {}
    for sh in set(shapes):
        plans[sh] = F.Plan(sh[0], sh[1], F.FORWARD)

    def per_image():
        for x, y in zip(xs, ys):
            plans[x.shape].exec(x, y, s)

    ms = timed(per_image)
    res["per_image_fp32"] = {"ms": round(ms, 3), "gflops_nominal": round(nom / (ms * 1e-3) / 1e9, 1),
                             "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    for p in plans.values():
        p.close()
    for name, prec in (("batch_fp32", F.PREC_FP32), ("batch_split_bf16", F.PREC_SPLIT_BF16)):
        with F.Batch(shapes, F.FORWARD, prec) as b:
            b.exec(xs, ys, s)
            ms = timed(lambda: b.exec(None, None, s))
            msg = timed(lambda: b.exec(None, None, s, graph=True))
            ok = b.status() == 0
        res[name] = {"ms": round(ms, 3), "ms_graph": round(msg, 3), "waits_ok": ok,
                     "gflops_nominal": round(nom / (min(ms, msg) * 1e-3) / 1e9, 1),
                     "hbm_frac": round(alg / (min(ms, msg) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    del xs, ys
    torch.cuda.empty_cache()
    return res


def serve_trace(F, torch, rates=(2000, 5000, 10000, 20000, 50000), min_requests=20000, seconds=2.0,
                spot_checks=8):
    """Poisson arrivals of Gaussian-filter requests (square sides 64..4096,
    log-uniform; FP32 / split BF16 50/50; cutoff 0.05..0.5), buffers already
    in HBM.  Each rate runs min(min_requests, rate * seconds) requests, and
    at least min_requests from 10k req/s up.  Every side has its own pools of
    input and output images, each at least 512 MB (more than twice the 256 MB
    Infinity Cache) and at least 64 images (8 slots x groups of 8): request
    i reads input i mod K and writes the next output of its side's pool, so
    no two requests in flight share an output and every request streams from
    HBM.  Each trace is replayed through the serving loop (8 launch slots,
    groups of up to 8, 64 GB budget) as drawn, again with every request in
    FP32, through a server whose groups put 4 or more small FP32 requests in
    one persistent launch (groups of up to 16), and FIFO on one stream
    through the plain per-image FP32 filter.  Latency is arrival to
    completion.  After each served leg the last request of each side is run
    again alone and must give the same bits."""
    import numpy as np
    from paper_1505_08019_amd import inputs

    sides = [1 << e for e in range(6, 13)]
    g = torch.Generator(device="cuda:0")
    g.manual_seed(5)
    pool_bytes = 512 << 20
    bufs = {}
    for sd in sides:
        img = 8 * sd * sd
        k_in = max(2, pool_bytes // img)
        k_out = max(64, pool_bytes // img)
        xin = torch.randint(0, 256, (k_in, sd, sd), generator=g, device="cuda:0",
                            dtype=torch.int32).to(torch.complex64)
        xout = torch.empty((k_out, sd, sd), dtype=torch.complex64, device="cuda:0")
        bufs[sd] = (xin, xout)
    plans = {sd: F.Plan(sd, sd, F.FORWARD, F.PREC_FP32) for sd in sides}
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    out = {"pool_bytes_per_side_min": pool_bytes,
           "pool_images": {str(sd): [int(bufs[sd][0].shape[0]), int(bufs[sd][1].shape[0])] for sd in sides}}

    def spot_check(last):
        """Each side's last served request against the same request alone (bits)."""
        ok = 0
        for sd, (i_in, i_out, p, cut) in last.items():
            xin, xout = bufs[sd]
            with F.Plan(sd, sd, F.FORWARD, p) as pl:
                alone = pl.exec_filter(xin[i_in], cut)
            torch.cuda.synchronize()
            ok += int(torch.equal(alone, xout[i_out]))
        return ok, len(last)

    with F.Server(hbm_budget_bytes=64 << 30, inflight=8, max_batch=8) as srv, \
            F.Server(hbm_budget_bytes=64 << 30, inflight=8, max_batch=16, persistent_min=4) as srvp:
        for sv in (srv, srvp):
            for sd in sides:  # plans of every class, outside the measurement
                for prec in (F.PREC_FP32, F.PREC_SPLIT_BF16):
                    x0, y0 = bufs[sd][0][0], bufs[sd][1][0]
                    sv.wait(sv.submit_ptr(F.KIND_FILTER, sd, sd, x0.data_ptr(), y0.data_ptr(), prec, 0.2))
        for rate in rates:
            n = int(min(min_requests, rate * seconds))
            if rate >= 10000:
                n = max(n, min_requests)
            tr = inputs.poisson_trace(rate, n)
            reqs = [(int(tr["side"][i]), int(tr["precision"][i]), float(tr["cutoff"][i])) for i in range(n)]
            served = {}
            for label, force32, sv in (("serve", False, srv), ("serve_all_fp32", True, srv),
                                       ("serve_persistent_groups", False, srvp)):
                sv.reset_stats()
                nxt = {sd: 0 for sd in sides}
                last = {}
                t0 = time.perf_counter()
                lag = 0.0
                tickets = []
                for i, (sd, prec, cut) in enumerate(reqs):
                    at = t0 + tr["t"][i]
                    while time.perf_counter() < at:
                        pass
                    lag = max(lag, time.perf_counter() - at)
                    xin, xout = bufs[sd]
                    i_in, i_out = i % xin.shape[0], nxt[sd] % xout.shape[0]
                    nxt[sd] += 1
                    p = F.PREC_SPLIT_BF16 if (prec and not force32) else F.PREC_FP32
                    # inputs were synchronised before the trace: no stream ordering needed
                    tickets.append(sv.submit_ptr(F.KIND_FILTER, sd, sd, xin[i_in].data_ptr(),
                                                 xout[i_out].data_ptr(), p, cut))
                    last[sd] = (i_in, i_out, p, cut)
                status = [sv.wait(t) for t in tickets]
                st = sv.stats()
                ok, nchk = spot_check(last)
                served[label] = {"p50_ms": round(st["p50_ms"], 4), "p99_ms": round(st["p99_ms"], 4),
                                 "req_per_s": round(st["req_per_s"], 1), "completed": st["completed"],
                                 "failed": sum(1 for v in status if v != 0),
                                 "spot_check_bit_identical": "%d/%d" % (ok, nchk),
                                 "max_submit_lag_ms": round(lag * 1e3, 4)}
            # FIFO baseline: one stream, plain FP32 filter, same arrivals
            evs = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
            nxt = {sd: 0 for sd in sides}
            torch.cuda.synchronize()
            evs[0].record(stream)
            t0 = time.perf_counter()
            for i, (sd, prec, cut) in enumerate(reqs):
                at = t0 + tr["t"][i]
                while time.perf_counter() < at:
                    pass
                xin, xout = bufs[sd]
                i_in, i_out = i % xin.shape[0], nxt[sd] % xout.shape[0]
                nxt[sd] += 1
                plans[sd].exec_filter(xin[i_in], cut, xout[i_out], stream)
                evs[i + 1].record(stream)
            evs[-1].synchronize()
            done = np.array([evs[0].elapsed_time(evs[i + 1]) for i in range(n)])  # ms from t0
            lat = done - np.asarray(tr["t"][:n]) * 1e3
            fifo = {"p50_ms": round(float(np.percentile(lat, 50)), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4),
                    "req_per_s": round(n / (done[-1] * 1e-3), 1)}
            out[str(rate)] = {"requests": n, **served, "fifo_fp32": fifo}
            log("serve trace %d req/s (%d requests): serve p50 %.3f p99 %.3f ms %.0f req/s; all-FP32 serve p50 %.3f "
                "p99 %.3f ms %.0f req/s; FIFO FP32 p50 %.3f p99 %.3f ms %.0f req/s" % (
                    rate, n, served["serve"]["p50_ms"], served["serve"]["p99_ms"], served["serve"]["req_per_s"],
                    served["serve_all_fp32"]["p50_ms"], served["serve_all_fp32"]["p99_ms"],
                    served["serve_all_fp32"]["req_per_s"], fifo["p50_ms"], fifo["p99_ms"], fifo["req_per_s"]))
    for p in plans.values():
        p.close()
    del bufs
    torch.cuda.empty_cache()
    return out


def cpu_model() -> str:
    """The host CPU's model name from /proc/cpuinfo, with its family, model
    and stepping numbers (a virtualised host may report a short name)."""
    fields = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if not line.strip():
                    break  # first processor only
                k, _, v = line.partition(":")
                fields[k.strip()] = v.strip()
    except OSError:
        pass
    name = fields.get("model name", "unknown")
    ids = [(k, fields[k]) for k in ("cpu family", "model", "stepping") if k in fields]
    return name + (" (%s)" % ", ".join("%s %s" % kv for kv in ids) if ids else "")


def cpu_baseline(rows, cols, seconds, windows=3):
    """FP64 oracle round trips on all host cores: `windows` timed windows of
    about seconds / windows each; the median window's rate is the value."""
    import statistics

    import oracle
    from paper_1505_08019_amd import inputs
    from paper_1505_08019_amd.metrics import flops_5nm

    x = inputs.uniform_pixels(rows, cols, cfg_seed=2)
    threads = oracle.max_threads()
    rates, total_n, total_s = [], 0, 0.0
    for _ in range(windows):
        n = 0
        t0 = time.perf_counter()
        while True:
            X = oracle.fft2(x, -1, threads=0)
            oracle.fft2(X, +1, threads=0)
            n += 1
            el = time.perf_counter() - t0
            if el >= seconds / windows:
                break
        rates.append(2 * flops_5nm(rows, cols) * n / el / 1e9)
        total_n += n
        total_s += el
    return {"value": round(statistics.median(rates), 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "windows_gflops": [round(r, 3) for r in rates],
            "sample": "median of %d windows, %d forward+inverse round trips in all, of one %dx%d uniform-pixel "
                      "image, FP64 C oracle (OpenMP over rows, then columns), %.1f s" % (
                          windows, total_n, rows, cols, total_s)}


def cpu_context(rows, cols, seconds):
    """For context beside cpu_baseline: the same oracle on one core, and
    scipy.fft.fft2 / ifft2 (the optimised host library) on complex64 with as
    many threads as the oracle uses, each for about `seconds` of
    forward+inverse round trips."""
    import oracle
    from paper_1505_08019_amd import inputs
    from paper_1505_08019_amd.metrics import flops_5nm

    x = inputs.uniform_pixels(rows, cols, cfg_seed=2)
    per_rt = 2 * flops_5nm(rows, cols)
    out = {}

    def timed(step):
        n, t0 = 0, time.perf_counter()
        while True:
            step()
            n += 1
            el = time.perf_counter() - t0
            if el >= seconds:
                return n, el

    n, el = timed(lambda: oracle.fft2(oracle.fft2(x, -1, threads=1), +1, threads=1))
    out["oracle_1_core"] = {"value": round(per_rt * n / el / 1e9, 3), "unit": "GFLOP/s", "round_trips": n,
                            "seconds": round(el, 2)}
    try:
        import scipy.fft

        workers = oracle.max_threads()  # the same host-core share as the oracle
        xs = x.astype("complex64")
        n, el = timed(lambda: scipy.fft.ifft2(scipy.fft.fft2(xs, workers=workers), workers=workers))
        out["scipy_fft2_complex64"] = {"value": round(per_rt * n / el / 1e9, 3), "unit": "GFLOP/s",
                                       "workers": workers, "round_trips": n, "seconds": round(el, 2)}
    except Exception as e:  # context only: never fails the bench
        out["scipy_fft2_complex64"] = {"error": str(e)[:200]}
    return out


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
    copy_gbs = copy_reference(torch)
    log("reference copy %.0f GB/s" % copy_gbs)
    res = time_round_trip(F, torch, rows, cols, args.steps, args.warmup, args.buffers)
    log("%dx%d round trip %.3f us" % (rows, cols, res["ms_step"] * 1e3))
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
                   "schedule_source": "tuned_schedules.txt beside the library (fft2_autotune), else the heuristic",
                   "round_trip_rel_l2": res["round_trip_rel_l2"], "buffer_sets": res["buffer_sets"],
                   "buffer_set_bytes": res["buffer_set_bytes"]},
        # the default counter record was taken on the default 1024^2 workload
        "roofline": roofline_for(res, rows, cols, copy_gbs,
                                 traffic_record="bench_default_traffic.json" if rows == 1024 else None),
    }
    if not args.no_extra:
        extra = {}
        extra["%dx%d_timing" % (rows, cols)] = timing_detail(F, torch, rows, cols, args.buffers)
        log("timing detail: %s" % json.dumps(extra["%dx%d_timing" % (rows, cols)]))
        # buffer sets: 4 x 384 MB at 4096^2 and 2 x 1.5 GB at 8192^2, so no set
        # is still in the 256 MB Infinity Cache when it comes round again
        for n, steps, nbuf in ((4096, 20, 4), (8192, 10, 2)):
            r = time_round_trip(F, torch, n, n, steps, 3, nbuf)
            log("%dx%d round trip %.3f us" % (n, n, r["ms_step"] * 1e3))
            extra["%dx%d" % (n, n)] = {
                "ms_per_round_trip": round(r["ms_step"], 4),
                "gflops": round(2 * flops_5nm(n, n) / (r["ms_step"] * 1e-3) / 1e9, 1),
                "hbm_frac_whole_transform": round(2 * 16 * n * n * r["npass"] / (r["ms_step"] * 1e-3) / 1e9 /
                                                  HBM_PEAK_GBS, 4),
                "roofline": roofline_for(r, n, n, traffic_record={8192: "fp32_8192_traffic.json"}.get(n)),
                "round_trip_rel_l2": r["round_trip_rel_l2"],
            }
        extra["precision_forms"] = precision_forms(F, torch, flops_5nm)
        log("precision forms done")
        extra["real_image_transforms"] = real_transforms(F, torch, flops_5nm)
        log("real transforms done")
        extra["ragged_batch_512"] = ragged_batch(F, torch, flops_5nm)
        log("ragged batch done")
        extra["serve_poisson_filter"] = serve_trace(F, torch)
        line["extra"] = extra
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(rows, cols, args.cpu_seconds)
        line.setdefault("extra", {})["cpu_context"] = cpu_context(rows, cols, 3.0)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
