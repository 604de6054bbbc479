"""Summaries of rocprofv3 output for the committed profile records.

Usage (from the repository root, on the files rocprofv3 wrote):

  python -m paper_1505_08019_amd.prof stats <kernel_stats.csv> <out.md> --command "<cmd>"
      Short table of the kernels of one run (calls, average and total time).

  python -m paper_1505_08019_amd.prof run <rows> <cols> <forms> [--reps R] [--copy]
      Workload for a counter run: R forward+inverse round trips of a
      rows x cols image in each listed form (fp32, split_bf16, fp16); with
      --copy, first the reference copy (for the traffic calibration).

  python -m paper_1505_08019_amd.prof sq <counters.csv> <out.md> --command "<cmd>" [--title T]
      Per-dispatch averages of the SQ counters of one run, per kernel, with
      the VALU, LDS and wait activity as fractions of the wave cycles.

  python -m paper_1505_08019_amd.prof traffic <fetch.csv> <write.csv> <out.json> --command "<cmd>"
      Per-launch HBM bytes of each kernel from two counter runs (FETCH_SIZE,
      then WRITE_SIZE, both in KiB per dispatch), each scaled by what the same
      counter reads for the reference copy that bench.py runs in the same
      process (COPY_BYTES read and COPY_BYTES written per launch).

Kernel names are normalised (``normalise``) so that bench.py can look up its
dominant kernel; the traffic record carries the hash of the kernel sources
it was taken with, and bench.py ignores it once the sources change.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))

# The reference copy: a float32 multiply by one over 128 Mi elements, which
# reads and writes 512 MiB once each, twice the 256 MB Infinity Cache.
COPY_ELEMS = 128 << 20
COPY_BYTES = COPY_ELEMS * 4
COPY_MATCH = "MulFunctor"


PASS_SOURCES = ("engine.hpp", "pass_kernel.hpp", "kernel_table.hpp", "kernels_gen.hpp")


def kernel_source_hash() -> str:
    """Hash of the sources the FP32 pass kernels are compiled from."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for f in sorted(os.listdir(csrc)):
        if f in PASS_SOURCES or (f.startswith("kernels_") and f.endswith(".hip")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def normalise(name: str) -> str:
    """'void fft2::pass_kernel<0, 10, 2, 4, false>(fft2::PassArgs)' -> 'pass_kernel<0,10,2,4,false>'."""
    n = name.strip()
    n = re.sub(r"^void\s+", "", n)
    n = re.sub(r"\(.*\)$", "", n)
    n = n.replace("fft2::", "").replace(" ", "")
    return n


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def stats_md(stats_csv: str, out_md: str, command: str, top: int = 14, focus: tuple = ()) -> str:
    """Kernels named in `focus` (normalised names) first, then the `top` by total time."""
    rows = _rows(stats_csv)
    rows.sort(key=lambda r: -float(r.get("TotalDurationNs", 0)))
    lines = ["# Kernel time: %s" % os.path.basename(out_md).rsplit(".", 1)[0], "",
             "Command (from the repository root):", "", "    " + command, "",
             "| kernel | calls | avg us | min us | max us | total ms | % |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    pinned = [r for r in rows if normalise(r["Name"]) in focus]
    rest = [r for r in rows if normalise(r["Name"]) not in focus]
    for r in pinned + rest[:top]:
        lines.append("| `%s` | %s | %.2f | %.2f | %.2f | %.3f | %.1f |" % (
            normalise(r["Name"])[:90], r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    text = "\n".join(lines) + "\n"
    with open(out_md, "w") as f:
        f.write(text)
    return text


def _per_kernel(path: str, counter: str):
    acc = {}
    for r in _rows(path):
        if r.get("Counter_Name") != counter:
            continue
        k = normalise(r["Kernel_Name"])
        v = float(r["Counter_Value"])
        s = acc.setdefault(k, [0.0, 0])
        s[0] += v
        s[1] += 1
    return {k: (v[0] / v[1], v[1]) for k, v in acc.items()}


def traffic_json(fetch_csv: str, write_csv: str, out_json: str, command: str) -> dict:
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE")
    write = _per_kernel(write_csv, "WRITE_SIZE")
    copy_f = [v for k, v in fetch.items() if COPY_MATCH in k]
    copy_w = [v for k, v in write.items() if COPY_MATCH in k]
    if not copy_f or not copy_w:
        raise SystemExit("reference copy kernel (%s) not found in the counter files" % COPY_MATCH)
    f_scale = COPY_BYTES / (copy_f[0][0] * 1024.0)
    w_scale = COPY_BYTES / (copy_w[0][0] * 1024.0)
    kernels = {}
    for k in sorted(set(fetch) & set(write)):
        if COPY_MATCH in k:
            continue
        fb = fetch[k][0] * 1024.0 * f_scale
        wb = write[k][0] * 1024.0 * w_scale
        kernels[k] = {"fetch_kib_raw": round(fetch[k][0], 1), "write_kib_raw": round(write[k][0], 1),
                      "dispatches": fetch[k][1], "fetch_bytes": int(fb), "write_bytes": int(wb),
                      "hbm_bytes_per_launch": int(fb + wb)}
    rec = {"source_hash": kernel_source_hash(), "command": command,
           "copy_reference": {"bytes_read": COPY_BYTES, "bytes_written": COPY_BYTES,
                              "fetch_kib_raw": round(copy_f[0][0], 1), "write_kib_raw": round(copy_w[0][0], 1),
                              "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4)},
           "kernels": kernels}
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    return rec


def run_round_trips(rows: int, cols: int, forms: str, reps: int = 3, copy: bool = False) -> None:
    import torch

    from paper_1505_08019_amd import fft2 as F

    if copy:  # the reference copy of bench.py: COPY_BYTES read, COPY_BYTES written
        a = torch.ones(COPY_ELEMS, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()

    precs = {"fp32": F.PREC_FP32, "split_bf16": F.PREC_SPLIT_BF16, "fp16": F.PREC_FP16}
    x = torch.rand(rows, cols, device="cuda:0").to(torch.complex64)
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    for name in forms.split(","):
        with F.Plan(rows, cols, F.FORWARD, precs[name]) as pf, F.Plan(rows, cols, F.INVERSE, precs[name]) as pi:
            for _ in range(reps):
                pf.exec(x, y)
                pi.exec(y, z)
    torch.cuda.synchronize()
    print("ran %d round trips of %dx%d in %s" % (reps, rows, cols, forms), flush=True)


SQ_RATIOS = (("SQ_ACTIVE_INST_VALU", "active VALU / wave cycles"), ("SQ_ACTIVE_INST_LDS", "active LDS / wave cycles"),
             ("SQ_WAIT_INST_ANY", "wait / wave cycles"))


def sq_md(csv_path: str, out_md: str, command: str, title: str = "") -> str:
    """Per-kernel, per-dispatch averages of every counter in the file; the
    activity counters also as a fraction of SQ_WAVE_CYCLES."""
    rows = _rows(csv_path)
    counters = sorted({r["Counter_Name"] for r in rows})
    per = {c: _per_kernel(csv_path, c) for c in counters}
    kernels = sorted({k for c in counters for k in per[c]}, key=lambda k: -per[counters[0]].get(k, (0, 0))[0])
    ratios = [(c, label) for c, label in SQ_RATIOS if c in counters and "SQ_WAVE_CYCLES" in counters]
    head = ["kernel", "dispatches"] + counters + [label for _, label in ratios]
    lines = ["# SQ counters: %s" % (title or os.path.basename(out_md).rsplit(".", 1)[0]), "",
             "Command (from the repository root):", "", "    " + command, "",
             "Figures are averages per dispatch, summed over the GPU's counter instances.", "",
             "| " + " | ".join(head) + " |", "|---|" + "---:|" * (len(head) - 1)]
    for k in kernels:
        n = max(per[c].get(k, (0, 0))[1] for c in counters)
        vals = []
        for c in counters:
            v = per[c].get(k, (0.0, 0))[0]
            vals.append("%.3gM" % (v / 1e6) if v >= 1e5 else "%.0f" % v)
        for c, _ in ratios:
            wc = per["SQ_WAVE_CYCLES"].get(k, (0.0, 0))[0]
            vals.append("%.2f" % (per[c].get(k, (0.0, 0))[0] / wc) if wc else "-")
        lines.append("| `%s` | %d | %s |" % (k[:80], n, " | ".join(vals)))
    text = "\n".join(lines) + "\n"
    with open(out_md, "w") as f:
        f.write(text)
    return text


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("out")
    a.add_argument("--command", required=True)
    a.add_argument("--focus", default="", help="kernel names listed first, separated by semicolons")
    r = sub.add_parser("run")
    r.add_argument("rows", type=int)
    r.add_argument("cols", type=int)
    r.add_argument("forms")
    r.add_argument("--reps", type=int, default=3)
    r.add_argument("--copy", action="store_true")
    q = sub.add_parser("sq")
    q.add_argument("csv")
    q.add_argument("out")
    q.add_argument("--command", required=True)
    q.add_argument("--title", default="")
    b = sub.add_parser("traffic")
    b.add_argument("fetch")
    b.add_argument("write")
    b.add_argument("out")
    b.add_argument("--command", required=True)
    args = ap.parse_args(argv)
    if args.cmd == "run":
        run_round_trips(args.rows, args.cols, args.forms, args.reps, args.copy)
    elif args.cmd == "sq":
        sys.stdout.write(sq_md(args.csv, args.out, args.command, args.title))
    elif args.cmd == "stats":
        focus = tuple(normalise(k) for k in args.focus.split(";") if k)
        sys.stdout.write(stats_md(args.csv, args.out, args.command, focus=focus))
    else:
        json.dump(traffic_json(args.fetch, args.write, args.out, args.command), sys.stdout, indent=1)
        print()


if __name__ == "__main__":
    main()
