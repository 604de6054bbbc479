"""Write the table of tuned FP32 pass schedules that ships beside the library.

Usage (on the target GPU, from the repository root):

  python -m paper_1505_08019_amd.tune_table [out_path] [--reps R]

For every shape below and both directions it runs fft2_autotune (which times
every candidate schedule) and records the fastest.  The library reads
``tuned_schedules.txt`` next to ``libfft2.so`` when it first plans a shape;
every schedule of a shape gives bit-identical results, so the table changes
speed only.  Shapes: all rows x cols with sides 2^6 .. 2^11 (the ragged-batch
sizes), squares 2^12 .. 2^14 and 8192 x 16384.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))


def shapes() -> list[tuple[int, int]]:
    out = [(1 << a, 1 << b) for a in range(6, 12) for b in range(6, 12)]
    out += [(4096, 4096), (8192, 8192), (16384, 16384), (8192, 16384), (16384, 8192)]
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("out", nargs="?", default=os.path.join(HERE, "tuned_schedules.txt"))
    ap.add_argument("--reps", type=int, default=10)
    args = ap.parse_args(argv)
    tmp = args.out + ".partial"
    if os.path.exists(tmp):
        os.remove(tmp)
    os.environ["FFT2_AUTOTUNE_CACHE"] = tmp  # fft2_autotune appends each choice here
    from paper_1505_08019_amd import fft2 as F

    t0 = time.time()
    for r, c in shapes():
        for d in (F.FORWARD, F.INVERSE):
            s = F.autotune(r, c, d, F.PREC_FP32, reps=args.reps)
            print("%5d x %-5d %+d  %s" % (r, c, d, s), flush=True)
    with open(tmp) as f:
        body = f.read()
    with open(args.out, "w") as f:
        f.write("# Tuned FP32 pass schedules: rows cols precision direction device schedule\n")
        f.write("# written by: python -m paper_1505_08019_amd.tune_table --reps %d (%.0f s)\n" % (
            args.reps, time.time() - t0))
        f.write(body)
    os.remove(tmp)
    print("wrote", args.out)


if __name__ == "__main__":
    sys.exit(main())
