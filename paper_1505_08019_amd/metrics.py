"""Reporting conventions (no FFT arithmetic here).

* ``flops_5nm``: the nominal flop count 5*M*N*log2(M*N) of one M x N complex
  2D FFT, the usual convention for FFT GFLOP/s.  The paper's own count for a
  1024 x 1024 image (introduction) is 2.1e7 = M*N*log2(M*N), two per radix-2
  butterfly; ``flops_paper`` returns that count.
* ``alg_bytes``: the bytes a 2D FFT must move between HBM and the chip when
  each pass keeps its working set on-chip: one read and one write of the
  complex64 image per pass.
"""
from __future__ import annotations

import math


def log2_exact(n: int) -> int:
    if n <= 0 or (n & (n - 1)) != 0:
        raise ValueError("%d is not a power of two" % n)
    return n.bit_length() - 1


def flops_5nm(rows: int, cols: int) -> float:
    n = rows * cols
    return 5.0 * n * math.log2(n) if n > 1 else 0.0


def flops_paper(rows: int, cols: int) -> float:
    n = rows * cols
    return n * math.log2(n) if n > 1 else 0.0


def alg_bytes(rows: int, cols: int, passes: int) -> int:
    """Algorithmic HBM bytes of a 2D FFT done in ``passes`` on-chip passes."""
    return 16 * rows * cols * passes


def rel_l2(a, b) -> float:
    """||a - b||_2 / ||b||_2 (0 if both are zero)."""
    import numpy as np
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    den = float(np.linalg.norm(b))
    num = float(np.linalg.norm(a - b))
    if den == 0.0:
        return 0.0 if num == 0.0 else math.inf
    return num / den


def max_rel(a, b) -> float:
    """max|a - b| / max|b|."""
    import numpy as np
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    den = float(np.abs(b).max()) if b.size else 0.0
    num = float(np.abs(a - b).max()) if b.size else 0.0
    if den == 0.0:
        return 0.0 if num == 0.0 else math.inf
    return num / den
