"""The plan's twiddle tables (sec. 3.1: rotation factors computed once in
advance and kept unchanged), read back from the device and compared bit for
bit with the correctly rounded FP32 values of cos and sin.

Reference values: cos(2 pi u / 2^s) and sin(2 pi u / 2^s) summed as Taylor
series in 50-digit decimal arithmetic, rounded to FP64 and then to FP32.  The
double rounding can only differ from one correct rounding if the FP64 value
sits exactly on an FP32 midpoint, which the test checks does not happen."""
import ctypes
from decimal import Decimal, localcontext

import numpy as np
import pytest

from paper_1505_08019_amd import fft2 as F

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

_PI = Decimal("3.14159265358979323846264338327950288419716939937510")


def _cos_sin(u, L):
    """(cos, sin) of 2 pi u / L to about 45 significant digits."""
    with localcontext() as ctx:
        ctx.prec = 55
        x = 2 * _PI * Decimal(u) / Decimal(L)
        x2 = x * x
        c = s = Decimal(0)
        tc, ts = Decimal(1), x
        n = 0
        while True:
            c += tc
            s += ts
            tc = -tc * x2 / ((2 * n + 1) * (2 * n + 2))
            ts = -ts * x2 / ((2 * n + 2) * (2 * n + 3))
            n += 1
            if abs(tc) < Decimal("1e-52") and abs(ts) < Decimal("1e-52"):
                break
        return float(c), float(s)


def _to_f32(v64):
    f = np.float32(v64)
    # not an exact midpoint between two FP32 neighbours (see module doc)
    lo, hi = np.nextafter(f, np.float32(-np.inf)), np.nextafter(f, np.float32(np.inf))
    assert v64 != (float(f) + float(lo)) / 2 and v64 != (float(f) + float(hi)) / 2
    return f


def _expected(bits, sign):
    """Stage-major table of a length-2^bits dimension: stage s (1..bits) holds
    W_{2^s}^u = exp(sign 2 pi i u / 2^s), u < 2^(s-1), at index 2^(s-1)-1+u."""
    L = 1 << bits
    top = [_cos_sin(u, L) for u in range(L // 2)]  # W_L^u; W_{2^s}^u = W_L^(u L / 2^s)
    out = np.empty(L - 1, dtype=np.complex64)
    re = out.view(np.float32)[0::2]
    im = out.view(np.float32)[1::2]
    for s in range(1, bits + 1):
        h = 1 << (s - 1)
        for u in range(h):
            c, si = top[u * (L >> s)]
            re[h - 1 + u] = _to_f32(c)
            im[h - 1 + u] = _to_f32(sign * si) if si != 0.0 else np.float32(sign * 0.0)
    return out


def _device_table(ptr, n):
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipMemcpy.restype = ctypes.c_int
    out = np.empty(n, dtype=np.complex64)
    torch.cuda.synchronize()
    assert hip.hipMemcpy(out.ctypes.data, ptr, n * 8, 2) == 0  # hipMemcpyDeviceToHost
    return out


@pytest.mark.parametrize("direction", [F.FORWARD, F.INVERSE], ids=["forward", "inverse"])
def test_plan_tables_bit_exact(direction):
    rows, cols = 16384, 8192
    with F.Plan(rows, cols, direction) as p:
        tr, tc = ctypes.c_void_p(), ctypes.c_void_p()
        F.check(F.lib().fft2_plan_tables(p.handle, ctypes.byref(tr), ctypes.byref(tc)))
        got_r = _device_table(tr.value, cols - 1)
        got_c = _device_table(tc.value, rows - 1)
    sign = -1.0 if direction == F.FORWARD else 1.0
    for got, bits in ((got_r, 13), (got_c, 14)):
        want = _expected(bits, sign)
        gb, wb = got.view(np.uint32), want.view(np.uint32)
        bad = np.nonzero(gb != wb)[0]
        assert bad.size == 0, "first mismatches at %s: %s vs %s" % (bad[:4], got[bad[:4] // 2], want[bad[:4] // 2])
    # spot values that are exact: W_4^1 = -+i, W_2^0 = 1
    assert got_c[2] == np.complex64(0 + sign * 1j)
    assert got_c[0] == np.complex64(1)


def _step_block_size(b):
    m, rem = b >> 2, b & 3
    n = (1 << b) if (rem and m) else 0
    for j in range(2, m + 1):
        n += 1 << (4 * j)
    return n


def _expected_steps(bits, sign):
    """Step tables of the MFMA forms for a length-2^bits dimension: for line
    lengths 2^b, b = 1..bits, the tables of the steps with stride S > 1 (the
    2^(b mod 4)-point step of block length 2^b if b mod 4 > 0 and b >= 4,
    then the radix-16 steps of block lengths 16^m .. 16^2, m = b / 4), each
    holding W_Lt^(k1 n2) at k1 S + n2 (Lt the block length, S = Lt / radix)."""
    L = 1 << bits
    top = [_cos_sin(u, L) for u in range(L // 2)]
    vals = []
    for b in range(1, bits + 1):
        m, rem = b >> 2, b & 3
        steps = ([(b, b - rem)] if (rem and m) else []) + [(4 * j, 4 * j - 4) for j in range(m, 1, -1)]
        for bt, ls in steps:
            for k1 in range((1 << bt) >> ls):
                for n2 in range(1 << ls):
                    v = (k1 * n2) * (L >> bt)  # W_Lt^(k1 n2) = W_L^v, v < L
                    c, si = top[v % (L // 2)]
                    if v >= L // 2:
                        c, si = -c, -si
                    vals.append((c, si))
    assert len(vals) == sum(_step_block_size(b) for b in range(1, bits + 1))
    out = np.empty(len(vals), dtype=np.complex64)
    re = out.view(np.float32)[0::2]
    im = out.view(np.float32)[1::2]
    for i, (c, si) in enumerate(vals):
        re[i] = _to_f32(c)
        im[i] = _to_f32(sign * si) if si != 0.0 else np.float32(sign * 0.0)
    return out


@pytest.mark.parametrize("direction", [F.FORWARD, F.INVERSE], ids=["forward", "inverse"])
def test_step_tables_bit_exact(direction):
    """The per-step twiddle tables the MFMA forms read (stored after each
    dimension's stage table), bit for bit against correctly rounded values."""
    rows, cols = 4096, 2048
    with F.Plan(rows, cols, direction) as p:
        tr, tc = ctypes.c_void_p(), ctypes.c_void_p()
        F.check(F.lib().fft2_plan_tables(p.handle, ctypes.byref(tr), ctypes.byref(tc)))
        sign = -1.0 if direction == F.FORWARD else 1.0
        for ptr, L, bits in ((tr.value, cols, 11), (tc.value, rows, 12)):
            want = _expected_steps(bits, sign)
            got = _device_table(ptr + 8 * (L - 1), want.size)
            gb, wb = got.view(np.uint32), want.view(np.uint32)
            bad = np.nonzero(gb != wb)[0]
            assert bad.size == 0, "bits %d: first mismatches at %s: %s vs %s" % (
                bits, bad[:4], got[bad[:4] // 2], want[bad[:4] // 2])
