"""FP64 CPU reference ("oracle") for the 2D image FFT.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product library
(``paper_1505_08019_amd``) never imports it and shares no code with it.

The arithmetic lives in ``fft2_oracle.c`` (plain C, FP64): bit-reversal
scramble (sec. 3.2) followed by radix-2 decimation-in-time butterflies
(eqs. 2-4), rows first and then columns (separability, sec. 2).  This module
only marshals numpy arrays into it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fft2_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile ``fft2_oracle.c`` with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_fft2.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.oracle_fft2.restype = ctypes.c_int
        lib.oracle_filter.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int]
        lib.oracle_filter.restype = ctypes.c_int
        lib.oracle_gaussian_mask.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        lib.oracle_gaussian_mask.restype = None
        lib.oracle_bitrev.argtypes = [ctypes.c_int, ctypes.c_int]
        lib.oracle_bitrev.restype = ctypes.c_int
        lib.oracle_log2.argtypes = [ctypes.c_int]
        lib.oracle_log2.restype = ctypes.c_int
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _as_c128(x) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x), dtype=np.complex128)
    if a.ndim != 2:
        raise ValueError("expected a 2D image, got shape %r" % (a.shape,))
    return a


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def fft2(x, direction: int = -1, row_stages: int = -1, col_stages: int = -1, threads: int = 1) -> np.ndarray:
    """2D DFT of ``x`` (eq. 1 made 2D by separability) in FP64.

    direction -1 is forward (unscaled), +1 inverse (scaled by 1/(rows*cols)).
    ``row_stages``/``col_stages`` < 0 run every butterfly level; smaller values
    return the staged snapshot described in ``fft2_oracle.c`` (both scrambles
    always applied).  Returns a new complex128 array.
    """
    a = _as_c128(x)
    out = np.empty_like(a)
    rows, cols = a.shape
    rc = _load().oracle_fft2(_dp(a), _dp(out), rows, cols, int(direction), int(row_stages), int(col_stages), int(threads))
    if rc != 0:
        raise ValueError("oracle_fft2 failed with code %d for shape %r" % (rc, a.shape))
    return out


def ifft2(x, threads: int = 1) -> np.ndarray:
    """Inverse 2D DFT, scaled by 1/(rows*cols)."""
    return fft2(x, +1, threads=threads)


def gaussian_mask(rows: int, cols: int, cutoff: float) -> np.ndarray:
    """The Gaussian low-pass mask H of the filter request, FP64, rows x cols."""
    h = np.empty((rows, cols), dtype=np.float64)
    _load().oracle_gaussian_mask(_dp(h), rows, cols, float(cutoff))
    return h


def filter_gaussian(x, cutoff: float, threads: int = 1) -> np.ndarray:
    """Filter request: inverse 2D DFT of (forward 2D DFT of x) * H."""
    a = _as_c128(x)
    out = np.empty_like(a)
    rows, cols = a.shape
    rc = _load().oracle_filter(_dp(a), _dp(out), rows, cols, float(cutoff), int(threads))
    if rc != 0:
        raise ValueError("oracle_filter failed with code %d for shape %r" % (rc, a.shape))
    return out


def bitrev(i: int, b: int) -> int:
    """rev_b(i): the low b bits of i reversed (sec. 3.2)."""
    return _load().oracle_bitrev(int(i), int(b))


def max_threads() -> int:
    """Threads the oracle's OpenMP loops use when asked for 'all'."""
    return _load().oracle_max_threads()


def dft2_at(x, k1, k2, direction: int = -1) -> np.ndarray:
    """X[k1[i], k2[i]] by the plain double sum of eq. (1) in 2D, FP64.

    For checking single outputs of images too large for a full oracle run:
    each requested output is the sum over all pixels of x[n1, n2] times
    W_M^(k1 n1) W_N^(k2 n2), evaluated in FP64 with the exponents reduced
    modulo M and N exactly in integers.  The sum over n2 is done first (a
    matrix-vector product per distinct k2), then the sum over n1.  Forward
    only is unscaled; direction +1 applies the 1/(M N) inverse scale.
    """
    a = np.asarray(x)
    M, N = a.shape
    k1 = np.atleast_1d(np.asarray(k1, dtype=np.int64))
    k2 = np.atleast_1d(np.asarray(k2, dtype=np.int64))
    sign = float(direction)
    n1 = np.arange(M, dtype=np.int64)
    n2 = np.arange(N, dtype=np.int64)
    out = np.empty(k1.shape, dtype=np.complex128)
    for kk2 in np.unique(k2):
        ph2 = np.exp(sign * 2j * np.pi * ((kk2 * n2) % N) / N)
        inner = np.empty(M, dtype=np.complex128)
        step = max(1, (1 << 24) // max(N, 1))
        for r0 in range(0, M, step):
            inner[r0:r0 + step] = a[r0:r0 + step].astype(np.complex128) @ ph2
        for i in np.nonzero(k2 == kk2)[0]:
            ph1 = np.exp(sign * 2j * np.pi * ((k1[i] * n1) % M) / M)
            out[i] = inner @ ph1
    if direction == 1:
        out /= (M * N)
    return out


def rfft2(x, threads: int = 1) -> np.ndarray:
    """Forward 2D DFT of a REAL image, non-redundant half: X[k1, k2] for
    0 <= k2 <= cols/2 (rows x (cols/2 + 1), complex128).

    By definition: the DFT of eq. (1), made 2D by separability (sec. 2), of
    the real image, with the columns k2 > cols/2 left out, since for real
    input X[k1, k2] = conj(X[-k1 mod rows, -k2 mod cols]) repeats them (the
    paper's images are gray images, sec. 4).  Computed with the radix-2
    oracle on the image widened to complex with a zero imaginary part.
    """
    a = np.asarray(x)
    if np.iscomplexobj(a):
        raise ValueError("rfft2 takes a real image")
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 2 or a.shape[1] < 2:
        raise ValueError("rfft2 takes a 2D image with at least 2 columns, got shape %r" % (a.shape,))
    full = fft2(a.astype(np.complex128), -1, threads=threads)
    return np.ascontiguousarray(full[:, : a.shape[1] // 2 + 1])


def hermitian_extend(X, cols: int) -> np.ndarray:
    """The full rows x cols spectrum whose columns 0 .. cols/2 are X, the
    others given by X[k1, k2] = conj(X[-k1 mod rows, cols - k2])."""
    X = np.asarray(X, dtype=np.complex128)
    rows, h = X.shape
    if h != cols // 2 + 1 or cols < 2:
        raise ValueError("half spectrum of %d columns does not fit %d image columns" % (h, cols))
    full = np.empty((rows, cols), dtype=np.complex128)
    full[:, :h] = X
    k1 = (-np.arange(rows)) % rows
    for k2 in range(h, cols):
        full[:, k2] = np.conj(X[k1, cols - k2])
    return full


def irfft2(X, cols: int, threads: int = 1) -> np.ndarray:
    """Real image from its non-redundant half spectrum X (rows x (cols/2+1)):
    the real part of the inverse 2D DFT (scaled by 1/(rows cols)) of the
    Hermitian extension of X (see hermitian_extend).  Returns float64."""
    return np.ascontiguousarray(fft2(hermitian_extend(X, cols), +1, threads=threads).real)


def _dct_matrix(L: int) -> np.ndarray:
    """C[k, n] = 2 cos(pi k (2n + 1) / (2L)): the DCT-II of length L as a matrix."""
    k = np.arange(L, dtype=np.float64)[:, None]
    n = np.arange(L, dtype=np.float64)[None, :]
    return 2.0 * np.cos(np.pi * k * (2.0 * n + 1.0) / (2.0 * L))


def _idct_matrix(L: int) -> np.ndarray:
    """A[n, k] = w_k cos(pi k (2n + 1) / (2L)) / (2L), w_0 = 1, w_k = 2: the
    DCT-III that inverts _dct_matrix (A C = I)."""
    n = np.arange(L, dtype=np.float64)[:, None]
    k = np.arange(L, dtype=np.float64)[None, :]
    w = np.where(k == 0, 1.0, 2.0)
    return w * np.cos(np.pi * k * (2.0 * n + 1.0) / (2.0 * L)) / (2.0 * L)


def dct2(x) -> np.ndarray:
    """2D DCT-II of a real image by its definition, FP64:
    X[k1, k2] = 4 sum_{n1, n2} x[n1, n2] cos(pi k1 (2 n1 + 1) / (2M)) cos(pi k2 (2 n2 + 1) / (2N)),
    i.e. C_M x C_N^T (a matrix product per dimension; the paper names the
    DCT as the direct extension of its method, sec. 5)."""
    a = np.asarray(x)
    if np.iscomplexobj(a) or a.ndim != 2:
        raise ValueError("dct2 takes a real 2D image")
    a = a.astype(np.float64)
    M, N = a.shape
    return _dct_matrix(M) @ a @ _dct_matrix(N).T


def idct2(X) -> np.ndarray:
    """Inverse of dct2 (a 2D DCT-III scaled by 1/(4 M N)):
    x[n1, n2] = sum_{k1, k2} w_k1 w_k2 X[k1, k2] cos(...) cos(...) / (4 M N),
    w_0 = 1 and w_k = 2 otherwise."""
    a = np.asarray(X)
    if np.iscomplexobj(a) or a.ndim != 2:
        raise ValueError("idct2 takes a real 2D array")
    a = a.astype(np.float64)
    M, N = a.shape
    return _idct_matrix(M) @ a @ _idct_matrix(N).T
