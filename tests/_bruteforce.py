"""Brute-force 2D DFT straight from eq. (1), in pure Python ``cmath``.

Independent of the oracle (no shared code, no FFT): it evaluates the double
sum X[k1,k2] = sum_{n1,n2} x[n1,n2] exp(sign*2*pi*i*(k1*n1/M + k2*n2/N)) term
by term.  Used only on tiny images to pin the oracle and the GPU path.
"""
import cmath
import math


def dft2(x, sign=-1):
    rows = len(x)
    cols = len(x[0]) if rows else 0
    out = [[0j] * cols for _ in range(rows)]
    for k1 in range(rows):
        for k2 in range(cols):
            acc = 0j
            for n1 in range(rows):
                for n2 in range(cols):
                    ang = sign * 2.0 * math.pi * ((k1 * n1) / rows + (k2 * n2) / cols)
                    acc += x[n1][n2] * cmath.exp(1j * ang)
            out[k1][k2] = acc
    return out
