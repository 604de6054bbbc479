"""MI355X-native 2D image FFT (radix-2 decimation in time) behind a C ABI.

The compute path lives in the HIP library ``libfft2.so`` built from ``csrc/``;
``fft2`` is a thin ctypes binding over it.  Importing this package does not
load the library; the first call into ``paper_1505_08019_amd.fft2`` does, and
fails loudly if it has not been built.
"""
