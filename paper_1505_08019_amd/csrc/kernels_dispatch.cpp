// kernels_dispatch.cpp -- routes a pass-kernel request to its translation unit.
#include "kernel_table.hpp"

void* fft2_row_kernel_a(int, int, int, bool);
void* fft2_row_kernel_b(int, int, int, bool);
void* fft2_row_kernel_c(int, int, int, bool);
void* fft2_row_kernel_d(int, int, int, bool);
void* fft2_col_kernel_a(int, int, int, bool);
void* fft2_col_kernel_b(int, int, int, bool);
void* fft2_col_kernel_c(int, int, int, bool);

void* fft2_row_kernel(int bn, int j, int nreg, bool partial) {
  if (bn <= 8) return fft2_row_kernel_a(bn, j, nreg, partial);
  if (bn <= 10) return fft2_row_kernel_b(bn, j, nreg, partial);
  if (bn <= 12) return fft2_row_kernel_c(bn, j, nreg, partial);
  return fft2_row_kernel_d(bn, j, nreg, partial);
}

void* fft2_col_kernel(int cb, int nz, int nreg, bool partial) {
  if (cb <= 2) return fft2_col_kernel_a(cb, nz, nreg, partial);
  if (cb == 3) return fft2_col_kernel_b(cb, nz, nreg, partial);
  return fft2_col_kernel_c(cb, nz, nreg, partial);
}
