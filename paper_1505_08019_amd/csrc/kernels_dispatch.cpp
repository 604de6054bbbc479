// kernels_dispatch.cpp -- routes a pass-kernel request to its translation unit.
#include "kernel_table.hpp"

void* fft2_row_kernel_a(int, int, int, bool);
void* fft2_row_kernel_b(int, int, int, bool);
void* fft2_row_kernel_c(int, int, int, bool);
void* fft2_row_kernel_d(int, int, int, bool);
void* fft2_row_kernel_e(int, int, int, bool);
void* fft2_row_kernel_f(int, int, int, bool);
void* fft2_col_kernel_a(int, int, int, bool);
void* fft2_col_kernel_b(int, int, int, bool);
void* fft2_col_kernel_c(int, int, int, bool);
void* fft2_col_kernel_d(int, int, int, bool);
void* fft2_rowip_kernel_a(int, int, int, bool);
void* fft2_rowip_kernel_b(int, int, int, bool);
void* fft2_rowip_kernel_c(int, int, int, bool);
void* fft2_rowip_kernel_d(int, int, int, bool);
void* fft2_filt_kernel_a(int, int, int, bool);
void* fft2_filt_kernel_b(int, int, int, bool);
void* fft2_filt_kernel_c(int, int, int, bool);
void* fft2_rowtail_kernel_a(int, int, int, bool);
void* fft2_rowtail_kernel_b(int, int, int, bool);
void* fft2_rowtail_kernel_c(int, int, int, bool);
void* fft2_rowtail_kernel_d(int, int, int, bool);

void* fft2_pass_kernel(int kind, int b1, int b2, int nreg, bool partial) {
  if (b1 < 0) return nullptr;
  switch (kind) {
    case 0:
      if (b1 <= 2) return fft2_row_kernel_a(b1, b2, nreg, partial);
      if (b1 <= 5) return fft2_row_kernel_e(b1, b2, nreg, partial);
      if (b1 <= 8) return fft2_row_kernel_f(b1, b2, nreg, partial);
      if (b1 <= 10) return fft2_row_kernel_b(b1, b2, nreg, partial);
      if (b1 <= 12) return fft2_row_kernel_c(b1, b2, nreg, partial);
      if (b1 <= 14) return fft2_row_kernel_d(b1, b2, nreg, partial);
      return nullptr;
    case 1:
      if (b1 <= 1) return fft2_col_kernel_a(b1, b2, nreg, partial);
      if (b1 <= 2) return fft2_col_kernel_d(b1, b2, nreg, partial);
      if (b1 <= 3) return fft2_col_kernel_b(b1, b2, nreg, partial);
      if (b1 <= 4) return fft2_col_kernel_c(b1, b2, nreg, partial);
      return nullptr;
    case 2:
      if (b1 <= 8) return fft2_rowip_kernel_a(b1, b2, nreg, partial);
      if (b1 <= 10) return fft2_rowip_kernel_b(b1, b2, nreg, partial);
      if (b1 <= 12) return fft2_rowip_kernel_c(b1, b2, nreg, partial);
      if (b1 <= 14) return fft2_rowip_kernel_d(b1, b2, nreg, partial);
      return nullptr;
    case 3:
      if (b1 <= 2) return fft2_filt_kernel_a(b1, b2, nreg, partial);
      if (b1 <= 3) return fft2_filt_kernel_b(b1, b2, nreg, partial);
      if (b1 <= 4) return fft2_filt_kernel_c(b1, b2, nreg, partial);
      return nullptr;
    case 4:
      if (b1 <= 8) return fft2_rowtail_kernel_a(b1, b2, nreg, partial);
      if (b1 <= 10) return fft2_rowtail_kernel_b(b1, b2, nreg, partial);
      if (b1 <= 12) return fft2_rowtail_kernel_c(b1, b2, nreg, partial);
      if (b1 <= 14) return fft2_rowtail_kernel_d(b1, b2, nreg, partial);
      return nullptr;
    default:
      return nullptr;
  }
}
