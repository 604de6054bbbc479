/*
 * fft2_oracle.c -- FP64 reference ("oracle") for the 2D image FFT.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code with the GPU path.
 *
 * What it computes (Shen et al., "Research on the fast Fourier transform of
 * image based on GPU"):
 *   - the DFT of eq. (1), X(k) = sum_n x(n) W_N^{nk}, N a power of two, with
 *     W_N = exp(-2*pi*i/N) for the forward direction and exp(+2*pi*i/N) for the
 *     inverse (the paper leaves the sign unstated; this is the usual reading);
 *   - reached by radix-2 decimation in time: the input is first put in
 *     bit-reversed order (sec. 3.2, the "descending" step), then log2 N levels
 *     of N/2 butterflies each apply eqs. (2)-(3):
 *         X(k)       = Xe(k) + W_N^k Xo(k)
 *         X(k + N/2) = Xe(k) - W_N^k Xo(k),   k < N/2
 *     where Xe, Xo are the half-length DFTs of the even and odd samples
 *     (eq. (2) as printed swaps the two names and mis-states the sum limits;
 *     the only consistent reading is the one used here);
 *   - in 2D by separability (sec. 2): every row is transformed, then every
 *     column (rows first; the paper allows either order).
 *   - The inverse is the same with conjugated twiddles, scaled by 1/(rows*cols)
 *     so that a forward/inverse round trip is the identity (the paper only
 *     says the inverse is easy to obtain, sec. 5).
 *
 * Everything is double precision.  Twiddles are cos/sin of 2*pi*j/m in FP64,
 * computed where they are used.  No blocking, no fusion, no reordering beyond
 * the loop order above.
 *
 * Staged snapshots: oracle_fft2 takes row_stages / col_stages.  Both scrambles
 * are always applied; then only the first row_stages butterfly levels along
 * each row and the first col_stages levels along each column are run.  With
 * both at their maximum (or negative) the result is the full 2D DFT.  The
 * 1/(rows*cols) inverse scale is applied only when both are at their maximum.
 *
 * OpenMP: rows (and then columns) are independent (sec. 2), so the row loop and
 * the column loop may run on several threads; the arithmetic of each row or
 * column is the same whatever the thread count.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_PI 3.14159265358979323846264338327950288

/* log2 of a power of two in [1, 2^30], else -1. */
int oracle_log2(int n)
{
    if (n <= 0) return -1;
    int b = 0;
    while ((1 << b) < n) b++;
    return ((1 << b) == n) ? b : -1;
}

/* rev_b(i): the low b bits of i written in reverse order (sec. 3.2). */
int oracle_bitrev(int i, int b)
{
    int r = 0;
    for (int k = 0; k < b; k++)
        r = (r << 1) | ((i >> k) & 1);
    return r;
}

/* In-place 1D transform of y[0..n), n = 2^b:
 * scramble y'[p] = y[rev_b(p)], then butterfly levels s = 1..nstages.
 * Level s joins blocks of m = 2^s points; inside each block the pair
 * (t+j, t+j+m/2) becomes (a + w*c, a - w*c) with w = W_m^j (eqs. 2-4). */
static void fft1d_dit(double complex *y, double complex *tmp, int b, int nstages, int sign)
{
    int n = 1 << b;
    for (int p = 0; p < n; p++)
        tmp[p] = y[oracle_bitrev(p, b)];
    for (int p = 0; p < n; p++)
        y[p] = tmp[p];
    for (int s = 1; s <= nstages; s++) {
        int m = 1 << s;
        int h = m / 2;
        for (int j = 0; j < h; j++) {
            double ang = 2.0 * ORACLE_PI * (double)j / (double)m;
            double complex w = cos(ang) + (double)sign * sin(ang) * I;
            for (int t = 0; t < n; t += m) {
                double complex a = y[t + j];
                double complex c = w * y[t + j + h];
                y[t + j] = a + c;
                y[t + j + h] = a - c;
            }
        }
    }
}

/* 2D transform.  in/out: rows*cols complex128 values, row-major, interleaved
 * (re, im) doubles; in == out is allowed.  sign: -1 forward, +1 inverse.
 * row_stages / col_stages: number of butterfly levels per dimension (negative
 * means all).  nthreads <= 0 means the OpenMP default.
 * Returns 0, or -1 for a size that is not a power of two, -2 for a bad sign,
 * -3 for an allocation failure. */
int oracle_fft2(const double *in, double *out, int rows, int cols, int sign,
                int row_stages, int col_stages, int nthreads)
{
    int bm = oracle_log2(rows), bn = oracle_log2(cols);
    if (bm < 0 || bn < 0) return -1;
    if (sign != -1 && sign != 1) return -2;
    if (row_stages < 0 || row_stages > bn) row_stages = bn;
    if (col_stages < 0 || col_stages > bm) col_stages = bm;
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
#endif
    size_t total = (size_t)rows * (size_t)cols;
    double complex *data = (double complex *)malloc(total * sizeof(double complex));
    if (!data) return -3;
    for (size_t i = 0; i < total; i++)
        data[i] = in[2 * i] + in[2 * i + 1] * I;
    int fail = 0;

    /* Every row: scramble, then row_stages levels. */
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        double complex *tmp = (double complex *)malloc((size_t)(cols > rows ? cols : rows) * sizeof(double complex));
        double complex *col = (double complex *)malloc((size_t)rows * sizeof(double complex));
        if (!tmp || !col) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            fail = 1;
        }
#ifdef _OPENMP
#pragma omp barrier
#endif
        if (!fail) {
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
            for (int r = 0; r < rows; r++)
                fft1d_dit(data + (size_t)r * cols, tmp, bn, row_stages, sign);
            /* Every column: gather, scramble, col_stages levels, scatter. */
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
            for (int c = 0; c < cols; c++) {
                for (int r = 0; r < rows; r++)
                    col[r] = data[(size_t)r * cols + c];
                fft1d_dit(col, tmp, bm, col_stages, sign);
                for (int r = 0; r < rows; r++)
                    data[(size_t)r * cols + c] = col[r];
            }
        }
        free(tmp);
        free(col);
    }
    if (fail) {
        free(data);
        return -3;
    }
    double scale = 1.0;
    if (sign == 1 && row_stages == bn && col_stages == bm)
        scale = 1.0 / (double)total;
    for (size_t i = 0; i < total; i++) {
        out[2 * i] = creal(data[i]) * scale;
        out[2 * i + 1] = cimag(data[i]) * scale;
    }
    free(data);
    return 0;
}

/* Gaussian low-pass mask for the image-filter request (the paper names image
 * filtering as the application of the 2D FFT, introduction):
 *   H(k1, k2) = exp(-rho^2 / (2 rc^2)),  rho = sqrt(f1^2 + f2^2) / 0.5,
 *   f = k/L for k < L/2, else (k - L)/L   (signed frequency in cycles/sample),
 * so rho is the radius as a fraction of the Nyquist frequency and rc is the
 * cutoff on that scale.  Writes rows*cols doubles. */
void oracle_gaussian_mask(double *h, int rows, int cols, double cutoff)
{
    for (int k1 = 0; k1 < rows; k1++) {
        double f1 = (k1 < rows / 2) ? (double)k1 / rows : (double)(k1 - rows) / rows;
        for (int k2 = 0; k2 < cols; k2++) {
            double f2 = (k2 < cols / 2) ? (double)k2 / cols : (double)(k2 - cols) / cols;
            double rho = sqrt(f1 * f1 + f2 * f2) / 0.5;
            h[(size_t)k1 * cols + k2] = exp(-(rho * rho) / (2.0 * cutoff * cutoff));
        }
    }
}

/* Filter request: forward 2D DFT, multiply every bin by the mask, inverse 2D
 * DFT.  in/out as in oracle_fft2. */
int oracle_filter(const double *in, double *out, int rows, int cols, double cutoff, int nthreads)
{
    size_t total = (size_t)rows * (size_t)cols;
    double *spec = (double *)malloc(2 * total * sizeof(double));
    double *h = (double *)malloc(total * sizeof(double));
    if (!spec || !h) {
        free(spec);
        free(h);
        return -3;
    }
    int rc = oracle_fft2(in, spec, rows, cols, -1, -1, -1, nthreads);
    if (rc == 0) {
        oracle_gaussian_mask(h, rows, cols, cutoff);
        for (size_t i = 0; i < total; i++) {
            spec[2 * i] *= h[i];
            spec[2 * i + 1] *= h[i];
        }
        rc = oracle_fft2(spec, out, rows, cols, +1, -1, -1, nthreads);
    }
    free(spec);
    free(h);
    return rc;
}

/* Thread count the OpenMP runtime would use for nthreads <= 0. */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
