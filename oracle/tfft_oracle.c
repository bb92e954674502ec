/*
 * FP64 CPU oracle for the batched complex-to-complex DFT (TEST INFRASTRUCTURE).
 *
 * This file is part of the independent reference that the HIP path is checked
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no source, header, table or generator with the
 * product library, and the product never calls it.
 *
 * What it computes (TurboFFT paper, Section II "Background", DFT definition):
 *   forward  y_j = sum_n x_n * w_N^{j n},        w_N = exp(-2 pi i / N)
 *   inverse  x_j = (1/N) sum_n y_n * w_N^{-j n}  (the 1/N is applied by the caller)
 * and the O(N log N) factorisation of the same matrix (Section II, "FFT
 * accelerates DFT computation through factorization") as a textbook recursive
 * radix-2 decimation-in-time split.  The recursion can add a value to the output
 * of any node, which models the paper's fault model (Section II-A: one soft
 * error in a compute unit per detection period).
 *
 * Everything is IEEE binary64 with round-to-nearest; no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* One additive fault on the output of one node of the radix-2 recursion.
 * level 0 is the whole transform; the two children of node v at level l are
 * nodes 2v (even-indexed inputs) and 2v+1 (odd-indexed inputs) at level l+1;
 * level log2(N) holds the length-1 leaves (a copy of one input element). */
typedef struct {
    int32_t level;
    int32_t pad_;
    int64_t node;
    int64_t index; /* element of that node's output, 0 <= index < N >> level */
    double dre, dim;
} orc_fault;

/* w_n^t = exp(-2 pi i t / n).  The angle is reduced with exact integer
 * arithmetic to [0, pi/4] (octant symmetry of cos/sin) before libm is called,
 * so the only roundings are one in the reduced angle and libm's own. */
void orc_omega(int64_t t, int64_t n, double *re, double *im)
{
    int64_t q = 8 * n; /* angle = 2 pi p / q */
    int64_t p = (8 * (t % n) + q) % q;
    int neg_sin = 0, neg_cos = 0, swap = 0;
    if (2 * p > q) { p = q - p; neg_sin = 1; }      /* theta -> 2pi - theta */
    if (4 * p > q) { p = q / 2 - p; neg_cos = 1; }  /* theta -> pi - theta  */
    if (8 * p > q) { p = q / 4 - p; swap = 1; }     /* theta -> pi/2 - theta */
    double ang = (2.0 * M_PI * (double)p) / (double)q;
    double c = cos(ang), s = sin(ang);
    if (p == 0) { c = 1.0; s = 0.0; }
    if (swap) { double tmp = c; c = s; s = tmp; }
    if (neg_cos) c = -c;
    if (neg_sin) s = -s;
    *re = c;
    *im = -s;
}

/* out[2t], out[2t+1] = w_n^t for 0 <= t < count */
void orc_omega_table(int64_t n, int64_t count, double *out)
{
    for (int64_t t = 0; t < count; ++t) orc_omega(t, n, &out[2 * t], &out[2 * t + 1]);
}

static double *make_table(int64_t n, int64_t count)
{
    double *tw = (double *)malloc(sizeof(double) * 2 * (size_t)(count > 0 ? count : 1));
    if (tw) orc_omega_table(n, count, tw);
    return tw;
}

/* ---------------------------------------------------------------- naive DFT */

static void dft_one(const double *x, double *y, int64_t n, int sign, const double *tw)
{
    for (int64_t j = 0; j < n; ++j) {
        double sr = 0.0, si = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            int64_t t = (int64_t)(((__int128)j * k) % n);
            double wr = tw[2 * t], wi = sign > 0 ? -tw[2 * t + 1] : tw[2 * t + 1];
            double xr = x[2 * k], xi = x[2 * k + 1];
            sr += wr * xr - wi * xi;
            si += wr * xi + wi * xr;
        }
        y[2 * j] = sr;
        y[2 * j + 1] = si;
    }
}

/* Direct O(N^2) sum for each of `batch` contiguous signals.  sign=-1 forward,
 * sign=+1 the unscaled inverse.  Returns 0, or -1 on bad arguments. */
int orc_dft_naive_batch(const double *x, double *y, int64_t n, int64_t batch, int sign, int nthreads)
{
    if (n < 1 || batch < 0 || (sign != 1 && sign != -1)) return -1;
    double *tw = make_table(n, n);
    if (!tw) return -2;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t b = 0; b < batch; ++b) dft_one(x + 2 * b * n, y + 2 * b * n, n, sign, tw);
    free(tw);
    return 0;
}

/* ------------------------------------------------------- recursive radix-2 */

static void fft_rec(const double *x, int64_t xs, int64_t n, double *y, const double *tw, int64_t tws, int sign,
                    int level, int64_t node, const orc_fault *f, int64_t nf)
{
    if (n == 1) {
        y[0] = x[0];
        y[1] = x[1];
    } else {
        int64_t h = n / 2;
        /* even-indexed inputs -> y[0, h), odd-indexed inputs -> y[h, n) */
        fft_rec(x, 2 * xs, h, y, tw, 2 * tws, sign, level + 1, 2 * node, f, nf);
        fft_rec(x + 2 * xs, 2 * xs, h, y + 2 * h, tw, 2 * tws, sign, level + 1, 2 * node + 1, f, nf);
        for (int64_t k = 0; k < h; ++k) {
            double wr = tw[2 * k * tws], wi = tw[2 * k * tws + 1];
            if (sign > 0) wi = -wi;
            double er = y[2 * k], ei = y[2 * k + 1];
            double orr = y[2 * (k + h)], oi = y[2 * (k + h) + 1];
            double tr = wr * orr - wi * oi, ti = wr * oi + wi * orr;
            y[2 * k] = er + tr;
            y[2 * k + 1] = ei + ti;
            y[2 * (k + h)] = er - tr;
            y[2 * (k + h) + 1] = ei - ti;
        }
    }
    for (int64_t i = 0; i < nf; ++i) {
        if (f[i].level == level && f[i].node == node && f[i].index >= 0 && f[i].index < n) {
            y[2 * f[i].index] += f[i].dre;
            y[2 * f[i].index + 1] += f[i].dim;
        }
    }
}

static int is_pow2(int64_t n) { return n >= 1 && (n & (n - 1)) == 0; }

/* Radix-2 FFT of `batch` contiguous length-n signals (n a power of two). */
int orc_fft_batch(const double *x, double *y, int64_t n, int64_t batch, int sign, int nthreads)
{
    if (!is_pow2(n) || batch < 0 || (sign != 1 && sign != -1)) return -1;
    double *tw = make_table(n, n / 2);
    if (!tw) return -2;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t b = 0; b < batch; ++b)
        fft_rec(x + 2 * b * n, 1, n, y + 2 * b * n, tw, 1, sign, 0, 0, NULL, 0);
    free(tw);
    return 0;
}

/* Radix-2 FFT of one signal with additive faults on recursion nodes. */
int orc_fft_faulty(const double *x, double *y, int64_t n, int sign, const orc_fault *f, int64_t nf)
{
    if (!is_pow2(n) || (sign != 1 && sign != -1) || nf < 0) return -1;
    double *tw = make_table(n, n / 2);
    if (!tw) return -2;
    fft_rec(x, 1, n, y, tw, 1, sign, 0, 0, f, nf);
    free(tw);
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_fault_struct_size(void) { return (int)sizeof(orc_fault); }
