/*
 * Driver for a sanitizer build of the oracle's C part (AddressSanitizer and
 * UndefinedBehaviorSanitizer, CPU only).  Exercises every exported routine on
 * small sizes, including the edges (n = 1, 2, batch 0, fault indices at the
 * ends of a node, a fault at every level), and checks the radix-2 FFT against
 * the naive DFT.  Exit status 0 on success.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int32_t level;
    int32_t pad_;
    int64_t node;
    int64_t index;
    double dre, dim;
} orc_fault;

void orc_omega(int64_t t, int64_t n, double *re, double *im);
void orc_omega_table(int64_t n, int64_t count, double *out);
int orc_dft_naive_batch(const double *x, double *y, int64_t n, int64_t batch, int sign, int nthreads);
int orc_fft_batch(const double *x, double *y, int64_t n, int64_t batch, int sign, int nthreads);
int orc_fft_faulty(const double *x, double *y, int64_t n, int sign, const orc_fault *f, int64_t nf);
int orc_max_threads(void);
int orc_fault_struct_size(void);

static double urand(uint64_t *s)
{
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}

int main(void)
{
    uint64_t seed = 12345;
    int bad = 0;
    if (orc_fault_struct_size() != (int)sizeof(orc_fault)) bad = 1;
    (void)orc_max_threads();
    double re, im;
    orc_omega(-3, 8, &re, &im);
    orc_omega(1LL << 40, 3, &re, &im);
    for (int64_t n = 1; n <= 1024; n *= 2) {
        const int64_t batch = 3;
        double *x = malloc(sizeof(double) * 2 * n * batch);
        double *y = malloc(sizeof(double) * 2 * n * batch);
        double *z = malloc(sizeof(double) * 2 * n * batch);
        double *t = malloc(sizeof(double) * 2 * n);
        for (int64_t i = 0; i < 2 * n * batch; ++i) x[i] = urand(&seed);
        orc_omega_table(n, n, t);
        for (int sign = -1; sign <= 1; sign += 2) {
            if (orc_fft_batch(x, y, n, batch, sign, 1) != 0) bad = 1;
            if (orc_dft_naive_batch(x, z, n, batch, sign, 1) != 0) bad = 1;
            double err = 0.0, nrm = 0.0;
            for (int64_t i = 0; i < 2 * n * batch; ++i) {
                err += (y[i] - z[i]) * (y[i] - z[i]);
                nrm += z[i] * z[i];
            }
            if (!(sqrt(err) <= 1e-12 * sqrt(nrm) + 1e-300)) {
                fprintf(stderr, "n=%lld sign=%d fft vs naive %g\n", (long long)n, sign, sqrt(err / nrm));
                bad = 1;
            }
        }
        /* one fault at every level, first and last index of node 0 and of the last node */
        int levels = 0;
        while ((1LL << levels) < n) ++levels;
        for (int lvl = 0; lvl <= levels; ++lvl) {
            const int64_t len = n >> lvl, nodes = 1LL << lvl;
            orc_fault f[2] = {{lvl, 0, 0, 0, 1.0, 0.0}, {lvl, 0, nodes - 1, len - 1, 0.0, -1.0}};
            if (orc_fft_faulty(x, y, n, -1, f, 2) != 0) bad = 1;
        }
        if (orc_fft_batch(x, y, n, 0, -1, 1) != 0) bad = 1; /* empty batch */
        free(x);
        free(y);
        free(z);
        free(t);
    }
    /* rejected arguments */
    if (orc_fft_batch(NULL, NULL, 12, 1, -1, 1) == 0) bad = 1;
    if (orc_fft_batch(NULL, NULL, 8, 1, 0, 1) == 0) bad = 1;
    if (orc_dft_naive_batch(NULL, NULL, 0, 1, -1, 1) == 0) bad = 1;
    if (orc_fft_faulty(NULL, NULL, 8, -1, NULL, -1) == 0) bad = 1;
    printf(bad ? "FAIL\n" : "ok\n");
    return bad;
}
