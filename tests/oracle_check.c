/* Drives the CPU oracle (oracle/hrms_oracle.c, compiled into the same
 * program) under the address and undefined-behaviour sanitizers: every
 * variant, 1D and 2D, on spectra and planes of awkward sizes (1 bin, lengths
 * just past a power of two, odd row strides), every output, both precisions,
 * each input in an allocation of exactly its size so that any read past the
 * end is reported. Also checks the H = 1 identity on the way. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_num_levels(int hmax);
int oracle_stats(const double* x, int64_t n, double* mu, double* sigma);
int oracle_snr_consts(int variant, double mu, double sigma, int hmax, float* m32, float* q32,
                      double* m64, double* q64);
int oracle_hrms_1d(const double* x, int64_t N, int variant, int hmax, const int64_t* idx,
                   int64_t cnt, const double* m, const double* q, int f32, double* h,
                   double* max_snr, uint8_t* best_h);
int oracle_hrms_2d(const double* x, int64_t ld, int64_t nf, int zmax, int variant, int hmax,
                   const int64_t* fidx, const int32_t* zidx, int64_t cnt, const double* m,
                   const double* q, int f32, double* h, double* max_snr, uint8_t* best_h);
double oracle_sum_opt_paths(const double* x, int64_t N, int H, int64_t n, int f32);
int oracle_scale_f32(const double* x, int64_t n, double mu, double* out);

static uint64_t state = 1812026470u;
static double uni(void)
{
    state = state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}

static int fails = 0;

int main(void)
{
    const int64_t lengths[] = {1, 2, 3, 5, 31, 33, 64, 65, 257, 1000, 4097};
    for (size_t li = 0; li < sizeof(lengths) / sizeof(lengths[0]); ++li) {
        const int64_t N = lengths[li];
        double* x = malloc((size_t)N * sizeof(double));
        for (int64_t k = 0; k < N; ++k) x[k] = -log(1.0 - uni());
        double mu, sd;
        if (oracle_stats(x, N, &mu, &sd) != 0) ++fails;
        for (int variant = 0; variant <= 4; ++variant) {
            for (int hmax = 1; hmax <= 32; hmax *= 2) {
                const int nl = oracle_num_levels(hmax);
                double m[12], q[12];
                float m32[6], q32[6];
                const int cv = variant == 4 ? 3 : variant;
                if (oracle_snr_consts(cv, mu, sd, hmax, m32, q32, m, q) != 0) ++fails;
                double* h = malloc((size_t)(nl * N) * sizeof(double));
                double* ms = malloc((size_t)N * sizeof(double));
                uint8_t* bh = malloc((size_t)N);
                for (int f32 = 0; f32 <= 1; ++f32) {
                    if (oracle_hrms_1d(x, N, variant, hmax, NULL, N, m, q, f32, h, ms, bh) != 0)
                        ++fails;
                    for (int64_t k = 0; k < N; ++k)
                        if (h[k] != (f32 ? (double)(float)x[k] : x[k])) ++fails;
                }
                free(h);
                free(ms);
                free(bh);
            }
            if (variant == 4 && N >= 8)
                for (int64_t n = 0; n < N / 8; ++n) (void)oracle_sum_opt_paths(x, N, 8, n, 0);
        }
        double* y = malloc((size_t)N * sizeof(double));
        if (oracle_scale_f32(x, N, mu, y) != 0) ++fails;
        free(y);
        free(x);
    }
    /* planes: rows of nf bins in rows of ld */
    const int64_t nfs[] = {1, 7, 100, 513};
    for (size_t fi = 0; fi < sizeof(nfs) / sizeof(nfs[0]); ++fi) {
        for (int zmax = 0; zmax <= 5; zmax += 5) {
            const int64_t nf = nfs[fi], ld = nf + 3, rows = 2 * zmax + 1;
            /* the last row holds only nf bins: nothing past it may be read */
            const int64_t n_alloc = (rows - 1) * ld + nf;
            double* x = malloc((size_t)n_alloc * sizeof(double));
            for (int64_t k = 0; k < n_alloc; ++k) x[k] = -log(1.0 - uni());
            for (int variant = 0; variant <= 5; ++variant) {
                if (variant == 4) continue;
                for (int hmax = 1; hmax <= 32; hmax *= 2) {
                    const int nl = oracle_num_levels(hmax);
                    double m[12], q[12];
                    for (int l = 0; l < 12; ++l) m[l] = q[l] = 1.0;
                    double* h = malloc((size_t)(nl * rows * nf) * sizeof(double));
                    double* ms = malloc((size_t)(rows * nf) * sizeof(double));
                    uint8_t* bh = malloc((size_t)(rows * nf));
                    for (int f32 = 0; f32 <= 1; ++f32)
                        if (oracle_hrms_2d(x, ld, nf, zmax, variant, hmax, NULL, NULL, 0, m, q, f32,
                                           h, ms, bh) != 0)
                            ++fails;
                    for (int64_t r = 0; r < rows; ++r)
                        for (int64_t k = 0; k < nf; ++k)
                            if (h[r * nf + k] != (double)(float)x[r * ld + k]) ++fails;
                    free(h);
                    free(ms);
                    free(bh);
                }
            }
            free(x);
        }
    }
    printf("oracle under sanitizers: %d failures\n", fails);
    return fails ? 1 : 0;
}
