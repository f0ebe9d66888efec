/*
 * hrms_oracle.c -- plain CPU oracle for the incoherent harmonic sum.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the library under test links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do. It shares no code, header, table or constant with
 * the HIP implementation.
 *
 * Source: K. Adamek and W. Armour, "A GPU implementation of the harmonic sum
 * algorithm" (arXiv:1812.02647).
 *   - standard sum, eq. (1), Sec. 1
 *   - Max HRMS, eq. (2), Sec. 2
 *   - freq-bin HRMS, eq. (3), Sec. 2
 *   - Greedy HRMS, eq. (4) and the sentence after it, Sec. 2
 *   - exhaustive-path ("optimal") sum: Sec. 1 names an optimal sum that tries
 *     every combination of bins without defining it; the reading used here is
 *     stated at sum_opt_paths
 *   - 2D harmonic sum after the acceleration search: named in the abstract and
 *     Sec. 1 but not defined; the reading used here is stated at oracle_2d_sum.
 *   - SNR (Sec. 3) is reported but not defined; the reading used here is stated
 *     at oracle_snr_consts.
 *
 * Every output is computed straight from its definition, one output at a time,
 * with the harmonics summed in the order the equation writes them (i = 1..H).
 * Levels are recomputed from scratch; nothing is blocked, fused or reordered.
 *
 * Precision. Each routine takes a flag f32:
 *   f32 = 0 : every operation in binary64 (the reference for error bounds);
 *   f32 = 1 : every +, -, * result is rounded to binary32 at once, i.e. the sum
 *             is evaluated in FP32 in the written order. One +, -, * or / of
 *             two binary32 values carried out in binary64 and then rounded to
 *             binary32 is the correctly rounded binary32 result, since
 *             53 >= 2*24 + 2 (double rounding is innocuous in that case), so
 *             rnd() below reproduces IEEE binary32 arithmetic exactly.
 * Comparisons (Max, Greedy, best level) act on the values as stored, so they
 * are exact in both modes.
 *
 * Inputs are given as binary64 arrays. FP32/FP16/BF16 spectra widen to binary64
 * exactly, so the same bytes the device consumes reach the oracle unchanged.
 *
 * Parity pins: every routine is pinned by the CPU tests (identity at H = 1,
 * constant input, integer-valued exactness, brute-force path enumeration,
 * injected combs, closed-form statistics, 2D mirror symmetry and reduction to
 * 1D). The SNR null constants of Max and Greedy are pinned statistically only
 * (null calibration on exponential noise); they are otherwise parity unpinned.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#define OV_EQ1 0
#define OV_MAX 1
#define OV_FREQBIN 2
#define OV_GREEDY 3
#define OV_OPT 4
#define OV_GREEDY_FZ 5   /* 2D only: Greedy with fdot drift */

#define OE_OK 0
#define OE_INVAL (-1)

static double rnd(int f32, double v) { return f32 ? (double)(float)v : v; }

/* Round half up of a/b for a >= 0, b > 0, in integers: floor((2a + b) / 2b).
 * This is the reading of the non-integer index n*i/H of eq. (1). */
static int64_t round_half_up(int64_t a, int64_t b) { return (2 * a + b) / (2 * b); }

/* Round half away from zero of a/b, b > 0 (used for the fdot row of the 2D sum,
 * so that z and -z map to mirror rows). */
static int64_t round_half_away(int64_t a, int64_t b)
{
    return a >= 0 ? round_half_up(a, b) : -round_half_up(-a, b);
}

static int is_pow2_le32(int h) { return h >= 1 && h <= 32 && (h & (h - 1)) == 0; }

int oracle_num_levels(int hmax)
{
    int l = 0;
    if (!is_pow2_le32(hmax)) return OE_INVAL;
    while ((1 << l) < hmax) ++l;
    return l + 1;
}

/* ------------------------------------------------------------------------ */
/* Unnormalised partial sum S_H(n) of one output of a 1D spectrum.           */
/* ------------------------------------------------------------------------ */

/* eq. (1): S_H(n) = sum_{i=1..H} x(n*i/H), the index rounded half up. */
static double sum_eq1(const double* x, int64_t n, int H, int f32)
{
    double acc = 0.0;
    for (int i = 1; i <= H; ++i) acc = rnd(f32, acc + x[round_half_up(n * i, H)]);
    return acc;
}

/* eq. (2): S_H(n) = sum_{i=1..H} max over the i bins of harmonic i's window.
 * The window is read as x(i*n + j) for j = 0..i-1 (see the header of the test
 * fixtures and the design notes: with this offset H = 1 is the identity). */
static double sum_max(const double* x, int64_t n, int H, int f32)
{
    double acc = 0.0;
    for (int i = 1; i <= H; ++i) {
        double m = x[(int64_t)i * n];
        for (int j = 1; j < i; ++j) {
            double v = x[(int64_t)i * n + j];
            if (v > m) m = v;
        }
        acc = rnd(f32, acc + m);
    }
    return acc;
}

/* eq. (3): S_H(n) = sum_{i=1..H} x(i*n). */
static double sum_freqbin(const double* x, int64_t n, int H, int f32)
{
    double acc = 0.0;
    for (int i = 1; i <= H; ++i) acc = rnd(f32, acc + x[(int64_t)i * n]);
    return acc;
}

/* eq. (4): starting from the fundamental x(n) with offset j = 0, harmonic k
 * (k = 2..H) adds the larger of x(k*n + j) and x(k*n + j + 1); when the right
 * neighbour is strictly larger it is taken and j grows by one. */
static double sum_greedy(const double* x, int64_t n, int H, int f32)
{
    double acc = x[n];
    int64_t j = 0;
    for (int k = 2; k <= H; ++k) {
        double a = x[(int64_t)k * n + j];
        double b = x[(int64_t)k * n + j + 1];
        if (b > a) {
            acc = rnd(f32, acc + b);
            j += 1;
        } else {
            acc = rnd(f32, acc + a);
        }
    }
    return acc;
}

/*
 * Exhaustive-path sum. Sec. 1 names an optimal harmonic sum that performs every
 * possible sum; it is read as the maximum, over every offset path that eq. (4)
 * could follow, of the sum along that path: j_1 = 0 and j_k = j_{k-1} or
 * j_{k-1} + 1 for k = 2..H, and
 *     S_H(n) = max over paths of  x(n) + sum_{k=2..H} x(k*n + j_k).
 * Each path is summed in the order k = 1..H (in the chosen precision) and the
 * largest path sum is kept (a later path replaces it only when strictly
 * larger). Greedy follows one of these paths, so it never exceeds S_H.
 *
 * sum_opt_paths is that definition, enumerating the 2^(H-1) paths (bit k-2 of
 * the path number is the step taken at harmonic k): only practical for small
 * H. sum_opt is the same maximum by the recurrence over offsets,
 *     P_1(0) = x(n),
 *     P_k(j) = max(P_{k-1}(j), P_{k-1}(j-1)) + x(k*n + j),  0 <= j < k,
 * (a missing predecessor is skipped), S_H = max_j P_H(j). Rounding to binary32
 * is monotone, so the largest rounded path sum and the recurrence agree
 * exactly; the pins check the two against each other.
 */
static double sum_opt_paths(const double* x, int64_t n, int H, int f32)
{
    double best = 0.0;
    const int64_t npaths = (int64_t)1 << (H - 1);
    for (int64_t path = 0; path < npaths; ++path) {
        double acc = x[n];
        int64_t j = 0;
        for (int k = 2; k <= H; ++k) {
            j += (path >> (k - 2)) & 1;
            acc = rnd(f32, acc + x[(int64_t)k * n + j]);
        }
        if (path == 0 || acc > best) best = acc;
    }
    return best;
}

static double sum_opt(const double* x, int64_t n, int H, int f32)
{
    double P[32], Q[32];
    P[0] = x[n];
    for (int k = 2; k <= H; ++k) {
        for (int j = 0; j < k; ++j) {
            double m;
            if (j == 0) {
                m = P[0];
            } else if (j == k - 1) {
                m = P[k - 2];
            } else {
                m = P[j - 1] > P[j] ? P[j - 1] : P[j];
            }
            Q[j] = rnd(f32, m + x[(int64_t)k * n + j]);
        }
        for (int j = 0; j < k; ++j) P[j] = Q[j];
    }
    double best = P[0];
    for (int j = 1; j < H; ++j)
        if (P[j] > best) best = P[j];
    return best;
}

double oracle_sum_opt_paths(const double* x, int64_t N, int H, int64_t n, int f32)
{
    (void)N;
    if (H < 1 || H > 24) return NAN;
    return sum_opt_paths(x, n, H, f32);
}

/* Whether level H of output n exists. eq. (2)-(4) index up to H*n + H - 1, so
 * the level exists when that index is inside the spectrum; eq. (1) never reads
 * past n, so every level exists for every n. */
static int level_valid_1d(int variant, int64_t n, int64_t N, int H)
{
    if (variant == OV_EQ1) return 1;
    return n < N / H;
}

double oracle_sum_1d(const double* x, int64_t N, int variant, int H, int64_t n, int f32)
{
    (void)N;
    switch (variant) {
    case OV_EQ1: return sum_eq1(x, n, H, f32);
    case OV_MAX: return sum_max(x, n, H, f32);
    case OV_FREQBIN: return sum_freqbin(x, n, H, f32);
    case OV_GREEDY: return sum_greedy(x, n, H, f32);
    case OV_OPT: return sum_opt(x, n, H, f32);
    default: return NAN;
    }
}

/* Scale factor 1/sqrt(H) of eq. (1)-(3); in FP32 mode the factor itself is the
 * binary32 rounding of the binary64 value. */
static double inv_sqrt_h(int H, int f32) { return rnd(f32, 1.0 / sqrt((double)H)); }

/* ------------------------------------------------------------------------ */
/* Statistics and SNR constants.                                              */
/* ------------------------------------------------------------------------ */

/* Population mean and standard deviation over all bins. Sums are carried in
 * extended precision (x87 long double) so that the oracle's own rounding is
 * far below the device's binary64 reduction error. */
int oracle_stats(const double* x, int64_t n, double* mu, double* sigma)
{
    long double s1 = 0.0L, s2 = 0.0L;
    if (n < 1 || !x || !mu || !sigma) return OE_INVAL;
    for (int64_t k = 0; k < n; ++k) {
        s1 += (long double)x[k];
        s2 += (long double)x[k] * (long double)x[k];
    }
    long double m = s1 / (long double)n;
    long double v = s2 / (long double)n - m * m;
    if (v < 0.0L) v = 0.0L;
    *mu = (double)m;
    *sigma = (double)sqrtl(v);
    return OE_OK;
}

/*
 * Null mean m_H and standard deviation s_H of h_H = S_H / sqrt(H) when the
 * bins are independent with mean mu and standard deviation sigma. The paper
 * reports SNR (Sec. 3) without defining it; it is read here as the
 * standardisation snr_H = (h_H - m_H) / s_H, so that noise alone has mean 0
 * and unit spread at every level and for every variant.
 *
 *   eq. (1), eq. (3): S_H is a sum of H distinct bins:
 *       E S = H mu, Var S = H sigma^2.
 *   eq. (2): term i is the maximum of i bins. Writing a bin as
 *       mu + sigma (E - 1) with E ~ Exp(1) (a power spectrum of Gaussian noise
 *       is chi-square with two degrees of freedom, i.e. exponential), the
 *       maximum of i such E has mean Hn_i = sum_{k<=i} 1/k and variance
 *       Psi_i = sum_{k<=i} 1/k^2 (Renyi's representation of exponential order
 *       statistics), so E S = sum_i (mu + sigma (Hn_i - 1)),
 *       Var S = sigma^2 sum_i Psi_i.
 *   eq. (4): the first term is one bin; each later term is the maximum of two
 *       fresh bins (mean mu + sigma/2, variance 5/4 sigma^2), so
 *       E S = mu + (H-1)(mu + sigma/2), Var S = sigma^2 (1 + 5/4 (H-1)).
 *   Greedy with fdot drift (2D, z != 0): each later term is the maximum of
 *       four fresh bins (two rows by two columns), so
 *       E S = mu + (H-1)(mu + 13/12 sigma), Var S = sigma^2 (1 + 205/144 (H-1));
 *       its z = 0 row cannot drift in fdot and takes the eq. (4) constants.
 *   "Fresh" assumes the bins a path may read at different harmonics are
 *   distinct, which holds for fundamentals m >= H away from the plane's edge.
 *
 * Written out for level H in binary64, in this operation order, then rounded
 * once: m32 = (float)m, q32 = (float)(1/s), and q32 = 0 when s = 0.
 */
int oracle_snr_consts(int variant, double mu, double sigma, int hmax, float* m32, float* q32,
                      double* m64, double* q64)
{
    int nl = oracle_num_levels(hmax);
    if (nl < 1) return OE_INVAL;
    for (int l = 0; l < nl; ++l) {
        int H = 1 << l;
        double rh = sqrt((double)H);
        double mean_s, var_s;
        if (variant == OV_EQ1 || variant == OV_FREQBIN) {
            mean_s = (double)H * mu;
            var_s = (double)H * (sigma * sigma);
        } else if (variant == OV_MAX) {
            double hn = 0.0, psi = 0.0, sum_mean = 0.0, sum_psi = 0.0;
            for (int i = 1; i <= H; ++i) {
                hn = hn + 1.0 / (double)i;
                psi = psi + 1.0 / ((double)i * (double)i);
                sum_mean = sum_mean + (mu + sigma * (hn - 1.0));
                sum_psi = sum_psi + psi;
            }
            mean_s = sum_mean;
            var_s = (sigma * sigma) * sum_psi;
        } else if (variant == OV_GREEDY) {
            mean_s = mu + (double)(H - 1) * (mu + 0.5 * sigma);
            var_s = (sigma * sigma) * (1.0 + 1.25 * (double)(H - 1));
        } else if (variant == OV_GREEDY_FZ) {
            /* each later term is the largest of four fresh bins: mean
             * mu + sigma (Hn_4 - 1) = mu + 13/12 sigma, variance
             * Psi_4 sigma^2 = 205/144 sigma^2 */
            mean_s = mu + (double)(H - 1) * (mu + (13.0 / 12.0) * sigma);
            var_s = (sigma * sigma) * (1.0 + (205.0 / 144.0) * (double)(H - 1));
        } else {
            return OE_INVAL;
        }
        double m = mean_s / rh;
        double s = sqrt(var_s) / rh;
        double q = s > 0.0 ? 1.0 / s : 0.0;
        if (m32) m32[l] = (float)m;
        if (q32) q32[l] = (float)q;
        if (m64) m64[l] = m;
        if (q64) q64[l] = q;
    }
    return OE_OK;
}

/* snr_H = (h_H - m_H) * q_H, each operation in the chosen precision. */
static double snr_of(double h, double m, double q, int f32) { return rnd(f32, rnd(f32, h - m) * q); }

/* ------------------------------------------------------------------------ */
/* 1D driver.                                                                */
/* ------------------------------------------------------------------------ */

/*
 * Computes, for the outputs listed in idx (or every n in [0, N) when idx is
 * NULL), every level H = 1, 2, 4, ..., hmax:
 *   h[l * cnt + k]      = S_H(n_k) / sqrt(H)   (NaN where the level does not exist)
 *   max_snr[k], best_h[k]: the largest snr over the existing levels of n_k,
 *                          scanning H upwards and replacing only on a strictly
 *                          larger value (ties keep the smaller H).
 * m, q hold one constant pair per level (as produced by oracle_snr_consts:
 * the binary32 pair in FP32 mode, the binary64 pair otherwise). Any output
 * pointer may be NULL.
 */
int oracle_hrms_1d(const double* x, int64_t N, int variant, int hmax, const int64_t* idx,
                   int64_t cnt, const double* m, const double* q, int f32, double* h,
                   double* max_snr, uint8_t* best_h)
{
    int nl = oracle_num_levels(hmax);
    if (nl < 1 || N < 1 || !x || variant < 0 || variant > OV_OPT) return OE_INVAL;
    if (!idx) cnt = N;
    for (int64_t k = 0; k < cnt; ++k) {
        int64_t n = idx ? idx[k] : k;
        if (n < 0 || n >= N) return OE_INVAL;
        double best = 0.0;
        int best_level = 0;
        for (int l = 0; l < nl; ++l) {
            int H = 1 << l;
            if (!level_valid_1d(variant, n, N, H)) {
                if (h) h[(int64_t)l * cnt + k] = NAN;
                continue;
            }
            double s = oracle_sum_1d(x, N, variant, H, n, f32);
            double hv = rnd(f32, s * inv_sqrt_h(H, f32));
            if (h) h[(int64_t)l * cnt + k] = hv;
            if (m && q) {
                double snr = snr_of(hv, m[l], q[l], f32);
                if (l == 0 || snr > best) {
                    best = snr;
                    best_level = H;
                }
            }
        }
        if (max_snr) max_snr[k] = best;
        if (best_h) best_h[k] = (uint8_t)best_level;
    }
    return OE_OK;
}

/* ------------------------------------------------------------------------ */
/* 2D f-fdot plane.                                                          */
/* ------------------------------------------------------------------------ */

/*
 * The plane holds rows r = z + zmax for z = -zmax..zmax, each of nf frequency
 * bins, row stride ld. The 2D sum is named but not defined in the paper
 * (abstract, Sec. 1). It is read as the 1D sums applied along frequency, with
 * harmonic i of output (f, z) at level H taken from the fdot row nearest to
 * i*z/H: a signal whose H-th harmonic drifts by z bins has its i-th harmonic
 * drifting by i*z/H. The row is row_i = round_half_away(i*z, H) + zmax
 * (halves away from zero, so that z and -z map to mirror rows).
 *
 *   EQ1    :  S_H(f, z) = sum_{i=1..H} x[row_i][round_half_up(i*f, H)]
 *             (eq. (1) on both axes; every f in [0, nf) has every level)
 *   MAX    :  S_H(m, z) = sum_{i=1..H} max_{j=0..i-1} x[row_i][i*m + j]
 *   FREQBIN:  S_H(m, z) = sum_{i=1..H} x[row_i][i*m]
 *   GREEDY :  eq. (4) along frequency with harmonic k read from row_k:
 *             start at x[row_1][m], j = 0; for k = 2..H take the larger of
 *             x[row_k][k*m + j] and x[row_k][k*m + j + 1] (the right one only
 *             if strictly larger, then j += 1)
 * Outputs (m, z) of eq. (2)-(4) at level H exist for m < floor(nf / H), as in
 * 1D. Each level is computed on its own, since the row sampled for harmonic i
 * depends on H.
 */
/*
 * Greedy with fdot drift (2D only). The paper names a Greedy sum on the
 * frequency x fdot plane (abstract, Sec. 1) without defining it; it is read
 * as eq. (4)'s step rule applied to the fdot row as well as to the column.
 * With s = sign(z), path offsets j (column) and d (row, in fdot units)
 * starting at 0, and rows clamped to the plane:
 *     start at x[row_1][m];
 *     for k = 2..H, with r0 = clamp(round(k z / H) + d), r1 = clamp(r0' + s)
 *     where r0' = round(k z / H) + d, and c = k m + j, the candidates in this
 *     order are x[r0][c], x[r0][c + 1], x[r1][c], x[r1][c + 1]; the first
 *     largest is added (a later one replaces it only when strictly larger),
 *     and j grows by one when its column is c + 1, d by s when its row is r1.
 * The fdot of harmonic k grows in magnitude with k, so an underestimate of a
 * signal's fdot accumulates away from zero, as an underestimate of its
 * frequency accumulates upwards in eq. (4). At z = 0 (s = 0) the two rows
 * coincide and the sum is eq. (4) along row z = 0. Rows are rounded halves
 * away from zero and the candidate order is the same under z -> -z, so the
 * sum is mirror-symmetric in z.
 */
static int64_t clamp_row(int64_t r, int zmax) { return r < -zmax ? -zmax : (r > zmax ? zmax : r); }

static double sum_2d_greedy_fz(const double* x, int64_t ld, int zmax, int H, int64_t mbin, int z,
                               int f32)
{
    const int64_t s = z > 0 ? 1 : (z < 0 ? -1 : 0);
    int64_t j = 0, d = 0;
    double acc = x[(round_half_away((int64_t)z, H) + zmax) * ld + mbin];
    for (int k = 2; k <= H; ++k) {
        const int64_t rk = round_half_away((int64_t)k * z, H);
        const int64_t r0 = clamp_row(rk + d, zmax) + zmax;
        const int64_t r1 = clamp_row(rk + d + s, zmax) + zmax;
        const int64_t c = (int64_t)k * mbin + j;
        const double cand[4] = {x[r0 * ld + c], x[r0 * ld + c + 1], x[r1 * ld + c],
                                x[r1 * ld + c + 1]};
        int pick = 0;
        for (int t = 1; t < 4; ++t)
            if (cand[t] > cand[pick]) pick = t;
        acc = rnd(f32, acc + cand[pick]);
        if (pick & 1) j += 1;
        if (pick & 2) d += s;
    }
    return acc;
}

static double sum_2d(const double* x, int64_t ld, int zmax, int variant, int H, int64_t mbin, int z,
                     int f32)
{
    double acc = 0.0;
    if (variant == OV_EQ1) {
        for (int i = 1; i <= H; ++i) {
            int64_t row = round_half_away((int64_t)i * z, H) + zmax;
            acc = rnd(f32, acc + x[row * ld + round_half_up((int64_t)i * mbin, H)]);
        }
        return acc;
    }
    if (variant == OV_MAX) {
        for (int i = 1; i <= H; ++i) {
            int64_t row = round_half_away((int64_t)i * z, H) + zmax;
            const double* w = x + row * ld + (int64_t)i * mbin;
            double m = w[0];
            for (int j = 1; j < i; ++j)
                if (w[j] > m) m = w[j];
            acc = rnd(f32, acc + m);
        }
        return acc;
    }
    if (variant == OV_FREQBIN) {
        for (int i = 1; i <= H; ++i) {
            int64_t row = round_half_away((int64_t)i * z, H) + zmax;
            acc = rnd(f32, acc + x[row * ld + (int64_t)i * mbin]);
        }
        return acc;
    }
    if (variant == OV_GREEDY_FZ) return sum_2d_greedy_fz(x, ld, zmax, H, mbin, z, f32);
    /* GREEDY */
    {
        int64_t row1 = round_half_away((int64_t)z, H) + zmax;
        int64_t j = 0;
        acc = x[row1 * ld + mbin];
        for (int k = 2; k <= H; ++k) {
            int64_t row = round_half_away((int64_t)k * z, H) + zmax;
            double a = x[row * ld + (int64_t)k * mbin + j];
            double b = x[row * ld + (int64_t)k * mbin + j + 1];
            if (b > a) {
                acc = rnd(f32, acc + b);
                j += 1;
            } else {
                acc = rnd(f32, acc + a);
            }
        }
        return acc;
    }
}

double oracle_sum_2d(const double* x, int64_t ld, int zmax, int variant, int H, int64_t mbin, int z,
                     int f32)
{
    return sum_2d(x, ld, zmax, variant, H, mbin, z, f32);
}

/*
 * For the outputs (m_k, z_k) listed in (fidx, zidx) -- or the whole plane,
 * row-major over r = z + zmax then m, when fidx is NULL -- computes every level
 * exactly as oracle_hrms_1d does, with the 2D sums above. For Greedy with fdot
 * drift m and q hold two sets of per-level constants: [0, levels) for z != 0,
 * then [levels, 2 levels) for the z = 0 row.
 */
int oracle_hrms_2d(const double* x, int64_t ld, int64_t nf, int zmax, int variant, int hmax,
                   const int64_t* fidx, const int32_t* zidx, int64_t cnt, const double* m,
                   const double* q, int f32, double* h, double* max_snr, uint8_t* best_h)
{
    int nl = oracle_num_levels(hmax);
    if (nl < 1 || nf < 1 || zmax < 0 || ld < nf || !x) return OE_INVAL;
    if (variant < OV_EQ1 || variant > OV_GREEDY_FZ || variant == OV_OPT) return OE_INVAL;
    int64_t rows = 2 * (int64_t)zmax + 1;
    if (!fidx) cnt = rows * nf;
    for (int64_t k = 0; k < cnt; ++k) {
        int64_t mb = fidx ? fidx[k] : k % nf;
        int z = fidx ? zidx[k] : (int)(k / nf) - zmax;
        if (mb < 0 || mb >= nf || z < -zmax || z > zmax) return OE_INVAL;
        double best = 0.0;
        int best_level = 0;
        for (int l = 0; l < nl; ++l) {
            int H = 1 << l;
            if (!level_valid_1d(variant, mb, nf, H)) {
                if (h) h[(int64_t)l * cnt + k] = NAN;
                continue;
            }
            double s = sum_2d(x, ld, zmax, variant, H, mb, z, f32);
            double hv = rnd(f32, s * inv_sqrt_h(H, f32));
            if (h) h[(int64_t)l * cnt + k] = hv;
            if (m && q) {
                /* Greedy with fdot drift: its z = 0 row takes the second set */
                int c = (variant == OV_GREEDY_FZ && z == 0) ? nl + l : l;
                double snr = snr_of(hv, m[c], q[c], f32);
                if (l == 0 || snr > best) {
                    best = snr;
                    best_level = H;
                }
            }
        }
        if (max_snr) max_snr[k] = best;
        if (best_h) best_h[k] = (uint8_t)best_level;
    }
    return OE_OK;
}

/* ------------------------------------------------------------------------ */
/* Reduced-precision storage (FP16 / BF16) used by the precision study.       */
/* ------------------------------------------------------------------------ */

/*
 * Normalisation of a spectrum to unit mean before narrow storage: each bin is
 * multiplied by the binary32 value of 1/mu and the binary32 product is rounded
 * to the storage format. Only the binary32 product is formed here; rounding to
 * FP16 or BF16 is done by the test with numpy's own conversions (round to
 * nearest even; FP16 saturates at 65504 by clipping first).
 */
int oracle_scale_f32(const double* x, int64_t n, double mu, double* out)
{
    if (n < 0 || !(mu > 0.0)) return OE_INVAL;
    double inv = (double)(float)(1.0 / mu);
    for (int64_t k = 0; k < n; ++k) out[k] = (double)(float)(x[k] * inv);
    return OE_OK;
}
