/*
 * synth.c -- seeded synthetic power spectra (host, multi-threaded).
 *
 * Input generator shared by the tests, the benchmark and the oracle's callers.
 * It holds none of the harmonic-sum arithmetic: it only draws noise.
 *
 * Noise model: the power spectrum of white Gaussian noise is chi-square with
 * two degrees of freedom, i.e. exponential; scaled to unit mean it is Exp(1).
 * Each value is drawn from a counter-based generator so that any bin can be
 * produced independently of the others and of the thread layout:
 *
 *   SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast splittable
 *   pseudorandom number generators", OOPSLA 2014): for a 64-bit counter c,
 *     z = c * 0x9E3779B97F4A7C15
 *     z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
 *     z = (z ^ (z >> 27)) * 0x94D049BB133111EB
 *     z =  z ^ (z >> 31)
 *   here applied to c = key(seed, stream) + index + 1, with
 *   key(seed, stream) = mix(seed ^ mix(stream + 0x5851F42D4C957F2D)),
 *   mix() being the three finaliser steps above.
 *
 *   U = ((z >> 11) + 0.5) * 2^-53 lies in (0, 1); the bin value is
 *   (float)(-log(U)), the inverse-CDF draw of Exp(1).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

static uint64_t mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static uint64_t stream_key(uint64_t seed, uint64_t stream)
{
    return mix(seed ^ mix(stream + 0x5851F42D4C957F2DULL));
}

static uint64_t draw_u64(uint64_t key, uint64_t index)
{
    return mix((key + index + 1) * 0x9E3779B97F4A7C15ULL);
}

uint64_t synth_u64(uint64_t seed, uint64_t stream, uint64_t index)
{
    return draw_u64(stream_key(seed, stream), index);
}

double synth_uniform(uint64_t seed, uint64_t stream, uint64_t index)
{
    uint64_t z = synth_u64(seed, stream, index);
    return ((double)(z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

typedef struct {
    uint64_t key;
    uint64_t start;
    int64_t count;
    float* out;
} job_t;

static void* run_job(void* p)
{
    job_t* j = (job_t*)p;
    for (int64_t k = 0; k < j->count; ++k) {
        uint64_t z = draw_u64(j->key, j->start + (uint64_t)k);
        double u = ((double)(z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        j->out[k] = (float)(-log(u));
    }
    return NULL;
}

/* out[k] = Exp(1) draw number (start + k) of stream `stream`, k < count. */
int synth_exponential_f32(uint64_t seed, uint64_t stream, uint64_t start, int64_t count,
                          float* out, int nthreads)
{
    if (count < 0 || (!out && count > 0)) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    if (count < (int64_t)1 << 16) nthreads = 1;
    uint64_t key = stream_key(seed, stream);
    job_t jobs[64];
    pthread_t th[64];
    int64_t per = (count + nthreads - 1) / nthreads;
    int started = 0;
    for (int t = 0; t < nthreads; ++t) {
        int64_t b = per * t, e = b + per < count ? b + per : count;
        if (b >= e) break;
        jobs[t].key = key;
        jobs[t].start = start + (uint64_t)b;
        jobs[t].count = e - b;
        jobs[t].out = out + b;
        if (t == 0) continue;
        if (pthread_create(&th[t], NULL, run_job, &jobs[t]) != 0) {
            run_job(&jobs[t]);
            th[t] = 0;
        }
        started = t;
    }
    if (count > 0) run_job(&jobs[0]);
    for (int t = 1; t <= started; ++t)
        if (th[t]) pthread_join(th[t], NULL);
    return 0;
}
