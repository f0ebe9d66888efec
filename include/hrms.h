/*
 * hrms.h -- C ABI of the MI355X (gfx950) incoherent harmonic-sum library.
 *
 * Implements the harmonic sums of K. Adamek and W. Armour, "A GPU
 * implementation of the harmonic sum algorithm" (arXiv:1812.02647):
 *
 *   HRMS_EQ1      eq. (1), Sec. 1  h(n)_H = H^-1/2 sum_{i=1..H} x(round(n i / H))
 *   HRMS_MAX      eq. (2), Sec. 2  h(n)_H = H^-1/2 sum_{i=1..H} max_{0<=j<i} x(i n + j)
 *   HRMS_FREQBIN  eq. (3), Sec. 2  h(n)_H = H^-1/2 sum_{i=1..H} x(i n)
 *   HRMS_GREEDY   eq. (4), Sec. 2  start at x(n), j = 0; harmonic k = 2..H adds
 *                                  the larger of x(k n + j), x(k n + j + 1) and
 *                                  moves j up by one when the right bin is
 *                                  strictly larger
 *   HRMS_OPT      Sec. 1 (the sum it calls optimal, which tries every bin
 *                                  combination; no definition given), 1D,
 *                                  h only: the largest sum over every offset
 *                                  path eq. (4) could follow (j_1 = 0, each
 *                                  later j equal to or one above the previous),
 *                                  each path added in the order k = 1..H
 *
 * over batches of 1D power spectra (the periodicity search after the FFT,
 * Sec. 1) and over a 2D frequency x fdot plane (the sum that follows the
 * Fourier-domain acceleration search; abstract, Sec. 1).
 *
 * Conventions shared by every entry point
 *   - Levels are H = 1, 2, 4, ..., hmax with hmax a power of two <= 32: the
 *     sum is reported after every doubling of the number of harmonics added
 *     (Sec. 1).
 *   - round() in eq. (1) rounds halves up; the fdot row of the 2D sum rounds
 *     halves away from zero. All index arithmetic is exact integer arithmetic.
 *   - Level H of output n exists for every n with eq. (1), and for
 *     n < floor(N / H) with eq. (2)-(4) (their last index H n + H - 1 must lie in
 *     the spectrum). Outputs are "compact": the level-H plane of eq. (2)-(4)
 *     holds floor(N / H) values, that of eq. (1) holds N values.
 *   - Sums are accumulated in FP32, harmonics added in the order i = 1..H of
 *     the equations, each level of eq. (1) summed on its own; h = S * r_H with
 *     r_H the FP32 value of 1/sqrt(H). No multiply-add contraction is used.
 *   - SNR (reported by the paper, Sec. 3, without a definition) is the
 *     standardisation snr_H = (h_H - m_H) * q_H with m_H, 1/q_H the null mean
 *     and standard deviation of h_H for independent bins of mean mu and
 *     standard deviation sigma (exact for exponential, i.e. chi-square 2 dof,
 *     noise; constants evaluated in FP64 and rounded once to FP32).
 *     max_snr[n] is the largest snr over the existing levels of n; best_h[n] is
 *     the H that attains it (the smallest such H on ties).
 *   - mu and sigma are the population mean and standard deviation of all bins
 *     of a spectrum (or plane), reduced in FP64 on the device, or supplied by
 *     the caller.
 *
 * Memory and threads
 *   - Buffers marked "device" are device pointers allocated by the caller
 *     (hipMalloc, or torch tensors on a HIP device). The library never frees
 *     caller memory. "host" arrays are read during the call only.
 *   - Work is enqueued asynchronously on the given HIP stream (NULL = the null
 *     stream). Buffers must stay alive until the stream reaches the work.
 *   - A handle is not thread-safe; use one handle per host thread. Calls on one
 *     handle may use different streams: a call that reuses the device scratch
 *     of an earlier call with the same batch signature (1D: offsets, Hmax,
 *     variant, storage type and launch shape; 2D: the plane's shape; the
 *     precision form: offsets) waits on its stream for that call's work to
 *     finish, so such calls run one after the other; other calls may overlap.
 *   - Every argument is checked before anything is enqueued. On error nothing
 *     is enqueued, no output is touched and a negative status is returned;
 *     hrms_last_error() gives the reason. No call aborts or throws.
 *
 * Environment (read by hrms_create)
 *   HRMS_NO_GRAPH=1        enqueue launches directly instead of replaying graphs
 *   HRMS_LOG=1             one line on stderr per plan built, graph captured,
 *                          tune cache read, no-alloc table copy and error
 *   HRMS_FAULT_INJECT=...  comma-separated injected failures for testing error
 *                          paths: "alloc" fails every device allocation of the
 *                          library (HRMS_E_NOMEM, nothing enqueued), "launch"
 *                          fails the harmonic-sum launch of every call
 *                          (HRMS_E_HIP; the statistics and constants launches
 *                          before it may have been enqueued); the handle stays
 *                          usable and destroyable
 *   HRMS_FORCE_SHAPE=wg:r:chunk[:top], HRMS_INFLIGHT_OUTPUTS=n
 *                          tuning overrides of the 1D launch shape and of the
 *                          outputs in flight per CU on large spectra (0: no
 *                          limit); results are the same bits
 */
#ifndef HRMS_H
#define HRMS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hrms_ctx* hrms_handle;

enum { HRMS_EQ1 = 0, HRMS_MAX = 1, HRMS_FREQBIN = 2, HRMS_GREEDY = 3, HRMS_OPT = 4 };

/* 2D only: Greedy with fdot drift. The paper names a Greedy sum on the
 * frequency x fdot plane (abstract, Sec. 1) without defining it; read as
 * eq. (4)'s step rule applied to the fdot row as well as to the column. With
 * s = sign(z) and path offsets j (column), d (row, fdot units) starting at 0,
 * output (m, z) of level H starts at the bin of harmonic 1; harmonic
 * k = 2..H chooses among columns k m + j, k m + j + 1 of rows
 * round(k z / H) + d and round(k z / H) + d + s (rows clamped to the plane),
 * in that order, the first largest winning (strict >); j grows by one for the
 * right column, d by s for the second row. At z = 0 this is HRMS_GREEDY along
 * row 0. SNR constants: each later term is the largest of four bins, so
 * m_H = H^-1/2 (mu + (H-1)(mu + 13/12 sigma)),
 * 1/q_H = sigma H^-1/2 (1 + 205/144 (H-1))^1/2; the z = 0 row takes
 * HRMS_GREEDY's. */
enum { HRMS_GREEDY_FDOT = 5 };

/* Storage type of the input bins. FP16 and BF16 widen exactly to FP32 before
 * any arithmetic. */
enum { HRMS_F32 = 0, HRMS_F16 = 1, HRMS_BF16 = 2 };

/* Output selection bits. HRMS_OUT_CAND (1D only) appends, for every bin whose
 * maximum SNR over the levels is at least cand_threshold, one hrms_candidate
 * record -- the thresholding step that follows the harmonic sum in a search
 * (Sec. 1) -- fused into the harmonic-sum kernels, so that a run asking only
 * for candidates writes no per-bin output.
 * HRMS_OUT_PEAKS (1D only; needs HRMS_OUT_MAXSNR, excludes HRMS_OUT_CAND)
 * appends instead only the bins that are also local maxima of max_snr along
 * their spectrum: max_snr[n] >= cand_threshold, max_snr[n] > max_snr[n - 1]
 * and max_snr[n] >= max_snr[n + 1] (a missing neighbour at either end of the
 * spectrum counts as lower; on a plateau the lowest bin is kept). It runs as
 * a pass over max_snr after the harmonic sum, since a bin's neighbours may
 * belong to other tiles. best_h is filled when HRMS_OUT_BESTH is set, else 0. */
enum {
    HRMS_OUT_H = 1u,
    HRMS_OUT_MAXSNR = 2u,
    HRMS_OUT_BESTH = 4u,
    HRMS_OUT_CAND = 8u,
    HRMS_OUT_PEAKS = 16u
};

/* A candidate bin of a 1D batch. */
typedef struct {
    int32_t spectrum;         /* index in the batch */
    int32_t bin;              /* output n (the fundamental for eq. (2)-(4), the
                                 H-th harmonic's bin for eq. (1)) */
    float snr;                /* its maximum SNR over the levels (bit-equal to max_snr) */
    int32_t best_h;           /* the level H attaining it (bit-equal to best_h) */
} hrms_candidate;

enum { HRMS_STATS_COMPUTE = 0, HRMS_STATS_PROVIDED = 1 };

enum {
    HRMS_OK = 0,
    HRMS_E_INVAL = -1,       /* an argument is invalid (see hrms_last_error) */
    HRMS_E_UNSUPPORTED = -2, /* valid request this build does not implement */
    HRMS_E_NODEVICE = -3,    /* no usable gfx950 device */
    HRMS_E_NOMEM = -4,       /* device or host allocation failed */
    HRMS_E_HIP = -5          /* a HIP runtime call failed */
};

#define HRMS_MAX_HMAX 32
#define HRMS_MAX_LEVELS 6
/* Largest spectrum (or plane row) length: keeps every index H*n + H below 2^31. */
#define HRMS_MAX_BINS (1 << 26)

/* A batch of 1D power spectra (DM trials), packed back to back. */
typedef struct {
    int32_t n_spectra;        /* >= 1 */
    int32_t variant;          /* HRMS_EQ1 .. HRMS_OPT; HRMS_OPT takes out_mask ==
                                 HRMS_OUT_H only (no closed-form null, so no SNR:
                                 other outputs give HRMS_E_UNSUPPORTED) */
    int32_t dtype;            /* HRMS_F32 / HRMS_F16 / HRMS_BF16 */
    int32_t hmax_all;         /* Hmax of every spectrum when hmax == NULL */
    uint32_t out_mask;        /* HRMS_OUT_* bits; 0 computes only the statistics */
    int32_t stats_mode;       /* HRMS_STATS_COMPUTE or HRMS_STATS_PROVIDED */
    const void* x;            /* device: offsets[n_spectra] bins of `dtype`; the
                                 bins of spectrum s are x[offsets[s] .. offsets[s+1]) */
    const int64_t* offsets;   /* host: n_spectra + 1 values, offsets[0] = 0,
                                 each spectrum 1 .. HRMS_MAX_BINS bins long */
    const uint8_t* hmax;      /* host: per-spectrum Hmax, or NULL for hmax_all */
    double* stats;            /* device: [n_spectra][2] = (mu, sigma); written
                                 (COMPUTE) or read (PROVIDED) */
    float* snr_consts;        /* device or NULL: [n_spectra][HRMS_MAX_LEVELS][2]
                                 = (m_H, q_H) of the run's variant, written;
                                 unused levels (and every level of HRMS_OPT)
                                 are written as 0 */
    float* h;                 /* device: compact level planes at the offsets
                                 given by hrms_layout_1d; needed iff OUT_H */
    float* max_snr;           /* device: offsets[n_spectra] floats; iff OUT_MAXSNR */
    uint8_t* best_h;          /* device: offsets[n_spectra] bytes (the H value);
                                 iff OUT_BESTH */
    hrms_candidate* cand;     /* device: cand_capacity records; iff OUT_CAND or OUT_PEAKS. The
                                 order of the records is unspecified. */
    uint32_t* cand_count;     /* device: one counter, iff OUT_CAND or OUT_PEAKS; set to the
                                 number of candidates found (records past
                                 cand_capacity are dropped, the count is not) */
    uint32_t cand_capacity;   /* records cand can hold (0 allowed: count only) */
    float cand_threshold;     /* SNR threshold of OUT_CAND / OUT_PEAKS (finite) */
} hrms_run1d_args;

/* One frequency x fdot plane: row r = z + zmax holds fdot z, z = -zmax..zmax.
 * The paper names this sum (abstract, Sec. 1) without defining it; it is read
 * as the variant's 1D sum along frequency with each harmonic taken from its
 * own fdot row. Output (m, z) of level H is the fundamental at frequency bin m
 * whose H-th harmonic has fdot z; harmonic i is read from row
 * round(i z / H) + zmax (halves away from zero) at frequency round(i m / H)
 * (EQ1, halves up), the window i*m .. i*m + i - 1 (MAX), i*m (FREQBIN) or
 * i*m + j (GREEDY, j as in eq. (4)). As in 1D, output (m, z) of level H exists
 * for every m with EQ1 and for m < floor(nf / H) otherwise. */
typedef struct {
    int32_t nf;               /* frequency bins per row, 1 .. HRMS_MAX_BINS */
    int32_t zmax;             /* >= 0 */
    int32_t hmax;             /* power of two <= 32 */
    int32_t variant;          /* HRMS_EQ1 .. HRMS_GREEDY, or HRMS_GREEDY_FDOT */
    int32_t dtype;
    uint32_t out_mask;
    int32_t stats_mode;
    int32_t reserved;         /* must be 0 */
    int64_t ld;               /* row stride in bins, >= nf */
    const void* x;            /* device: (2 zmax + 1) rows of ld bins, element-aligned */
    double* stats;            /* device: [2] = (mu, sigma) over the nf bins of every row */
    float* snr_consts;        /* device or NULL: [HRMS_MAX_LEVELS][2] = (m_H, q_H);
                                 HRMS_GREEDY_FDOT: [2][HRMS_MAX_LEVELS][2], the
                                 rows z != 0, then the row z = 0 */
    float* h;                 /* device: level H plane [2 zmax + 1][nf] (EQ1) or
                                 [2 zmax + 1][floor(nf / H)], packed level after
                                 level (hrms_layout_2d) */
    float* max_snr;           /* device: [2 zmax + 1][nf] */
    uint8_t* best_h;          /* device: [2 zmax + 1][nf] */
} hrms_run2d_args;

/* Normalisation to unit mean and narrow storage (FP16 / BF16) of FP32 spectra:
 * y = round_to_dtype(x * fl32(1/mu)), rounding to nearest even, FP16 saturating
 * at +-65504. The statistics of y are taken as mu' = 1, sigma' = sigma / mu.
 * With HRMS_STATS_PROVIDED the call reads stats back once the work already
 * queued on the stream is done (it blocks until then) and returns
 * HRMS_E_INVAL, enqueuing nothing, unless every mu is a positive finite number
 * and every sigma a non-negative finite one. With HRMS_STATS_COMPUTE a
 * spectrum whose computed mean is not positive (an all-zero spectrum) is
 * stored unscaled and stats_out receives its own (mu, sigma). */
typedef struct {
    int32_t n_spectra;
    int32_t dtype;            /* HRMS_F16 or HRMS_BF16 */
    int32_t stats_mode;       /* COMPUTE: raw (mu, sigma) are reduced into stats;
                                 PROVIDED: they are read from stats */
    int32_t reserved;         /* must be 0 */
    const float* x;           /* device, FP32, packed as in hrms_run1d_args */
    const int64_t* offsets;   /* host */
    double* stats;            /* device [n_spectra][2]: raw (mu, sigma) */
    double* stats_out;        /* device [n_spectra][2]: (1, sigma / mu) of y */
    void* y;                  /* device: offsets[n_spectra] 2-byte bins */
} hrms_quantize_args;

/* Creates a handle bound to HIP device `device_ordinal` (made current for
 * every later call on the handle). tune_cache_path: file holding tuned launch
 * shapes, or NULL. Returns HRMS_E_NODEVICE when the device is absent or not
 * gfx950. *out is set only on success. */
int hrms_create(hrms_handle* out, int device_ordinal, const char* tune_cache_path);

/* Releases the handle's workspace, plans and graphs. Accepts NULL. */
int hrms_destroy(hrms_handle h);

/* Host-only: layout of the compact h planes of a 1D batch. plane_offsets (host,
 * may be NULL) receives [n_spectra][HRMS_MAX_LEVELS] float offsets into h
 * (-1 for levels above the spectrum's Hmax); *h_total_floats (may be NULL) the
 * number of floats h must hold. Validates `a` exactly as hrms_run_1d does,
 * except for device pointers. Needs no device. */
int hrms_layout_1d(const hrms_run1d_args* a, int64_t* plane_offsets, int64_t* h_total_floats);

/* Host-only: same for a 2D plane; plane_offsets has HRMS_MAX_LEVELS entries. */
int hrms_layout_2d(const hrms_run2d_args* a, int64_t* plane_offsets, int64_t* h_total_floats);

/* Harmonic sum of a 1D batch: statistics (unless provided), SNR constants,
 * then every level of every spectrum in one persistent launch. `hip_stream` is
 * a hipStream_t or NULL. The launches (statistics, constants, one or two
 * harmonic-sum kernels) are captured into a HIP graph the first time a plan
 * (batch signature) meets a set of argument pointers and the graph is replayed
 * afterwards (environment HRMS_NO_GRAPH=1 enqueues them directly instead). */
int hrms_run_1d(hrms_handle h, const hrms_run1d_args* a, void* hip_stream);

/* hrms_run_1d for callers that cannot allocate device memory: code that runs
 * while a HIP graph is being captured, tight serving loops, harnesses that
 * forbid hipMalloc. Same arguments, validation and results (bit for bit) as
 * hrms_run_1d; it calls no hipMalloc, hipFree or other allocating routine.
 *   - Its plan tables (spectrum descriptors, tile queues, statistics segments)
 *     and per-call scratch (queue counters, statistics partials, SNR
 *     constants) live in one static device array of 48 MiB per GPU, held from
 *     the first hrms_create on that GPU until the process ends. A batch whose
 *     plan needs more (about 32 bytes per tile of 2048-4096 outputs, plus
 *     about 200 bytes per spectrum and 32 bytes per 65536 bins; 1000 spectra
 *     of 2^21 bins fit in every variant) is rejected with HRMS_E_INVAL before
 *     anything is enqueued.
 *   - Every call on a GPU, from any handle, shares that GPU's array, which
 *     keeps the last call's contents: calls that overlap on one GPU (on
 *     different streams, or from different threads) race and give wrong
 *     results. Order them on one stream.
 *   - Launches are enqueued directly (no graph). When the previous call on
 *     the GPU used another batch signature, the tables are first copied from
 *     host memory into the array on `hip_stream`.
 *   - The handle keeps the host side of its 4 latest batch signatures; making
 *     room for a fifth waits until the device is idle. */
int hrms_run_1d_noalloc(hrms_handle h, const hrms_run1d_args* a, void* hip_stream);

/* Picks the fastest compiled launch shape (threads per workgroup, outputs per
 * thread, LDS chunk or 0 for the gathered form -- for eq. (1), 0 for loads
 * straight from global memory and 1 for the form that stages each 512-output
 * run's harmonic spans in LDS -- and the lowest top level of the
 * bands handed to a second launch, 0 for none: eq. (2) runs them in the window
 * form, eq. (3)-(4) in the LDS form) for batches
 * like `a` -- same variant, storage type, largest
 * Hmax and mean spectrum length within a factor of two -- by timing `reps` runs
 * of each shape on `hip_stream` (the call blocks until they finish). Later
 * hrms_run_1d calls on the handle use it, and it is written to the handle's
 * tune cache file if one was given. The shape does not change any result bit:
 * every output adds its harmonics in the same order whatever the shape. The
 * outputs of `a` hold the result of the last run. chosen (host, may be NULL,
 * else four entries) receives {wg, r, chunk, top}. */
int hrms_autotune_1d(hrms_handle h, const hrms_run1d_args* a, void* hip_stream, int reps,
                     int32_t* chosen);

/* The launches hrms_run_1d would make for `a` on this handle, without running
 * them. info (host, five entries) receives the launch shape {wg, r, chunk,
 * top} the run uses (the handle's tuned shape for batches like `a`, else the
 * one HRMS_FORCE_SHAPE names, else the default) and the number of
 * harmonic-sum kernel launches: 2 when bands at or above `top` run in a launch
 * of their own, 1 otherwise, 0 when the batch has no outputs. Builds (or finds
 * in the handle's cache) the host side of the plan; touches no device memory
 * and enqueues nothing. Errors: as hrms_run_1d's argument checks, and
 * HRMS_E_INVAL for a NULL info. */
int hrms_plan_1d(hrms_handle h, const hrms_run1d_args* a, int32_t* info);

/* Harmonic sum of a 2D plane, HRMS_EQ1 .. HRMS_GREEDY and HRMS_GREEDY_FDOT
 * (HRMS_OPT: HRMS_E_UNSUPPORTED). */
int hrms_run_2d(hrms_handle h, const hrms_run2d_args* a, void* hip_stream);

/* Normalise and store FP32 spectra as FP16 / BF16 (precision form of the 1D
 * batch and of a plane with ld == nf, passed as one spectrum). */
int hrms_quantize(hrms_handle h, const hrms_quantize_args* a, void* hip_stream);

/* Static description of a status code. */
const char* hrms_strerror(int status);

/* Detail of the last error on this handle (empty string if none; a static
 * string for NULL handles). Valid until the next call on the handle. */
const char* hrms_last_error(hrms_handle h);

#ifdef __cplusplus
}
#endif

#endif /* HRMS_H */
