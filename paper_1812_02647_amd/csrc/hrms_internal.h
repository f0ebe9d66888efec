// hrms_internal.h -- structures shared by the host runtime (hrms_abi.cpp) and
// the gfx950 kernels (hrms_kernels.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hrms_types.h"

namespace hrms {

// Per-level constants of one spectrum: null mean, inverse null spread and the
// level's scale fl32(1 / sqrt(H)).
struct LevelConst {
    float m;
    float q;
    float rh;
    float pad;
};

// Work queues of the persistent grid: one per XCD. Workgroup w starts on
// queue w % nqueues, claims its tiles through the queue's atomic counter and
// moves on to the following queues once its own is drained.
constexpr int kMaxQueues = 8;
constexpr int kCounterSlots = 2 * kMaxQueues;   // main launch, top-band launch

struct Run1DParams {
    const void* x;
    const SpecDesc* spec;
    const TileRec* tiles;       // queue q holds tiles[qbeg[q] .. qbeg[q + 1])
    const LevelConst* consts;   // [n_spec][kMaxLevels]
    float* h;
    float* max_snr;
    uint8_t* best_h;
    const int32_t* qbeg;        // [nqueues + 1]
    unsigned int* counters;     // [kMaxQueues] tiles claimed from each queue
    int32_t nqueues;
    uint32_t out_mask;
    CandRec* cand;              // candidate list (out_mask bit 8)
    unsigned int* cand_count;
    uint32_t cand_cap;
    float cand_thr;
};

struct StatsParams {
    const void* x;
    const SpecDesc* spec;
    const Seg* segs;
    double* partial;            // [nsegs][2]
    int32_t nsegs;
};

struct ConstsParams {
    const SpecDesc* spec;
    const Seg* segs;            // segments of each spectrum are contiguous
    const int32_t* seg_first;   // [n_spec + 1]
    const double* partial;
    double* stats;              // [n_spec][2]
    LevelConst* consts;         // [n_spec][kMaxLevels]
    float* user_consts;         // optional [n_spec][kMaxLevels][2]
    unsigned int* counters;     // [kCounterSlots] reset to 0 for the following launch, or NULL
    unsigned int* cand_count;   // reset to 0, or NULL
    int32_t n_spec;
    int32_t variant;
    int32_t compute_stats;      // 1: reduce partials into stats; 0: read stats
};

struct Run2DParams {
    const void* x;
    int64_t ld;
    const LevelConst* consts;   // [kMaxLevels]
    float* h;
    float* max_snr;
    uint8_t* best_h;
    int64_t hoff[kMaxLevels];   // first float of each level plane in h (-1: absent)
    int32_t nf;
    int32_t zmax;
    int32_t nlev;
    uint32_t out_mask;
    int32_t zgroups;            // ceil((2 zmax + 1) / rows per workgroup)
};

// Local maxima of max_snr above a threshold, one workgroup per segment.
struct PeakParams {
    const float* max_snr;
    const uint8_t* best_h;      // or NULL (records get 0)
    const SpecDesc* spec;       // xoff, n
    const Seg* segs;
    CandRec* cand;
    unsigned int* cand_count;
    uint32_t cand_cap;
    float thr;
    int32_t nsegs;
};

// Normalisation constants of the precision form, one per spectrum.
struct QuantConstParams {
    const SpecDesc* spec;
    const int32_t* seg_first;
    const double* partial;
    double* stats;              // raw (mu, sigma): written (compute) or read
    double* stats_out;          // (1, sigma / mu)
    float* inv_mu;              // fl32(1 / mu)
    int32_t n_spec;
    int32_t compute_stats;
};

struct QuantParams {
    const float* x;
    const SpecDesc* spec;       // xoff = first bin, n = bins
    const Seg* segs;
    const float* inv_mu;
    void* y;
    int32_t nsegs;
};

// Launch shapes of the 1D harmonic-sum kernel family.
struct Shape1D {
    int wg;        // threads per workgroup
    int r;         // outputs per thread
    int chunk;     // eq. (2)-(4): positions per LDS chunk (two are kept); 0: gathered
                   // from global memory (and eq. (1))
    int top;       // eq. (2)-(4): bands whose top level is at least `top` run in a
                   // second launch (hrms1d_top_shape); 0: none
};

// Launch shape of the LDS form for the top bands of a split launch.
constexpr Shape1D kTopShape{1024, 8, 16384, 0};
// eq. (2)'s top bands run in the window form instead, one run of WG outputs
// per tile: an XCD's resident workgroups then share one spectrum's top band
// and walk its harmonics at about the same pace, so that the lines harmonic
// k + 1 reads are still in the L2 from harmonic k of other workgroups.
constexpr Shape1D kTopWinShape{256, 8, 0, 0};
inline Shape1D hrms1d_top_shape(int variant) { return variant == 1 ? kTopWinShape : kTopShape; }
// Outputs per tile of the split launch.
inline int hrms1d_top_tile(int variant)
{
    return variant == 1 ? kTopWinShape.wg : kTopShape.wg * kTopShape.r;
}
// The exhaustive-path sum's only launch shape: 256 lanes, 8 outputs per lane
// taken in sequence, bins read straight from memory.
constexpr Shape1D kOptShape{256, 8, 0, 0};

// Kernel launchers (hrms_kernels.hip). Return hipSuccess or the launch error.
hipError_t launch_stats_partial(int dtype, const StatsParams& p, hipStream_t s);
hipError_t launch_consts(const ConstsParams& p, hipStream_t s);
hipError_t launch_hrms1d(int variant, int dtype, const Shape1D& shape, const Run1DParams& p,
                         int grid, hipStream_t s);
// Outputs per tile of a launch shape: every thread holds r outputs.
inline int hrms1d_tile_outputs(int variant, const Shape1D& s)
{
    (void)variant;
    return s.wg * s.r;
}
// eq. (2) and the exhaustive-path sum in the gathered shapes run the window
// form, whose lanes walk a tile's outputs in sequence (wg * 4 or wg * 2 at a
// time in the cheap bands, wg in the deep ones), so a tile may hold any
// number of outputs.
inline bool hrms1d_window_form(int variant, const Shape1D& s)
{
    return (variant == 1 || variant == 4) && s.chunk == 0;
}
// Tile length of a band whose top level is ht, in a spectrum whose top level
// is htop: the forms without LDS staging give their cheap bands longer tiles
// so that per-tile work (claim, record, barrier) stays small against the bins
// they cover. Multiples measured on 1000 x 2^21 FP32 batches: the window form
// 8x (ht <= 2) and 2x (ht <= 8); freq-bin 2x (ht <= 2; 8x and 2x for ht <= 8
// were slower); Greedy 8x and 2x below htop = 32 (Hmax 4: 11.9 -> 7.2 ms,
// 16: 12.6 -> 10.5) but only 2x (ht <= 2) at Hmax 32, where the longer tiles
// lost 0.6 ms.
inline int hrms1d_band_tile(int variant, const Shape1D& s, int ht, int htop)
{
    const int t = hrms1d_tile_outputs(variant, s);
    if (s.chunk != 0) return t;
    const bool wide = hrms1d_window_form(variant, s) || (variant == 3 && htop < 32);
    if (wide) return ht <= 2 ? 8 * t : ht <= 8 ? 2 * t : t;
    return ht <= 2 ? 2 * t : t;
}
// Resident workgroups per CU of the 1D kernel; 0 (with *err set) on failure.
int hrms1d_max_blocks_per_cu(int variant, int dtype, const Shape1D& shape, hipError_t* err);
bool hrms1d_shape_supported(int variant, const Shape1D& shape);
// Shapes compiled for the variant's kernel family; returns their count and
// writes up to `cap` of them.
int hrms1d_shapes(int variant, Shape1D* out, int cap);
hipError_t launch_hrms2d(int variant, int dtype, const Run2DParams& p, hipStream_t s);
hipError_t launch_peaks(const PeakParams& p, hipStream_t s);
hipError_t launch_quant_consts(const QuantConstParams& p, hipStream_t s);
hipError_t launch_quantize(int dtype, const QuantParams& p, hipStream_t s);

// Static device scratch of hrms_run_1d_noalloc, one copy per GPU
// (hrms_noalloc.hip): 48 MiB holds the plan of 1000 spectra of 2^21 bins in
// every variant and launch shape.
constexpr size_t kNoallocScratchBytes = size_t(48) << 20;
// Device address of `device`'s copy, looked up once per device with that
// device current (later calls return the stored address and status).
hipError_t noalloc_scratch(int device, void** ptr);

}  // namespace hrms
