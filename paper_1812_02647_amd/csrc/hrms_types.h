// hrms_types.h -- plain data records shared by the host planner and the
// gfx950 kernels (no HIP dependency, so the planner can be checked with a
// host compiler alone). Not part of the public ABI.
#pragma once

#include <cstdint>

namespace hrms {

constexpr int kMaxLevels = 6;

// One spectrum of a 1D batch (or one row group of a plane), as the kernels see it.
struct SpecDesc {
    int64_t xoff;               // first input bin in x (elements)
    int64_t ooff;               // first bin of max_snr / best_h
    int64_t hoff[kMaxLevels];   // first float of each level plane in h, -1 if absent
    int32_t n;                  // bins
    int32_t nlev;               // levels: log2(Hmax) + 1
};

// A tile of consecutive outputs [a, aend) of one spectrum (1D kernels). For
// eq. (2)-(4) a tile lies inside one band and nlev is the band's level count;
// for eq. (1) nlev is the spectrum's.
struct TileRec {
    int64_t xoff;    // first bin of the spectrum in x (and in max_snr / best_h)
    int32_t n;       // bins of the spectrum
    int32_t a;       // first output of the tile
    int32_t aend;    // one past its last output
    int32_t spec;    // spectrum index (constants, h offsets)
    int32_t nlev;    // levels of the tile's outputs
    int32_t pad;
};

// A candidate bin (same layout as hrms_candidate in hrms.h).
struct CandRec {
    int32_t spec;
    int32_t n;
    float snr;
    int32_t h;
};

// A segment of one spectrum for the statistics reduction.
struct Seg {
    int32_t spec;
    int32_t start;
    int32_t len;
    int32_t pad;
};

}  // namespace hrms
