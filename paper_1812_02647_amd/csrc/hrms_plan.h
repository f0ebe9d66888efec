// hrms_plan.h -- host-side work decomposition of the 1D kernels of
// eq. (2)-(4) (arXiv:1812.02647, Sec. 2): the LDS pieces of one tile. Header
// only and free of HIP so that it can be checked with a host compiler.
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

#include "hrms_types.h"

namespace hrms {

// Variant code of freq-bin HRMS (equals HRMS_FREQBIN in hrms.h).
constexpr int kPlanFreqbin = 2;

inline int level_index(int i)
{
    int l = 0;
    while ((1 << l) < i) ++l;
    return l;
}

// Pieces of tile [a, a + T) of a spectrum of n bins with nlev levels whose
// first bin sits at an absolute element index congruent to xmod modulo V
// (eq. (2)-(4) kernels). For each harmonic i = 1..Ht in turn, the outputs
// that still have harmonic i are cut into runs [n0, n1) whose bins
// i n0 .. i (n1 - 1) (+ i - 1 bins of window for Max and Greedy) fit one
// LDS chunk of `chunk` bins; the staged range starts at a 16-byte boundary.
// Returns the number of bins the tile stages.
inline int64_t tile_pieces(int variant, int vec, int chunk, int n, int nlev, int xmod, int a, int T,
                    std::vector<PieceRec>* out)
{
    const int win = variant == kPlanFreqbin ? 0 : 1;
    const int pmax = chunk - vec - 32;
    const int aend = std::min(a + T, n);
    int lt = 0;
    while (lt + 1 < nlev && a < (n >> (lt + 1))) ++lt;
    const int ht = 1 << lt;
    int64_t staged = 0;
    for (int i = 1; i <= ht; ++i) {
        const int li = level_index(i);
        const int hi = std::min(aend, n >> li);
        for (int n0 = a; n0 < hi;) {
            const int n1 = std::min(hi, n0 + pmax / i);
            const int64_t pos = (int64_t)i * n0;
            const int p0 = (int)(pos - ((xmod + pos) % vec));
            const int64_t last = (int64_t)i * (n1 - 1) + win * (i - 1);
            const int nv = (int)((last + 1 - p0 + vec - 1) / vec);
            if (out) {
                PieceRec pr;
                pr.p0 = p0;
                pr.nr = (n0 - a) | ((n1 - a) << 16);
                pr.ih = i | (li << 8) | (((i & (i - 1)) == 0 ? 1 : 0) << 16);
                pr.nv = nv;
                out->push_back(pr);
            }
            staged += (int64_t)nv * vec;
            n0 = n1;
        }
    }
    return staged;
}

}  // namespace hrms
