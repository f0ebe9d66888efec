// hrms_plan.h -- work decomposition of the 1D kernels of eq. (2)-(4)
// (arXiv:1812.02647, Sec. 2), shared by the gfx950 kernels and the host
// planner. Header only and free of HIP headers, so that it can be checked
// with a host compiler alone.
//
// Output n of a spectrum of N bins has level H when n < floor(N / H); the
// outputs with the same top level Ht form a band [floor(N / 2Ht), floor(N / Ht))
// (the last band, Ht = Hmax, starts at 0). A tile is a run [a, aend) of one
// band. Term i of output n reads the window of positions i n .. i n + w_i,
// w_i = 0 for eq. (3) and i - 1 for eq. (2) and (4) (Greedy's offsets j, j + 1
// stay below i), so harmonic i of the tile reads the span
// [i a, i (aend - 1) + w_i + 1). The spans of neighbouring harmonics overlap
// once i (aend - a) >= a, and their union is a few intervals.
//
// A tile walks the union of its spans in chunks of at most C positions,
// increasing: each interval is cut into chunks [p, E) with p at a 16-byte
// boundary of the packed batch, the next chunk starting W = w_Ht positions
// (rounded down to that boundary) before the end of the previous one. Term
// (n, i) belongs to the chunk whose range holds the end i n + w_i of its
// window, i.e. the chunk with Eprev <= i n + w_i < E; the overlap of W makes
// the whole window lie in [p, E). The end of the window grows with i, so an
// output meets its harmonics in increasing i across chunks, and a chunk takes
// its harmonics in increasing i as well: every output adds its terms in the
// order of the equations.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define HRMS_HD __host__ __device__
#else
#define HRMS_HD
#endif

namespace hrms {

// Variant code of freq-bin HRMS (equals HRMS_FREQBIN in hrms.h).
constexpr int kPlanFreqbin = 2;

HRMS_HD inline int plan_min(int x, int y) { return x < y ? x : y; }
HRMS_HD inline int plan_max(int x, int y) { return x > y ? x : y; }

// Positions past i n that term i reads.
HRMS_HD inline int term_window(int variant, int i) { return variant == kPlanFreqbin ? 0 : i - 1; }

// Levels of output n of a spectrum of N bins analysed up to nlev levels.
HRMS_HD inline int output_levels(int n, int N, int nlev)
{
    int l = 1;
    while (l < nlev && n < (N >> l)) ++l;
    return l;
}

// ceil(x / d) for d > 0, 0 when x <= 0.
HRMS_HD inline int ceil_div_pos(int x, int d) { return x <= 0 ? 0 : (x + d - 1) / d; }

// Outputs [nb, ne) of tile [a, aend) whose term i belongs to the chunk ending
// at E that follows the chunk ending at Eprev (Eprev = 0 for the first chunk).
HRMS_HD inline void chunk_terms(int i, int w, int eprev, int e, int a, int aend, int& nb, int& ne)
{
    nb = plan_max(a, ceil_div_pos(eprev - w, i));
    ne = plan_min(aend, ceil_div_pos(e - w, i));
}

// Chunks of one tile, generated in increasing position.
struct SpanWalk {
    int a, aend, ht, win, vec, chunk, xmod;   // tile and layout
    int inext;                                // next harmonic not yet in an interval
    int iend;                                 // end of the current interval
    int eprev;                                // end of the previous chunk

    // win: 1 for eq. (2) and (4), 0 for eq. (3); vec: elements per 16 bytes;
    // xmod: absolute element index of the spectrum's first bin, modulo vec.
    HRMS_HD void begin(int a_, int aend_, int ht_, int win_, int vec_, int chunk_, int xmod_)
    {
        a = a_;
        aend = aend_;
        ht = ht_;
        win = win_;
        vec = vec_;
        chunk = chunk_;
        xmod = xmod_;
        inext = 1;
        iend = 0;
        eprev = 0;
    }

    HRMS_HD int span_end(int i) const { return i * (aend - 1) + win * (i - 1) + 1; }

    HRMS_HD int align_down(int q) const
    {
        int r = (xmod + q) % vec;
        if (r < 0) r += vec;
        return q - r;
    }

    // Next chunk [p, e) and the end of the chunk before it; false when the
    // tile has no more.
    HRMS_HD bool next(int& p, int& e, int& ep)
    {
        if (eprev >= iend) {
            if (inext > ht) return false;
            const int s = inext * a;
            iend = span_end(inext);
            ++inext;
            while (inext <= ht && inext * a <= iend) {
                iend = plan_max(iend, span_end(inext));
                ++inext;
            }
            p = align_down(s);
        } else {
            p = align_down(eprev - win * (ht - 1));
        }
        e = plan_min(p + chunk, iend);
        ep = eprev;
        eprev = e;
        return true;
    }
};

}  // namespace hrms
