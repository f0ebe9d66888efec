// Host-only check of the 1D work decomposition (hrms_plan.h): for many
// spectrum geometries, the chunks of every band tile cover each (output,
// harmonic) pair that exists exactly once, in increasing harmonic order per
// output; each chunk holds every position its terms read (window included),
// starts at a 16-byte boundary of the packed batch and fits the LDS chunk.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_1812_02647_amd/csrc/hrms_plan.h"

using namespace hrms;

static int fails = 0;
#define CHECK(c, ...)                                  \
    do {                                               \
        if (!(c)) {                                    \
            if (fails < 20) std::printf(__VA_ARGS__);  \
            ++fails;                                   \
        }                                              \
    } while (0)

int main()
{
    const int lengths[] = {1, 2, 3, 7, 31, 64, 100, 1000, 4097, 65535, 200003, 1 << 18, 1 << 21};
    const int vecs[] = {4, 8};   // FP32, FP16/BF16
    const int chunks[] = {4096, 8192, 16384};
    const int tiles[] = {2048, 4096, 8192};
    long checked = 0, chunks_seen = 0;
    for (int variant = 1; variant <= 3; ++variant)
        for (int vec : vecs)
            for (int C : chunks)
                for (int T : tiles)
                    for (int N : lengths)
                        for (int nlev = 1; nlev <= 6; ++nlev)
                            for (int xmod = 0; xmod < vec; xmod += (vec == 4 ? 1 : 3)) {
                                if (N > 70000 && (nlev < 6 || xmod != 1 || C != 8192)) continue;
                                if (N > (1 << 18) && (T != 8192 || vec != 4)) continue;
                                const int win = variant == kPlanFreqbin ? 0 : 1;
                                // bands, then tiles of at most T outputs inside each
                                for (int l = 0; l < nlev; ++l) {
                                    const int hi = N >> l;
                                    const int lo = l + 1 < nlev ? (N >> (l + 1)) : 0;
                                    const int ht = 1 << l;
                                    for (int a = lo; a < hi; a += T) {
                                        const int aend = a + T < hi ? a + T : hi;
                                        for (int m = a; m < aend; ++m)
                                            CHECK(output_levels(m, N, nlev) == l + 1,
                                                  "band of n=%d N=%d\n", m, N);
                                        std::vector<int> lasti(aend - a, 0);
                                        SpanWalk w;
                                        w.begin(a, aend, ht, win, vec, C, xmod);
                                        int p, e, ep, prev_e = 0;
                                        while (w.next(p, e, ep)) {
                                            ++chunks_seen;
                                            CHECK(ep == prev_e, "chunk chain\n");
                                            CHECK(e > ep, "progress %d %d\n", ep, e);
                                            CHECK(e - p <= C, "capacity %d\n", e - p);
                                            CHECK(((xmod + p) % vec + vec) % vec == 0, "alignment\n");
                                            CHECK(e <= N, "past the spectrum %d %d\n", e, N);
                                            prev_e = e;
                                            for (int i = 1; i <= ht; ++i) {
                                                int nb, ne;
                                                chunk_terms(i, term_window(variant, i), ep, e, a,
                                                            aend, nb, ne);
                                                for (int m = nb; m < ne; ++m) {
                                                    CHECK(lasti[m - a] == i - 1,
                                                          "order n=%d i=%d last=%d\n", m, i,
                                                          lasti[m - a]);
                                                    lasti[m - a] = i;
                                                    const long s0 = (long)i * m;
                                                    const long s1 = s0 + term_window(variant, i);
                                                    CHECK(s0 >= p && s1 < e, "window n=%d i=%d\n", m,
                                                          i);
                                                }
                                            }
                                        }
                                        for (int m = a; m < aend; ++m) {
                                            CHECK(lasti[m - a] == ht, "coverage n=%d ht=%d got=%d\n",
                                                  m, ht, lasti[m - a]);
                                            ++checked;
                                        }
                                    }
                                }
                            }
    std::printf("checked %ld outputs in %ld chunks, %d failures\n", checked, chunks_seen, fails);
    return fails ? 1 : 0;
}
