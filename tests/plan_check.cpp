// Host-only check of the 1D work decomposition (hrms_plan.h): for many
// spectrum geometries, the pieces of every tile cover each (output, harmonic)
// pair that exists exactly once, in increasing harmonic order per output; each
// piece's staged range holds every bin its outputs read (window included), is
// 16-byte aligned in the packed batch and fits the LDS chunk.
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
    const int lengths[] = {1, 2, 3, 7, 31, 64, 100, 1000, 4097, 65535, 200003, 1 << 18};
    const int vecs[] = {4, 8};           // FP32, FP16/BF16
    const int chunks[] = {4096, 8192};
    const int tiles[] = {2048, 4096};
    long checked = 0;
    for (int variant = 1; variant <= 3; ++variant)
        for (int vec : vecs)
            for (int chunk : chunks)
                for (int T : tiles)
                    for (int n : lengths)
                        for (int nlev = 1; nlev <= 6; ++nlev)
                            for (int xmod = 0; xmod < vec; xmod += (vec == 4 ? 1 : 3)) {
                                if (n > 70000 && (nlev < 6 || xmod != 1 || chunk != 8192)) continue;
                                const int win = variant == kPlanFreqbin ? 0 : 1;
                                for (int a = 0; a < n; a += T) {
                                    std::vector<PieceRec> ps;
                                    tile_pieces(variant, vec, chunk, n, nlev, xmod, a, T, &ps);
                                    const int aend = std::min(a + T, n);
                                    // last harmonic seen per output
                                    std::vector<int> lasti(aend - a, 0);
                                    for (const PieceRec& p : ps) {
                                        const int i = p.ih & 0xff, li = (p.ih >> 8) & 0xff;
                                        const int snap = (p.ih >> 16) & 1;
                                        const int n0 = a + (p.nr & 0xffff), n1 = a + (p.nr >> 16);
                                        CHECK(li == level_index(i), "level %d of %d\n", li, i);
                                        CHECK(snap == ((i & (i - 1)) == 0), "snap flag\n");
                                        CHECK(n0 < n1 && n0 >= a && n1 <= aend, "range %d %d\n", n0, n1);
                                        CHECK((xmod + p.p0) % vec == 0, "alignment\n");
                                        CHECK(p.nv >= 1 && p.nv * vec <= chunk, "capacity %d\n", p.nv);
                                        for (int m = n0; m < n1; ++m) {
                                            // the output exists at harmonic i's level
                                            CHECK(m < (n >> li), "n=%d i=%d level missing\n", m, i);
                                            CHECK(lasti[m - a] == i - 1, "order n=%d i=%d last=%d\n", m, i,
                                                  lasti[m - a]);
                                            lasti[m - a] = i;
                                            const long lo = (long)i * m;
                                            const long hi = lo + win * (i - 1);
                                            CHECK(lo >= p.p0 && hi < (long)p.p0 + (long)p.nv * vec,
                                                  "staging n=%d i=%d\n", m, i);
                                        }
                                    }
                                    // every existing harmonic of every output was covered
                                    for (int m = a; m < aend; ++m) {
                                        int top = 0;
                                        for (int l = 0; l < nlev; ++l)
                                            if (m < (n >> l)) top = 1 << l;
                                        CHECK(lasti[m - a] == top, "coverage n=%d top=%d got=%d\n", m, top,
                                              lasti[m - a]);
                                        ++checked;
                                    }
                                }
                            }
    std::printf("checked %ld outputs, %d failures\n", checked, fails);
    return fails ? 1 : 0;
}
