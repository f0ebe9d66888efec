// Host-only check of the runtime behind the C ABI (validation, layout, the 1D
// planner and the no-alloc scratch layout), built with g++ and the address
// and undefined-behaviour sanitizers. The kernels and their launchers are not
// built: the few launcher entry points the runtime calls are replaced by
// stubs, and no device is touched.
//
// For many batches (ragged lengths, per-spectrum Hmax, every variant, storage
// type and launch shape) it checks that
//   - every output of every band of every spectrum lies in exactly one tile
//     of the launch that owns its band (top bands in the second launch when
//     the shape splits), tiles stay inside their band and spectrum, and each
//     tile's level count is its band's (eq. (1): the spectrum's);
//   - each launch's queues partition its tile list, the grid is positive and
//     a multiple of the queue count when it can be;
//   - the statistics segments cover each spectrum once, in order;
//   - the compact plane layout matches floor(N / H) (N for eq. (1));
//   - the no-alloc scratch sections are 256-byte aligned, disjoint and inside
//     the total;
// and that invalid arguments are rejected with the documented status.
#include "../paper_1812_02647_amd/csrc/hrms_abi.cpp"

#include <random>

namespace hrms {
// Launchers and occupancy: stubs (the planner only asks for the occupancy).
hipError_t launch_stats_partial(int, const StatsParams&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_consts(const ConstsParams&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_hrms1d(int, int, const Shape1D&, const Run1DParams&, int, hipStream_t)
{
    return hipErrorNotSupported;
}
hipError_t launch_hrms2d(int, int, const Run2DParams&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_peaks(const PeakParams&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_quant_consts(const QuantConstParams&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_quantize(int, const QuantParams&, hipStream_t) { return hipErrorNotSupported; }
int hrms1d_max_blocks_per_cu(int, int, const Shape1D& s, hipError_t* err)
{
    if (err) *err = hipSuccess;
    return s.wg >= 1024 ? 1 : s.wg >= 512 ? 2 : 3;
}
bool hrms1d_shape_supported(int variant, const Shape1D& s)
{
    if (variant == 4) return s.wg == kOptShape.wg && s.r == kOptShape.r && s.chunk == 0 && s.top == 0;
    if (variant == 0) return s.chunk == 0 && s.top == 0;
    return true;
}
int hrms1d_shapes(int, Shape1D*, int) { return 0; }
hipError_t noalloc_scratch(int, void** ptr)
{
    *ptr = nullptr;
    return hipErrorNotSupported;
}
}  // namespace hrms

static int fails = 0;
#define CHECK(c, ...)                                 \
    do {                                              \
        if (!(c)) {                                   \
            if (fails < 30) std::printf(__VA_ARGS__); \
            ++fails;                                  \
        }                                             \
    } while (0)

static void check_plan(hrms_ctx* c, const hrms_run1d_args* a, const Shape1D& shape)
{
    Plan1D P;
    const int st = plan_host_1d(c, a, shape, &P);
    CHECK(st == HRMS_OK, "plan status %d\n", st);
    if (st != HRMS_OK) return;
    const int ns = a->n_spectra;
    // coverage: per spectrum, per output, count of tiles holding it
    for (int part = 0; part < 2; ++part) {
        const std::vector<TileRec>& tiles = part ? P.tiles_top : P.tiles;
        const std::vector<int32_t>& qb = part ? P.qbeg_top : P.qbeg;
        CHECK((int)qb.size() == P.nqueues + 1, "queue bounds\n");
        CHECK(qb.front() == 0 && qb.back() == (int)tiles.size(), "queues span the list\n");
        for (size_t q = 0; q + 1 < qb.size(); ++q) CHECK(qb[q] <= qb[q + 1], "queue order\n");
        const int grid = part ? P.grid_top : P.grid;
        if (!tiles.empty()) {
            CHECK(grid >= 1, "grid %d\n", grid);
            if (grid >= P.nqueues && (int)tiles.size() >= P.nqueues)
                CHECK(grid % P.nqueues == 0, "grid %d not a multiple of %d\n", grid, P.nqueues);
        }
    }
    for (int s = 0; s < ns; ++s) {
        const int N = (int)(a->offsets[s + 1] - a->offsets[s]);
        const int nlev = levels_of_hmax(a->hmax ? a->hmax[s] : a->hmax_all);
        std::vector<uint8_t> seen((size_t)N, 0);
        for (int part = 0; part < 2; ++part) {
            const std::vector<TileRec>& tiles = part ? P.tiles_top : P.tiles;
            for (const TileRec& t : tiles) {
                if (t.spec != s) continue;
                CHECK(t.xoff == a->offsets[s] && t.n == N, "tile record of spectrum %d\n", s);
                CHECK(0 <= t.a && t.a < t.aend && t.aend <= N, "tile [%d, %d) of N=%d\n", t.a,
                      t.aend, N);
                if (!(0 <= t.a && t.a < t.aend && t.aend <= N)) continue;
                if (a->variant == HRMS_EQ1) {
                    CHECK(t.nlev == nlev, "eq1 tile levels\n");
                    CHECK(part == 0, "eq1 has no second launch\n");
                } else {
                    const int l = t.nlev - 1;
                    const int hi = N >> l;
                    const int lo = t.nlev < nlev ? (N >> t.nlev) : 0;
                    CHECK(lo <= t.a && t.aend <= hi, "tile [%d,%d) outside band %d of N=%d\n",
                          t.a, t.aend, l, N);
                    const bool top = shape.top > 0 && (1 << l) >= shape.top;
                    CHECK(top == (part == 1), "band %d in launch %d\n", l, part);
                    // tile length: the band's (cheap bands of the forms without
                    // LDS staging take several runs) or the split launch's
                    const int cap = part ? hrms1d_top_tile(a->variant)
                                         : hrms1d_band_tile(a->variant, shape, 1 << l,
                                                            1 << (nlev - 1));
                    CHECK(t.aend - t.a <= cap, "tile of %d outputs in band %d (at most %d)\n",
                          t.aend - t.a, l, cap);
                }
                if (a->variant == HRMS_EQ1)
                    CHECK(t.aend - t.a <= hrms1d_tile_outputs(a->variant, shape),
                          "eq1 tile of %d outputs\n", t.aend - t.a);
                for (int n = t.a; n < t.aend; ++n) seen[(size_t)n]++;
            }
        }
        // eq. (2)-(4): outputs n < floor(N / 1) all belong to the band of their top level
        for (int n = 0; n < N; ++n)
            CHECK(seen[(size_t)n] == 1, "spectrum %d output %d covered %d times\n", s, n,
                  (int)seen[(size_t)n]);
        // statistics segments
        int64_t pos = 0;
        for (int g = P.seg_first[s]; g < P.seg_first[s + 1]; ++g) {
            CHECK(P.segs[g].spec == s && P.segs[g].start == pos && P.segs[g].len > 0,
                  "segment %d\n", g);
            pos += P.segs[g].len;
        }
        CHECK(pos == N, "segments cover %lld of %d\n", (long long)pos, N);
        // plane layout
        for (int l = 0; l < kMaxLevels; ++l) {
            const int64_t o = P.spec[s].hoff[l];
            if (l >= nlev) {
                CHECK(o == -1, "absent level has an offset\n");
                continue;
            }
            if (s + 1 < ns || l + 1 < nlev) {
                const int64_t next = l + 1 < nlev ? P.spec[s].hoff[l + 1] : P.spec[s + 1].hoff[0];
                CHECK(next - o == (a->variant == HRMS_EQ1 ? N : (N >> l)), "plane size\n");
            }
        }
    }
    // no-alloc scratch sections
    const ScratchLayout L = scratch_layout(P);
    const size_t sec[] = {L.counters, L.consts, L.partial, L.spec, L.qbeg,
                          L.qbeg_top, L.tiles, L.tiles_top, L.segs, L.seg_first};
    for (size_t k = 0; k < sizeof(sec) / sizeof(sec[0]); ++k) {
        CHECK(sec[k] % 256 == 0, "section %zu misaligned\n", k);
        if (k) CHECK(sec[k] >= sec[k - 1], "sections out of order\n");
        CHECK(sec[k] <= L.total, "section past the end\n");
    }
    CHECK(L.tiles_top - L.tiles >= P.tiles.size() * sizeof(TileRec), "tile section too small\n");
    CHECK(L.total - L.seg_first >= P.seg_first.size() * sizeof(int32_t), "last section\n");
}

static void check_validation()
{
    int64_t off[] = {0, 100, 250};
    uint8_t hm[] = {8, 32};
    hrms_run1d_args a{};
    a.n_spectra = 2;
    a.variant = HRMS_MAX;
    a.dtype = HRMS_F32;
    a.hmax_all = 32;
    a.out_mask = 7;
    a.offsets = off;
    a.hmax = hm;
    CHECK(hrms_layout_1d(&a, nullptr, nullptr) == HRMS_OK, "valid batch\n");
    CHECK(hrms_layout_1d(nullptr, nullptr, nullptr) == HRMS_E_INVAL, "NULL args\n");
    hrms_run1d_args b = a;
    b.offsets = nullptr;
    CHECK(hrms_layout_1d(&b, nullptr, nullptr) == HRMS_E_INVAL, "NULL offsets\n");
    int64_t bad[] = {0, 100, 100};
    b = a;
    b.offsets = bad;
    CHECK(hrms_layout_1d(&b, nullptr, nullptr) == HRMS_E_INVAL, "empty spectrum\n");
    uint8_t badh[] = {8, 12};
    b = a;
    b.hmax = badh;
    CHECK(hrms_layout_1d(&b, nullptr, nullptr) == HRMS_E_INVAL, "Hmax 12\n");
    b = a;
    b.variant = HRMS_GREEDY_FDOT;
    CHECK(hrms_layout_1d(&b, nullptr, nullptr) == HRMS_E_UNSUPPORTED, "fdot Greedy in 1D\n");
    b = a;
    b.out_mask = HRMS_OUT_CAND | HRMS_OUT_PEAKS | HRMS_OUT_MAXSNR;
    CHECK(hrms_layout_1d(&b, nullptr, nullptr) == HRMS_E_INVAL, "exclusive lists\n");
    hrms_run2d_args p{};
    p.nf = 1000;
    p.zmax = 3;
    p.hmax = 16;
    p.variant = HRMS_GREEDY_FDOT;
    p.ld = 1000;
    p.out_mask = 7;
    int64_t po[HRMS_MAX_LEVELS];
    int64_t tot = 0;
    CHECK(hrms_layout_2d(&p, po, &tot) == HRMS_OK && po[1] == 7000 && po[5] == -1, "2D layout\n");
    p.zmax = -1;
    CHECK(hrms_layout_2d(&p, po, &tot) == HRMS_E_INVAL, "negative zmax\n");
    CHECK(hrms_run_1d(nullptr, &a, nullptr) == HRMS_E_INVAL, "NULL handle\n");
    CHECK(std::strlen(hrms_last_error(nullptr)) > 0, "last error text\n");
}

int main()
{
    hrms_ctx c;
    c.cu_count = 256;
    c.arch = "gfx950";
    check_validation();
    std::mt19937_64 rng(1812);
    const Shape1D shapes[] = {{512, 8, 0, 0},    {256, 8, 0, 0},      {256, 16, 0, 0},
                              {512, 8, 0, 32},   {256, 8, 0, 16},     {1024, 8, 16384, 0},
                              {512, 8, 8192, 0}, {1024, 16, 16384, 0}};
    long plans = 0;
    for (int trial = 0; trial < 120; ++trial) {
        const int ns = 1 + (int)(rng() % 9);
        std::vector<int64_t> off(ns + 1, 0);
        std::vector<uint8_t> hm(ns);
        for (int s = 0; s < ns; ++s) {
            const int kind = (int)(rng() % 4);
            int64_t len = kind == 0 ? 1 + (int64_t)(rng() % 40)
                          : kind == 1 ? 1 + (int64_t)(rng() % 5000)
                          : kind == 2 ? 1 + (int64_t)(rng() % 300000)
                                      : (int64_t(1) << (10 + rng() % 11)) + (int64_t)(rng() % 3);
            off[s + 1] = off[s] + len;
            hm[s] = (uint8_t)(1u << (rng() % 6));
        }
        for (int variant = 0; variant <= 4; ++variant) {
            for (int dtype = 0; dtype <= 2; dtype += 1 + (int)(trial % 2)) {
                for (const Shape1D& sh : shapes) {
                    if (!hrms1d_shape_supported(variant, sh)) continue;
                    if (variant == 4 && dtype) continue;
                    hrms_run1d_args a{};
                    a.n_spectra = ns;
                    a.variant = variant;
                    a.dtype = dtype;
                    a.hmax_all = 32;
                    a.out_mask = variant == 4 ? 1u : 7u;
                    a.offsets = off.data();
                    a.hmax = (trial % 3) ? hm.data() : nullptr;
                    CHECK(hrms_layout_1d(&a, nullptr, nullptr) == HRMS_OK, "layout of trial %d\n",
                          trial);
                    check_plan(&c, &a, sh);
                    ++plans;
                }
                if (variant == 4) break;
            }
        }
    }
    std::printf("%ld plans checked, %d failures\n", plans, fails);
    return fails ? 1 : 0;
}
