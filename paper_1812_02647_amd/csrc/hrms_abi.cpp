// hrms_abi.cpp -- host runtime behind the C ABI declared in include/hrms.h.
//
// Validation and layout are plain host code (usable with no device present).
// The runtime turns a batch into a plan -- per-spectrum descriptors, a
// cost-sorted tile list for the persistent harmonic-sum launch, statistics
// segments and a constants table -- caches it by batch signature, and enqueues
// statistics -> constants -> harmonic sum on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/hrms.h"
#include "hrms_internal.h"
#include "hrms_plan.h"

using namespace hrms;

namespace {

static_assert(kMaxLevels == HRMS_MAX_LEVELS, "level count of the ABI and the kernels differ");

constexpr int kStatsSeg = 1 << 16;   // bins per statistics segment
constexpr int kPlanCache = 4;

thread_local std::string g_last_error;

// Injected failures (environment HRMS_FAULT_INJECT, a comma-separated list read
// by hrms_create) for testing callers' error paths: "alloc" makes every device
// allocation of the library fail (HRMS_E_NOMEM, before anything is enqueued),
// "launch" the harmonic-sum launch of every call (HRMS_E_HIP, after the
// statistics and constants launches were enqueued). The handle stays usable
// and destroyable; hrms_run_1d_noalloc allocates nothing, so "alloc" leaves
// it working.
constexpr unsigned kFaultAlloc = 1u, kFaultLaunch = 2u;

unsigned parse_faults(const char* s)
{
    unsigned f = 0;
    if (!s) return 0;
    const std::string v(s);
    size_t pos = 0;
    while (pos <= v.size()) {
        const size_t end = std::min(v.find(',', pos), v.size());
        const std::string tok = v.substr(pos, end - pos);
        if (tok == "alloc") f |= kFaultAlloc;
        if (tok == "launch") f |= kFaultLaunch;
        pos = end + 1;
    }
    return f;
}

struct DeviceBuf {
    void* p = nullptr;
    size_t bytes = 0;
    ~DeviceBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t ensure(size_t n)
    {
        if (n <= bytes && p) return hipSuccess;
        release();
        if (n == 0) n = 16;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        bytes = n;
        return hipSuccess;
    }
};

// Calls on one handle that reuse a plan share its device scratch (queue
// counters, statistics partials, constants). A plan therefore remembers the
// stream of its last use and an event recorded after that work; a later call
// on another stream waits for the event first, and a plan is freed only once
// its event has completed.
struct UseOrder {
    hipEvent_t done = nullptr;
    hipStream_t last = nullptr;
    bool used = false;
    ~UseOrder()
    {
        if (done) {
            if (used) (void)hipEventSynchronize(done);
            (void)hipEventDestroy(done);
        }
    }
    // Orders the coming work on `s` after the previous use.
    hipError_t before(hipStream_t s)
    {
        if (!done) {
            hipError_t e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
            if (e != hipSuccess) {
                done = nullptr;
                return e;
            }
        }
        if (used && s != last) return hipStreamWaitEvent(s, done, 0);
        return hipSuccess;
    }
    // Marks the work just enqueued on `s` as the plan's latest use.
    hipError_t after(hipStream_t s)
    {
        hipError_t e = hipEventRecord(done, s);
        if (e != hipSuccess) return e;
        last = s;
        used = true;
        return hipSuccess;
    }
};

// Records a plan's use on every exit of a launch sequence, including an exit
// after a failed launch that follows launches already enqueued.
struct UseGuard {
    UseOrder& o;
    hipStream_t s;
    bool armed = true;
    UseGuard(UseOrder& o_, hipStream_t s_) : o(o_), s(s_) {}
    hipError_t finish()
    {
        armed = false;
        return o.after(s);
    }
    ~UseGuard()
    {
        if (armed) (void)o.after(s);
    }
};

struct Plan1D {
    // signature
    std::vector<int64_t> offsets;
    std::vector<uint8_t> nlev;
    int variant = 0, dtype = 0;
    Shape1D shape{};
    // host mirrors (kept alive for the asynchronous uploads)
    std::vector<SpecDesc> spec;
    std::vector<TileRec> tiles, tiles_top;   // main launch, top-band launch
    std::vector<int32_t> qbeg, qbeg_top;
    std::vector<Seg> segs;
    std::vector<int32_t> seg_first;
    int grid = 0, grid_top = 0;
    int nqueues = 1;
    uint64_t serial = 0;   // process-unique, names the tables in the no-alloc scratch
    // device
    DeviceBuf d_spec, d_tiles, d_qbeg, d_tiles_top, d_qbeg_top, d_segs, d_seg_first, d_partial,
        d_consts, d_counter;
    bool uploaded = false;
    // instantiated launch sequence for the most recent argument pointers
    hipGraphExec_t gexec = nullptr;
    std::vector<const void*> gkey;
    UseOrder order;   // declared last: destroyed first, after waiting for the last use
    ~Plan1D()
    {
        if (order.used) (void)hipEventSynchronize(order.done);
        if (gexec) (void)hipGraphExecDestroy(gexec);
    }
};

// A 2D plane: its rows as statistics "spectra", combined into one (mu, sigma).
struct Plan2D {
    int nf = 0, zmax = 0, nlev = 0;
    int64_t ld = 0;
    std::vector<SpecDesc> rows;
    std::vector<Seg> segs;
    std::vector<int32_t> seg_first;   // {0, nsegs}
    std::vector<SpecDesc> plane;      // one descriptor: n = rows * nf
    DeviceBuf d_rows, d_segs, d_seg_first, d_plane, d_partial, d_consts;
    UseOrder order;
};

// Precision form of a batch: statistics segments and fl32(1 / mu) per spectrum.
struct PlanQ {
    std::vector<int64_t> offsets;
    std::vector<SpecDesc> spec;
    std::vector<Seg> segs;
    std::vector<int32_t> seg_first;
    DeviceBuf d_spec, d_segs, d_seg_first, d_partial, d_inv;
    UseOrder order;
};

// Tuned launch shape of a class of 1D batches.
struct TuneKey {
    int variant, dtype, hmax, lenlog;
    bool operator<(const TuneKey& o) const
    {
        if (variant != o.variant) return variant < o.variant;
        if (dtype != o.dtype) return dtype < o.dtype;
        if (hmax != o.hmax) return hmax < o.hmax;
        return lenlog < o.lenlog;
    }
};

}  // namespace

struct hrms_ctx {
    int device = 0;
    int cu_count = 0;
    std::string arch;
    std::string err;
    std::string tune_path;
    std::map<TuneKey, Shape1D> tune;
    hipStream_t capture = nullptr;   // private stream for graph capture
    bool graphs = true;
    bool log = false;                // HRMS_LOG: one line per plan, capture and error on stderr
    unsigned fault = 0;              // HRMS_FAULT_INJECT: kFaultAlloc | kFaultLaunch
    std::vector<std::unique_ptr<Plan1D>> plans;   // most recent last
    // host-only plans of hrms_run_1d_noalloc (their tables live in the
    // device's static scratch), most recent last
    std::vector<std::unique_ptr<Plan1D>> na_plans;
    void* scratch = nullptr;             // this device's copy of the no-alloc scratch
    hipError_t scratch_status = hipSuccess;
    std::unique_ptr<Plan2D> plan2d;
    std::unique_ptr<PlanQ> planq;
};

namespace {

void hlog(const hrms_ctx* c, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void hlog(const hrms_ctx* c, const char* fmt, ...)
{
    if (!c || !c->log) return;
    std::va_list ap;
    va_start(ap, fmt);
    std::fprintf(stderr, "[hrms] ");
    std::vfprintf(stderr, fmt, ap);
    std::fprintf(stderr, "\n");
    va_end(ap);
}

int fail(hrms_ctx* c, int status, const std::string& msg)
{
    if (c) {
        c->err = msg;
        hlog(c, "error %d: %s", status, msg.c_str());
    } else {
        g_last_error = msg;
    }
    return status;
}

// An injected allocation failure, checked before a call allocates.
int alloc_fault(hrms_ctx* c)
{
    if (!(c->fault & kFaultAlloc)) return HRMS_OK;
    return fail(c, HRMS_E_NOMEM, "injected allocation failure (HRMS_FAULT_INJECT=alloc)");
}

int hip_fail(hrms_ctx* c, hipError_t e, const char* what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(c, e == hipErrorOutOfMemory ? HRMS_E_NOMEM : HRMS_E_HIP, m);
}

int levels_of_hmax(int h)
{
    if (h < 1 || h > HRMS_MAX_HMAX || (h & (h - 1))) return -1;
    int l = 0;
    while ((1 << l) < h) ++l;
    return l + 1;
}

int dtype_bytes(int dt) { return dt == HRMS_F32 ? 4 : 2; }

// ---------------------------------------------------------------------------
// Validation (host only)
// ---------------------------------------------------------------------------

int validate_1d(hrms_ctx* c, const hrms_run1d_args* a, bool device_ptrs)
{
    if (!a) return fail(c, HRMS_E_INVAL, "args is NULL");
    if (a->n_spectra < 1) return fail(c, HRMS_E_INVAL, "n_spectra must be >= 1");
    if (a->variant == HRMS_GREEDY_FDOT)
        return fail(c, HRMS_E_UNSUPPORTED, "HRMS_GREEDY_FDOT drifts along fdot: 2D planes only");
    if (a->variant < HRMS_EQ1 || a->variant > HRMS_OPT)
        return fail(c, HRMS_E_INVAL, "variant must be HRMS_EQ1..HRMS_OPT");
    if (a->dtype < HRMS_F32 || a->dtype > HRMS_BF16)
        return fail(c, HRMS_E_INVAL, "dtype must be HRMS_F32, HRMS_F16 or HRMS_BF16");
    if (a->out_mask & ~31u) return fail(c, HRMS_E_INVAL, "out_mask has unknown bits");
    if ((a->out_mask & HRMS_OUT_PEAKS) && (a->out_mask & HRMS_OUT_CAND))
        return fail(c, HRMS_E_INVAL, "HRMS_OUT_PEAKS and HRMS_OUT_CAND are exclusive");
    if ((a->out_mask & HRMS_OUT_PEAKS) && !(a->out_mask & HRMS_OUT_MAXSNR))
        return fail(c, HRMS_E_INVAL, "HRMS_OUT_PEAKS needs HRMS_OUT_MAXSNR");
    if (a->variant == HRMS_OPT && (a->out_mask & ~HRMS_OUT_H))
        return fail(c, HRMS_E_UNSUPPORTED,
                    "HRMS_OPT produces h only: its null distribution has no closed form, so "
                    "there is no SNR, best-H or candidate output");
    if (a->stats_mode != HRMS_STATS_COMPUTE && a->stats_mode != HRMS_STATS_PROVIDED)
        return fail(c, HRMS_E_INVAL, "stats_mode must be COMPUTE or PROVIDED");
    const bool listing = (a->out_mask & (HRMS_OUT_CAND | HRMS_OUT_PEAKS)) != 0;
    if (listing && !std::isfinite(a->cand_threshold))
        return fail(c, HRMS_E_INVAL, "cand_threshold must be finite");
    if (!a->offsets) return fail(c, HRMS_E_INVAL, "offsets is NULL");
    if (a->offsets[0] != 0) return fail(c, HRMS_E_INVAL, "offsets[0] must be 0");
    for (int s = 0; s < a->n_spectra; ++s) {
        const int64_t len = a->offsets[s + 1] - a->offsets[s];
        if (len < 1 || len > HRMS_MAX_BINS)
            return fail(c, HRMS_E_INVAL,
                        "spectrum " + std::to_string(s) + " has " + std::to_string(len) +
                            " bins (allowed 1.." + std::to_string(HRMS_MAX_BINS) + ")");
        const int hm = a->hmax ? a->hmax[s] : a->hmax_all;
        if (levels_of_hmax(hm) < 0)
            return fail(c, HRMS_E_INVAL, "Hmax of spectrum " + std::to_string(s) + " is " +
                                             std::to_string(hm) +
                                             " (must be a power of two <= 32)");
    }
    if (device_ptrs) {
        if (!a->x) return fail(c, HRMS_E_INVAL, "x is NULL");
        if (reinterpret_cast<uintptr_t>(a->x) % 16)
            return fail(c, HRMS_E_INVAL, "x must be 16-byte aligned");
        if (!a->stats) return fail(c, HRMS_E_INVAL, "stats is NULL");
        if ((a->out_mask & HRMS_OUT_H) && !a->h)
            return fail(c, HRMS_E_INVAL, "h is NULL but HRMS_OUT_H is set");
        if ((a->out_mask & HRMS_OUT_MAXSNR) && !a->max_snr)
            return fail(c, HRMS_E_INVAL, "max_snr is NULL but HRMS_OUT_MAXSNR is set");
        if ((a->out_mask & HRMS_OUT_BESTH) && !a->best_h)
            return fail(c, HRMS_E_INVAL, "best_h is NULL but HRMS_OUT_BESTH is set");
        if (listing && !a->cand_count)
            return fail(c, HRMS_E_INVAL, "cand_count is NULL but a candidate list is requested");
        if (listing && a->cand_capacity > 0 && !a->cand)
            return fail(c, HRMS_E_INVAL, "cand is NULL but cand_capacity > 0");
    }
    return HRMS_OK;
}

int validate_2d(hrms_ctx* c, const hrms_run2d_args* a, bool device_ptrs)
{
    if (!a) return fail(c, HRMS_E_INVAL, "args is NULL");
    if (a->nf < 1 || a->nf > HRMS_MAX_BINS)
        return fail(c, HRMS_E_INVAL, "nf must be in 1.." + std::to_string(HRMS_MAX_BINS));
    if (a->zmax < 0 || a->zmax > 4096) return fail(c, HRMS_E_INVAL, "zmax must be in 0..4096");
    if (a->ld < a->nf) return fail(c, HRMS_E_INVAL, "ld must be >= nf");
    if (levels_of_hmax(a->hmax) < 0)
        return fail(c, HRMS_E_INVAL, "hmax must be a power of two <= 32");
    if (a->variant == HRMS_OPT)
        return fail(c, HRMS_E_UNSUPPORTED, "HRMS_OPT is implemented for 1D spectra only");
    if (a->variant < HRMS_EQ1 || a->variant > HRMS_GREEDY_FDOT)
        return fail(c, HRMS_E_INVAL, "variant must be HRMS_EQ1..HRMS_GREEDY or HRMS_GREEDY_FDOT");
    if (a->dtype < HRMS_F32 || a->dtype > HRMS_BF16)
        return fail(c, HRMS_E_INVAL, "dtype must be HRMS_F32, HRMS_F16 or HRMS_BF16");
    if (a->out_mask & ~7u) return fail(c, HRMS_E_INVAL, "out_mask has unknown bits");
    if (a->stats_mode != HRMS_STATS_COMPUTE && a->stats_mode != HRMS_STATS_PROVIDED)
        return fail(c, HRMS_E_INVAL, "stats_mode must be COMPUTE or PROVIDED");
    if (a->reserved != 0) return fail(c, HRMS_E_INVAL, "reserved must be 0");
    if ((2 * (int64_t)a->zmax + 1) * (int64_t)a->nf > 0x7fffffffLL)
        return fail(c, HRMS_E_INVAL, "(2 zmax + 1) * nf must be below 2^31");
    if (device_ptrs) {
        if (!a->x) return fail(c, HRMS_E_INVAL, "x is NULL");
        if (reinterpret_cast<uintptr_t>(a->x) % dtype_bytes(a->dtype))
            return fail(c, HRMS_E_INVAL, "x must be aligned to its element size");
        if (!a->stats) return fail(c, HRMS_E_INVAL, "stats is NULL");
        if ((a->out_mask & HRMS_OUT_H) && !a->h)
            return fail(c, HRMS_E_INVAL, "h is NULL but HRMS_OUT_H is set");
        if ((a->out_mask & HRMS_OUT_MAXSNR) && !a->max_snr)
            return fail(c, HRMS_E_INVAL, "max_snr is NULL but HRMS_OUT_MAXSNR is set");
        if ((a->out_mask & HRMS_OUT_BESTH) && !a->best_h)
            return fail(c, HRMS_E_INVAL, "best_h is NULL but HRMS_OUT_BESTH is set");
    }
    return HRMS_OK;
}

// ---------------------------------------------------------------------------
// Layout
// ---------------------------------------------------------------------------

int64_t plane_len_1d(int variant, int64_t n, int l) { return variant == HRMS_EQ1 ? n : (n >> l); }

int64_t layout_1d_into(const hrms_run1d_args* a, int64_t* plane_offsets)
{
    int64_t off = 0;
    for (int s = 0; s < a->n_spectra; ++s) {
        const int64_t n = a->offsets[s + 1] - a->offsets[s];
        const int nl = levels_of_hmax(a->hmax ? a->hmax[s] : a->hmax_all);
        for (int l = 0; l < HRMS_MAX_LEVELS; ++l) {
            int64_t o = -1;
            if (l < nl) {
                o = off;
                off += plane_len_1d(a->variant, n, l);
            }
            if (plane_offsets) plane_offsets[(int64_t)s * HRMS_MAX_LEVELS + l] = o;
        }
    }
    return off;
}

int64_t layout_2d_into(const hrms_run2d_args* a, int64_t* plane_offsets)
{
    const int nl = levels_of_hmax(a->hmax);
    const int64_t rows = 2 * (int64_t)a->zmax + 1;
    int64_t off = 0;
    for (int l = 0; l < HRMS_MAX_LEVELS; ++l) {
        int64_t o = -1;
        if (l < nl) {
            o = off;
            off += rows * plane_len_1d(a->variant, a->nf, l);
        }
        if (plane_offsets) plane_offsets[l] = o;
    }
    return off;
}

// ---------------------------------------------------------------------------
// Plans
// ---------------------------------------------------------------------------

// Half of one XCD's 4 MB L2.
constexpr int64_t kL2HalfBytes = 2 << 20;

// Outputs in flight per CU past which the gathered and window forms lose:
// an XCD works through whole spectra, and once the input lines that its tiles
// in flight read no longer fit its L2, more resident workgroups only add
// re-reads through the fabric. Measured on 2^21-bin FP32 spectra at
// Hmax = 32 (Greedy 21.7 -> 14.7 ms, Max 23.0 -> 22.0, freq-bin in the
// gathered form 23.2 -> 15.3 at 4096 outputs; at Hmax = 16 freq-bin is faster
// with 8192, 11.0 -> 10.7); 2-byte bins halve the lines, so twice the
// outputs. htop is the plan's largest top level. 0: no limit.
int inflight_outputs_per_cu(int variant, int dtype, int htop)
{
    int f32 = 0;
    if (variant == HRMS_MAX) f32 = 6144;
    else if (variant == HRMS_FREQBIN) f32 = htop >= 32 ? 4096 : 8192;
    else if (variant == HRMS_GREEDY) f32 = 4096;
    return dtype == HRMS_F32 ? f32 : 2 * f32;
}

Shape1D default_shape(int variant, int dtype)
{
    // measured on the 1000 x 2^21, Hmax = 32 batch
    if (variant == HRMS_EQ1) return Shape1D{512, 8, 0, 0};
    if (variant == HRMS_MAX)   // FP32: the top band in a window-form launch of its own
        return dtype == HRMS_F32 ? Shape1D{256, 8, 0, 32} : Shape1D{256, 8, 0, 0};
    if (variant == HRMS_GREEDY)   // 2-byte bins halve the lines: more outputs per workgroup pay
        return dtype == HRMS_F32 ? Shape1D{256, 8, 0, 0} : Shape1D{512, 8, 0, 0};
    if (variant == HRMS_OPT) return kOptShape;
    return Shape1D{512, 8, 0, 0};
}

template <typename T>
hipError_t upload(DeviceBuf& b, const std::vector<T>& v, hipStream_t s)
{
    hipError_t e = b.ensure(v.size() * sizeof(T));
    if (e != hipSuccess || v.empty()) return e;
    return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

// Host part of a 1D plan: descriptors, tile queues, statistics segments and
// grid sizes. Touches no device memory.
int plan_host_1d(hrms_ctx* c, const hrms_run1d_args* a, const Shape1D& shape, Plan1D* P)
{
    const int ns = a->n_spectra;
    P->offsets.assign(a->offsets, a->offsets + ns + 1);
    P->nlev.resize(ns);
    for (int s = 0; s < ns; ++s)
        P->nlev[s] = (uint8_t)levels_of_hmax(a->hmax ? a->hmax[s] : a->hmax_all);
    P->variant = a->variant;
    P->dtype = a->dtype;
    P->shape = shape;

    std::vector<int64_t> poff((size_t)ns * HRMS_MAX_LEVELS);
    layout_1d_into(a, poff.data());
    P->spec.resize(ns);
    for (int s = 0; s < ns; ++s) {
        SpecDesc& d = P->spec[s];
        d.xoff = a->offsets[s];
        d.ooff = a->offsets[s];
        for (int l = 0; l < kMaxLevels; ++l) d.hoff[l] = poff[(size_t)s * HRMS_MAX_LEVELS + l];
        d.n = (int32_t)(a->offsets[s + 1] - a->offsets[s]);
        d.nlev = P->nlev[s];
    }

    // Tiles. Spectra are spread over one queue per XCD, balancing their total
    // cost; a queue lists its spectra one after the other (so the bins of a
    // spectrum stay in that XCD's L2 while its tiles run), each spectrum's
    // tiles most expensive first. For eq. (2)-(4) tiles are cut inside bands
    // and a tile's cost is the positions it stages plus the terms it adds;
    // with shape.top set, the bands whose top level is at least shape.top go
    // to a second launch (hrms1d_top_shape). Tile lists depend only
    // on (length, levels, alignment) and are shared by the spectra that agree
    // on them.
    const bool eq1 = a->variant == HRMS_EQ1;
    const int T = hrms1d_tile_outputs(a->variant, shape);
    const Shape1D tshape = hrms1d_top_shape(a->variant);
    const int Ttop = hrms1d_top_tile(a->variant);
    const int vec = 16 / dtype_bytes(a->dtype);
    const int nq = (c->cu_count >= kMaxQueues && c->cu_count % kMaxQueues == 0) ? kMaxQueues : 1;
    struct Geo {
        int n, nlev, xmod;
        bool operator<(const Geo& o) const
        {
            return n != o.n ? n < o.n : nlev != o.nlev ? nlev < o.nlev : xmod < o.xmod;
        }
    };
    struct TileSched {
        int32_t a, aend, nlev;
        bool top;
        int64_t cost;
    };
    std::map<Geo, std::vector<TileSched>> sched;
    // [part][spectrum]: tiles (cost, record); part 0 = main launch, 1 = top bands
    std::vector<std::vector<std::pair<int64_t, TileRec>>> per_spec[2];
    per_spec[0].resize(ns);
    per_spec[1].resize(ns);
    std::vector<std::pair<int64_t, int>> spec_cost[2];
    spec_cost[0].resize(ns);
    spec_cost[1].resize(ns);
    for (int s = 0; s < ns; ++s) {
        const int n = P->spec[s].n;
        const Geo g{n, (int)P->nlev[s], (int)(a->offsets[s] % vec)};
        auto it = sched.find(g);
        if (it == sched.end()) {
            std::vector<TileSched> ts;
            if (eq1) {
                // from the end of the spectrum down: 21.3 -> 19.6 ms against
                // increasing order on 1000 x 2^21 FP32 spectra at Hmax = 32
                // (the ragged last tile, cheaper, still goes last)
                for (int t0 = n > 0 ? (n - 1) / T * T : -1; t0 >= 0; t0 -= T) {
                    const int te = std::min(t0 + T, n);
                    ts.push_back(TileSched{t0, te, g.nlev, false,
                                           (int64_t)(te - t0) * ((1 << (g.nlev - 1)) + 1)});
                }
            } else {
                const int win = a->variant == HRMS_FREQBIN ? 0 : 1;
                for (int l = 0; l < g.nlev; ++l) {
                    const int hi = n >> l;
                    const int lo = l + 1 < g.nlev ? (n >> (l + 1)) : 0;
                    const int ht = 1 << l;
                    const bool top = shape.top > 0 && ht >= shape.top;
                    const Shape1D& sh = top ? tshape : shape;
                    const int tt = top ? Ttop : hrms1d_band_tile(a->variant, shape, ht, 1 << (g.nlev - 1));
                    const int64_t terms = a->variant == HRMS_MAX || a->variant == HRMS_OPT
                                              ? (int64_t)ht * (ht + 1) / 2
                                              : ht;
                    for (int t0 = lo; t0 < hi; t0 += tt) {
                        const int te = std::min(t0 + tt, hi);
                        int64_t staged = 0;
                        if (sh.chunk > 0) {   // LDS form: positions staged
                            SpanWalk w;
                            w.begin(t0, te, ht, win, vec, sh.chunk, g.xmod);
                            int cp, ce, cep;
                            while (w.next(cp, ce, cep)) staged += ce - cp;
                        }
                        ts.push_back(TileSched{t0, te, l + 1, top, staged + (te - t0) * terms});
                    }
                }
            }
            it = sched.emplace(g, std::move(ts)).first;
        }
        int64_t tot[2] = {0, 0};
        for (const TileSched& x : it->second) {
            TileRec tr;
            tr.xoff = a->offsets[s];
            tr.n = n;
            tr.a = x.a;
            tr.aend = x.aend;
            tr.spec = s;
            tr.nlev = x.nlev;
            tr.pad = 0;
            per_spec[x.top][s].push_back({x.cost, tr});
            tot[x.top] += x.cost;
        }
        for (int part = 0; part < 2; ++part) {
            if (a->variant == HRMS_GREEDY && a->dtype == HRMS_F32) {
                // FP32 Greedy: tiles in the order of where their top harmonic
                // reads (a * Ht), deepest band first on ties, so that tiles of
                // different bands that read the same lines run together
                // (measured 24.3 -> 22.6 ms on the 1D batch; the other
                // variants, and Greedy on 2-byte bins, were as fast or faster
                // in cost order)
                std::stable_sort(per_spec[part][s].begin(), per_spec[part][s].end(),
                                 [](const std::pair<int64_t, TileRec>& x,
                                    const std::pair<int64_t, TileRec>& y) {
                                     const int64_t gx = (int64_t)x.second.a << (x.second.nlev - 1);
                                     const int64_t gy = (int64_t)y.second.a << (y.second.nlev - 1);
                                     if (gx != gy) return gx < gy;
                                     return x.second.nlev > y.second.nlev;
                                 });
            } else {
                std::stable_sort(per_spec[part][s].begin(), per_spec[part][s].end(),
                                 [](const std::pair<int64_t, TileRec>& x,
                                    const std::pair<int64_t, TileRec>& y) {
                                     return x.first > y.first;
                                 });
            }
            spec_cost[part][s] = {tot[part], s};
        }
    }
    for (int part = 0; part < 2; ++part) {
        std::stable_sort(spec_cost[part].begin(), spec_cost[part].end(),
                         [](const std::pair<int64_t, int>& x, const std::pair<int64_t, int>& y) {
                             return x.first > y.first;
                         });
        std::vector<std::vector<int>> qspec(nq);
        std::vector<int64_t> qload(nq, 0);
        for (const auto& sc : spec_cost[part]) {
            int best = 0;
            for (int q = 1; q < nq; ++q)
                if (qload[q] < qload[best]) best = q;
            qspec[best].push_back(sc.second);
            qload[best] += sc.first;
        }
        std::vector<TileRec>& tiles = part ? P->tiles_top : P->tiles;
        std::vector<int32_t>& qbeg = part ? P->qbeg_top : P->qbeg;
        tiles.clear();
        qbeg.assign(nq + 1, 0);
        for (int q = 0; q < nq; ++q) {
            qbeg[q] = (int32_t)tiles.size();
            for (int sp : qspec[q])
                for (const auto& ct : per_spec[part][sp]) tiles.push_back(ct.second);
        }
        qbeg[nq] = (int32_t)tiles.size();
    }
    P->nqueues = nq;

    // statistics segments
    P->segs.clear();
    P->seg_first.assign(ns + 1, 0);
    for (int s = 0; s < ns; ++s) {
        P->seg_first[s] = (int32_t)P->segs.size();
        const int64_t n = P->spec[s].n;
        for (int64_t b = 0; b < n; b += kStatsSeg)
            P->segs.push_back(Seg{s, (int32_t)b, (int32_t)std::min<int64_t>(kStatsSeg, n - b), 0});
    }
    P->seg_first[ns] = (int32_t)P->segs.size();

    // one resident wave of workgroups per launch, the same number per queue;
    // on spectra that an XCD's L2 cannot hold, no more outputs in flight per
    // CU than inflight_outputs_per_cu allows
    int64_t big_bins = 0, all_bins = 0;
    const int elem_bytes = a->dtype == HRMS_F32 ? 4 : 2;
    for (const SpecDesc& sd : P->spec) {
        all_bins += sd.n;
        if ((int64_t)sd.n * elem_bytes >= kL2HalfBytes) big_bins += sd.n;
    }
    const bool l2_bound = 2 * big_bins >= all_bins;
    // largest top level of the main launch's bands
    int htop = 1;
    for (int s = 0; s < ns; ++s) htop = std::max(htop, 1 << (P->nlev[s] - 1));
    if (shape.top > 0) htop = std::min(htop, shape.top / 2);
    for (int part = 0; part < 2; ++part) {
        const std::vector<TileRec>& tiles = part ? P->tiles_top : P->tiles;
        int& grid_out = part ? P->grid_top : P->grid;
        grid_out = 0;
        if (tiles.empty()) continue;
        hipError_t oe = hipSuccess;
        int per_cu =
            hrms1d_max_blocks_per_cu(a->variant, a->dtype, part ? hrms1d_top_shape(a->variant) : shape, &oe);
        if (per_cu <= 0)
            return hip_fail(c, oe != hipSuccess ? oe : hipErrorInvalidConfiguration,
                            "occupancy query of the 1D kernel");
        int lim = inflight_outputs_per_cu(a->variant, a->dtype, htop);
        if (const char* f = std::getenv("HRMS_INFLIGHT_OUTPUTS")) lim = std::atoi(f);   // tuning
        if (part == 0 && l2_bound && lim > 0)
            per_cu = std::min(per_cu, std::max(1, lim / hrms1d_tile_outputs(a->variant, shape)));
        int64_t grid = std::min<int64_t>((int64_t)c->cu_count * per_cu, (int64_t)tiles.size());
        if (grid >= nq) grid -= grid % nq;
        grid_out = (int)std::max<int64_t>(grid, 1);
    }

    return HRMS_OK;
}

// Device copies of a plan in buffers the plan owns (allocated on first use).
int upload_plan_1d(hrms_ctx* c, Plan1D* P, hipStream_t stream)
{
    const int ns = (int)P->spec.size();
    hipError_t e;
    if (int f = alloc_fault(c)) return f;
    if ((e = upload(P->d_spec, P->spec, stream)) != hipSuccess) return hip_fail(c, e, "upload spec");
    if ((e = upload(P->d_tiles, P->tiles, stream)) != hipSuccess)
        return hip_fail(c, e, "upload tiles");
    if ((e = upload(P->d_qbeg, P->qbeg, stream)) != hipSuccess) return hip_fail(c, e, "upload qbeg");
    if (!P->tiles_top.empty()) {
        if ((e = upload(P->d_tiles_top, P->tiles_top, stream)) != hipSuccess)
            return hip_fail(c, e, "upload tiles");
        if ((e = upload(P->d_qbeg_top, P->qbeg_top, stream)) != hipSuccess)
            return hip_fail(c, e, "upload qbeg");
    }
    if ((e = upload(P->d_segs, P->segs, stream)) != hipSuccess) return hip_fail(c, e, "upload segs");
    if ((e = upload(P->d_seg_first, P->seg_first, stream)) != hipSuccess)
        return hip_fail(c, e, "upload seg_first");
    if ((e = P->d_partial.ensure(P->segs.size() * 2 * sizeof(double))) != hipSuccess)
        return hip_fail(c, e, "alloc partials");
    if ((e = P->d_consts.ensure((size_t)ns * kMaxLevels * sizeof(LevelConst))) != hipSuccess)
        return hip_fail(c, e, "alloc consts");
    if ((e = P->d_counter.ensure(sizeof(unsigned int) * kCounterSlots)) != hipSuccess)
        return hip_fail(c, e, "alloc counters");
    P->uploaded = true;
    return HRMS_OK;
}

void build_segments(const std::vector<SpecDesc>& spec, std::vector<Seg>& segs,
                    std::vector<int32_t>& seg_first)
{
    segs.clear();
    seg_first.assign(spec.size() + 1, 0);
    for (size_t s = 0; s < spec.size(); ++s) {
        seg_first[s] = (int32_t)segs.size();
        for (int64_t b = 0; b < spec[s].n; b += kStatsSeg)
            segs.push_back(
                Seg{(int32_t)s, (int32_t)b, (int32_t)std::min<int64_t>(kStatsSeg, spec[s].n - b), 0});
    }
    seg_first[spec.size()] = (int32_t)segs.size();
}

int get_plan_2d(hrms_ctx* c, const hrms_run2d_args* a, hipStream_t stream, Plan2D** out)
{
    const int nlev = levels_of_hmax(a->hmax);
    Plan2D* P = c->plan2d.get();
    if (P && P->nf == a->nf && P->zmax == a->zmax && P->ld == a->ld && P->nlev == nlev) {
        *out = P;
        return HRMS_OK;
    }
    if (int f = alloc_fault(c)) return f;
    // (the old plan waits for its last use before its buffers are freed)
    c->plan2d.reset(new (std::nothrow) Plan2D());
    P = c->plan2d.get();
    if (!P) return fail(c, HRMS_E_NOMEM, "host allocation failed");
    P->nf = a->nf;
    P->zmax = a->zmax;
    P->ld = a->ld;
    P->nlev = nlev;
    const int rows = 2 * a->zmax + 1;
    P->rows.resize(rows);
    for (int r = 0; r < rows; ++r) {
        SpecDesc& d = P->rows[r];
        d = SpecDesc{};
        d.xoff = (int64_t)r * a->ld;
        d.n = a->nf;
        d.nlev = nlev;
    }
    build_segments(P->rows, P->segs, P->seg_first);
    P->seg_first = {0, (int32_t)P->segs.size()};
    SpecDesc pl{};
    pl.n = (int32_t)((int64_t)rows * a->nf);
    pl.nlev = nlev;
    P->plane = {pl};
    hipError_t e;
    if ((e = upload(P->d_rows, P->rows, stream)) != hipSuccess) return hip_fail(c, e, "upload rows");
    if ((e = upload(P->d_segs, P->segs, stream)) != hipSuccess) return hip_fail(c, e, "upload segs");
    if ((e = upload(P->d_seg_first, P->seg_first, stream)) != hipSuccess)
        return hip_fail(c, e, "upload seg_first");
    if ((e = upload(P->d_plane, P->plane, stream)) != hipSuccess) return hip_fail(c, e, "upload plane");
    if ((e = P->d_partial.ensure(P->segs.size() * 2 * sizeof(double))) != hipSuccess)
        return hip_fail(c, e, "alloc partials");
    // two sets: Greedy with fdot drift keeps eq. (4)'s for its z = 0 row
    if ((e = P->d_consts.ensure(2 * kMaxLevels * sizeof(LevelConst))) != hipSuccess)
        return hip_fail(c, e, "alloc consts");
    *out = P;
    return HRMS_OK;
}

int get_plan_q(hrms_ctx* c, const hrms_quantize_args* a, hipStream_t stream, PlanQ** out)
{
    PlanQ* P = c->planq.get();
    const int ns = a->n_spectra;
    if (P && (int)P->offsets.size() == ns + 1 &&
        std::memcmp(P->offsets.data(), a->offsets, (ns + 1) * sizeof(int64_t)) == 0) {
        *out = P;
        return HRMS_OK;
    }
    if (int f = alloc_fault(c)) return f;
    c->planq.reset(new (std::nothrow) PlanQ());
    P = c->planq.get();
    if (!P) return fail(c, HRMS_E_NOMEM, "host allocation failed");
    P->offsets.assign(a->offsets, a->offsets + ns + 1);
    P->spec.resize(ns);
    for (int s = 0; s < ns; ++s) {
        SpecDesc& d = P->spec[s];
        d = SpecDesc{};
        d.xoff = a->offsets[s];
        d.ooff = a->offsets[s];
        d.n = (int32_t)(a->offsets[s + 1] - a->offsets[s]);
        d.nlev = 1;
    }
    build_segments(P->spec, P->segs, P->seg_first);
    hipError_t e;
    if ((e = upload(P->d_spec, P->spec, stream)) != hipSuccess) return hip_fail(c, e, "upload spec");
    if ((e = upload(P->d_segs, P->segs, stream)) != hipSuccess) return hip_fail(c, e, "upload segs");
    if ((e = upload(P->d_seg_first, P->seg_first, stream)) != hipSuccess)
        return hip_fail(c, e, "upload seg_first");
    if ((e = P->d_partial.ensure(P->segs.size() * 2 * sizeof(double))) != hipSuccess)
        return hip_fail(c, e, "alloc partials");
    if ((e = P->d_inv.ensure((size_t)ns * sizeof(float))) != hipSuccess)
        return hip_fail(c, e, "alloc inv_mu");
    *out = P;
    return HRMS_OK;
}

int validate_q(hrms_ctx* c, const hrms_quantize_args* a)
{
    if (!a) return fail(c, HRMS_E_INVAL, "args is NULL");
    if (a->n_spectra < 1) return fail(c, HRMS_E_INVAL, "n_spectra must be >= 1");
    if (a->dtype != HRMS_F16 && a->dtype != HRMS_BF16)
        return fail(c, HRMS_E_INVAL, "dtype must be HRMS_F16 or HRMS_BF16");
    if (a->stats_mode != HRMS_STATS_COMPUTE && a->stats_mode != HRMS_STATS_PROVIDED)
        return fail(c, HRMS_E_INVAL, "stats_mode must be COMPUTE or PROVIDED");
    if (a->reserved != 0) return fail(c, HRMS_E_INVAL, "reserved must be 0");
    if (!a->offsets) return fail(c, HRMS_E_INVAL, "offsets is NULL");
    if (a->offsets[0] != 0) return fail(c, HRMS_E_INVAL, "offsets[0] must be 0");
    for (int s = 0; s < a->n_spectra; ++s) {
        const int64_t len = a->offsets[s + 1] - a->offsets[s];
        if (len < 1 || len > 0x7fffffffLL)
            return fail(c, HRMS_E_INVAL, "spectrum " + std::to_string(s) + " has an invalid length");
    }
    if (!a->x || !a->y || !a->stats || !a->stats_out)
        return fail(c, HRMS_E_INVAL, "x, y, stats and stats_out must be non-NULL");
    return HRMS_OK;
}

// Provided statistics of the precision form are read back (after the work
// already queued on the stream) and must give a positive finite mean and a
// non-negative finite sigma: 1 / mu scales every bin.
int check_provided_q(hrms_ctx* c, const hrms_quantize_args* a, hipStream_t stream)
{
    std::vector<double> st((size_t)a->n_spectra * 2);
    hipError_t e = hipMemcpyAsync(st.data(), a->stats, st.size() * sizeof(double),
                                  hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(c, e, "reading the provided statistics");
    for (int s = 0; s < a->n_spectra; ++s) {
        const double mu = st[2 * (size_t)s], sd = st[2 * (size_t)s + 1];
        if (!(std::isfinite(mu) && mu > 0.0))
            return fail(c, HRMS_E_INVAL, "provided mean of spectrum " + std::to_string(s) +
                                             " is not a positive finite number");
        if (!(std::isfinite(sd) && sd >= 0.0))
            return fail(c, HRMS_E_INVAL, "provided sigma of spectrum " + std::to_string(s) +
                                             " is not a non-negative finite number");
    }
    return HRMS_OK;
}

bool same_signature(const Plan1D& P, const hrms_run1d_args* a, const Shape1D& shape)
{
    if (P.variant != a->variant || P.dtype != a->dtype) return false;
    if (P.shape.wg != shape.wg || P.shape.r != shape.r || P.shape.chunk != shape.chunk ||
        P.shape.top != shape.top)
        return false;
    if ((int)P.nlev.size() != a->n_spectra) return false;
    if (std::memcmp(P.offsets.data(), a->offsets, (a->n_spectra + 1) * sizeof(int64_t)) != 0)
        return false;
    for (int s = 0; s < a->n_spectra; ++s)
        if (P.nlev[s] != levels_of_hmax(a->hmax ? a->hmax[s] : a->hmax_all)) return false;
    return true;
}

void log_plan(const hrms_ctx* c, const Plan1D& P, const char* what)
{
    hlog(c, "%s: %zu spectra, variant %d, dtype %d, shape %dx%d chunk %d top %d; %zu + %zu tiles "
            "in %d queues, grids %d + %d",
         what, P.spec.size(), P.variant, P.dtype, P.shape.wg, P.shape.r, P.shape.chunk,
         P.shape.top, P.tiles.size(), P.tiles_top.size(), P.nqueues, P.grid, P.grid_top);
}

int get_plan_1d(hrms_ctx* c, const hrms_run1d_args* a, const Shape1D& shape, hipStream_t stream,
                Plan1D** out)
{
    for (size_t k = 0; k < c->plans.size(); ++k) {
        if (same_signature(*c->plans[k], a, shape)) {
            std::unique_ptr<Plan1D> p = std::move(c->plans[k]);
            c->plans.erase(c->plans.begin() + (long)k);
            c->plans.push_back(std::move(p));
            *out = c->plans.back().get();
            return HRMS_OK;
        }
    }
    std::unique_ptr<Plan1D> p(new (std::nothrow) Plan1D());
    if (!p) return fail(c, HRMS_E_NOMEM, "host allocation failed");
    int st = plan_host_1d(c, a, shape, p.get());
    if (st == HRMS_OK) st = upload_plan_1d(c, p.get(), stream);
    if (st != HRMS_OK) return st;
    log_plan(c, *p, "plan");
    if ((int)c->plans.size() >= kPlanCache) {
        // the evicted plan waits for its last use before its buffers are freed
        c->plans.erase(c->plans.begin());
    }
    c->plans.push_back(std::move(p));
    *out = c->plans.back().get();
    return HRMS_OK;
}


// ---------------------------------------------------------------------------
// Launch shapes: tuned table, environment override for debugging, default
// ---------------------------------------------------------------------------

TuneKey tune_key(const hrms_run1d_args* a)
{
    int hm = 0;
    const int64_t total = a->offsets[a->n_spectra];
    for (int s = 0; s < a->n_spectra; ++s) hm = std::max(hm, (int)(a->hmax ? a->hmax[s] : a->hmax_all));
    const int64_t mean = std::max<int64_t>(1, total / a->n_spectra);
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= mean) ++lg;
    return TuneKey{a->variant, a->dtype, hm, lg};
}

Shape1D shape_for(hrms_ctx* c, const hrms_run1d_args* a)
{
    if (const char* f = std::getenv("HRMS_FORCE_SHAPE")) {
        Shape1D fs{};
        if (std::sscanf(f, "%d:%d:%d:%d", &fs.wg, &fs.r, &fs.chunk, &fs.top) >= 3 &&
            hrms1d_shape_supported(a->variant, fs))
            return fs;
    }
    auto it = c->tune.find(tune_key(a));
    if (it != c->tune.end() && hrms1d_shape_supported(a->variant, it->second)) return it->second;
    return default_shape(a->variant, a->dtype);
}

const char* kTuneMagic = "hrms-tune-v2";

// Tune cache: a header line "hrms-tune-v2 <arch> <CUs>" then one line per
// batch class "variant dtype hmax lenlog wg r chunk top". A file whose header
// does not match this device, or a malformed line, is ignored.
void load_tune(hrms_ctx* c)
{
    FILE* f = std::fopen(c->tune_path.c_str(), "r");
    if (!f) return;
    char magic[32] = {0}, arch[64] = {0};
    int cus = 0;
    if (std::fscanf(f, "%31s %63s %d", magic, arch, &cus) == 3 && std::strcmp(magic, kTuneMagic) == 0 &&
        c->arch == arch && cus == c->cu_count) {
        std::map<TuneKey, Shape1D> t;
        TuneKey k{};
        Shape1D sh{};
        int got;
        while ((got = std::fscanf(f, "%d %d %d %d %d %d %d %d", &k.variant, &k.dtype, &k.hmax,
                                  &k.lenlog, &sh.wg, &sh.r, &sh.chunk, &sh.top)) == 8) {
            if (hrms1d_shape_supported(k.variant, sh)) t[k] = sh;
        }
        if (got == EOF) {
            c->tune.swap(t);
            hlog(c, "tune cache %s: %zu batch classes", c->tune_path.c_str(), c->tune.size());
        }
    }
    std::fclose(f);
}

void save_tune(hrms_ctx* c)
{
    const std::string tmp = c->tune_path + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "%s %s %d\n", kTuneMagic, c->arch.c_str(), c->cu_count);
    for (const auto& kv : c->tune)
        std::fprintf(f, "%d %d %d %d %d %d %d %d\n", kv.first.variant, kv.first.dtype, kv.first.hmax,
                     kv.first.lenlog, kv.second.wg, kv.second.r, kv.second.chunk, kv.second.top);
    const bool ok = std::fclose(f) == 0;
    if (ok) std::rename(tmp.c_str(), c->tune_path.c_str());
}

// Device addresses of a plan's tables and scratch: the plan's own buffers, or
// sections of the static scratch of the entry point that allocates nothing.
struct PlanDev {
    const SpecDesc* spec;
    const TileRec* tiles;
    const int32_t* qbeg;
    const TileRec* tiles_top;
    const int32_t* qbeg_top;
    const Seg* segs;
    const int32_t* seg_first;
    double* partial;
    LevelConst* consts;
    unsigned int* counters;
};

PlanDev plan_dev(const Plan1D& P)
{
    return PlanDev{(const SpecDesc*)P.d_spec.p,      (const TileRec*)P.d_tiles.p,
                   (const int32_t*)P.d_qbeg.p,       (const TileRec*)P.d_tiles_top.p,
                   (const int32_t*)P.d_qbeg_top.p,   (const Seg*)P.d_segs.p,
                   (const int32_t*)P.d_seg_first.p,  (double*)P.d_partial.p,
                   (LevelConst*)P.d_consts.p,        (unsigned int*)P.d_counter.p};
}

// Enqueues statistics (or not), constants and the harmonic sum.
hipError_t enqueue_1d(const hrms_run1d_args* a, const Plan1D* P, const PlanDev& D,
                      const Shape1D& shape, hipStream_t stream, bool fail_launch)
{
    hipError_t e;
    const bool compute = a->stats_mode == HRMS_STATS_COMPUTE;
    if (compute) {
        StatsParams sp{a->x, D.spec, D.segs, D.partial, (int32_t)P->segs.size()};
        if ((e = launch_stats_partial(a->dtype, sp, stream)) != hipSuccess) return e;
    }
    ConstsParams cp{};
    cp.spec = D.spec;
    cp.segs = D.segs;
    cp.seg_first = D.seg_first;
    cp.partial = D.partial;
    cp.stats = a->stats;
    cp.consts = D.consts;
    cp.user_consts = a->snr_consts;
    cp.counters = D.counters;
    cp.cand_count = (a->out_mask & (HRMS_OUT_CAND | HRMS_OUT_PEAKS)) ? a->cand_count : nullptr;
    cp.n_spec = a->n_spectra;
    cp.variant = a->variant;
    cp.compute_stats = compute ? 1 : 0;
    if ((e = launch_consts(cp, stream)) != hipSuccess) return e;
    if (a->out_mask != 0) {
        Run1DParams rp{};
        rp.x = a->x;
        rp.spec = D.spec;
        rp.tiles = D.tiles;
        rp.consts = D.consts;
        rp.h = a->h;
        rp.max_snr = a->max_snr;
        rp.best_h = a->best_h;
        rp.qbeg = D.qbeg;
        rp.counters = D.counters;
        rp.nqueues = P->nqueues;
        rp.out_mask = a->out_mask;
        rp.cand = reinterpret_cast<CandRec*>(a->cand);
        rp.cand_count = a->cand_count;
        rp.cand_cap = a->cand_capacity;
        rp.cand_thr = a->cand_threshold;
        if (fail_launch) return hipErrorLaunchFailure;   // injected (HRMS_FAULT_INJECT=launch)
        if (!P->tiles.empty() &&
            (e = launch_hrms1d(a->variant, a->dtype, shape, rp, P->grid, stream)) != hipSuccess)
            return e;
        if (!P->tiles_top.empty()) {
            rp.tiles = D.tiles_top;
            rp.qbeg = D.qbeg_top;
            rp.counters = D.counters + kMaxQueues;
            if ((e = launch_hrms1d(a->variant, a->dtype, hrms1d_top_shape(a->variant), rp, P->grid_top, stream)) !=
                hipSuccess)
                return e;
        }
    }
    if (a->out_mask & HRMS_OUT_PEAKS) {
        PeakParams pp{};
        pp.max_snr = a->max_snr;
        pp.best_h = (a->out_mask & HRMS_OUT_BESTH) ? a->best_h : nullptr;
        pp.spec = D.spec;
        pp.segs = D.segs;
        pp.cand = reinterpret_cast<CandRec*>(a->cand);
        pp.cand_count = a->cand_count;
        pp.cand_cap = a->cand_capacity;
        pp.thr = a->cand_threshold;
        pp.nsegs = (int32_t)P->segs.size();
        if ((e = launch_peaks(pp, stream)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// Runs one batch with the given shape; with graphs on, the launch sequence is
// captured once per plan and argument pointers and replayed afterwards.
int run_1d_with(hrms_ctx* h, const hrms_run1d_args* a, hipStream_t stream, const Shape1D& shape,
                bool graphs)
{
    Plan1D* P = nullptr;
    int st = get_plan_1d(h, a, shape, stream, &P);
    if (st != HRMS_OK) return st;
    hipError_t e;
    if ((e = P->order.before(stream)) != hipSuccess) return hip_fail(h, e, "stream ordering");
    if (!graphs) {
        UseGuard use(P->order, stream);
        if ((e = enqueue_1d(a, P, plan_dev(*P), shape, stream, (h->fault & kFaultLaunch) != 0)) != hipSuccess)
            return hip_fail(h, e, "launch");
        if ((e = use.finish()) != hipSuccess) return hip_fail(h, e, "hipEventRecord");
        return HRMS_OK;
    }
    uint32_t thr_bits;
    std::memcpy(&thr_bits, &a->cand_threshold, sizeof thr_bits);
    const std::vector<const void*> key = {a->x, a->stats, a->snr_consts, a->h, a->max_snr,
                                          a->best_h, (const void*)(intptr_t)a->stats_mode,
                                          (const void*)(intptr_t)a->out_mask, a->cand,
                                          a->cand_count, (const void*)(intptr_t)a->cand_capacity,
                                          (const void*)(intptr_t)thr_bits};
    if (!P->gexec || P->gkey != key) {
        if (!h->capture &&
            (e = hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(h, e, "hipStreamCreate");
        if (P->gexec) {
            (void)hipGraphExecDestroy(P->gexec);
            P->gexec = nullptr;
        }
        if ((e = hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(h, e, "hipStreamBeginCapture");
        const hipError_t le = enqueue_1d(a, P, plan_dev(*P), shape, h->capture, (h->fault & kFaultLaunch) != 0);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(h->capture, &g);
        if (le != hipSuccess || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(h, le != hipSuccess ? le : e, "graph capture");
        }
        e = hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            P->gexec = nullptr;
            return hip_fail(h, e, "hipGraphInstantiate");
        }
        P->gkey = key;
        hlog(h, "graph captured: variant %d, %zu spectra", P->variant, P->spec.size());
    }
    if ((e = hipGraphLaunch(P->gexec, stream)) != hipSuccess) return hip_fail(h, e, "hipGraphLaunch");
    if ((e = P->order.after(stream)) != hipSuccess) return hip_fail(h, e, "hipEventRecord");
    return HRMS_OK;
}

// ---------------------------------------------------------------------------
// The entry point that allocates nothing: host plans only; the plan's tables
// and the per-call scratch live in the device's static scratch array
// ---------------------------------------------------------------------------

std::atomic<uint64_t> g_plan_serial{0};

// Which plan's tables each device's static scratch holds (0: none). Every
// write of the tables goes through run_1d_noalloc, so a plan whose serial is
// recorded here needs no upload.
std::mutex g_owner_mu;
std::map<int, uint64_t> g_scratch_owner;

struct ScratchLayout {
    size_t counters, consts, partial, spec, qbeg, qbeg_top, tiles, tiles_top, segs, seg_first;
    size_t total;
};

ScratchLayout scratch_layout(const Plan1D& P)
{
    ScratchLayout L{};
    size_t off = 0;
    auto take = [&off](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    const size_t ns = P.spec.size();
    L.counters = take(sizeof(unsigned int) * kCounterSlots);
    L.consts = take(ns * kMaxLevels * sizeof(LevelConst));
    L.partial = take(P.segs.size() * 2 * sizeof(double));
    L.spec = take(ns * sizeof(SpecDesc));
    L.qbeg = take(P.qbeg.size() * sizeof(int32_t));
    L.qbeg_top = take(P.qbeg_top.size() * sizeof(int32_t));
    L.tiles = take(P.tiles.size() * sizeof(TileRec));
    L.tiles_top = take(P.tiles_top.size() * sizeof(TileRec));
    L.segs = take(P.segs.size() * sizeof(Seg));
    L.seg_first = take(P.seg_first.size() * sizeof(int32_t));
    L.total = off;
    return L;
}

PlanDev plan_dev_at(char* base, const ScratchLayout& L)
{
    return PlanDev{(const SpecDesc*)(base + L.spec),      (const TileRec*)(base + L.tiles),
                   (const int32_t*)(base + L.qbeg),       (const TileRec*)(base + L.tiles_top),
                   (const int32_t*)(base + L.qbeg_top),   (const Seg*)(base + L.segs),
                   (const int32_t*)(base + L.seg_first),  (double*)(base + L.partial),
                   (LevelConst*)(base + L.consts),        (unsigned int*)(base + L.counters)};
}

// Host plan of the no-alloc entry point (it never gets device buffers).
int get_plan_1d_host(hrms_ctx* c, const hrms_run1d_args* a, const Shape1D& shape, Plan1D** out)
{
    for (size_t k = 0; k < c->na_plans.size(); ++k) {
        if (same_signature(*c->na_plans[k], a, shape)) {
            std::unique_ptr<Plan1D> p = std::move(c->na_plans[k]);
            c->na_plans.erase(c->na_plans.begin() + (long)k);
            c->na_plans.push_back(std::move(p));
            *out = c->na_plans.back().get();
            return HRMS_OK;
        }
    }
    std::unique_ptr<Plan1D> p(new (std::nothrow) Plan1D());
    if (!p) return fail(c, HRMS_E_NOMEM, "host allocation failed");
    const int st = plan_host_1d(c, a, shape, p.get());
    if (st != HRMS_OK) return st;
    p->serial = ++g_plan_serial;
    log_plan(c, *p, "no-alloc plan");
    if ((int)c->na_plans.size() >= kPlanCache) {
        // the evicted plan's host tables may still be the source of a queued
        // copy: the device finishes its work before they are freed
        (void)hipDeviceSynchronize();
        c->na_plans.erase(c->na_plans.begin());
    }
    c->na_plans.push_back(std::move(p));
    *out = c->na_plans.back().get();
    return HRMS_OK;
}

template <typename T>
hipError_t copy_section(char* base, size_t off, const std::vector<T>& v, hipStream_t s)
{
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(base + off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

int run_1d_noalloc(hrms_ctx* h, const hrms_run1d_args* a, hipStream_t stream)
{
    if (h->scratch_status != hipSuccess || !h->scratch)
        return hip_fail(h, h->scratch_status != hipSuccess ? h->scratch_status : hipErrorInvalidSymbol,
                        "device address of the no-alloc scratch");
    const Shape1D shape = shape_for(h, a);
    Plan1D* P = nullptr;
    int st = get_plan_1d_host(h, a, shape, &P);
    if (st != HRMS_OK) return st;
    const ScratchLayout L = scratch_layout(*P);
    if (L.total > kNoallocScratchBytes)
        return fail(h, HRMS_E_INVAL,
                    "the batch needs " + std::to_string(L.total) +
                        " bytes of device scratch; hrms_run_1d_noalloc holds at most " +
                        std::to_string(kNoallocScratchBytes));
    char* base = static_cast<char*>(h->scratch);
    hipError_t e = hipSuccess;
    {
        std::lock_guard<std::mutex> lock(g_owner_mu);
        uint64_t& owner = g_scratch_owner[h->device];
        if (owner != P->serial) {
            owner = 0;
            if ((e = copy_section(base, L.spec, P->spec, stream)) == hipSuccess &&
                (e = copy_section(base, L.qbeg, P->qbeg, stream)) == hipSuccess &&
                (e = copy_section(base, L.qbeg_top, P->qbeg_top, stream)) == hipSuccess &&
                (e = copy_section(base, L.tiles, P->tiles, stream)) == hipSuccess &&
                (e = copy_section(base, L.tiles_top, P->tiles_top, stream)) == hipSuccess &&
                (e = copy_section(base, L.segs, P->segs, stream)) == hipSuccess &&
                (e = copy_section(base, L.seg_first, P->seg_first, stream)) == hipSuccess) {
                owner = P->serial;
                hlog(h, "no-alloc tables copied: %zu bytes of scratch", L.total);
            }
        }
    }
    if (e != hipSuccess) return hip_fail(h, e, "copying the plan into the static scratch");
    // the queue counters and the candidate count are cleared by the constants kernel
    if ((e = enqueue_1d(a, P, plan_dev_at(base, L), shape, stream, (h->fault & kFaultLaunch) != 0)) != hipSuccess)
        return hip_fail(h, e, "launch");
    return HRMS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char* hrms_strerror(int status)
{
    switch (status) {
    case HRMS_OK: return "success";
    case HRMS_E_INVAL: return "invalid argument";
    case HRMS_E_UNSUPPORTED: return "unsupported request";
    case HRMS_E_NODEVICE: return "no usable gfx950 device";
    case HRMS_E_NOMEM: return "out of memory";
    case HRMS_E_HIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

const char* hrms_last_error(hrms_handle h)
{
    if (!h) return g_last_error.c_str();
    return h->err.c_str();
}

int hrms_create(hrms_handle* out, int device_ordinal, const char* tune_cache_path)
{
    if (!out) return fail(nullptr, HRMS_E_INVAL, "out is NULL");
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0)
        return fail(nullptr, HRMS_E_NODEVICE, "no HIP device is visible");
    if (device_ordinal < 0 || device_ordinal >= count)
        return fail(nullptr, HRMS_E_NODEVICE, "device ordinal out of range");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device_ordinal);
    if (e != hipSuccess) return fail(nullptr, HRMS_E_NODEVICE, hipGetErrorString(e));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, HRMS_E_NODEVICE,
                    std::string("device is ") + prop.gcnArchName + ", not gfx950");
    hrms_ctx* c = new (std::nothrow) hrms_ctx();
    if (!c) return fail(nullptr, HRMS_E_NOMEM, "host allocation failed");
    c->device = device_ordinal;
    c->cu_count = prop.multiProcessorCount;
    c->arch = std::string(prop.gcnArchName).substr(0, std::string(prop.gcnArchName).find(':'));
    if (const char* g = std::getenv("HRMS_NO_GRAPH")) c->graphs = !(g[0] && g[0] != '0');
    if (const char* g = std::getenv("HRMS_LOG")) c->log = g[0] && g[0] != '0';
    c->fault = parse_faults(std::getenv("HRMS_FAULT_INJECT"));
    if (tune_cache_path) {
        c->tune_path = tune_cache_path;
        load_tune(c);
    }
    // device address of this device's copy of the no-alloc scratch (looked up
    // once per device, with the device current)
    c->scratch_status = noalloc_scratch(device_ordinal, &c->scratch);
    *out = c;
    return HRMS_OK;
}

int hrms_destroy(hrms_handle h)
{
    if (!h) return HRMS_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    h->plans.clear();
    h->na_plans.clear();
    h->plan2d.reset();
    h->planq.reset();
    if (h->capture) (void)hipStreamDestroy(h->capture);
    (void)hipSetDevice(cur);
    delete h;
    return HRMS_OK;
}

int hrms_layout_1d(const hrms_run1d_args* a, int64_t* plane_offsets, int64_t* h_total_floats)
{
    int st = validate_1d(nullptr, a, false);
    if (st != HRMS_OK) return st;
    const int64_t total = layout_1d_into(a, plane_offsets);
    if (h_total_floats) *h_total_floats = total;
    return HRMS_OK;
}

int hrms_layout_2d(const hrms_run2d_args* a, int64_t* plane_offsets, int64_t* h_total_floats)
{
    int st = validate_2d(nullptr, a, false);
    if (st != HRMS_OK) return st;
    const int64_t total = layout_2d_into(a, plane_offsets);
    if (h_total_floats) *h_total_floats = total;
    return HRMS_OK;
}

int hrms_run_1d(hrms_handle h, const hrms_run1d_args* a, void* hip_stream)
{
    if (!h) return fail(nullptr, HRMS_E_INVAL, "handle is NULL");
    h->err.clear();
    int st = validate_1d(h, a, true);
    if (st != HRMS_OK) return st;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
    return run_1d_with(h, a, static_cast<hipStream_t>(hip_stream), shape_for(h, a), h->graphs);
}

int hrms_run_1d_noalloc(hrms_handle h, const hrms_run1d_args* a, void* hip_stream)
{
    if (!h) return fail(nullptr, HRMS_E_INVAL, "handle is NULL");
    h->err.clear();
    int st = validate_1d(h, a, true);
    if (st != HRMS_OK) return st;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
    return run_1d_noalloc(h, a, static_cast<hipStream_t>(hip_stream));
}

int hrms_autotune_1d(hrms_handle h, const hrms_run1d_args* a, void* hip_stream, int reps,
                     int32_t* chosen)
{
    if (!h) return fail(nullptr, HRMS_E_INVAL, "handle is NULL");
    h->err.clear();
    int st = validate_1d(h, a, true);
    if (st != HRMS_OK) return st;
    if (reps < 1 || reps > 1000) return fail(h, HRMS_E_INVAL, "reps must be in 1..1000");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    Shape1D shapes[32];
    const int ns = std::min(32, hrms1d_shapes(a->variant, shapes, 32));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(h, e, "hipEventCreate");
    }
    float best_ms = 0.0f;
    int best = -1;
    for (int k = 0; k < ns && st == HRMS_OK; ++k) {
        st = run_1d_with(h, a, stream, shapes[k], false);   // plan build + warm-up
        if (st != HRMS_OK) break;
        if ((e = hipEventRecord(e0, stream)) != hipSuccess) {
            st = hip_fail(h, e, "hipEventRecord");
            break;
        }
        for (int r = 0; r < reps && st == HRMS_OK; ++r) st = run_1d_with(h, a, stream, shapes[k], false);
        if (st != HRMS_OK) break;
        float ms = 0.0f;
        if ((e = hipEventRecord(e1, stream)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
            (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
            st = hip_fail(h, e, "timing");
            break;
        }
        if (best < 0 || ms < best_ms) {
            best_ms = ms;
            best = k;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != HRMS_OK) return st;
    if (best < 0) return fail(h, HRMS_E_UNSUPPORTED, "no launch shape compiled for this variant");
    h->tune[tune_key(a)] = shapes[best];
    if (chosen) {
        chosen[0] = shapes[best].wg;
        chosen[1] = shapes[best].r;
        chosen[2] = shapes[best].chunk;
        chosen[3] = shapes[best].top;
    }
    if (!h->tune_path.empty()) save_tune(h);
    return HRMS_OK;
}

int hrms_plan_1d(hrms_handle h, const hrms_run1d_args* a, int32_t* info)
{
    if (!h) return fail(nullptr, HRMS_E_INVAL, "handle is NULL");
    h->err.clear();
    if (!info) return fail(h, HRMS_E_INVAL, "info is NULL");
    int st = validate_1d(h, a, true);
    if (st != HRMS_OK) return st;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
    const Shape1D shape = shape_for(h, a);
    Plan1D* P = nullptr;
    st = get_plan_1d_host(h, a, shape, &P);
    if (st != HRMS_OK) return st;
    info[0] = shape.wg;
    info[1] = shape.r;
    info[2] = shape.chunk;
    info[3] = shape.top;
    info[4] = (P->tiles.empty() ? 0 : 1) + (P->tiles_top.empty() ? 0 : 1);
    return HRMS_OK;
}

int hrms_run_2d(hrms_handle h, const hrms_run2d_args* a, void* hip_stream)
{
    if (!h) return fail(nullptr, HRMS_E_INVAL, "handle is NULL");
    h->err.clear();
    int st = validate_2d(h, a, true);
    if (st != HRMS_OK) return st;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    Plan2D* P = nullptr;
    st = get_plan_2d(h, a, stream, &P);
    if (st != HRMS_OK) return st;
    if ((e = P->order.before(stream)) != hipSuccess) return hip_fail(h, e, "stream ordering");
    UseGuard use(P->order, stream);
    const bool compute = a->stats_mode == HRMS_STATS_COMPUTE;
    if (compute) {
        StatsParams sp{a->x, (const SpecDesc*)P->d_rows.p, (const Seg*)P->d_segs.p,
                       (double*)P->d_partial.p, (int32_t)P->segs.size()};
        if ((e = launch_stats_partial(a->dtype, sp, stream)) != hipSuccess)
            return hip_fail(h, e, "statistics launch");
    }
    ConstsParams cp{};
    cp.spec = (const SpecDesc*)P->d_plane.p;
    cp.segs = (const Seg*)P->d_segs.p;
    cp.seg_first = (const int32_t*)P->d_seg_first.p;
    cp.partial = (const double*)P->d_partial.p;
    cp.stats = a->stats;
    cp.consts = (LevelConst*)P->d_consts.p;
    cp.user_consts = a->snr_consts;
    cp.counters = nullptr;
    cp.n_spec = 1;
    cp.variant = a->variant;
    cp.compute_stats = compute ? 1 : 0;
    if ((e = launch_consts(cp, stream)) != hipSuccess) return hip_fail(h, e, "constants launch");
    if (a->variant == HRMS_GREEDY_FDOT) {
        // the z = 0 row: eq. (4)'s constants, from the statistics just written
        cp.consts = (LevelConst*)P->d_consts.p + kMaxLevels;
        cp.user_consts = a->snr_consts ? a->snr_consts + 2 * HRMS_MAX_LEVELS : nullptr;
        cp.variant = HRMS_GREEDY;
        cp.compute_stats = 0;
        if ((e = launch_consts(cp, stream)) != hipSuccess)
            return hip_fail(h, e, "constants launch");
    }
    if (a->out_mask != 0) {
        Run2DParams rp{};
        rp.x = a->x;
        rp.ld = a->ld;
        rp.consts = (const LevelConst*)P->d_consts.p;
        rp.h = a->h;
        rp.max_snr = a->max_snr;
        rp.best_h = a->best_h;
        // the level planes depend on the variant (eq. (1) keeps nf outputs per
        // row), so they are laid out per call rather than cached in the plan
        layout_2d_into(a, rp.hoff);
        rp.nf = a->nf;
        rp.zmax = a->zmax;
        rp.nlev = P->nlev;
        rp.out_mask = a->out_mask;
        rp.zgroups = (2 * a->zmax + 1 + 3) / 4;
        if (h->fault & kFaultLaunch) e = hipErrorLaunchFailure;   // injected
        else e = launch_hrms2d(a->variant, a->dtype, rp, stream);
        if (e != hipSuccess)
            return hip_fail(h, e, "2D harmonic-sum launch");
    }
    if ((e = use.finish()) != hipSuccess) return hip_fail(h, e, "hipEventRecord");
    return HRMS_OK;
}

int hrms_quantize(hrms_handle h, const hrms_quantize_args* a, void* hip_stream)
{
    if (!h) return fail(nullptr, HRMS_E_INVAL, "handle is NULL");
    h->err.clear();
    int st = validate_q(h, a);
    if (st != HRMS_OK) return st;
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    if (a->stats_mode == HRMS_STATS_PROVIDED && (st = check_provided_q(h, a, stream)) != HRMS_OK)
        return st;
    PlanQ* P = nullptr;
    st = get_plan_q(h, a, stream, &P);
    if (st != HRMS_OK) return st;
    if ((e = P->order.before(stream)) != hipSuccess) return hip_fail(h, e, "stream ordering");
    UseGuard use(P->order, stream);
    const bool compute = a->stats_mode == HRMS_STATS_COMPUTE;
    if (compute) {
        StatsParams sp{a->x, (const SpecDesc*)P->d_spec.p, (const Seg*)P->d_segs.p,
                       (double*)P->d_partial.p, (int32_t)P->segs.size()};
        if ((e = launch_stats_partial(HRMS_F32, sp, stream)) != hipSuccess)
            return hip_fail(h, e, "statistics launch");
    }
    QuantConstParams qc{};
    qc.spec = (const SpecDesc*)P->d_spec.p;
    qc.seg_first = (const int32_t*)P->d_seg_first.p;
    qc.partial = (const double*)P->d_partial.p;
    qc.stats = a->stats;
    qc.stats_out = a->stats_out;
    qc.inv_mu = (float*)P->d_inv.p;
    qc.n_spec = a->n_spectra;
    qc.compute_stats = compute ? 1 : 0;
    if ((e = launch_quant_consts(qc, stream)) != hipSuccess)
        return hip_fail(h, e, "normalisation constants launch");
    QuantParams qp{};
    qp.x = a->x;
    qp.spec = (const SpecDesc*)P->d_spec.p;
    qp.segs = (const Seg*)P->d_segs.p;
    qp.inv_mu = (const float*)P->d_inv.p;
    qp.y = a->y;
    qp.nsegs = (int32_t)P->segs.size();
    if (h->fault & kFaultLaunch) e = hipErrorLaunchFailure;   // injected
    else e = launch_quantize(a->dtype, qp, stream);
    if (e != hipSuccess)
        return hip_fail(h, e, "quantisation launch");
    if ((e = use.finish()) != hipSuccess) return hip_fail(h, e, "hipEventRecord");
    return HRMS_OK;
}

}  // extern "C"
