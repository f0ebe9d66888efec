// hrms_kernels.hip -- gfx950 kernels of the incoherent harmonic sum.
//
// Paper: K. Adamek and W. Armour, "A GPU implementation of the harmonic sum
// algorithm" (arXiv:1812.02647); eq. (1) in Sec. 1, eq. (2)-(4) in Sec. 2.
//
// Design (memory-bound; no matrix cores):
//   * eq. (2)-(4): a tile is a run of outputs of one band (outputs with the
//     same top level). Harmonic i of the tile reads a contiguous span of
//     positions; the tile streams the union of its spans through LDS in
//     chunks loaded with 16-byte coalesced loads, so the stride-i gather never
//     reaches HBM or L2 directly and a position read by several harmonics of
//     the tile is staged once. Running sums, best SNR and best level live in
//     LDS, one slot per output of the tile.
//   * Every output adds its harmonics in the order i = 1..H of the equations
//     (chunks in increasing position, harmonics in increasing i inside a
//     chunk, one thread per output); a level snapshot
//     (h = S * fl32(1/sqrt(H)), SNR, best level) is taken when i reaches a
//     power of two.
//   * eq. (1): every term of every level is one of Hmax bins
//     x[round(n k / Hmax)]; they are read straight from global memory with
//     coalesced buffer loads.
//   * LDS holds FP32 whatever the storage type; a 1-in-32 padding keeps
//     strided reads (stride i) nearly free of bank conflicts.
//   * The grids are persistent: workgroups pull tiles from per-XCD queues of
//     cost-sorted tiles through atomic counters (the paper's load-balancing
//     concern, Sec. 1).
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "hrms_internal.h"
#include "hrms_plan.h"

namespace hrms {
namespace {

constexpr int kEq1 = 0, kMax = 1, kFreqbin = 2, kGreedy = 3, kOpt = 4;
// 2D only: Greedy with fdot drift (eq. (4)'s step rule on the fdot row as well)
constexpr int kGreedyFZ = 5;
constexpr int kF32 = 0, kF16 = 1, kBF16 = 2;

template <int DT>
struct Elem {
    static constexpr int kBytes = DT == kF32 ? 4 : 2;
    static constexpr int kVec = 16 / kBytes;   // elements per 16-byte load
};

__device__ __forceinline__ float h2f(uint32_t bits16)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)bits16);
}

__device__ __forceinline__ float bf2f(uint32_t bits16) { return __uint_as_float(bits16 << 16); }

template <int DT>
__device__ __forceinline__ float load_scalar(const void* base, int64_t idx)
{
    if constexpr (DT == kF32) {
        return static_cast<const float*>(base)[idx];
    } else if constexpr (DT == kF16) {
        return h2f(static_cast<const uint16_t*>(base)[idx]);
    } else {
        return bf2f(static_cast<const uint16_t*>(base)[idx]);
    }
}

// LDS index of chunk-relative bin k: one pad word per 32 bins.
__device__ __forceinline__ int pidx(int k) { return k + (k >> 5); }

// Level index of harmonic i: the smallest l with i <= 2^l.
__device__ __forceinline__ int level_of(int i) { return 32 - __clz(i - 1); }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Read-only record through the constant address space: with a uniform index
// this is a scalar (SMEM) load through the scalar cache, which the compiler
// cannot otherwise prove safe while the kernel also stores to global memory.
template <typename T>
__device__ __forceinline__ T ldc(const T* ptr)
{
    static_assert(sizeof(T) % 4 == 0, "records are whole words");
    typedef const __attribute__((address_space(4))) uint32_t* cword;
    const cword w = (cword)(ptr);
    uint32_t buf[sizeof(T) / 4];
#pragma unroll
    for (unsigned k = 0; k < sizeof(T) / 4; ++k) buf[k] = w[k];
    T out;
    __builtin_memcpy(&out, buf, sizeof(T));
    return out;
}

// Chunk start for absolute alignment of the 16-byte loads.
template <int DT>
__device__ __forceinline__ int align_chunk(int64_t xoff, int p)
{
    constexpr int V = Elem<DT>::kVec;
    return p - (int)((xoff + p) & (V - 1));
}

// Register stage of one chunk: VPT 16-byte vectors per thread.
//
// Vector vi holds positions p0 + vi V .. + V - 1 of a spectrum whose first bin
// is x[xoff]; p0 is 16-byte aligned in the batch. Positions outside the
// spectrum are never read by a term, so a vector that lies wholly outside it
// is replaced by the spectrum's nearest vector: every load stays inside the
// batch. (A vector holding any element of the batch lies inside the batch's
// last 16-byte block at worst, which x's 16-byte alignment keeps mapped.)
template <int DT, int WG, int VPT>
struct Stage {
    uint4 v[VPT];
    __device__ __forceinline__ void load(const void* x, int64_t xoff, int n_bins, int p0, int nvec)
    {
        constexpr int V = Elem<DT>::kVec;
        constexpr int B = Elem<DT>::kBytes;
        // element offsets relative to the spectrum's first 16-byte boundary
        const int64_t first = xoff & ~(int64_t)(V - 1);
        const int last = (int)(((xoff + n_bins - 1) & ~(int64_t)(V - 1)) - first);
        const char* base = static_cast<const char*>(x) + first * B;
        const int rel0 = (int)(xoff - first) + p0;
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            const int vi = u * WG + (int)threadIdx.x;
            if (vi < nvec) {
                int e = rel0 + vi * V;
                e = e < 0 ? 0 : e > last ? last : e;
                v[u] = *reinterpret_cast<const uint4*>(base + e * B);
            }
        }
    }
    // Each pad word receives a copy of the bin that follows it, so that the
    // word after any bin's word holds the next bin.
    __device__ __forceinline__ void store(float* buf, int nvec) const
    {
        constexpr int V = Elem<DT>::kVec;
        constexpr int STEP = WG * V;   // chunk positions per vector slot u
        static_assert(STEP % 32 == 0, "a vector slot spans whole padding blocks");
        // pidx(k0 + u STEP + e) = pidx(k0) + u (STEP + STEP / 32) + e for e < V
        const int tid = (int)threadIdx.x;
        float* b = buf + pidx(tid * V);
        // a vector starting a 32-bin block (other than the chunk's first) also
        // fills the pad word just before it
        const bool lead = ((tid * V) & 31) == 0;
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            const int vi = u * WG + tid;
            if (vi < nvec) {
                float* d = b + u * (STEP + STEP / 32);
                const uint32_t w[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
                float f[V];
                if constexpr (DT == kF32) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) f[e] = __uint_as_float(w[e]);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        f[2 * e] = DT == kF16 ? h2f(w[e] & 0xffffu) : bf2f(w[e] & 0xffffu);
                        f[2 * e + 1] = DT == kF16 ? h2f(w[e] >> 16) : bf2f(w[e] >> 16);
                    }
                }
#pragma unroll
                for (int e = 0; e < V; ++e) d[e] = f[e];
                if (lead && vi > 0) d[-1] = f[0];
            }
        }
    }
};

// Claims the next tile of this workgroup (call from one thread): from the
// current queue while it lasts, then from the following queues in turn;
// -1 once every queue is drained.
__device__ __forceinline__ int claim_tile(const Run1DParams& p, int& q, int& visited)
{
    while (visited < p.nqueues) {
        const unsigned k = atomicAdd(&p.counters[q], 1u);
        const int len = p.qbeg[q + 1] - p.qbeg[q];
        if ((int)k < len) return p.qbeg[q] + (int)k;
        q = q + 1 == p.nqueues ? 0 : q + 1;
        ++visited;
    }
    return -1;
}

// Candidate records are gathered per workgroup in LDS and written out in one
// block after a barrier, so that the global counter sees one atomic per
// workgroup flush instead of one per wavefront.
constexpr int kCandLds = 512;

struct CandStage {
    CandRec rec[kCandLds];
    unsigned int n;      // records appended since the last flush (may pass kCandLds)
    unsigned int base;   // global place of the flushed block
};

// Appends a record for every active lane with `take` set: one LDS atomic per
// wavefront claims the places, the lanes write in lane order; a record that
// finds the LDS block full goes straight to the global list.
__device__ __forceinline__ void append_candidates(const Run1DParams& p, CandStage& cs, bool take,
                                                  int spec, int n, float snr, int hval)
{
    const uint64_t m = __ballot(take);
    if (m == 0) return;
    const int lane = (int)(threadIdx.x & 63);
    const int leader = __ffsll((unsigned long long)m) - 1;
    unsigned int base = 0;
    if (lane == leader) base = atomicAdd(&cs.n, (unsigned int)__popcll(m));
    base = (unsigned int)__shfl((int)base, leader, 64);
    if (take) {
        const unsigned int k = base + (unsigned int)__popcll(m & ((1ull << lane) - 1ull));
        const CandRec rec{spec, n, snr, hval};
        if (k < (unsigned int)kCandLds) {
            cs.rec[k] = rec;
        } else {
            const unsigned int g = atomicAdd(p.cand_count, 1u);
            if (g < p.cand_cap) p.cand[g] = rec;
        }
    }
}

// Writes the workgroup's staged records to the global list. Called by every
// thread right after a barrier that follows all appends; no append may start
// before the barrier that ends this call.
__device__ __forceinline__ void flush_candidates(const Run1DParams& p, CandStage& cs, int wg)
{
    const unsigned int nc = (unsigned int)uniform((int)cs.n);
    if (nc == 0) return;
    const unsigned int m = nc < (unsigned int)kCandLds ? nc : (unsigned int)kCandLds;
    if (threadIdx.x == 0) cs.base = atomicAdd(p.cand_count, m);
    __syncthreads();   // base visible; every thread has read cs.n
    if (threadIdx.x == 0) cs.n = 0u;
    const unsigned int base = cs.base;
    for (unsigned int k = threadIdx.x; k < m; k += (unsigned int)wg)
        if (base + k < p.cand_cap) p.cand[base + k] = cs.rec[k];
    __syncthreads();   // the block is read out before the next appends
}

// --------------------------------------------------------------------------
// eq. (2)-(4): outputs indexed by the fundamental.
//
// A tile is a run [a, aend) of at most T = WG * R outputs of one band (all of
// its outputs have the same top level Ht = 2^(nlev - 1)); thread t holds
// outputs a + r WG + t (r < R) in registers: running sum, best SNR, best
// level and Greedy's offset j. The tile walks the union of its harmonic spans
// in chunks of at most CB positions (hrms_plan.h): a position that several
// harmonics of the tile read is staged once, and a chunk serves the terms
// whose window ends inside it -- for each harmonic i, a run of outputs. The
// chunk's harmonics are visited in increasing i, chunks in increasing
// position, so every output adds its terms in the order i = 1..H of the
// equations; a level snapshot (h = S * fl32(1/sqrt(H)), SNR, best level) is
// taken when i is a power of two, and max-SNR / best-H are written at i = Ht.
//
// Chunks go global -> registers -> LDS through a double-buffered LDS chunk:
// while chunk k is computed, chunk k + 1 sits in LDS and chunk k + 2 is in
// flight to registers; one barrier per chunk. The grid is persistent: tiles
// come from per-XCD queues of cost-sorted tiles, claimed one tile ahead.
// --------------------------------------------------------------------------

// One chunk of a tile, as the kernel carries it.
struct ChunkDesc {
    TileRec t;
    int cp, ce, cep;   // chunk [cp, ce); cep: end of the previous chunk of the tile (0: first)
};

// Walks the chunks of the tiles claimed by the workgroup, in order. Tile c of
// the workgroup is named by ring[c & 1]: thread 0 claims tile c + 1 when the
// walk enters tile c. With one call of next per barrier phase, tile c was
// claimed at least one barrier before it is read, and its slot is rewritten
// (with tile c + 2) at least one barrier after every wave has read it.
template <int DT, int CB, int WIN>
struct ChunkCursor {
    TileRec t;
    SpanWalk w;
    int seq;
    bool live;

    __device__ __forceinline__ void open()
    {
        constexpr int V = Elem<DT>::kVec;
        w.begin(t.a, t.aend, 1 << (t.nlev - 1), WIN, V, CB, (int)(t.xoff & (V - 1)));
    }
    __device__ __forceinline__ void start(const Run1DParams& p, const int* ring)
    {
        seq = 0;
        const int id = uniform(ring[0]);
        live = id >= 0;
        if (live) {
            t = ldc(p.tiles + id);
            open();
        }
    }
    __device__ __forceinline__ bool next(const Run1DParams& p, int* ring, int& cq, int& visited,
                                         ChunkDesc& d)
    {
        if (!live) return false;
        if (!w.next(d.cp, d.ce, d.cep)) {
            ++seq;
            const int id = uniform(ring[seq & 1]);
            if (id < 0) {
                live = false;
                return false;
            }
            if (threadIdx.x == 0) ring[(seq + 1) & 1] = claim_tile(p, cq, visited);
            t = ldc(p.tiles + id);
            open();
            w.next(d.cp, d.ce, d.cep);
        }
        d.t = t;
        return true;
    }
};

// Term i of an output whose window starts at chunk position k (LDS index
// idx = pidx(k)). The word after a bin's LDS word always holds the next bin
// (pad words carry a copy of the bin after them), so a window of i <= 32 bins
// is words idx .. idx + i - 1 when it crosses no pad word (cross = 0), and
// words idx .. idx + i when it crosses one (cross = 1; the pad repeats a bin
// of the window). Greedy reads its offset j from st (bits 8..) and sets step when the
// right neighbour is taken (j then grows by one).
template <int VAR>
__device__ __forceinline__ float term_value(const float* buf, int k, int idx, int i, int cross,
                                            int st, bool& step)
{
    step = false;
    if constexpr (VAR == kFreqbin) {
        return buf[idx];
    } else if constexpr (VAR == kMax) {
        // running maximum with a strict >, the window's first bin first: only
        // that bin decides a NaN result, and repeated later bins leave the
        // value unchanged. The window is the L = i + cross words from idx; all
        // of them are read before the maximum is formed, in blocks of 8 whose
        // last one ends at word L - 1 (overlapping its predecessor rather than
        // leaving a ragged tail).
        const float* w = buf + idx;
        const int L = i + cross;
        if (L <= 8) {
            const float x0 = w[0];
            if (L == 1) return x0;
            if (L < 4) {
                const float a1 = w[1], a2 = w[L - 1];
                float tv = a1 > x0 ? a1 : x0;
                return a2 > tv ? a2 : tv;
            }
            float v[8];
#pragma unroll
            for (int u = 1; u < 4; ++u) v[u] = w[u];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[4 + u] = w[L - 4 + u];
            float tv = x0;
#pragma unroll
            for (int u = 1; u < 8; ++u) tv = v[u] > tv ? v[u] : tv;
            return tv;
        }
        // first round: blocks at words 0 and 8 (when before the last block)
        // and the last block; second round: blocks at 16 and 24
        float v[3][8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[0][u] = w[u];
        if (L > 16) {
#pragma unroll
            for (int u = 0; u < 8; ++u) v[1][u] = w[8 + u];
        }
        const float* wl = w + (L - 8);
#pragma unroll
        for (int u = 0; u < 8; ++u) v[2][u] = wl[u];
        float tv = v[0][0];
#pragma unroll
        for (int u = 1; u < 8; ++u) tv = v[0][u] > tv ? v[0][u] : tv;
        if (L > 16) {
#pragma unroll
            for (int u = 0; u < 8; ++u) tv = v[1][u] > tv ? v[1][u] : tv;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) tv = v[2][u] > tv ? v[2][u] : tv;
        if (L > 24) {
#pragma unroll
            for (int u = 0; u < 8; ++u) v[0][u] = w[16 + u];
            if (L > 32) {
#pragma unroll
                for (int u = 0; u < 8; ++u) v[1][u] = w[24 + u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) tv = v[0][u] > tv ? v[0][u] : tv;
            if (L > 32) {
#pragma unroll
                for (int u = 0; u < 8; ++u) tv = v[1][u] > tv ? v[1][u] : tv;
            }
        }
        return tv;
    } else {
        if (i == 1) return buf[idx];
        const int q = pidx(k + (st >> 8));
        const float x0 = buf[q];
        const float x1 = buf[q + 1];
        step = x1 > x0;
        return step ? x1 : x0;
    }
}

constexpr int kBufferFlags = 0x00020000;   // raw (untyped) 32-bit buffer, gfx9 word 3

// Raw buffer over [base, base + bytes): a store past the end is dropped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t out_rsrc(const void* base, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes,
                                             kBufferFlags);
}

// Output stores carry the non-temporal hint (cache policy NT): the sums and
// SNR planes are written once and never read back by the launch, so they
// should not displace the input lines that later tiles read again.
constexpr int kStreamStore = 2;

__device__ __forceinline__ void stream_store_b32(uint32_t v, __amdgpu_buffer_rsrc_t rs, int voff,
                                                 int soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(v, rs, voff, soff, kStreamStore);
}

__device__ __forceinline__ void stream_store_b8(uint8_t v, __amdgpu_buffer_rsrc_t rs, int voff,
                                                int soff)
{
    __builtin_amdgcn_raw_buffer_store_b8(v, rs, voff, soff, kStreamStore);
}

template <int VAR, int DT, int WG, int R, int CB, bool CAND>
__global__ __launch_bounds__(WG) void k_hrms1d_span(const Run1DParams p)
{
    constexpr int V = Elem<DT>::kVec;
    static_assert(CB % V == 0, "chunk must be a multiple of the vector");
    static_assert((WG & (WG - 1)) == 0 && WG >= 64, "WG must be a power of two");
    constexpr int NVEC = CB / V;
    constexpr int VPT = (NVEC + WG - 1) / WG;
    constexpr int BUF = VPT * WG * V;
    constexpr int LDSB = BUF + (BUF >> 5) + 1;
    constexpr int WIN = VAR == kFreqbin ? 0 : 1;
    constexpr int TSH = __builtin_ctz(WG);
    __shared__ float lds[2][LDSB];
    __shared__ int ring[2];
    __shared__ CandStage cands;

    const int tid = (int)threadIdx.x;
    const int lane = tid & 63;
    const int wbase = uniform(tid & ~63);   // first thread of this wave
    if (tid == 0) cands.n = 0u;
    const bool track = CAND || (p.out_mask & 6u) != 0;
    int cq = (int)(blockIdx.x % (unsigned)p.nqueues), visited = 0;
    if (tid == 0) {
        ring[0] = claim_tile(p, cq, visited);
        ring[1] = claim_tile(p, cq, visited);
    }
    __syncthreads();

    // Every call of g.next sits in a barrier phase of its own, so that a
    // ring slot is read by all waves before it is rewritten and rewritten
    // before it is read again.
    ChunkCursor<DT, CB, WIN> g;
    g.start(p, ring);
    Stage<DT, WG, VPT> stage;
    ChunkDesc d0, d1, d2;
    bool h0 = g.next(p, ring, cq, visited, d0);
    if (h0) {
        stage.load(p.x, d0.t.xoff, d0.t.n, d0.cp, (d0.ce - d0.cp + V - 1) / V);
        stage.store(lds[0], (d0.ce - d0.cp + V - 1) / V);
    }
    __syncthreads();
    bool h1 = h0 && g.next(p, ring, cq, visited, d1);
    if (h1) stage.load(p.x, d1.t.xoff, d1.t.n, d1.cp, (d1.ce - d1.cp + V - 1) / V);
    __syncthreads();   // chunk 0 is in LDS

    float acc[R], best[R];
    int st[R];   // best level (bits 0..7) | Greedy offset j (bits 8..)
#pragma unroll
    for (int r = 0; r < R; ++r) {
        acc[r] = 0.0f;
        best[r] = 0.0f;
        st[r] = 0;
    }
    // constants of the current spectrum, lane l holding level l
    float lm = 0.0f, lq = 0.0f, lrh = 0.0f;
    int lho_lo = 0, lho_hi = 0;
    int cur_spec = -1;

    for (int k = 0; h0; ++k) {
        // chunk k + 1 -> LDS (its buffer held chunk k - 1), chunk k + 2 -> registers
        if (h1) stage.store(lds[(k + 1) & 1], (d1.ce - d1.cp + V - 1) / V);
        const bool h2 = h1 && g.next(p, ring, cq, visited, d2);
        if (h2) stage.load(p.x, d2.t.xoff, d2.t.n, d2.cp, (d2.ce - d2.cp + V - 1) / V);

        // ---- chunk k ----
        const float* buf = lds[k & 1];
        const int a = d0.t.a;
        const int ht = 1 << (d0.t.nlev - 1);
        if (d0.cep == 0) {
            // first chunk of a tile: fresh outputs (Greedy starts from -0 so
            // that its first term passes unchanged, the others from +0)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                acc[r] = VAR == kGreedy ? -0.0f : 0.0f;
                st[r] = 0;
            }
            if (d0.t.spec != cur_spec) {
                cur_spec = d0.t.spec;
                if (lane < kMaxLevels) {
                    const LevelConst lc = p.consts[(int64_t)cur_spec * kMaxLevels + lane];
                    lm = lc.m;
                    lq = lc.q;
                    lrh = lc.rh;
                    const int64_t ho = p.spec[cur_spec].hoff[lane];
                    lho_lo = (int)(uint32_t)ho;
                    lho_hi = (int)(ho >> 32);
                }
            }
        }
        const int tn = d0.t.aend - a;   // outputs of the tile
        int nbv = 0, nev = 0;
        if (lane < ht) chunk_terms(lane + 1, WIN * lane, d0.cep, d0.ce, a, d0.t.aend, nbv, nev);
        uint32_t segs = (uint32_t)__ballot(lane < ht && nbv < nev);
        while (segs) {
            const int l = __builtin_ctz(segs);
            segs &= segs - 1;
            const int i = l + 1;
            // outputs [a + ub, a + ue) take term i from this chunk
            const int ub = __builtin_amdgcn_readlane(nbv, l) - a;
            const int ue = __builtin_amdgcn_readlane(nev, l) - a;
            // this wave's output blocks [r WG + wbase, + 64) that meet [ub, ue)
            const int lo = ub - wbase - 63, hi = ue - 1 - wbase;
            const int r_lo = lo <= 0 ? 0 : (lo + WG - 1) >> TSH;
            const int r_hi = hi < 0 ? -1 : (hi >> TSH) < R - 1 ? (hi >> TSH) : R - 1;
            if (r_lo > r_hi) continue;
            // every lane of every block inside the run: no per-lane checks
            const bool full = r_lo == 0 && r_hi == R - 1 && ub <= wbase &&
                              ue >= (R - 1) * WG + wbase + 64;
            // chunk position of term i of output a + r WG + tid: k0 + r i WG;
            // i WG is a multiple of 32, so its LDS index is pidx(k0) + r rstep
            const int k0 = (int)__umul24((unsigned)i, (unsigned)tid) + i * a - d0.cp;
            const int rstep = i * (WG + WG / 32);
            const int x0 = pidx(k0);
            // window crossing of a pad word; the same for every r (k0 mod 32 is)
            const int cross = ((k0 & 31) + i - 1) >> 5;
            const int span = ue - ub;
            const int u0 = tid - ub;   // output offset in the run, block 0
            const bool snap = (i & (i - 1)) == 0;
            if (!snap) {
                if (full) {
                    float tv[R];
                    bool stp[R];
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        tv[r] = term_value<VAR>(buf, k0 + r * i * WG, x0 + r * rstep, i, cross,
                                                st[r], stp[r]);
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        acc[r] = acc[r] + tv[r];
                        if (stp[r]) st[r] += 256;
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        if (r < r_lo || r > r_hi) continue;
                        if ((unsigned)(u0 + r * WG) < (unsigned)span) {
                            bool stp;
                            const float tv = term_value<VAR>(buf, k0 + r * i * WG, x0 + r * rstep,
                                                             i, cross, st[r], stp);
                            acc[r] = acc[r] + tv;
                            if (stp) st[r] += 256;
                        }
                    }
                }
                continue;
            }
            // snapshot harmonic (i = 2^li)
            const int li = __builtin_ctz((unsigned)i);
            const float rh = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lrh), li));
            const float m0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lm), li));
            const float q0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lq), li));
            const int64_t ho =
                (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(lho_hi, li) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane(lho_lo, li));
            const bool fin = i == ht;
            // the tile's outputs in each output array; block r at byte r WG size
            const __amdgpu_buffer_rsrc_t hrs = out_rsrc(p.h + ho + a, tn * 4);
            const __amdgpu_buffer_rsrc_t mrs = out_rsrc(p.max_snr + d0.t.xoff + a, tn * 4);
            const __amdgpu_buffer_rsrc_t brs = out_rsrc(p.best_h + d0.t.xoff + a, tn);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (r < r_lo || r > r_hi) continue;
                if (full || (unsigned)(u0 + r * WG) < (unsigned)span) {
                    bool stp;
                    const float tv = term_value<VAR>(buf, k0 + r * i * WG, x0 + r * rstep, i,
                                                     cross, st[r], stp);
                    if (stp) st[r] += 256;
                    acc[r] = acc[r] + tv;
                    const float hv = acc[r] * rh;
                    if (p.out_mask & 1u)
                        stream_store_b32(__float_as_uint(hv), hrs, tid * 4, r * WG * 4);
                    if (track) {
                        const float snr = (hv - m0) * q0;
                        if (li == 0 || snr > best[r]) {
                            best[r] = snr;
                            st[r] = (st[r] & ~255) | li;
                        }
                        if (fin) {
                            if (p.out_mask & 2u)
                                stream_store_b32(__float_as_uint(best[r]), mrs, tid * 4,
                                                 r * WG * 4);
                            if (p.out_mask & 4u)
                                stream_store_b8((uint8_t)(1u << (st[r] & 255)), brs, tid, r * WG);
                            if constexpr (CAND)
                                append_candidates(p, cands, best[r] >= p.cand_thr, d0.t.spec,
                                                  a + r * WG + tid, best[r], 1 << (st[r] & 255));
                        }
                    }
                }
            }
        }
        __syncthreads();   // chunk k done; chunk k + 1 visible
        if constexpr (CAND) flush_candidates(p, cands, WG);
        d0 = d1;
        h0 = h1;
        d1 = d2;
        h1 = h2;
    }
}

// --------------------------------------------------------------------------
// eq. (1): output n is the H-th harmonic; term i of level H reads bin
// round(n i / H). With Lh = Hmax, term i of level H is fraction k / Lh,
// k = i Lh / H, so every term of every level is one of the Lh bins
// v_k = x[round(n k / Lh)], k = 1..Lh, and v_k belongs to the levels
// H >= Lh / 2^tz(k). Bins v_k are read in increasing k, so each level still
// adds its terms in the order i = 1..H; each level keeps its own sum.
//
// Neighbouring outputs read neighbouring (often equal) bins -- the stride is
// k / Lh <= 1 -- so the loads of a wavefront are coalesced; they are issued
// straight from global memory as 32-bit-offset buffer loads, R outputs per
// thread in flight.
// --------------------------------------------------------------------------
template <int DT>
__device__ __forceinline__ float buffer_elem(__amdgpu_buffer_rsrc_t rs, int pos)
{
    if constexpr (DT == kF32) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, pos * 4, 0, 0));
    } else if constexpr (DT == kF16) {
        return h2f(__builtin_amdgcn_raw_buffer_load_b16(rs, pos * 2, 0, 0));
    } else {
        return bf2f(__builtin_amdgcn_raw_buffer_load_b16(rs, pos * 2, 0, 0));
    }
}


// Element at byte offset bo of a buffer resource.
template <int DT>
__device__ __forceinline__ float buffer_elem_at(__amdgpu_buffer_rsrc_t rs, int bo)
{
    if constexpr (DT == kF32) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, bo, 0, 0));
    } else if constexpr (DT == kF16) {
        return h2f(__builtin_amdgcn_raw_buffer_load_b16(rs, bo, 0, 0));
    } else {
        return bf2f(__builtin_amdgcn_raw_buffer_load_b16(rs, bo, 0, 0));
    }
}

// Terms of eq. (1) whose loads a thread issues together.
constexpr int kEq1Unroll = 4;

template <int DT, int WG, int R, int CB, bool CAND>
__global__ __launch_bounds__(WG) void k_hrms1d_eq1(const Run1DParams p)
{
    const int tid = (int)threadIdx.x;
    __shared__ int s_claim[2];
    __shared__ CandStage cands;
    int cq = (int)(blockIdx.x % (unsigned)p.nqueues), visited = 0;
    if (tid == 0) {
        s_claim[0] = claim_tile(p, cq, visited);
        cands.n = 0u;
    }
    __syncthreads();
    int t = uniform(s_claim[0]);
    for (int c = 0; t >= 0; ++c) {
        // claim the following tile now; it is read after this tile's barrier
        if (tid == 0) s_claim[(c + 1) & 1] = claim_tile(p, cq, visited);
        const TileRec ct = ldc(p.tiles + t);
        const int a = ct.a;
        const int N = ct.n;
        const int nl = ct.nlev;
        const int aend = ct.aend;
        const int sh = nl - 1;
        const int Lh = 1 << sh;
        const unsigned half = (unsigned)Lh >> 1;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(static_cast<const char*>(p.x) + ct.xoff * Elem<DT>::kBytes), (short)0,
            N * Elem<DT>::kBytes, kBufferFlags);

        // Output n = a + r WG + tid reads (n k + Lh/2) >> sh for k = 1..Lh:
        // t below holds n0 k + Lh/2 for n0 = a + tid, and output r adds
        // r WG k. A lane past the tile's end (at most R WG outputs further)
        // reads past the spectrum's end, which the resource returns as zero,
        // and its stores are discarded; n k + Lh/2 < 2^32 for every
        // n < HRMS_MAX_BINS + R WG.
        const unsigned n0 = (unsigned)(a + tid);
        // WG k is a multiple of Lh, so output r's bin of term k is the
        // bin of output 0 plus r S k exactly (S = WG / Lh): one shift per
        // term, one add per output
        const int S = WG >> sh;
        float acc[R][kMaxLevels];
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int l = 0; l < kMaxLevels; ++l) acc[r][l] = 0.0f;
        }
        unsigned tk0 = half;
        if (Lh >= kEq1Unroll) {
            // kEq1Unroll terms per step, all loads issued before the first
            // add, so that a wavefront keeps kEq1Unroll * R loads in flight
            for (int k = 1; k <= Lh; k += kEq1Unroll) {
                float v[kEq1Unroll][R];
#pragma unroll
                for (int u = 0; u < kEq1Unroll; ++u) {
                    tk0 += n0;
                    const int b0 = (int)(tk0 >> sh) * Elem<DT>::kBytes;
                    // the step between outputs in bytes, uniform, kept opaque
                    // to the loop optimiser (which would otherwise keep
                    // R kEq1Unroll running offsets in vector registers)
                    const int sb = __builtin_amdgcn_readfirstlane(S * (k + u) * Elem<DT>::kBytes);
#pragma unroll
                    for (int r = 0; r < R; ++r) v[u][r] = buffer_elem_at<DT>(rs, b0 + r * sb);
                }
#pragma unroll
                for (int u = 0; u < kEq1Unroll; ++u) {
                    // k = 1 mod kEq1Unroll, so tz(k + u) = tz(u + 1) but for the
                    // last u, where it is at least tz(kEq1Unroll)
                    constexpr int kTz = __builtin_ctz((unsigned)kEq1Unroll);
                    const int tz = u + 1 < kEq1Unroll
                                       ? __builtin_ctz((unsigned)(u + 1))
                                       : kTz + __builtin_ctz((unsigned)(k + u) >> kTz);
#pragma unroll
                    for (int m = 0; m < kMaxLevels; ++m) {
                        if (m <= tz) {
#pragma unroll
                            for (int r = 0; r < R; ++r) acc[r][m] = acc[r][m] + v[u][r];
                        }
                    }
                }
            }
        } else {
            for (int k = 1; k <= Lh; ++k) {
                tk0 += n0;
                const int b0 = (int)(tk0 >> sh) * Elem<DT>::kBytes;
                const int sb = S * k * Elem<DT>::kBytes;
                const int tz = __builtin_ctz((unsigned)k);
                float v[R];
#pragma unroll
                for (int r = 0; r < R; ++r) v[r] = buffer_elem_at<DT>(rs, b0 + r * sb);
#pragma unroll
                for (int m = 0; m < kMaxLevels; ++m) {
                    if (m <= tz) {
#pragma unroll
                        for (int r = 0; r < R; ++r) acc[r][m] = acc[r][m] + v[r];
                    }
                }
            }
        }

        float best[R];
        int bl[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            best[r] = 0.0f;
            bl[r] = 0;
        }
        // stores through resources spanning the tile's outputs: a lane past
        // the tile's end stores out of range, which the resource discards
        const int tn = aend - a;
        // acc[r][m] holds level l = sh - m (term k belongs to the levels
        // m <= tz(k)); levels are visited in increasing l, so the first of
        // equal SNRs is kept
#pragma unroll
        for (int m = kMaxLevels - 1; m >= 0; --m) {
            const int l = sh - m;
            if (l >= 0) {
                const LevelConst c = ldc(p.consts + (int64_t)ct.spec * kMaxLevels + l);
                const int64_t ho = ldc(p.spec[ct.spec].hoff + l);
                const __amdgpu_buffer_rsrc_t hrs = out_rsrc(p.h + ho + a, tn * 4);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const float hv = acc[r][m] * c.rh;
                    if (p.out_mask & 1u)
                        stream_store_b32(__float_as_uint(hv), hrs, tid * 4, r * WG * 4);
                    const float snr = (hv - c.m) * c.q;
                    if (l == 0 || snr > best[r]) {
                        best[r] = snr;
                        bl[r] = l;
                    }
                }
            }
        }
        const __amdgpu_buffer_rsrc_t mrs = out_rsrc(p.max_snr + ct.xoff + a, tn * 4);
        const __amdgpu_buffer_rsrc_t brs = out_rsrc(p.best_h + ct.xoff + a, tn);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (p.out_mask & 2u)
                stream_store_b32(__float_as_uint(best[r]), mrs, tid * 4, r * WG * 4);
            if (p.out_mask & 4u)
                stream_store_b8((uint8_t)(1u << bl[r]), brs, tid, r * WG);
            if constexpr (CAND)
                append_candidates(p, cands, (int)n0 + r * WG < aend && best[r] >= p.cand_thr,
                                  ct.spec, (int)n0 + r * WG, best[r], 1 << bl[r]);
        }
        __syncthreads();
        if constexpr (CAND) flush_candidates(p, cands, WG);
        t = uniform(s_claim[(c + 1) & 1]);
    }
}

// --------------------------------------------------------------------------
// eq. (1), LDS-staged. The tile's outputs are taken WG at a time (a run); for
// a run starting at output ns, term k of its outputs reads the contiguous
// positions round(n k / Lh), n = ns .. ns + WG - 1, at most S k + 1 of them
// (S = WG / Lh). Each run's Lh spans are copied into LDS with aligned 16-byte
// loads, one vector per lane, and the terms are then read from LDS; the next
// run's vectors are loaded into registers while the current one is summed.
// The terms, the order of the adds and the outputs are those of the direct
// form above; only where a bin is read from differs.
//
// LDS layout of one run: span k (k = 1..Lh) holds S k / V + 1 vectors of V
// elements starting at the V-aligned position below its first bin, at float
// offset o_k = S k (k - 1) / 2 + V (k - 1). Spans k and Lh + 1 - k together
// hold S (Lh + 1) / V + 2 vectors, so a flat vector index maps to its span
// with one division.
// --------------------------------------------------------------------------
// Workgroup barrier for data exchanged through LDS only: waits for this
// wave's LDS operations (lgkmcnt 0; vmcnt and expcnt left at their maximum in
// the gfx9 encoding) and not for its global loads and stores, so loads issued
// ahead of the barrier stay in flight. The empty asm statements keep the
// compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

template <int DT, int WG>
struct Eq1Lds {
    static constexpr int V = Elem<DT>::kVec;
    static constexpr int kHmax = 1 << (kMaxLevels - 1);
    // floats of one run's staging at Lh = kHmax (the largest over Lh)
    static constexpr int kFloats = WG * (kHmax + 1) / 2 + V * kHmax;
    // vectors per thread per run at most
    static constexpr int kQ = (WG * (kHmax + 1) / (2 * V) + kHmax + WG - 1) / WG;
    static_assert(WG % kHmax == 0, "S = WG / Lh must be a whole multiple of V");
    static_assert((WG / kHmax) % V == 0, "S = WG / Lh must be a whole multiple of V");
};

// (at most 128 VGPRs: two 512-thread workgroups per CU, as the LDS allows)
template <int DT, int WG, int R, bool CAND>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(4)))
void k_hrms1d_eq1_lds(const Run1DParams p)
{
    using L = Eq1Lds<DT, WG>;
    constexpr int V = L::V;
    constexpr int B = Elem<DT>::kBytes;
    const int tid = (int)threadIdx.x;
    __shared__ int s_claim[2];
    __shared__ CandStage cands;
    // (plus one vector of pad that lanes without a vector write to)
    __shared__ __attribute__((aligned(16))) float stage[2][L::kFloats + 8];
    int cq = (int)(blockIdx.x % (unsigned)p.nqueues), visited = 0;
    if (tid == 0) {
        s_claim[0] = claim_tile(p, cq, visited);
        cands.n = 0u;
    }
    __syncthreads();
    int t = uniform(s_claim[0]);
    for (int c = 0; t >= 0; ++c) {
        if (tid == 0) s_claim[(c + 1) & 1] = claim_tile(p, cq, visited);
        const TileRec ct = ldc(p.tiles + t);
        const int a = ct.a;
        const int N = ct.n;
        const int nl = ct.nlev;
        const int aend = ct.aend;
        const int sh = nl - 1;
        const int Lh = 1 << sh;
        const unsigned half = (unsigned)Lh >> 1;
        const int S = WG >> sh;
        // vectors of one run, and of a pair of spans k, Lh + 1 - k
        const int Qt = (S * Lh * (Lh + 1) / 2) / V + Lh;
        const int Pq = S * (Lh + 1) / V + 2;
        // resource from the V-aligned element at or below the spectrum's
        // first bin: vectors then fall on 16-byte boundaries of the batch.
        // Its range ends at the 16-byte block holding the spectrum's last bin
        // (the range check acts per dword, and a 2-byte bin may share its
        // dword with the next spectrum); x's 16-byte alignment keeps that
        // block mapped. Positions past the spectrum's end are used only by
        // outputs past the tile's end, whose stores are discarded.
        const int d = (int)(ct.xoff & (int64_t)(V - 1));
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(static_cast<const char*>(p.x) + (ct.xoff - d) * B), (short)0,
            ((N + d) * B + 15) & ~15, kBufferFlags);
        const int tn = aend - a;
        const int runs = (tn + WG - 1) / WG < R ? (tn + WG - 1) / WG : R;

        // Span layout of the tile's runs: the same for every run, since
        // run ns + WG reads every span S k positions (a whole number of
        // vectors) further on. Vector j of this thread: LDS float offset lo,
        // byte offset ga in the resource for the next run to load, and the
        // step sk between runs. A lane without a vector loads the resource's
        // first one and writes it to the pad: no lane takes a branch around
        // its loads, which would make the compiler wait for every load in
        // flight (the next runs' too) before each LDS write.
        int lo[L::kQ], ga[L::kQ], sk[L::kQ];
        {
            // q / Pq by a multiply: exact for q Pq < 2^32
            const unsigned mg = Lh == 1 ? 0u : 0xffffffffu / (unsigned)Pq + 1u;
#pragma unroll
            for (int j = 0; j < L::kQ; ++j) {
                const int q = tid + j * WG;
                int k = 1, off = q;
                if (Lh > 1) {
                    const int pr = (int)__umulhi((unsigned)q, mg);
                    const int w = q - pr * Pq;
                    const int c1 = S * (pr + 1) / V + 1;
                    k = w < c1 ? pr + 1 : Lh - pr;
                    off = w < c1 ? w : w - c1;
                }
                const int first = (int)(((unsigned)a * (unsigned)k + half) >> sh);
                const bool has = q < Qt;
                lo[j] = has ? S * k * (k - 1) / 2 + V * (k - 1) + off * V : L::kFloats;
                ga[j] = has ? (((d + first) & ~(V - 1)) + off * V) * B : 0;
                sk[j] = has ? S * k * B : 0;
            }
        }
        // vectors of the next run to load into registers
        auto load_run = [&](uint4 (&v)[L::kQ]) {
#pragma unroll
            for (int j = 0; j < L::kQ; ++j) {
                const auto r4 = __builtin_amdgcn_raw_buffer_load_b128(rs, ga[j], 0, 0);
                v[j] = make_uint4(r4[0], r4[1], r4[2], r4[3]);
                ga[j] += sk[j];
            }
        };
        auto store_run = [&](const uint4 (&v)[L::kQ], float* buf) {
#pragma unroll
            for (int j = 0; j < L::kQ; ++j) {
                if constexpr (DT == kF32) {
                    *reinterpret_cast<uint4*>(buf + lo[j]) = v[j];
                } else {
                    const uint32_t w4[4] = {v[j].x, v[j].y, v[j].z, v[j].w};
                    float f[8];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        f[2 * e] = DT == kF16 ? h2f(w4[e] & 0xffffu) : bf2f(w4[e] & 0xffffu);
                        f[2 * e + 1] = DT == kF16 ? h2f(w4[e] >> 16) : bf2f(w4[e] >> 16);
                    }
                    *reinterpret_cast<float4*>(buf + lo[j]) = make_float4(f[0], f[1], f[2], f[3]);
                    *reinterpret_cast<float4*>(buf + lo[j] + 4) = make_float4(f[4], f[5], f[6], f[7]);
                }
            }
        };

        // At Lh = kHmax (every tile of a spectrum summed to H = 32), the LDS
        // byte offset of each term is kept per thread for the whole tile:
        // term k of output n + r WG sits where term k of output n sits in
        // run 0. Offsets are below 2^16 (one buffer), two to a register.
        constexpr int kH = L::kHmax;
        static_assert(L::kFloats * 4 < 65536, "term offsets are 16-bit");
        unsigned ix2[kH / 2];
        if (Lh == kH) {
            int o = 0;
#pragma unroll
            for (int k = 1; k <= kH; ++k) {
                const unsigned pk = (unsigned)(a + tid) * (unsigned)k + half;
                const unsigned pa = (unsigned)a * (unsigned)k + half;
                const unsigned bo =
                    (unsigned)(o - ((d + (int)(pa >> sh)) & ~(V - 1)) + d + (int)(pk >> sh)) * 4u;
                if (k & 1)
                    ix2[(k - 1) / 2] = bo;
                else
                    ix2[(k - 1) / 2] |= bo << 16;
                o += S * k + V;
            }
        }

        // Run r is summed from stage[r & 1]; the registers hold the two runs
        // after it, so each run's loads have two runs' time to arrive.
        // term k of output n of a run: LDS float o_k + (d + pos(n, k)) -
        // base_k, base_k the aligned position below span k's first bin; the
        // same for every run, so it is taken at the tile's first run
        auto sum_run = [&](int r, uint4 (&vn)[L::kQ]) {
            const float* buf = stage[r & 1];
            const unsigned n0 = (unsigned)(a + tid);
            const int n = a + r * WG + tid;
            // acc[m] is level sh - m: term k belongs to the levels
            // m <= tz(k), so with k = 1 mod 4 only the fourth term of a group
            // has a level set known at run time
            float acc[kMaxLevels];
#pragma unroll
            for (int m = 0; m < kMaxLevels; ++m) acc[m] = 0.0f;
            unsigned tk = half, tks = half;
            int ok = 0;
            auto term = [&](int k) {
                tk += n0;
                tks += (unsigned)a;
                const int bk = (d + (int)(tks >> sh)) & ~(V - 1);
                const float val = buf[ok - bk + d + (int)(tk >> sh)];
                ok += S * k + V;
                return val;
            };
            auto add_to = [&](float tv, int tz) {
#pragma unroll
                for (int m = 0; m < kMaxLevels; ++m)
                    if (m <= tz) acc[m] = acc[m] + tv;
            };
            if (Lh == kH) {
                // every term's level set known at compile time
#pragma unroll
                for (int k0 = 1; k0 <= kH; k0 += 8) {
                    float tv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const unsigned w = ix2[(k0 - 1 + u) / 2];
                        const unsigned bo = (u & 1) ? w >> 16 : w & 0xffffu;
                        tv[u] = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(buf) + bo);
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) add_to(tv[u], __builtin_ctz((unsigned)(k0 + u)));
                }
            } else if (Lh >= 4) {
                for (int k = 1; k <= Lh; k += 4) {
                    const float t0 = term(k), t1 = term(k + 1), t2 = term(k + 2), t3 = term(k + 3);
                    add_to(t0, 0);
                    add_to(t1, 1);
                    add_to(t2, 0);
                    add_to(t3, 2 + __builtin_ctz((unsigned)(k + 3) >> 2));   // k + 3 = 0 mod 4
                }
            } else {
                for (int k = 1; k <= Lh; ++k) add_to(term(k), __builtin_ctz((unsigned)k));
            }

            float best = 0.0f;
            int bl = 0;
            // levels l = sh - m in increasing order (the first of equal SNRs
            // is kept)
#pragma unroll
            for (int m = kMaxLevels - 1; m >= 0; --m) {
                const int l = sh - m;
                const bool lv = l >= 0;
                const LevelConst cst = ldc(p.consts + (int64_t)ct.spec * kMaxLevels + (lv ? l : 0));
                const int64_t ho = lv ? ldc(p.spec[ct.spec].hoff + l) : 0;
                const __amdgpu_buffer_rsrc_t hrs =
                    out_rsrc(p.h + ho + a, lv && (p.out_mask & 1u) ? tn * 4 : 0);
                const float hv = acc[m] * cst.rh;
                stream_store_b32(__float_as_uint(hv), hrs, tid * 4, r * WG * 4);
                const float snr = (hv - cst.m) * cst.q;
                if (lv && (l == 0 || snr > best)) {
                    best = snr;
                    bl = l;
                }
            }
            const __amdgpu_buffer_rsrc_t mrs =
                out_rsrc(p.max_snr + ct.xoff + a, (p.out_mask & 2u) ? tn * 4 : 0);
            const __amdgpu_buffer_rsrc_t brs = out_rsrc(p.best_h + ct.xoff + a, (p.out_mask & 4u) ? tn : 0);
            stream_store_b32(__float_as_uint(best), mrs, tid * 4, r * WG * 4);
            stream_store_b8((uint8_t)(1u << bl), brs, tid, r * WG);
            if constexpr (CAND)
                append_candidates(p, cands, n < aend && best >= p.cand_thr, ct.spec, n, best, 1 << bl);
            // run r + 1 into the other buffer, last read before the previous
            // barrier; then its registers take run r + 3 (runs past the
            // tile's end are loaded and summed too, and their stores
            // discarded)
            store_run(vn, stage[(r + 1) & 1]);
            lds_barrier();
            load_run(vn);
        };

        uint4 v0[L::kQ], v1[L::kQ];
        load_run(v0);
        store_run(v0, stage[0]);
        load_run(v0);
        load_run(v1);
        lds_barrier();
        for (int r = 0; r < runs; r += 2) {
            sum_run(r, v0);
            sum_run(r + 1, v1);
        }
        if constexpr (CAND) flush_candidates(p, cands, WG);
        t = uniform(s_claim[(c + 1) & 1]);
    }
}

// --------------------------------------------------------------------------
// eq. (2)-(4), gathered straight from global memory: a tile is a run of
// outputs of one band, taken WG * R at a time (a tile of a cheap band holds
// several such runs); thread t holds outputs a + r WG + t of the current run
// in registers and, for i = 1..Ht in turn, loads the bins of term i of all R
// outputs at once (positions i n, stepped by n from harmonic to harmonic) with
// 32-bit-offset buffer loads over the spectrum. Neighbouring outputs read
// positions i apart, so a wavefront's load covers about 2i cache lines that
// the other harmonics of other tiles read as well (the L2 and the
// memory-side cache serve the reuse). Each output adds its terms in the
// order i = 1..H; snapshots as in the LDS form.
// --------------------------------------------------------------------------
template <int VAR, int DT, int WG, int R, bool CAND>
__global__ __launch_bounds__(WG) void k_hrms1d_gather(const Run1DParams p)
{
    const int tid = (int)threadIdx.x;
    const int lane = tid & 63;
    const bool track = CAND || (p.out_mask & 6u) != 0;
    __shared__ int s_claim[2];
    __shared__ CandStage cands;
    int cq = (int)(blockIdx.x % (unsigned)p.nqueues), visited = 0;
    if (tid == 0) {
        s_claim[0] = claim_tile(p, cq, visited);
        cands.n = 0u;
    }
    __syncthreads();
    int t = uniform(s_claim[0]);
    int cur_spec = -1;
    float lm = 0.0f, lq = 0.0f, lrh = 0.0f;
    int lho_lo = 0, lho_hi = 0;
    for (int c = 0; t >= 0; ++c) {
        // claim the following tile now; it is read after this tile's barrier
        if (tid == 0) s_claim[(c + 1) & 1] = claim_tile(p, cq, visited);
        const TileRec ct = ldc(p.tiles + t);
        const int ht = 1 << (ct.nlev - 1);
        if (ct.spec != cur_spec) {
            cur_spec = ct.spec;
            if (lane < kMaxLevels) {
                const LevelConst lc = p.consts[(int64_t)cur_spec * kMaxLevels + lane];
                lm = lc.m;
                lq = lc.q;
                lrh = lc.rh;
                const int64_t ho = p.spec[cur_spec].hoff[lane];
                lho_lo = (int)(uint32_t)ho;
                lho_hi = (int)(ho >> 32);
            }
        }
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(static_cast<const char*>(p.x) + ct.xoff * Elem<DT>::kBytes), (short)0,
            ct.n * Elem<DT>::kBytes, kBufferFlags);
        // a tile of the cheap bands holds several runs of WG R outputs,
        // taken in turn (fewer tiles to claim and fewer barriers per output)
        for (int a = ct.a; a < ct.aend; a += WG * R) {
            const int tn = ct.aend - a < WG * R ? ct.aend - a : WG * R;
            const int aend = a + tn;
            const __amdgpu_buffer_rsrc_t mrs = out_rsrc(p.max_snr + ct.xoff + a, tn * 4);
            const __amdgpu_buffer_rsrc_t brs = out_rsrc(p.best_h + ct.xoff + a, tn);

            float acc[R], best[R];
            int st[R], pos[R], nn[R];
            bool act[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int n = a + r * WG + tid;
                act[r] = n < aend;
                nn[r] = act[r] ? n : a;
                pos[r] = 0;
                // Greedy starts from -0 so that its first term passes unchanged
                acc[r] = VAR == kGreedy ? -0.0f : 0.0f;
                best[r] = 0.0f;
                st[r] = 0;
            }
            for (int i = 1; i <= ht; ++i) {
                float tv[R];
#pragma unroll
                for (int r = 0; r < R; ++r) pos[r] += nn[r];
                if constexpr (VAR == kFreqbin) {
#pragma unroll
                    for (int r = 0; r < R; ++r) tv[r] = buffer_elem<DT>(rs, pos[r]);
                } else if constexpr (VAR == kMax) {
#pragma unroll
                    for (int r = 0; r < R; ++r) tv[r] = buffer_elem<DT>(rs, pos[r]);
                    for (int jj = 1; jj < i; ++jj) {
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const float w = buffer_elem<DT>(rs, pos[r] + jj);
                            tv[r] = w > tv[r] ? w : tv[r];
                        }
                    }
                } else {
                    if (i == 1) {
#pragma unroll
                        for (int r = 0; r < R; ++r) tv[r] = buffer_elem<DT>(rs, pos[r]);
                    } else {
                        float x0[R], x1[R];
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const int q = pos[r] + (st[r] >> 8);
                            x0[r] = buffer_elem<DT>(rs, q);
                            x1[r] = buffer_elem<DT>(rs, q + 1);
                        }
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const bool step = x1[r] > x0[r];
                            tv[r] = step ? x1[r] : x0[r];
                            st[r] += step ? 256 : 0;
                        }
                    }
                }
#pragma unroll
                for (int r = 0; r < R; ++r) acc[r] = acc[r] + tv[r];
                if ((i & (i - 1)) == 0) {
                    const int li = __builtin_ctz((unsigned)i);
                    const float rh =
                        __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lrh), li));
                    const float m0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lm), li));
                    const float q0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lq), li));
                    const int64_t ho =
                        (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(lho_hi, li) << 32) |
                                  (uint32_t)__builtin_amdgcn_readlane(lho_lo, li));
                    const __amdgpu_buffer_rsrc_t hrs = out_rsrc(p.h + ho + a, tn * 4);
                    const bool fin = i == ht;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const float hv = acc[r] * rh;
                        const float snr = (hv - m0) * q0;
                        if (li == 0 || snr > best[r]) {
                            best[r] = snr;
                            st[r] = (st[r] & ~255) | li;
                        }
                        if (act[r]) {
                            if (p.out_mask & 1u)
                                stream_store_b32(__float_as_uint(hv), hrs, tid * 4, r * WG * 4);
                            if (fin && track) {
                                if (p.out_mask & 2u)
                                    stream_store_b32(__float_as_uint(best[r]), mrs, tid * 4,
                                                     r * WG * 4);
                                if (p.out_mask & 4u)
                                    stream_store_b8((uint8_t)(1u << (st[r] & 255)), brs, tid, r * WG);
                            }
                        }
                        if (CAND && fin)
                            append_candidates(p, cands, act[r] && best[r] >= p.cand_thr, ct.spec,
                                              nn[r], best[r], 1 << (st[r] & 255));
                    }
                }
            }
        }
        __syncthreads();
        if constexpr (CAND) flush_candidates(p, cands, WG);
        t = uniform(s_claim[(c + 1) & 1]);
    }
}

// --------------------------------------------------------------------------
// Statistics: FP64 sums of x and x^2 per segment, in a fixed order, so that
// repeated runs give identical bits.
// --------------------------------------------------------------------------
constexpr int kStatsWG = 256;

template <int DT>
__global__ __launch_bounds__(kStatsWG) void k_stats_partial(const StatsParams p)
{
    // Thread t sums bins start + t + k * WG in increasing k: the order depends
    // only on positions inside the spectrum, not on where the batch packs it.
    constexpr int U = 8;
    __shared__ double s_red[2][kStatsWG / 64];
    const Seg sg = p.segs[blockIdx.x];
    const SpecDesc sd = p.spec[sg.spec];
    const int tid = (int)threadIdx.x;
    const int64_t base = sd.xoff + sg.start;
    double s1 = 0.0, s2 = 0.0;
    int e = tid;
    for (; e + (U - 1) * kStatsWG < sg.len; e += U * kStatsWG) {
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = load_scalar<DT>(p.x, base + e + u * kStatsWG);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double d = (double)v[u];
            s1 = s1 + d;
            s2 = s2 + d * d;
        }
    }
    for (; e < sg.len; e += kStatsWG) {
        const double d = (double)load_scalar<DT>(p.x, base + e);
        s1 = s1 + d;
        s2 = s2 + d * d;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        s1 = s1 + __shfl_xor(s1, off, 64);
        s2 = s2 + __shfl_xor(s2, off, 64);
    }
    if ((tid & 63) == 0) {
        s_red[0][tid >> 6] = s1;
        s_red[1][tid >> 6] = s2;
    }
    __syncthreads();
    if (tid == 0) {
        double t1 = 0.0, t2 = 0.0;
        for (int w = 0; w < kStatsWG / 64; ++w) {
            t1 = t1 + s_red[0][w];
            t2 = t2 + s_red[1][w];
        }
        p.partial[2 * (int64_t)blockIdx.x] = t1;
        p.partial[2 * (int64_t)blockIdx.x + 1] = t2;
    }
}

// Null mean and spread of h_H (see hrms.h): evaluated in FP64 in a fixed
// operation order, then rounded once to FP32.
__device__ void level_consts(int variant, double mu, double sigma, int H, double* m_out,
                             double* q_out)
{
    if (variant == kOpt) {
        // the maximum over every path has no closed-form null moments: no SNR
        *m_out = 0.0;
        *q_out = 0.0;
        return;
    }
    const double rh = sqrt((double)H);
    double mean_s, var_s;
    if (variant == kEq1 || variant == kFreqbin) {
        mean_s = (double)H * mu;
        var_s = (double)H * (sigma * sigma);
    } else if (variant == kMax) {
        // maximum of i exponential bins: mean mu + sigma (Hn_i - 1),
        // variance sigma^2 Psi_i (Renyi's representation of order statistics)
        double hn = 0.0, psi = 0.0, sum_mean = 0.0, sum_psi = 0.0;
        for (int i = 1; i <= H; ++i) {
            hn = hn + 1.0 / (double)i;
            psi = psi + 1.0 / ((double)i * (double)i);
            sum_mean = sum_mean + (mu + sigma * (hn - 1.0));
            sum_psi = sum_psi + psi;
        }
        mean_s = sum_mean;
        var_s = (sigma * sigma) * sum_psi;
    } else if (variant == kGreedyFZ) {
        // Greedy with fdot drift: one bin, then H - 1 maxima of four fresh
        // bins (two rows by two columns): mean mu + 13/12 sigma, variance
        // Psi_4 sigma^2 = 205/144 sigma^2
        mean_s = mu + (double)(H - 1) * (mu + (13.0 / 12.0) * sigma);
        var_s = (sigma * sigma) * (1.0 + (205.0 / 144.0) * (double)(H - 1));
    } else {
        // Greedy: one bin, then H - 1 maxima of two fresh bins
        mean_s = mu + (double)(H - 1) * (mu + 0.5 * sigma);
        var_s = (sigma * sigma) * (1.0 + 1.25 * (double)(H - 1));
    }
    const double m = mean_s / rh;
    const double s = sqrt(var_s) / rh;
    *m_out = m;
    *q_out = s > 0.0 ? 1.0 / s : 0.0;
}

// Sums of a spectrum's segment partials by one wave: lane j adds segments
// j, j + 64, ... in order, then a fixed tree halves the lanes; lane 0's
// result is returned to every lane. The order depends only on the spectrum's
// own segments, so repeated runs and any packing give the same bits.
__device__ __forceinline__ void wave_partial_sums(const double* partial, int first, int last,
                                                  int lane, double& t1, double& t2)
{
    double a = 0.0, b = 0.0;
    for (int g = first + lane; g < last; g += 64) {
        a = a + partial[2 * (int64_t)g];
        b = b + partial[2 * (int64_t)g + 1];
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const double ao = __shfl_down(a, d, 64);
        const double bo = __shfl_down(b, d, 64);
        if (lane < d) {
            a = a + ao;
            b = b + bo;
        }
    }
    t1 = __shfl(a, 0, 64);
    t2 = __shfl(b, 0, 64);
}

// One wave per spectrum: statistics (reduced, or read when provided) and the
// per-level constants, lane l < 6 computing level l's.
__global__ __launch_bounds__(64) void k_consts(const ConstsParams p)
{
    const int s = (int)blockIdx.x;
    const int lane = (int)threadIdx.x;
    if (s == 0 && lane == 0) {
        if (p.counters)
            for (int q = 0; q < kCounterSlots; ++q) p.counters[q] = 0u;
        if (p.cand_count) *p.cand_count = 0u;
    }
    if (s >= p.n_spec) return;
    const SpecDesc sd = p.spec[s];
    double mu, sigma;
    if (p.compute_stats) {
        double t1, t2;
        wave_partial_sums(p.partial, p.seg_first[s], p.seg_first[s + 1], lane, t1, t2);
        const double nb = (double)sd.n;
        mu = t1 / nb;
        double var = t2 / nb - mu * mu;
        if (var < 0.0) var = 0.0;
        sigma = sqrt(var);
        if (lane == 0) {
            p.stats[2 * (int64_t)s] = mu;
            p.stats[2 * (int64_t)s + 1] = sigma;
        }
    } else {
        mu = p.stats[2 * (int64_t)s];
        sigma = p.stats[2 * (int64_t)s + 1];
    }
    const int l = lane;
    if (l < kMaxLevels) {
        float m32 = 0.0f, q32 = 0.0f;
        if (l < sd.nlev) {
            double m, q;
            level_consts(p.variant, mu, sigma, 1 << l, &m, &q);
            m32 = (float)m;
            q32 = (float)q;
        }
        const float rh = (float)(1.0 / sqrt((double)(1 << l)));
        p.consts[(int64_t)s * kMaxLevels + l] = LevelConst{m32, q32, rh, 0.0f};
        if (p.user_consts) {
            p.user_consts[((int64_t)s * kMaxLevels + l) * 2] = m32;
            p.user_consts[((int64_t)s * kMaxLevels + l) * 2 + 1] = q32;
        }
    }
}

// --------------------------------------------------------------------------
// Window form: eq. (2) and the exhaustive-path sum, one output per lane at a
// time (R outputs per lane taken in sequence), every harmonic's window of k
// bins x(k n) .. x(k n + k - 1) read straight from memory with the harmonic
// loop fully unrolled, so that the window's loads are issued together and
// merged into wide loads.
//
// eq. (2): term k is the window's running maximum (strict >, its first bin
// first), added to the FP32 accumulator in the order k = 1..H.
//
// Exhaustive-path sum (the optimal sum named in Sec. 1): the largest sum over
// every offset path eq. (4) could follow (j_1 = 0, each later offset equal to
// or one above the previous), by the recurrence over offsets
//     P_k(j) = max(P_{k-1}(j), P_{k-1}(j-1)) + x(k n + j),  0 <= j < k,
// with P_1(0) = x(n) and a missing predecessor skipped; level H's sum is the
// largest P_H(j). Rounding is monotone, so this is the largest FP32 path sum
// with each path added in the order k = 1..H. The k <= 32 states live in
// registers. Only h is written (there is no closed-form null for an SNR).
// --------------------------------------------------------------------------
// Per-tile values the window form needs, the level constants lane-distributed
// (lane l holds level l's).
struct WinTile {
    __amdgpu_buffer_rsrc_t rs, mrs, brs;
    int a, tn, ht, spec;
    float lm, lq, lrh;
    int lho_lo, lho_hi;
};

// NR outputs per lane (offsets u0, u0 + stride, ... in the tile) whose top
// level is at most KMAX, all harmonics unrolled so that every window load of
// the group is issued before the sums need them. Lanes past the tile's end
// compute on the tile's first output and their stores fall outside the output
// ranges, which the buffer resources discard.
template <int VAR, int DT, int KMAX, int NR, bool CAND>
__device__ __forceinline__ void win_group(const Run1DParams& p, const WinTile& w, int u0,
                                          int stride, bool track, CandStage& cands)
{
    int nn[NR];
    float acc[NR], best[NR];
    int bl[NR];
    float P[NR][VAR == kOpt ? KMAX : 1];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const int u = u0 + q * stride;
        nn[q] = w.a + (u < w.tn ? u : 0);
        acc[q] = 0.0f;
        best[q] = 0.0f;
        bl[q] = 0;
    }
#pragma unroll
    for (int k = 1; k <= KMAX; ++k) {
        if (k > w.ht) continue;
        float xv[NR][KMAX];
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const int base = k * nn[q];
#pragma unroll
            for (int j = 0; j < k; ++j) xv[q][j] = buffer_elem<DT>(w.rs, base + j);
        }
        float S[NR];
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            if constexpr (VAR == kMax) {
                float tv = xv[q][0];
#pragma unroll
                for (int j = 1; j < k; ++j) tv = xv[q][j] > tv ? xv[q][j] : tv;
                acc[q] = acc[q] + tv;
                S[q] = acc[q];
            } else {
                if (k == 1) {
                    P[q][0] = xv[q][0];
                } else {
                    // top down, so that every update reads the previous states
                    P[q][k - 1] = P[q][k - 2] + xv[q][k - 1];
#pragma unroll
                    for (int j = k - 2; j >= 1; --j) {
                        const float m = P[q][j - 1] > P[q][j] ? P[q][j - 1] : P[q][j];
                        P[q][j] = m + xv[q][j];
                    }
                    P[q][0] = P[q][0] + xv[q][0];
                }
                S[q] = 0.0f;
                if ((k & (k - 1)) == 0) {
                    S[q] = P[q][0];
#pragma unroll
                    for (int j = 1; j < k; ++j) S[q] = P[q][j] > S[q] ? P[q][j] : S[q];
                }
            }
        }
        if ((k & (k - 1)) == 0) {
            const int li = __builtin_ctz((unsigned)k);
            const float rh = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(w.lrh), li));
            const int64_t ho =
                (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(w.lho_hi, li) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane(w.lho_lo, li));
            const __amdgpu_buffer_rsrc_t hrs = out_rsrc(p.h + ho + w.a, w.tn * 4);
            const float m0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(w.lm), li));
            const float q0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(w.lq), li));
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                const float hv = S[q] * rh;
                if (p.out_mask & 1u)
                    stream_store_b32(__float_as_uint(hv), hrs, (u0 + q * stride) * 4, 0);
                if (track) {
                    const float snr = (hv - m0) * q0;
                    if (li == 0 || snr > best[q]) {
                        best[q] = snr;
                        bl[q] = li;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const int u = u0 + q * stride;
        if (track) {
            if (p.out_mask & 2u)
                stream_store_b32(__float_as_uint(best[q]), w.mrs, u * 4, 0);
            if (p.out_mask & 4u)
                stream_store_b8((uint8_t)(1u << bl[q]), w.brs, u, 0);
        }
        if constexpr (CAND)
            append_candidates(p, cands, u < w.tn && best[q] >= p.cand_thr, w.spec, nn[q], best[q],
                              1 << bl[q]);
    }
}

// Words of one wave's staging area in the window form: the 64 windows of a
// harmonic k <= 32 (64 k bins), one pad word per 32 bins.
constexpr int kWinWaveWords = 64 * 32 + 64;

// One output per lane of a deep band (top level up to 32). The wave's 64
// consecutive outputs n0 .. n0 + 63 read, for harmonic k, the contiguous bins
// k n0 .. k n0 + 64 k - 1: the wave loads them with whole-line accesses into
// its own LDS area (lane-strided by one bin), then every lane reads its window
// of k bins from there. Only the wave touches its area, and its LDS accesses
// are carried out in order, so no barrier is needed. Lanes past the tile's end
// work on the tile's first output and discard the result.
//
// For eq. (2) on FP32 bins the loads of harmonic k + 1 are issued before
// harmonic k is staged and reduced, so that a wave always has the next
// harmonic's bins in flight (HT, the band's top level, 16 or 32, is then a
// template argument so that whether a next harmonic exists is known at
// compile time).
template <int VAR, int DT, int HT, bool CAND>
__device__ __forceinline__ void win_deep(const Run1DParams& p, const WinTile& w,
                                         const __amdgpu_buffer_rsrc_t rs, const int a, const int tn,
                                         const int ht, int u, bool track, CandStage& cands,
                                         float* wl)
{
    const int lane = (int)threadIdx.x & 63;
    const int ub = u - lane;   // the wave's first output in the tile
    if (ub >= tn) return;      // nothing for this wave (uniform)
    const bool act = u < tn;
    const int n = a + (act ? u : 0);
    const int n0 = a + ub;
    float best = 0.0f;
    int bl = 0;
    float P[VAR == kOpt ? 32 : 1];
    float acc = 0.0f;
    // (2-byte bins: the extra registers cost a resident wave, and it loses)
    constexpr bool kAhead = VAR == kMax && DT == kF32;
    float vn[kAhead ? 32 : 1];   // bins of the next harmonic, in flight
    if constexpr (kAhead) vn[0] = buffer_elem<DT>(rs, n0 + lane);
#pragma unroll
    for (int k = 1; k <= HT; ++k) {
        // without the look-ahead the band's top level stays a run-time bound
        // (HT = 32), which keeps the other forms' registers as they were
        if (!kAhead && k > ht) continue;
        {
            float v[32];
            if constexpr (kAhead) {
#pragma unroll
                for (int t = 0; t < k; ++t) v[t] = vn[t];
                if (k < HT) {
                    const int rnext = (k + 1) * n0 + lane;
#pragma unroll
                    for (int t = 0; t <= k; ++t) vn[t] = buffer_elem<DT>(rs, rnext + 64 * t);
                }
            } else {
                const int rbase = k * n0 + lane;
#pragma unroll
                for (int t = 0; t < k; ++t) v[t] = buffer_elem<DT>(rs, rbase + 64 * t);
            }
            __builtin_amdgcn_wave_barrier();   // the previous windows are read
#pragma unroll
            for (int t = 0; t < k; ++t) wl[pidx(lane + 64 * t)] = v[t];
            __builtin_amdgcn_wave_barrier();
        }
        float xv[32];
        const int wb = act ? k * lane : 0;
#pragma unroll
        for (int j = 0; j < k; ++j) xv[j] = wl[pidx(wb + j)];
        float S = 0.0f;
        if constexpr (VAR == kMax) {
            float tv = xv[0];
#pragma unroll
            for (int j = 1; j < k; ++j) tv = xv[j] > tv ? xv[j] : tv;
            acc = acc + tv;
            S = acc;
        } else {
            if (k == 1) {
                P[0] = xv[0];
            } else {
                // top down, so that every update reads the previous states
                P[k - 1] = P[k - 2] + xv[k - 1];
#pragma unroll
                for (int j = k - 2; j >= 1; --j) {
                    const float m = P[j - 1] > P[j] ? P[j - 1] : P[j];
                    P[j] = m + xv[j];
                }
                P[0] = P[0] + xv[0];
            }
            if ((k & (k - 1)) == 0) {
                S = P[0];
#pragma unroll
                for (int j = 1; j < k; ++j) S = P[j] > S ? P[j] : S;
            }
        }
        if ((k & (k - 1)) == 0) {
            const int li = __builtin_ctz((unsigned)k);
            const float rh =
                __int_as_float(__builtin_amdgcn_readlane(__float_as_int(w.lrh), li));
            const float hv = S * rh;
            if (p.out_mask & 1u) {
                const int64_t ho = (int64_t)(
                    ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(w.lho_hi, li) << 32) |
                    (uint32_t)__builtin_amdgcn_readlane(w.lho_lo, li));
                const __amdgpu_buffer_rsrc_t hrs = out_rsrc(p.h + ho + a, tn * 4);
                stream_store_b32(__float_as_uint(hv), hrs, u * 4, 0);
            }
            if (track) {
                const float m0 =
                    __int_as_float(__builtin_amdgcn_readlane(__float_as_int(w.lm), li));
                const float q0 =
                    __int_as_float(__builtin_amdgcn_readlane(__float_as_int(w.lq), li));
                const float snr = (hv - m0) * q0;
                if (li == 0 || snr > best) {
                    best = snr;
                    bl = li;
                }
            }
        }
    }
    if (track) {
        if (p.out_mask & 2u)
            stream_store_b32(__float_as_uint(best), w.mrs, u * 4, 0);
        if (p.out_mask & 4u)
            stream_store_b8((uint8_t)(1u << bl), w.brs, u, 0);
    }
    if constexpr (CAND)
        append_candidates(p, cands, act && best >= p.cand_thr, w.spec, n, best, 1 << bl);
}

template <int VAR, int DT, int WG, int R, bool CAND>
__global__ __launch_bounds__(WG) void k_hrms1d_win(const Run1DParams p)
{
    static_assert(VAR == kMax || VAR == kOpt, "window form: eq. (2) and the exhaustive path");
    static_assert(VAR == kMax || !CAND, "the exhaustive-path sum has no SNR");
    static_assert(R % 4 == 0, "outputs per lane come in groups of 4");
    (void)R;
    const int tid = (int)threadIdx.x;
    const int lane = tid & 63;
    const bool track = VAR == kMax && (CAND || (p.out_mask & 6u) != 0);
    __shared__ int s_claim[2];
    __shared__ CandStage cands;
    __shared__ float wlds[WG / 64][kWinWaveWords];
    float* wl = wlds[tid >> 6];
    int cq = (int)(blockIdx.x % (unsigned)p.nqueues), visited = 0;
    if (tid == 0) {
        s_claim[0] = claim_tile(p, cq, visited);
        cands.n = 0u;
    }
    __syncthreads();
    int t = uniform(s_claim[0]);
    WinTile w;
    w.spec = -1;
    w.lm = w.lq = w.lrh = 0.0f;
    w.lho_lo = w.lho_hi = 0;
    for (int c = 0; t >= 0; ++c) {
        if (tid == 0) s_claim[(c + 1) & 1] = claim_tile(p, cq, visited);
        const TileRec ct = ldc(p.tiles + t);
        w.a = ct.a;
        w.ht = 1 << (ct.nlev - 1);
        w.tn = ct.aend - ct.a;
        if (ct.spec != w.spec) {
            w.spec = ct.spec;
            if (lane < kMaxLevels) {
                const LevelConst lc = p.consts[(int64_t)w.spec * kMaxLevels + lane];
                w.lm = lc.m;
                w.lq = lc.q;
                w.lrh = lc.rh;
                const int64_t ho = p.spec[w.spec].hoff[lane];
                w.lho_lo = (int)(uint32_t)ho;
                w.lho_hi = (int)(ho >> 32);
            }
        }
        w.rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(static_cast<const char*>(p.x) + ct.xoff * Elem<DT>::kBytes), (short)0,
            ct.n * Elem<DT>::kBytes, kBufferFlags);
        w.mrs = out_rsrc(p.max_snr + ct.xoff + w.a, w.tn * 4);
        w.brs = out_rsrc(p.best_h + ct.xoff + w.a, w.tn);
        // the cheap bands take several outputs per lane at once, the deep ones
        // one at a time (their windows already keep many loads in flight)
        // (a tile holds up to 8 R WG outputs in the cheap bands, R WG otherwise)
        if (w.ht <= 2) {
#pragma unroll 1
            for (int u0 = 0; u0 < w.tn; u0 += 4 * WG)
                win_group<VAR, DT, 2, 4, CAND>(p, w, u0 + tid, WG, track, cands);
        } else if (w.ht <= 8) {
#pragma unroll 1
            for (int u0 = 0; u0 < w.tn; u0 += 2 * WG)
                win_group<VAR, DT, 8, 2, CAND>(p, w, u0 + tid, WG, track, cands);
        } else if (VAR == kMax && DT == kF32 && w.ht == 16) {
#pragma unroll 1
            for (int u0 = 0; u0 < w.tn; u0 += WG)
                win_deep<VAR, DT, 16, CAND>(p, w, w.rs, w.a, w.tn, w.ht, u0 + tid, track, cands,
                                            wl);
        } else {
#pragma unroll 1
            for (int u0 = 0; u0 < w.tn; u0 += WG)
                win_deep<VAR, DT, 32, CAND>(p, w, w.rs, w.a, w.tn, w.ht, u0 + tid, track, cands,
                                            wl);
        }
        __syncthreads();
        if constexpr (CAND) flush_candidates(p, cands, WG);
        t = uniform(s_claim[(c + 1) & 1]);
    }
}

// --------------------------------------------------------------------------
// 2D frequency x fdot plane. Output (f, z) of level H is the fundamental at
// frequency f whose H-th harmonic has fdot z; harmonic i reads row
// round(i z / H) (halves away from zero), and along that row the 1D form of
// the variant: column round(i f / H) (eq. (1), halves up), the window
// i f .. i f + i - 1 (eq. (2)), column i f (eq. (3)) or i f + j (eq. (4), j as
// there). Greedy with fdot drift also lets the row move: harmonic k chooses
// among columns k f + j, k f + j + 1 of rows round(k z / H) + d and that row
// plus sign(z) (clamped to the plane), the first largest winning, and j, d
// follow the choice. Each level is summed on its own, in the order i = 1..H. A thread owns
// one output; a workgroup holds 64 consecutive frequencies of kZRows fdot rows,
// the rows being the fastest grid dimension so that neighbouring workgroups
// read the same columns.
// --------------------------------------------------------------------------
constexpr int kZRows = 4;
constexpr unsigned kXcds = 8;   // XCDs of the part, taking workgroups in turn

__device__ __forceinline__ int row_of(int iz, int l)
{
    // round(iz / 2^l), halves away from zero
    const int H = 1 << l;
    return iz >= 0 ? (2 * iz + H) >> (l + 1) : -((-2 * iz + H) >> (l + 1));
}

// A row of the plane as a buffer resource spanning its nf bins (reads past
// the row return 0; none is made).
template <int DT>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_row(const Run2DParams& p, int row)
{
    const char* base = static_cast<const char*>(p.x) + (int64_t)row * p.ld * Elem<DT>::kBytes;
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, p.nf * Elem<DT>::kBytes,
                                             kBufferFlags);
}

template <int VAR, int DT>
__global__ __launch_bounds__(64 * kZRows) void k_hrms2d(const Run2DParams p)
{
    const int lane = (int)threadIdx.x & 63;
    // the fdot row is the same for the whole wavefront, so every row a
    // harmonic reads is a scalar and its loads go through a scalar resource
    const int zl = uniform((int)threadIdx.x >> 6);
    // Workgroup b runs on XCD b mod 8. Each XCD takes whole frequency blocks
    // with all their fdot groups (block 8 j + x of the frequency axis on XCD
    // x), so the columns that the rows of one block read are fetched into one
    // L2 and shared there by all its fdot groups, while the eight XCDs still
    // work on neighbouring frequency blocks.
    const unsigned xcd = blockIdx.x % kXcds, slot = blockIdx.x / kXcds;
    const int zg = (int)(slot % (unsigned)p.zgroups);
    const int mb = (int)((slot / (unsigned)p.zgroups) * kXcds + xcd);
    const int rows = 2 * p.zmax + 1;
    const int r = zg * kZRows + zl;
    const int m = mb * 64 + lane;
    if (r >= rows || m >= p.nf) return;
    const int z = r - p.zmax;
    float best = 0.0f;
    int bl = 0;
#pragma unroll
    for (int l = 0; l < kMaxLevels; ++l) {
        // eq. (1) reads at most column f, so every level of every f exists
        if (l < p.nlev && (VAR == kEq1 || m < (p.nf >> l))) {
            const int H = 1 << l;
            float acc = 0.0f;
            if constexpr (VAR == kEq1) {
#pragma unroll
                for (int i = 1; i <= (1 << (kMaxLevels - 1)); ++i) {
                    if (i <= H) {
                        const auto rs = plane_row<DT>(p, row_of(i * z, l) + p.zmax);
                        const int col = (int)(((int64_t)(2 * i) * m + H) >> (l + 1));
                        acc = acc + buffer_elem<DT>(rs, col);
                    }
                }
            } else if constexpr (VAR == kMax) {
                // one harmonic at a time (unrolling the harmonics would hold
                // every window in registers at once); each window is read in
                // blocks of 4 adjacent bins
#pragma unroll 1
                for (int i = 1; i <= H; ++i) {
                    const auto rs = plane_row<DT>(p, row_of(i * z, l) + p.zmax);
                    const int base = i * m;
                    // running maximum in window order with a strict >, as eq. (2)
                    float w = buffer_elem<DT>(rs, base);
                    int j = 1;
                    for (; j + 4 <= i; j += 4) {
                        float v[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) v[u] = buffer_elem<DT>(rs, base + j + u);
#pragma unroll
                        for (int u = 0; u < 4; ++u) w = v[u] > w ? v[u] : w;
                    }
                    for (; j < i; ++j) {
                        const float v = buffer_elem<DT>(rs, base + j);
                        w = v > w ? v : w;
                    }
                    acc = acc + w;
                }
            } else if constexpr (VAR == kFreqbin) {
#pragma unroll
                for (int i = 1; i <= (1 << (kMaxLevels - 1)); ++i) {
                    if (i <= H) {
                        const auto rs = plane_row<DT>(p, row_of(i * z, l) + p.zmax);
                        acc = acc + buffer_elem<DT>(rs, i * m);
                    }
                }
            } else if constexpr (VAR == kGreedyFZ) {
                // the path's row offset d differs from lane to lane, so rows
                // are addressed per lane; rows are clamped to the plane
                const int sg = z > 0 ? 1 : (z < 0 ? -1 : 0);
                acc = load_scalar<DT>(p.x, (int64_t)(row_of(z, l) + p.zmax) * p.ld + m);
                int j = 0, d = 0;
#pragma unroll
                for (int k = 2; k <= (1 << (kMaxLevels - 1)); ++k) {
                    if (k <= H) {
                        const int rk = row_of(k * z, l);
                        const int r0 = min(max(rk + d, -p.zmax), p.zmax) + p.zmax;
                        const int r1 = min(max(rk + d + sg, -p.zmax), p.zmax) + p.zmax;
                        const int64_t c = (int64_t)k * m + j;
                        const int64_t b0 = (int64_t)r0 * p.ld + c;
                        const int64_t b1 = (int64_t)r1 * p.ld + c;
                        const float x00 = load_scalar<DT>(p.x, b0);
                        const float x01 = load_scalar<DT>(p.x, b0 + 1);
                        const float x10 = load_scalar<DT>(p.x, b1);
                        const float x11 = load_scalar<DT>(p.x, b1 + 1);
                        // the first largest in the order x00, x01, x10, x11
                        float v = x00;
                        int pick = 0;
                        if (x01 > v) { v = x01; pick = 1; }
                        if (x10 > v) { v = x10; pick = 2; }
                        if (x11 > v) { v = x11; pick = 3; }
                        acc = acc + v;
                        j += pick & 1;
                        d += (pick & 2) ? sg : 0;
                    }
                }
            } else {
                acc = buffer_elem<DT>(plane_row<DT>(p, row_of(z, l) + p.zmax), m);
                int j = 0;
#pragma unroll
                for (int k = 2; k <= (1 << (kMaxLevels - 1)); ++k) {
                    if (k <= H) {
                        const auto rs = plane_row<DT>(p, row_of(k * z, l) + p.zmax);
                        const int q = k * m + j;
                        const float x0 = buffer_elem<DT>(rs, q);
                        const float x1 = buffer_elem<DT>(rs, q + 1);
                        if (x1 > x0) {
                            acc = acc + x1;
                            j += 1;
                        } else {
                            acc = acc + x0;
                        }
                    }
                }
            }
            // Greedy with fdot drift: the z = 0 row cannot drift and has
            // eq. (4)'s constants, the second set
            const LevelConst c = p.consts[(VAR == kGreedyFZ && z == 0) ? kMaxLevels + l : l];
            const float hv = acc * c.rh;
            const int plane = VAR == kEq1 ? p.nf : (p.nf >> l);
            if (p.out_mask & 1u)
                __builtin_nontemporal_store(hv, p.h + p.hoff[l] + (int64_t)r * plane + m);
            const float snr = (hv - c.m) * c.q;
            if (l == 0 || snr > best) {
                best = snr;
                bl = l;
            }
        }
    }
    const int64_t o = (int64_t)r * p.nf + m;
    if (p.out_mask & 2u) __builtin_nontemporal_store(best, p.max_snr + o);
    if (p.out_mask & 4u) __builtin_nontemporal_store((uint8_t)(1u << bl), p.best_h + o);
}

// --------------------------------------------------------------------------
// Local maxima of max_snr: bin n of a spectrum is listed when
// max_snr[n] >= thr, max_snr[n] > max_snr[n - 1] and max_snr[n] >= max_snr[n + 1]
// (a missing neighbour counts as lower). One workgroup per 64K-bin segment;
// records are gathered in LDS and written with one global atomic per
// workgroup, as in the fused candidate output.
// --------------------------------------------------------------------------
constexpr int kPeakWG = 256;

__global__ __launch_bounds__(kPeakWG) void k_peaks(const PeakParams pp)
{
    __shared__ CandStage cands;
    Run1DParams p{};   // only the candidate-list fields are used
    p.cand = pp.cand;
    p.cand_count = pp.cand_count;
    p.cand_cap = pp.cand_cap;
    if (threadIdx.x == 0) cands.n = 0u;
    __syncthreads();
    const Seg sg = pp.segs[blockIdx.x];
    const SpecDesc sd = pp.spec[sg.spec];
    const float* ms = pp.max_snr + sd.ooff;
    for (int b = 0; b < sg.len; b += kPeakWG) {
        const int n = sg.start + b + (int)threadIdx.x;
        bool take = false;
        float v = 0.0f;
        if (n < sg.start + sg.len) {
            v = ms[n];
            const float lo = n > 0 ? ms[n - 1] : -INFINITY;
            const float hi = n + 1 < sd.n ? ms[n + 1] : -INFINITY;
            take = v >= pp.thr && v > lo && v >= hi;
        }
        const int bh = take && pp.best_h ? (int)pp.best_h[sd.ooff + n] : 0;
        append_candidates(p, cands, take, sg.spec, n, v, bh);
    }
    __syncthreads();
    flush_candidates(p, cands, kPeakWG);
}

// --------------------------------------------------------------------------
// Precision form: y = round_to_dtype(x * fl32(1 / mu)), round to nearest
// even; FP16 saturates at +-65504.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_quant_consts(const QuantConstParams p)
{
    // one wave per spectrum, as k_consts
    const int s = (int)blockIdx.x;
    const int lane = (int)threadIdx.x;
    if (s >= p.n_spec) return;
    double mu, sigma;
    if (p.compute_stats) {
        double t1, t2;
        wave_partial_sums(p.partial, p.seg_first[s], p.seg_first[s + 1], lane, t1, t2);
        const double nb = (double)p.spec[s].n;
        mu = t1 / nb;
        double var = t2 / nb - mu * mu;
        if (var < 0.0) var = 0.0;
        sigma = sqrt(var);
        if (lane == 0) {
            p.stats[2 * (int64_t)s] = mu;
            p.stats[2 * (int64_t)s + 1] = sigma;
        }
    } else {
        mu = p.stats[2 * (int64_t)s];
        sigma = p.stats[2 * (int64_t)s + 1];
    }
    // a spectrum whose mean is not a positive finite number cannot be scaled
    // to unit mean: it is stored unscaled, with its own statistics
    const bool scalable = mu > 0.0 && mu <= 1.79769313486231570e308;
    if (lane == 0) {
        p.stats_out[2 * (int64_t)s] = scalable ? 1.0 : mu;
        p.stats_out[2 * (int64_t)s + 1] = scalable ? sigma / mu : sigma;
        p.inv_mu[s] = scalable ? (float)(1.0 / mu) : 1.0f;
    }
}

__device__ __forceinline__ uint16_t to_f16_sat(float v)
{
    if (v > 65504.0f) v = 65504.0f;
    if (v < -65504.0f) v = -65504.0f;
    return __builtin_bit_cast(uint16_t, (_Float16)v);
}

__device__ __forceinline__ uint16_t to_bf16_rne(float v)
{
    const uint32_t u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x0040u);   // quiet NaN
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

template <int DT>
__global__ __launch_bounds__(kStatsWG) void k_quantize(const QuantParams p)
{
    const Seg sg = p.segs[blockIdx.x];
    const SpecDesc sd = p.spec[sg.spec];
    const float inv = p.inv_mu[sg.spec];
    uint16_t* y = static_cast<uint16_t*>(p.y);
    const int64_t base = sd.xoff + sg.start;
    for (int e = (int)threadIdx.x; e < sg.len; e += kStatsWG) {
        const float v = p.x[base + e] * inv;
        y[base + e] = DT == kF16 ? to_f16_sat(v) : to_bf16_rne(v);
    }
}

template <int VAR, int DT, int WG, int R, int C, bool CAND>
void* fund_kernel()
{
    if constexpr (C == 0 && VAR == kMax)
        return reinterpret_cast<void*>(&k_hrms1d_win<VAR, DT, WG, R, CAND>);
    else if constexpr (C == 0)
        return reinterpret_cast<void*>(&k_hrms1d_gather<VAR, DT, WG, R, CAND>);
    else
        return reinterpret_cast<void*>(&k_hrms1d_span<VAR, DT, WG, R, C, CAND>);
}

template <int DT, int WG, int R, int C, bool CAND>
void* eq1_kernel()
{
    // chunk 1 marks the LDS-staged form
    if constexpr (C == 1)
        return reinterpret_cast<void*>(&k_hrms1d_eq1_lds<DT, WG, R, CAND>);
    else
        return reinterpret_cast<void*>(&k_hrms1d_eq1<DT, WG, R, C, CAND>);
}

// Launch shapes compiled into the library: (threads, outputs per thread, LDS
// chunk in bins) for the fundamental-indexed family and for eq. (1).
struct ShapeEntry {
    int eq1;   // 1: eq. (1) kernel family, 0: eq. (2)-(4)
    int wg, r, chunk;
    void* (*k[3][3][2])();   // [variant slot][dtype][with candidate output]
};

template <int VAR, int WG, int R, int CB>
constexpr auto fund_dtypes()
{
    struct T {
        void* (*k[3][2])();
    };
    return T{{{&fund_kernel<VAR, kF32, WG, R, CB, false>, &fund_kernel<VAR, kF32, WG, R, CB, true>},
              {&fund_kernel<VAR, kF16, WG, R, CB, false>, &fund_kernel<VAR, kF16, WG, R, CB, true>},
              {&fund_kernel<VAR, kBF16, WG, R, CB, false>,
               &fund_kernel<VAR, kBF16, WG, R, CB, true>}}};
}

template <int WG, int R, int CB>
constexpr ShapeEntry fund_shape()
{
    ShapeEntry e{0, WG, R, CB, {}};
    const auto mx = fund_dtypes<kMax, WG, R, CB>();
    const auto fb = fund_dtypes<kFreqbin, WG, R, CB>();
    const auto gr = fund_dtypes<kGreedy, WG, R, CB>();
    for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 2; ++c) {
            e.k[0][d][c] = mx.k[d][c];
            e.k[1][d][c] = fb.k[d][c];
            e.k[2][d][c] = gr.k[d][c];
        }
    return e;
}

template <int WG, int R, int CB>
constexpr ShapeEntry eq1_shape()
{
    ShapeEntry e{1, WG, R, CB, {}};
    e.k[0][0][0] = &eq1_kernel<kF32, WG, R, CB, false>;
    e.k[0][0][1] = &eq1_kernel<kF32, WG, R, CB, true>;
    e.k[0][1][0] = &eq1_kernel<kF16, WG, R, CB, false>;
    e.k[0][1][1] = &eq1_kernel<kF16, WG, R, CB, true>;
    e.k[0][2][0] = &eq1_kernel<kBF16, WG, R, CB, false>;
    e.k[0][2][1] = &eq1_kernel<kBF16, WG, R, CB, true>;
    return e;
}

const ShapeEntry kShapes[] = {
    fund_shape<1024, 8, 16384>(),
    fund_shape<1024, 16, 16384>(),
    fund_shape<512, 8, 8192>(),
    fund_shape<256, 8, 0>(),
    fund_shape<256, 16, 0>(),
    fund_shape<512, 8, 0>(),
    eq1_shape<256, 8, 0>(),
    eq1_shape<256, 4, 0>(),
    eq1_shape<512, 8, 0>(),
    eq1_shape<512, 8, 1>(),
};

const ShapeEntry* find_shape(int variant, const Shape1D& s)
{
    const int fam = variant == kEq1 ? 1 : 0;
    for (const ShapeEntry& e : kShapes)
        if (e.eq1 == fam && e.wg == s.wg && e.r == s.r && e.chunk == s.chunk) return &e;
    return nullptr;
}

void* opt_kernel(int dtype)
{
    switch (dtype) {
    case kF32:
        return reinterpret_cast<void*>(&k_hrms1d_win<kOpt, kF32, kOptShape.wg, kOptShape.r, false>);
    case kF16:
        return reinterpret_cast<void*>(&k_hrms1d_win<kOpt, kF16, kOptShape.wg, kOptShape.r, false>);
    default:
        return reinterpret_cast<void*>(&k_hrms1d_win<kOpt, kBF16, kOptShape.wg, kOptShape.r, false>);
    }
}

void* kernel_for(int variant, int dtype, const Shape1D& s, bool cand = false)
{
    if (variant == kOpt) {
        const bool ok = s.wg == kOptShape.wg && s.r == kOptShape.r && s.chunk == 0 && s.top == 0;
        return ok && !cand && dtype >= 0 && dtype <= 2 ? opt_kernel(dtype) : nullptr;
    }
    if (dtype < 0 || dtype > 2 || variant < 0 || variant > 3) return nullptr;
    const ShapeEntry* e = find_shape(variant, s);
    if (!e) return nullptr;
    return variant == kEq1 ? e->k[0][dtype][cand]() : e->k[variant - 1][dtype][cand]();
}

}  // namespace

hipError_t launch_stats_partial(int dtype, const StatsParams& p, hipStream_t s)
{
    if (p.nsegs <= 0) return hipSuccess;
    dim3 grid(p.nsegs), block(kStatsWG);
    switch (dtype) {
    case kF32: hipLaunchKernelGGL(k_stats_partial<kF32>, grid, block, 0, s, p); break;
    case kF16: hipLaunchKernelGGL(k_stats_partial<kF16>, grid, block, 0, s, p); break;
    default: hipLaunchKernelGGL(k_stats_partial<kBF16>, grid, block, 0, s, p); break;
    }
    return hipGetLastError();
}

hipError_t launch_consts(const ConstsParams& p, hipStream_t s)
{
    // one wave per spectrum (at least one, which also resets the counters)
    const int blocks = p.n_spec > 0 ? p.n_spec : 1;
    hipLaunchKernelGGL(k_consts, dim3(blocks), dim3(64), 0, s, p);
    return hipGetLastError();
}

bool hrms1d_shape_supported(int variant, const Shape1D& shape)
{
    if (shape.top != 0) {
        // a split launch: eq. (2)-(4) only, at a power-of-two level
        if (variant == kEq1 || shape.top < 2 || shape.top > 32 || (shape.top & (shape.top - 1)))
            return false;
    }
    return kernel_for(variant, kF32, shape) != nullptr;
}

int hrms1d_shapes(int variant, Shape1D* out, int cap)
{
    if (variant == kOpt) {
        if (out && cap > 0) out[0] = kOptShape;
        return 1;
    }
    // every compiled shape; the gathered forms also split at the top band
    const int fam = variant == kEq1 ? 1 : 0;
    int n = 0;
    for (const ShapeEntry& e : kShapes) {
        if (e.eq1 != fam) continue;
        if (out && n < cap) out[n] = Shape1D{e.wg, e.r, e.chunk, 0};
        ++n;
        if (!fam && e.chunk == 0) {
            if (out && n < cap) out[n] = Shape1D{e.wg, e.r, e.chunk, 32};
            ++n;
        }
    }
    return n;
}

int hrms1d_max_blocks_per_cu(int variant, int dtype, const Shape1D& shape, hipError_t* err)
{
    if (err) *err = hipSuccess;
    void* k = kernel_for(variant, dtype, shape);
    if (!k) return 0;
    int nb = 0;
    const hipError_t e1 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, shape.wg, 0);
    if (e1 == hipSuccess && nb > 0) return nb;
    // The runtime's calculator declines some kernels with more than 64 KiB of
    // LDS; count from the kernel's own resources instead: 160 KiB of LDS and
    // 4 SIMDs of 512 VGPRs per lane (at most 8 waves each) per CU.
    hipFuncAttributes fa{};
    const hipError_t e2 = hipFuncGetAttributes(&fa, k);
    if (e2 != hipSuccess) {
        if (err) *err = e1 != hipSuccess ? e1 : e2;
        return 0;
    }
    const int waves = (shape.wg + 63) / 64;
    const int vgpr = fa.numRegs > 0 ? (fa.numRegs + 7) / 8 * 8 : 128;
    const int per_simd = vgpr > 512 ? 0 : (512 / vgpr < 8 ? 512 / vgpr : 8);
    const int by_waves = 4 * per_simd / waves;
    const int by_lds = fa.sharedSizeBytes > 0 ? (int)(163840 / fa.sharedSizeBytes) : by_waves;
    return by_waves < by_lds ? by_waves : by_lds;
}

hipError_t launch_hrms1d(int variant, int dtype, const Shape1D& shape, const Run1DParams& p,
                         int grid, hipStream_t s)
{
    void* k = kernel_for(variant, dtype, shape, (p.out_mask & 8u) != 0);
    if (!k) return hipErrorInvalidValue;
    if (grid <= 0) return hipSuccess;
    Run1DParams pc = p;
    void* args[] = {&pc};
    return hipLaunchKernel(k, dim3(grid), dim3(shape.wg), args, 0, s);
}

using Kernel2D = void (*)(const Run2DParams);

template <int VAR>
Kernel2D kernel_2d(int dtype)
{
    return dtype == kF32 ? k_hrms2d<VAR, kF32> : dtype == kF16 ? k_hrms2d<VAR, kF16> : k_hrms2d<VAR, kBF16>;
}

hipError_t launch_hrms2d(int variant, int dtype, const Run2DParams& p, hipStream_t s)
{
    // frequency blocks rounded up to whole rounds of the XCDs (the blocks
    // past the plane's end return at once)
    const int64_t mblocks = ((int64_t)p.nf + 63) / 64;
    const int64_t blocks = (mblocks + kXcds - 1) / kXcds * kXcds * p.zgroups;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    dim3 grid((unsigned)blocks), block(64 * kZRows);
    Kernel2D k = nullptr;
    switch (variant) {
    case kEq1: k = kernel_2d<kEq1>(dtype); break;
    case kMax: k = kernel_2d<kMax>(dtype); break;
    case kFreqbin: k = kernel_2d<kFreqbin>(dtype); break;
    case kGreedy: k = kernel_2d<kGreedy>(dtype); break;
    case kGreedyFZ: k = kernel_2d<kGreedyFZ>(dtype); break;
    default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k, grid, block, 0, s, p);
    return hipGetLastError();
}

hipError_t launch_peaks(const PeakParams& p, hipStream_t s)
{
    if (p.nsegs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_peaks, dim3(p.nsegs), dim3(kPeakWG), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_quant_consts(const QuantConstParams& p, hipStream_t s)
{
    hipLaunchKernelGGL(k_quant_consts, dim3(p.n_spec > 0 ? p.n_spec : 1), dim3(64), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_quantize(int dtype, const QuantParams& p, hipStream_t s)
{
    if (p.nsegs <= 0) return hipSuccess;
    if (dtype == kF16)
        hipLaunchKernelGGL(k_quantize<kF16>, dim3(p.nsegs), dim3(kStatsWG), 0, s, p);
    else
        hipLaunchKernelGGL(k_quantize<kBF16>, dim3(p.nsegs), dim3(kStatsWG), 0, s, p);
    return hipGetLastError();
}

}  // namespace hrms
