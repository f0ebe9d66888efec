// hrms_kernels.hip -- gfx950 kernels of the incoherent harmonic sum.
//
// Paper: K. Adamek and W. Armour, "A GPU implementation of the harmonic sum
// algorithm" (arXiv:1812.02647); eq. (1) in Sec. 1, eq. (2)-(4) in Sec. 2.
//
// Design (memory-bound; no matrix cores):
//   * A tile is T = WG * R consecutive outputs [a, a + T) of one spectrum; thread
//     t owns outputs a + r * WG + t, r < R, and keeps their running sums, best
//     SNR and best level (and Greedy's offset j) in registers.
//   * Harmonic i of the tile reads the contiguous span [i a, i (a + T)) (plus up
//     to i - 1 bins of window). The tile streams the union of these spans
//     through LDS in chunks of C bins (+ a 32-bin halo for the windows of
//     eq. (2) and (4)), loaded with 16-byte coalesced loads, so the stride-i
//     gather of eq. (2)-(4) never reaches HBM or L2 directly. Spans of
//     neighbouring harmonics overlap once i T >= a, and are then staged once.
//   * Position i n of output n lies in exactly one chunk, chunks are visited in
//     increasing position and harmonics in increasing i inside a chunk, so every
//     output adds its harmonics in the order i = 1..H of the equations.
//   * A level snapshot (h = S * fl32(1/sqrt(H)), SNR, best level) is taken when
//     i reaches a power of two.
//   * LDS holds FP32 whatever the storage type; a 1-in-32 padding keeps strided
//     reads (stride i) nearly free of bank conflicts.
//   * The grid is persistent: workgroups pull tiles from a cost-sorted list
//     through one atomic counter (the paper's load-balancing concern, Sec. 1).
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "hrms_internal.h"

namespace hrms {
namespace {

constexpr int kEq1 = 0, kMax = 1, kFreqbin = 2, kGreedy = 3;
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

// Loads the kVec elements starting at absolute element index `abs` (a multiple
// of kVec); elements outside [lo, hi) read as 0.
template <int DT>
__device__ __forceinline__ void load_vec(const void* base, int64_t abs, int64_t lo, int64_t hi,
                                         float (&v)[Elem<DT>::kVec])
{
    constexpr int V = Elem<DT>::kVec;
    if (abs >= lo && abs + V <= hi) {
        const uint4 u = *reinterpret_cast<const uint4*>(static_cast<const char*>(base) +
                                                        abs * Elem<DT>::kBytes);
        const uint32_t w[4] = {u.x, u.y, u.z, u.w};
        if constexpr (DT == kF32) {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = __uint_as_float(w[e]);
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if constexpr (DT == kF16) {
                    v[2 * e] = h2f(w[e] & 0xffffu);
                    v[2 * e + 1] = h2f(w[e] >> 16);
                } else {
                    v[2 * e] = bf2f(w[e] & 0xffffu);
                    v[2 * e + 1] = bf2f(w[e] >> 16);
                }
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const int64_t k = abs + e;
            v[e] = (k >= lo && k < hi) ? load_scalar<DT>(base, k) : 0.0f;
        }
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

// Raw 16-byte vector of the input (kVec elements) with zeros outside [lo, hi).
template <int DT>
__device__ __forceinline__ uint4 load_raw(const void* base, int64_t abs, int64_t lo, int64_t hi)
{
    constexpr int V = Elem<DT>::kVec;
    if (abs >= lo && abs + V <= hi)
        return *reinterpret_cast<const uint4*>(static_cast<const char*>(base) +
                                               abs * Elem<DT>::kBytes);
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int e = 0; e < V; ++e) {
        const int64_t k = abs + e;
        if (k >= lo && k < hi) {
            if constexpr (DT == kF32) {
                w[e] = static_cast<const uint32_t*>(base)[k];
            } else {
                const uint32_t b = static_cast<const uint16_t*>(base)[k];
                w[e >> 1] |= b << (16 * (e & 1));
            }
        }
    }
    return uint4{w[0], w[1], w[2], w[3]};
}

template <int DT>
__device__ __forceinline__ void store_raw(float* buf, int k0, const uint4& u)
{
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
    if constexpr (DT == kF32) {
#pragma unroll
        for (int e = 0; e < 4; ++e) buf[pidx(k0 + e)] = __uint_as_float(w[e]);
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float lo = DT == kF16 ? h2f(w[e] & 0xffffu) : bf2f(w[e] & 0xffffu);
            const float hi = DT == kF16 ? h2f(w[e] >> 16) : bf2f(w[e] >> 16);
            buf[pidx(k0 + 2 * e)] = lo;
            buf[pidx(k0 + 2 * e + 1)] = hi;
        }
    }
}

// Register stage of one chunk: VPT 16-byte vectors per thread.
template <int DT, int WG, int VPT>
struct Stage {
    uint4 v[VPT];
    __device__ __forceinline__ void load(const void* x, int64_t xoff, int n_bins, int p0, int nvec)
    {
        constexpr int V = Elem<DT>::kVec;
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            const int vi = u * WG + (int)threadIdx.x;
            if (vi < nvec) v[u] = load_raw<DT>(x, xoff + p0 + (int64_t)vi * V, xoff, xoff + n_bins);
        }
    }
    __device__ __forceinline__ void store(float* buf, int nvec) const
    {
        constexpr int V = Elem<DT>::kVec;
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
            const int vi = u * WG + (int)threadIdx.x;
            if (vi < nvec) store_raw<DT>(buf, vi * V, v[u]);
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

// --------------------------------------------------------------------------
// eq. (2)-(4): outputs indexed by the fundamental.
//
// A tile is the T = WG * R outputs [a, aend) of one spectrum; thread t holds
// outputs a + r WG + t (r < R) in registers: running sum, best SNR, best level
// and Greedy's offset j. Harmonic i is needed for the outputs
// n < floor(N / 2^level(i)) and reads positions i n (+ up to i - 1 bins of
// window for eq. (2) and (4)).
//
// The tile walks harmonic-major through a list of pieces built on the host:
// piece (i, [n0, n1)) stages the bins i n0 .. i (n1 - 1) + window, which fit
// one LDS buffer, and every output of the piece then adds its term. Each
// output thus adds its harmonics in the order i = 1..H of the equations; a
// level snapshot is taken when i is a power of two.
//
// Workgroup w serves the tiles of queue q = w % nq with stride G = grid / nq.
// The next piece -- of this tile or of the next one -- is loaded into
// registers while the current one is computed.
// --------------------------------------------------------------------------
template <int VAR, int DT, int WG, int R, int CB>
__global__ __launch_bounds__(WG) void k_hrms1d_fund(const Run1DParams p)
{
    constexpr int V = Elem<DT>::kVec;
    static_assert(CB % V == 0, "chunk must be a multiple of the vector");
    constexpr int NVEC = CB / V;
    constexpr int VPT = (NVEC + WG - 1) / WG;
    constexpr int BUF = VPT * WG * V;
    constexpr int T = WG * R;
    static_assert((WG & (WG - 1)) == 0, "WG must be a power of two");
    static_assert(T <= 0xffff, "tile offsets are 16-bit");
    constexpr int WSH = __builtin_ctz(WG);
    __shared__ float lds[BUF + (BUF >> 5) + 1];

    const int tid = (int)threadIdx.x;
    // Tile claims run two tiles ahead of use: s_claim[c & 1] is written when
    // tile c - 1 starts and read when tile c starts.
    __shared__ int s_claim[3];
    int cq = (int)(blockIdx.x % (unsigned)p.nqueues), visited = 0;
    if (tid == 0) {
        s_claim[2] = claim_tile(p, cq, visited);   // tile 0
        s_claim[1] = claim_tile(p, cq, visited);   // tile 1
        s_claim[0] = claim_tile(p, cq, visited);   // tile 2
    }
    __syncthreads();
    int t = uniform(s_claim[2]);
    if (t < 0) return;
    int tn = uniform(s_claim[1]);
    int c = 1;   // index of the tile that tn names

    TileRec ct = ldc(p.tiles + t);
    int pi = ct.pbeg, pe = ct.pbeg + ct.pcount;
    PieceRec cp = ldc(p.pieces + pi);
    TileRec ft = ct;   // record of tile tn, fetched a whole tile ahead of its use
    if (tn >= 0) ft = ldc(p.tiles + tn);

    float acc[R], best[R];
    int st[R];   // best level (bits 0..7) | Greedy offset j (bits 8..)
#pragma unroll
    for (int r = 0; r < R; ++r) {
        acc[r] = 0.0f;
        best[r] = 0.0f;
        st[r] = 0;
    }

    Stage<DT, WG, VPT> stage;
    stage.load(p.x, ct.xoff, ct.n, cp.p0, cp.nv);
    stage.store(lds, cp.nv);
    __syncthreads();
    for (;;) {
        // next piece: of this tile, else the first of the following tile
        const bool newtile = pi + 1 >= pe;
        const bool more = !newtile || tn >= 0;
        const TileRec& nt = newtile ? ft : ct;
        PieceRec np = cp;
        if (more) {
            np = ldc(p.pieces + (newtile ? nt.pbeg : pi + 1));
            stage.load(p.x, nt.xoff, nt.n, np.p0, np.nv);
        }

        // this piece
        {
            const int a = ct.a;
            const int i = cp.ih & 0xff;
            const int li = (cp.ih >> 8) & 0xff;
            const bool snap = (cp.ih >> 16) & 1;
            const int n0 = a + (cp.nr & 0xffff), n1 = a + (cp.nr >> 16);
            const int p0 = cp.p0;
            float m = 0.0f, qq = 0.0f, rh = 0.0f;
            int64_t ho = 0;
            if (snap) {
                const LevelConst c = ldc(p.consts + (int64_t)ct.spec * kMaxLevels + li);
                m = c.m;
                qq = c.q;
                rh = c.rh;
                ho = ldc(p.spec[ct.spec].hoff + li);
            }
            const int r0 = (n0 - a) >> WSH, r1 = (n1 - 1 - a) >> WSH;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (r >= r0 && r <= r1) {
                    const int n = a + (r << WSH) + tid;
                    if (n >= n0 && n < n1) {
                        const int k = i * n - p0;
                        float tv;
                        if constexpr (VAR == kFreqbin) {
                            tv = lds[pidx(k)];
                        } else if constexpr (VAR == kMax) {
                            tv = lds[pidx(k)];
                            for (int jj = 1; jj < i; ++jj) {
                                const float w = lds[pidx(k + jj)];
                                tv = w > tv ? w : tv;
                            }
                        } else {
                            if (i == 1) {
                                tv = lds[pidx(k)];
                            } else {
                                const int j = st[r] >> 8;
                                const float x0 = lds[pidx(k + j)];
                                const float x1 = lds[pidx(k + j + 1)];
                                if (x1 > x0) {
                                    tv = x1;
                                    st[r] += 256;
                                } else {
                                    tv = x0;
                                }
                            }
                        }
                        acc[r] = acc[r] + tv;
                        if (snap) {
                            const float hv = acc[r] * rh;
                            if (p.out_mask & 1u) p.h[ho + n] = hv;
                            const float snr = (hv - m) * qq;
                            if (li == 0 || snr > best[r]) {
                                best[r] = snr;
                                st[r] = (st[r] & ~255) | li;
                            }
                        }
                    }
                }
            }
        }

        if (newtile) {
            const int a = ct.a;
            const int aend = min(a + T, ct.n);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int n = a + (r << WSH) + tid;
                if (n < aend) {
                    if (p.out_mask & 2u) p.max_snr[ct.xoff + n] = best[r];
                    if (p.out_mask & 4u) p.best_h[ct.xoff + n] = (uint8_t)(1u << (st[r] & 255));
                }
                acc[r] = 0.0f;
                best[r] = 0.0f;
                st[r] = 0;
            }
        }
        if (!more) break;
        __syncthreads();   // every thread is done with this piece
        stage.store(lds, np.nv);
        __syncthreads();
        if (newtile) {
            t = tn;
            ct = ft;
            pe = ct.pbeg + ct.pcount;
            pi = ct.pbeg;
            ++c;
            tn = uniform(s_claim[c & 1]);
            if (tid == 0) s_claim[(c + 1) & 1] = claim_tile(p, cq, visited);
            if (tn >= 0) ft = ldc(p.tiles + tn);
        } else {
            ++pi;
        }
        cp = np;
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

constexpr int kBufferFlags = 0x00020000;   // raw (untyped) 32-bit buffer, gfx9 word 3

template <int DT, int WG, int R, int CB>
__global__ __launch_bounds__(WG) void k_hrms1d_eq1(const Run1DParams p)
{
    constexpr int T = WG * R;
    const int tid = (int)threadIdx.x;
    __shared__ int s_claim[2];
    int cq = (int)(blockIdx.x % (unsigned)p.nqueues), visited = 0;
    if (tid == 0) s_claim[0] = claim_tile(p, cq, visited);
    __syncthreads();
    int t = uniform(s_claim[0]);
    for (int c = 0; t >= 0; ++c) {
        // claim the following tile now; it is read after this tile's barrier
        if (tid == 0) s_claim[(c + 1) & 1] = claim_tile(p, cq, visited);
        const TileRec ct = ldc(p.tiles + t);
        const int a = ct.a;
        const int N = ct.n;
        const int nl = ct.nlev;
        const int aend = min(a + T, N);
        const int sh = nl - 1;
        const int Lh = 1 << sh;
        const unsigned half = (unsigned)Lh >> 1;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(static_cast<const char*>(p.x) + ct.xoff * Elem<DT>::kBytes), (short)0,
            N * Elem<DT>::kBytes, kBufferFlags);

        float acc[R][kMaxLevels];
        unsigned nn[R], tk[R];
        bool act[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int l = 0; l < kMaxLevels; ++l) acc[r][l] = 0.0f;
            const int n = a + r * WG + tid;
            act[r] = n < aend;
            nn[r] = act[r] ? (unsigned)n : (unsigned)a;
            tk[r] = half;   // n k + Lh/2 for k = 0
        }
        for (int k = 1; k <= Lh; ++k) {
            float v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                tk[r] += nn[r];
                // round(n k / Lh), halves up: floor((n k + Lh/2) / Lh)
                v[r] = buffer_elem<DT>(rs, (int)(tk[r] >> sh));
            }
            const int lmin = sh - __builtin_ctz((unsigned)k);
#pragma unroll
            for (int l = 0; l < kMaxLevels; ++l) {
                if (l >= lmin && l < nl) {
#pragma unroll
                    for (int r = 0; r < R; ++r) acc[r][l] = acc[r][l] + v[r];
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
#pragma unroll
        for (int l = 0; l < kMaxLevels; ++l) {
            if (l < nl) {
                const LevelConst c = ldc(p.consts + (int64_t)ct.spec * kMaxLevels + l);
                const int64_t ho = ldc(p.spec[ct.spec].hoff + l);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const float hv = acc[r][l] * c.rh;
                    if (act[r] && (p.out_mask & 1u)) p.h[ho + nn[r]] = hv;
                    const float snr = (hv - c.m) * c.q;
                    if (l == 0 || snr > best[r]) {
                        best[r] = snr;
                        bl[r] = l;
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (act[r]) {
                if (p.out_mask & 2u) p.max_snr[ct.xoff + nn[r]] = best[r];
                if (p.out_mask & 4u) p.best_h[ct.xoff + nn[r]] = (uint8_t)(1u << bl[r]);
            }
        }
        __syncthreads();
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

__global__ __launch_bounds__(64) void k_consts(const ConstsParams p)
{
    const int s = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (s == 0 && p.counters)
        for (int q = 0; q < kMaxQueues; ++q) p.counters[q] = 0u;
    if (s >= p.n_spec) return;
    const SpecDesc sd = p.spec[s];
    double mu, sigma;
    if (p.compute_stats) {
        double t1 = 0.0, t2 = 0.0;
        for (int g = p.seg_first[s]; g < p.seg_first[s + 1]; ++g) {
            t1 = t1 + p.partial[2 * (int64_t)g];
            t2 = t2 + p.partial[2 * (int64_t)g + 1];
        }
        const double nb = (double)sd.n;
        mu = t1 / nb;
        double var = t2 / nb - mu * mu;
        if (var < 0.0) var = 0.0;
        sigma = sqrt(var);
        p.stats[2 * (int64_t)s] = mu;
        p.stats[2 * (int64_t)s + 1] = sigma;
    } else {
        mu = p.stats[2 * (int64_t)s];
        sigma = p.stats[2 * (int64_t)s + 1];
    }
    for (int l = 0; l < kMaxLevels; ++l) {
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
// 2D frequency x fdot plane (freq-bin and Greedy). Output (m, z) of level H is
// the fundamental at frequency m whose H-th harmonic has fdot z; harmonic i
// reads row round(i z / H) (halves away from zero) at frequency i m (freq-bin)
// or i m + j (Greedy, j as in eq. (4)). Each level is summed on its own, in
// the order i = 1..H. A thread owns one output; a workgroup holds 64
// consecutive frequencies of kZRows fdot rows, the rows being the fastest grid
// dimension so that neighbouring workgroups read the same columns.
// --------------------------------------------------------------------------
constexpr int kZRows = 4;

__device__ __forceinline__ int row_of(int iz, int l)
{
    // round(iz / 2^l), halves away from zero
    const int H = 1 << l;
    return iz >= 0 ? (2 * iz + H) >> (l + 1) : -((-2 * iz + H) >> (l + 1));
}

template <int VAR, int DT>
__global__ __launch_bounds__(64 * kZRows) void k_hrms2d(const Run2DParams p)
{
    const int lane = (int)threadIdx.x & 63;
    const int zl = (int)threadIdx.x >> 6;
    const int zg = (int)(blockIdx.x % (unsigned)p.zgroups);
    const int mb = (int)(blockIdx.x / (unsigned)p.zgroups);
    const int rows = 2 * p.zmax + 1;
    const int r = zg * kZRows + zl;
    const int m = mb * 64 + lane;
    if (r >= rows || m >= p.nf) return;
    const int z = r - p.zmax;
    const int64_t ld = p.ld;
    float best = 0.0f;
    int bl = 0;
#pragma unroll
    for (int l = 0; l < kMaxLevels; ++l) {
        if (l < p.nlev && m < (p.nf >> l)) {
            const int H = 1 << l;
            float acc;
            if constexpr (VAR == kFreqbin) {
                acc = 0.0f;
#pragma unroll
                for (int i = 1; i <= (1 << (kMaxLevels - 1)); ++i) {
                    if (i <= H) {
                        const int row = row_of(i * z, l) + p.zmax;
                        acc = acc + load_scalar<DT>(p.x, (int64_t)row * ld + (int64_t)i * m);
                    }
                }
            } else {
                const int row1 = row_of(z, l) + p.zmax;
                acc = load_scalar<DT>(p.x, (int64_t)row1 * ld + m);
                int j = 0;
#pragma unroll
                for (int k = 2; k <= (1 << (kMaxLevels - 1)); ++k) {
                    if (k <= H) {
                        const int row = row_of(k * z, l) + p.zmax;
                        const int64_t base = (int64_t)row * ld + (int64_t)k * m + j;
                        const float x0 = load_scalar<DT>(p.x, base);
                        const float x1 = load_scalar<DT>(p.x, base + 1);
                        if (x1 > x0) {
                            acc = acc + x1;
                            j += 1;
                        } else {
                            acc = acc + x0;
                        }
                    }
                }
            }
            const LevelConst c = p.consts[l];
            const float hv = acc * c.rh;
            if (p.out_mask & 1u) p.h[p.hoff[l] + (int64_t)r * (p.nf >> l) + m] = hv;
            const float snr = (hv - c.m) * c.q;
            if (l == 0 || snr > best) {
                best = snr;
                bl = l;
            }
        }
    }
    const int64_t o = (int64_t)r * p.nf + m;
    if (p.out_mask & 2u) p.max_snr[o] = best;
    if (p.out_mask & 4u) p.best_h[o] = (uint8_t)(1u << bl);
}

// --------------------------------------------------------------------------
// Precision form: y = round_to_dtype(x * fl32(1 / mu)), round to nearest
// even; FP16 saturates at +-65504.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_quant_consts(const QuantConstParams p)
{
    const int s = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (s >= p.n_spec) return;
    double mu, sigma;
    if (p.compute_stats) {
        double t1 = 0.0, t2 = 0.0;
        for (int g = p.seg_first[s]; g < p.seg_first[s + 1]; ++g) {
            t1 = t1 + p.partial[2 * (int64_t)g];
            t2 = t2 + p.partial[2 * (int64_t)g + 1];
        }
        const double nb = (double)p.spec[s].n;
        mu = t1 / nb;
        double var = t2 / nb - mu * mu;
        if (var < 0.0) var = 0.0;
        sigma = sqrt(var);
        p.stats[2 * (int64_t)s] = mu;
        p.stats[2 * (int64_t)s + 1] = sigma;
    } else {
        mu = p.stats[2 * (int64_t)s];
        sigma = p.stats[2 * (int64_t)s + 1];
    }
    p.stats_out[2 * (int64_t)s] = 1.0;
    p.stats_out[2 * (int64_t)s + 1] = sigma / mu;
    p.inv_mu[s] = (float)(1.0 / mu);
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

template <int VAR, int DT, int WG, int R, int C>
void* fund_kernel()
{
    return reinterpret_cast<void*>(&k_hrms1d_fund<VAR, DT, WG, R, C>);
}

template <int DT, int WG, int R, int C>
void* eq1_kernel()
{
    return reinterpret_cast<void*>(&k_hrms1d_eq1<DT, WG, R, C>);
}

// Launch shapes compiled into the library: (threads, outputs per thread, LDS
// chunk in bins) for the fundamental-indexed family and for eq. (1).
struct ShapeEntry {
    int eq1;   // 1: eq. (1) kernel family, 0: eq. (2)-(4)
    int wg, r, chunk;
    void* (*k[3][3])();   // [variant slot][dtype]
};

template <int WG, int R, int CB>
constexpr ShapeEntry fund_shape()
{
    return ShapeEntry{0, WG, R, CB,
                      {{&fund_kernel<kMax, kF32, WG, R, CB>, &fund_kernel<kMax, kF16, WG, R, CB>,
                        &fund_kernel<kMax, kBF16, WG, R, CB>},
                       {&fund_kernel<kFreqbin, kF32, WG, R, CB>,
                        &fund_kernel<kFreqbin, kF16, WG, R, CB>,
                        &fund_kernel<kFreqbin, kBF16, WG, R, CB>},
                       {&fund_kernel<kGreedy, kF32, WG, R, CB>,
                        &fund_kernel<kGreedy, kF16, WG, R, CB>,
                        &fund_kernel<kGreedy, kBF16, WG, R, CB>}}};
}

template <int WG, int R, int CB>
constexpr ShapeEntry eq1_shape()
{
    return ShapeEntry{1, WG, R, CB,
                      {{&eq1_kernel<kF32, WG, R, CB>, &eq1_kernel<kF16, WG, R, CB>,
                        &eq1_kernel<kBF16, WG, R, CB>},
                       {nullptr, nullptr, nullptr},
                       {nullptr, nullptr, nullptr}}};
}

const ShapeEntry kShapes[] = {
    fund_shape<256, 8, 8192>(),
    fund_shape<256, 8, 4096>(),
    fund_shape<256, 16, 8192>(),
    fund_shape<512, 8, 8192>(),
    fund_shape<128, 16, 8192>(),
    eq1_shape<256, 8, 0>(),
    eq1_shape<256, 4, 0>(),
    eq1_shape<512, 8, 0>(),
};

const ShapeEntry* find_shape(int variant, const Shape1D& s)
{
    const int fam = variant == kEq1 ? 1 : 0;
    for (const ShapeEntry& e : kShapes)
        if (e.eq1 == fam && e.wg == s.wg && e.r == s.r && e.chunk == s.chunk) return &e;
    return nullptr;
}

void* kernel_for(int variant, int dtype, const Shape1D& s)
{
    if (dtype < 0 || dtype > 2 || variant < 0 || variant > 3) return nullptr;
    const ShapeEntry* e = find_shape(variant, s);
    if (!e) return nullptr;
    return variant == kEq1 ? e->k[0][dtype]() : e->k[variant - 1][dtype]();
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
    const int blocks = (p.n_spec + 63) / 64;
    hipLaunchKernelGGL(k_consts, dim3(blocks), dim3(64), 0, s, p);
    return hipGetLastError();
}

bool hrms1d_shape_supported(int variant, const Shape1D& shape)
{
    return kernel_for(variant, kF32, shape) != nullptr;
}

int hrms1d_shapes(int variant, Shape1D* out, int cap)
{
    const int fam = variant == kEq1 ? 1 : 0;
    int n = 0;
    for (const ShapeEntry& e : kShapes) {
        if (e.eq1 != fam) continue;
        if (out && n < cap) out[n] = Shape1D{e.wg, e.r, e.chunk};
        ++n;
    }
    return n;
}

int hrms1d_max_blocks_per_cu(int variant, int dtype, const Shape1D& shape)
{
    void* k = kernel_for(variant, dtype, shape);
    if (!k) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, shape.wg, 0) != hipSuccess) return 0;
    return nb;
}

hipError_t launch_hrms1d(int variant, int dtype, const Shape1D& shape, const Run1DParams& p,
                         int grid, hipStream_t s)
{
    void* k = kernel_for(variant, dtype, shape);
    if (!k) return hipErrorInvalidValue;
    if (grid <= 0) return hipSuccess;
    Run1DParams pc = p;
    void* args[] = {&pc};
    return hipLaunchKernel(k, dim3(grid), dim3(shape.wg), args, 0, s);
}

hipError_t launch_hrms2d(int variant, int dtype, const Run2DParams& p, hipStream_t s)
{
    const int64_t mblocks = ((int64_t)p.nf + 63) / 64;
    const int64_t blocks = mblocks * p.zgroups;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    dim3 grid((unsigned)blocks), block(64 * kZRows);
    if (variant == kFreqbin) {
        switch (dtype) {
        case kF32: hipLaunchKernelGGL((k_hrms2d<kFreqbin, kF32>), grid, block, 0, s, p); break;
        case kF16: hipLaunchKernelGGL((k_hrms2d<kFreqbin, kF16>), grid, block, 0, s, p); break;
        default: hipLaunchKernelGGL((k_hrms2d<kFreqbin, kBF16>), grid, block, 0, s, p); break;
        }
    } else if (variant == kGreedy) {
        switch (dtype) {
        case kF32: hipLaunchKernelGGL((k_hrms2d<kGreedy, kF32>), grid, block, 0, s, p); break;
        case kF16: hipLaunchKernelGGL((k_hrms2d<kGreedy, kF16>), grid, block, 0, s, p); break;
        default: hipLaunchKernelGGL((k_hrms2d<kGreedy, kBF16>), grid, block, 0, s, p); break;
        }
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_quant_consts(const QuantConstParams& p, hipStream_t s)
{
    hipLaunchKernelGGL(k_quant_consts, dim3((p.n_spec + 63) / 64), dim3(64), 0, s, p);
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
