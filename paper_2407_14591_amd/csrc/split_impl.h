// Split product Y = H X for a Q = 2 sector with a left/right view (LeftInfo):
// H = (left family) + (right family) + (bonds across the cut) + diagonal,
// each family acting on one side of the cut only (Sec. 4.4's bond sum, with
// the targets of every bond tabulated per side once per (sector, terms), in
// the spirit of the paper's cluster matrices, App. C).
//
// Three kernels per product, all bound by the gathers of X:
//  * split_diag_kernel: the diagonal of each side per configuration, from
//    this call's couplings and fields (count + rcount entries), and the
//    coupling factors of the call in the compute type;
//  * split_rows_kernel / split_rows_lds_kernel: one tile = 512 consecutive
//    offsets of one run (one left configuration), or (rows of at most 8 bytes
//    whose run fits LDS) one whole run staged in LDS.  The right family reads
//    its targets from a table per right configuration (16-bit offsets in the
//    run, 0xFFFF where the bond does not hop); a bond across the cut reads the
//    run of the left configuration with its left site flipped and the offset
//    of the right configuration with its right site flipped.  Adds the
//    diagonal, writes Y.
//  * split_cols_kernel: one tile = one cluster of left configurations at one
//    1 KiB chunk of their runs; the left family's targets are the same bytes
//    of other runs, listed once per left configuration and read with scalar
//    loads (the whole wave shares them), so every gather is one contiguous
//    1 KiB segment; targets inside the cluster come from LDS.  Adds into Y.
// Every gather is a buffer load bounded by its target run: a table entry that
// marks "no hop" (or any offset past the run) reads zero and touches nothing.
#pragma once

#include "hx_impl.h"

namespace dcs {
namespace sp {

using hx::Acc;

constexpr int kThreads = (int)kSplitRowTile;
constexpr uint32_t kOob = 0x80000000u;  // past every run: all record counts here are < 2^31
constexpr uint32_t kBufferWord3 = 0x00020000u;  // 32-bit data format, no swizzle

// Per-call coupling factors in the compute type, written by split_diag_kernel
// after the diagonal (one table per value type) and read with scalar loads.
constexpr int kAmpRight = 0;     // 1/2 Jxy of the right-family bonds (by position, 288 slots)
constexpr int kAmpCross = 288;   // 1/2 Jxy of the bonds across the cut (128 slots)
constexpr int kJzCross = 416;    // 1/4 Jz of the bonds across the cut (128 slots)
constexpr int kAmpBond = 544;    // 1/2 Jxy by bond index (256 slots)
constexpr int kAmpEntries = 1024;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             (int)kBufferWord3);
}

template <typename T, int K>
__device__ __forceinline__ Acc<T, K> buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    Acc<T, K> v;
    constexpr int B = K * (int)sizeof(T);
    if constexpr (B == 4) {
        const uint32_t u = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
        __builtin_memcpy(&v, &u, 4);
    } else if constexpr (B == 8) {
        const auto u = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        __builtin_memcpy(&v, &u, 8);
    } else {
#pragma unroll
        for (int i = 0; i < B / 16; ++i) {
            const auto u = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16u * i, 0, 0);
            __builtin_memcpy(reinterpret_cast<char *>(&v) + 16 * i, &u, 16);
        }
    }
    return v;
}

// Tables that no kernel writes, read through the constant address space so
// that loads at a wave-uniform index become scalar loads (and the buffer
// descriptors built from them stay scalar).
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;
template <typename T>
__device__ __forceinline__ cptr<T> ro(const T *p) {
    return (cptr<T>)p;
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Block (left particle number) of a tile.  The tiles one workgroup takes only
// increase (its XCD's queue counter), so the search resumes where it stopped and
// the block bounds stay in registers.
struct BlockCursor {
    const uint64_t *tbase;
    int m_count, mi;
    uint64_t hi;  // tbase[mi + 1]
    __device__ __forceinline__ BlockCursor(const uint64_t *tb, int mc) : tbase(tb), m_count(mc), mi(0) {
        hi = tbase[1];
    }
    __device__ __forceinline__ int operator()(uint64_t t) {
        while (t >= hi && mi + 1 < m_count) {
            ++mi;
            hi = tbase[mi + 1];
        }
        return mi;
    }
};

// ------------------------------------------------------------------ diagonal
struct DiagParams {
    const uint32_t *lwords, *rwords;
    const double *jxy, *jz, *h;
    double *out;
    double *amp64;  // kAmpEntries doubles, then kAmpEntries floats
    uint32_t count, rcount;
    int nD, nR, nX, nbonds;
    DiagTerm d[kMaxBonds + kMaxSites];
    uint16_t rbond[kMaxBonds];
    uint16_t xbond[kMaxCross];
};
static_assert(sizeof(DiagParams) <= 4096, "kernel arguments are limited to 4 KiB");

template <int Unused = 0>
__global__ __launch_bounds__(256) void split_diag_kernel(const DiagParams P_arg) {
    (void)P_arg;
    const DiagParams &P = kernel_arg0<DiagParams>();
    if (blockIdx.x == 0) {
        float *amp32 = reinterpret_cast<float *>(P.amp64 + kAmpEntries);
        for (int q = threadIdx.x; q < kAmpEntries; q += 256) {
            double v = 0.0;
            if (q < kAmpCross) {
                if (q - kAmpRight < P.nR) v = 0.5 * P.jxy[P.rbond[q - kAmpRight]];
            } else if (q < kJzCross) {
                if (q - kAmpCross < P.nX) v = 0.5 * P.jxy[P.xbond[q - kAmpCross]];
            } else if (q < kAmpBond) {
                if (q - kJzCross < P.nX) v = 0.25 * P.jz[P.xbond[q - kJzCross]];
            } else if (q - kAmpBond < P.nbonds) {
                v = 0.5 * P.jxy[q - kAmpBond];
            }
            P.amp64[q] = v;
            amp32[q] = (float)v;
        }
    }
    const uint32_t g = blockIdx.x * 256u + threadIdx.x;
    if (g >= P.count + P.rcount) return;
    const uint32_t side = g < P.count ? 0u : 1u;
    const uint32_t w = side ? P.rwords[g - P.count] : P.lwords[g];
    double d = 0.0;
    for (int q = 0; q < P.nD; ++q) {
        const DiagTerm t = P.d[q];
        if (t.side != side) continue;
        const uint32_t bi = (w >> t.bi) & 1u;
        if (t.is_field) {
            if (P.h) d += P.h[t.index] * ((double)bi - 0.5);
        } else {
            const double jz = 0.25 * P.jz[t.index];
            d += bi == ((w >> t.bj) & 1u) ? jz : -jz;
        }
    }
    P.out[g] = d;
}

// Per-XCD tile queue (as hx::next_tile) with the next tile claimed one tile
// ahead, so the latency of the claim overlaps the current tile's work.  Two
// LDS slots alternate: the slot written during tile i was last read during
// tile i-1, before the barrier that ends it.
struct AheadQueue {
    uint32_t *counters;
    uint64_t base, end;  // this XCD's tile range
    uint32_t *slot;      // LDS, 2 entries
    uint32_t xcd, it, pending;

    __device__ __forceinline__ AheadQueue(uint32_t *c, const uint64_t *xbase, uint32_t *lds)
        : counters(c), slot(lds), xcd(blockIdx.x & 7u), it(0), pending(0) {
        base = xbase[xcd];
        end = xbase[xcd + 1];
        if (threadIdx.x == 0) slot[0] = atomicAdd(counters + xcd, 1u);
        __syncthreads();
    }
    __device__ __forceinline__ bool get(uint64_t &t) {
        const uint64_t lt = slot[it & 1u];
        if (base + lt >= end) return false;
        t = uniform64(base + lt);
        if (threadIdx.x == 0) pending = atomicAdd(counters + xcd, 1u);
        return true;
    }
    __device__ __forceinline__ void finish() {
        if (threadIdx.x == 0) slot[(it + 1u) & 1u] = pending;
        ++it;
        __syncthreads();
    }
};

// Tile ranges of the 8 XCDs: equal counts, or (weights given) equal sums of weight.
inline void xcd_ranges(uint64_t tiles, uint64_t *xbase) {
    const uint64_t per = (tiles + 7) / 8;
    for (int x = 0; x <= 8; ++x) xbase[x] = std::min<uint64_t>(tiles, (uint64_t)x * per);
}

// ------------------------------------------------------------------ rows
struct RowParams {
    const void *x;
    void *y;
    const void *amp;  // coupling factors of the compute type (kAmp* layout)
    const uint32_t *lwords, *rwords;
    const uint64_t *runs, *xl;
    const uint16_t *vo, *xo;
    const double *dl, *dr;
    const uint32_t *lptr;  // left family (the fused form): entries of every left configuration
    const uint64_t *lrun;  // bond << 48 | run start of the target
    const uint32_t *order;  // if not NULL: tile t is left configuration order[t] >> 8, chunk & 0xFF
    uint32_t *counters;
    uint64_t xbase[9];  // tile range of every XCD
    uint32_t count, rcount;
    int m_count, nR, nX;
    int nRloc;        // right-family bonds [0, nRloc) read from the staged rows of the tile
    uint32_t margin;  // staged rows on either side of the tile
    uint32_t lbase[kMaxLeftM], rbase[kMaxLeftM], ncols[kMaxLeftM], nsub[kMaxLeftM];
    uint64_t tbase[kMaxLeftM + 1];
    uint16_t rbond[kMaxBonds];
    CrossBond xb[kMaxCross];
    // adjoint (ADJ): the product is of g (x above); xprim is the primal vector x and
    // part receives per-tile sums [value][tile] (kAdjRowValues values, one tile per run)
    const void *xprim;
    double *part;
    float *dots;  // ADJ blocks: sum_c x_s,c g_s,c per row (row order of the sector), or NULL
    uint32_t part_n;
    int nJs;
    uint8_t jbit[8];  // bit of crossing right-site slot j in a packed right word
};
static_assert(sizeof(RowParams) <= 4096, "kernel arguments are limited to 4 KiB");

// Values of one run's tile in the adjoint row pass: sum_s x_s g_t over the hops of
// right-family bonds 0..31 and bonds across the cut 0..7, then sum_s x_s g_s, then
// sum_s (2 b_j(s) - 1) x_s g_s for crossing right-site slots 0..3.
constexpr int kAdjR = 32, kAdjX = 8, kAdjJ = 4;
static_assert(kAdjX == 8 && 1 + kAdjJ <= 8, "the row pass flushes these values in groups of 8");
constexpr int kAdjRowValues = kAdjR + kAdjX + 1 + kAdjJ;

// Gathers in flight per batch, sized for about 96 registers of gathered data:
// every gather is one whole row of K values (RB bytes, one to four 16-byte loads).
// Rows of 32 bytes and more take the bonds across the cut one at a time (4% less
// time than batches of four for k = 8 FP32, measured).
template <typename T, int K>
struct RowBatch {
    static constexpr uint32_t RB = K * sizeof(T);
    static constexpr int R = RB <= 8 ? 32 : (RB == 16 ? 16 : 8);  // right family, whole table rows
    static constexpr int X = RB <= 16 ? 8 : 1;                    // across the cut
};

// Row sums of 16 FP32 values of every lane at once (as hx::row_transpose_sum, on
// 32-bit moves): lane i of each 16-lane row ends with the row's total of v[i];
// then the four rows are added.  Fixed order (deterministic).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int H, int CTRL>
__device__ __forceinline__ void half_step_f(float (&v)[16], bool upper) {
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const float lo = v[k], hi = v[k + H];
        v[k] = (upper ? hi : lo) + dpp_f<CTRL>(upper ? lo : hi);
    }
}
__device__ __forceinline__ float wave_transpose_sum16f(float (&v)[16]) {
    const int l = threadIdx.x & 15;
    half_step_f<8, 0x140>(v, l & 8);  // row_mirror
    half_step_f<4, 0x141>(v, l & 4);  // row_half_mirror
    half_step_f<2, 0x1B>(v, l & 2);   // quad_perm [3,2,1,0]
    half_step_f<1, 0xB1>(v, l & 1);   // quad_perm [1,0,3,2]
    float s = v[0];
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    return s;
}
// The same for 8 values: lane i of each 8-lane group ends with the group's total
// of v[i & 7], then the two groups of a row, then the four rows are added.
template <int H, int CTRL>
__device__ __forceinline__ void half_step_f8(float (&v)[8], bool upper) {
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const float lo = v[k], hi = v[k + H];
        v[k] = (upper ? hi : lo) + dpp_f<CTRL>(upper ? lo : hi);
    }
}
__device__ __forceinline__ float wave_transpose_sum8f(float (&v)[8]) {
    const int l = threadIdx.x & 7;
    half_step_f8<4, 0x141>(v, l & 4);  // row_half_mirror
    half_step_f8<2, 0x1B>(v, l & 2);   // quad_perm [3,2,1,0]
    half_step_f8<1, 0xB1>(v, l & 1);   // quad_perm [1,0,3,2]
    float s = v[0];
    s += dpp_f<0x128>(s);  // row_ror:8, the other 8-lane group of the row
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    return s;
}

// Entries of the target tables' 16-byte rows: eight 16-bit offsets (runs below
// 65,535 rows; 0xFFFF: no hop), or, for longer runs (W32), four 32-bit ones
// (0xFFFFFFFF: no hop).  byte(): the entry as a byte offset into the run, an
// offset past every run for "no hop".
template <bool W32>
struct OffRow {
    static constexpr int PER = W32 ? 4 : 8;
    static constexpr uint32_t NOHOP = W32 ? 0xFFFFFFFFu : 0xFFFFu;
    static __device__ __forceinline__ uint32_t get(const uint4 &t, int u) {
        if constexpr (W32) {
            return u == 0 ? t.x : (u == 1 ? t.y : (u == 2 ? t.z : t.w));
        } else {
            const int h = u >> 1;
            const uint32_t w = h == 0 ? t.x : (h == 1 ? t.y : (h == 2 ? t.z : t.w));
            return (u & 1) ? (w >> 16) : (w & 0xFFFFu);
        }
    }
    template <uint32_t RB>
    static __device__ __forceinline__ uint32_t byte(uint32_t off) {
        if constexpr (W32) return off == NOHOP ? kOob : off * RB;
        else return off * RB;  // 0xFFFF * RB lies past every run of fewer than 0xFFFF rows
    }
    template <uint32_t RB>
    static __device__ __forceinline__ bool hop(uint32_t ob) {
        if constexpr (W32) return ob < kOob;
        else return ob < 0xFFFFu * RB;
    }
};

// Rows of x staged in LDS per tile: the tile's rows and `margin` rows on either
// side (bonds inside the last subsystem never leave that window), then one zero
// row.  Dwords, or 16-byte pieces when rows are whole 16-byte units.
template <typename T, int K>
__device__ __forceinline__ void stage_rows(char *lds, const T *x, uint64_t R, uint32_t s0, uint32_t s1,
                                           uint32_t zero_row) {
    constexpr uint32_t RB = K * sizeof(T);
    const auto rs = rsrc(x + (R + s0) * K, (s1 - s0) * RB);
    const uint32_t bytes = (s1 - s0) * RB;
    if constexpr (RB % 16 == 0) {
        uint4 *d = reinterpret_cast<uint4 *>(lds);
        for (uint32_t i = threadIdx.x; i < bytes / 16; i += kThreads) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, i * 16u, 0, 0);
            __builtin_memcpy(&d[i], &v, 16);
        }
    } else {
        uint32_t *d = reinterpret_cast<uint32_t *>(lds);
        for (uint32_t i = threadIdx.x; i < bytes / 4; i += kThreads)
            d[i] = __builtin_amdgcn_raw_buffer_load_b32(rs, i * 4u, 0, 0);
    }
    if (threadIdx.x < RB / 4) reinterpret_cast<uint32_t *>(lds + (size_t)zero_row * RB)[threadIdx.x] = 0u;
}

template <typename T, int K>
__device__ __forceinline__ Acc<T, K> lds_row(const char *lds, uint32_t row) {
    Acc<T, K> v;
    __builtin_memcpy(&v, lds + (size_t)row * (K * sizeof(T)), K * sizeof(T));
    return v;
}

// LEFT: the pass also applies the left family (the fused form, no column pass):
// a left bond maps the tile's run onto another run of the same block, row r onto
// row r, so its gathers are contiguous across the wave.
// ADJ (FP32 blocks of K columns, the adjoint's way 2): the product is y = H g (x is
// g); each hop also adds sum_c x_s,c g_t,c to its bond's value, and the row adds
// its sum_c x_s,c g_s,c to the diagonal values (as the staged-run adjoint pass, see
// there), summed over the wave (FP32) into per-wave FP64 slots; at the end of the
// tile the slots go, in wave order, to P.part[value][tile in run order].  The row's
// sum_c x_s,c g_s,c also goes to P.dots[row] (the per-right-configuration sums read
// it there instead of re-reading both blocks).
template <typename T, int K, bool LEFT, bool W32 = false, bool ADJ = false>
__global__ __launch_bounds__(kThreads, ADJ ? 4 : 2) void split_rows_kernel(const RowParams P_arg) {
    (void)P_arg;
    const RowParams &P = kernel_arg0<RowParams>();
    using B = RowBatch<T, K>;
    using OR = OffRow<W32>;
    static_assert(!ADJ || (!LEFT && sizeof(T) == 4), "the adjoint row pass: FP32, no fused left family");
    __shared__ double red[ADJ ? (kThreads / 64) * 64 : 1];
    const uint32_t wave_id = threadIdx.x >> 6, lane_id = threadIdx.x & 63u;
    auto flush16 = [&](float (&v)[16], int base) {
        const float tsum = wave_transpose_sum16f(v);
        if (lane_id < 16) red[wave_id * 64 + base + lane_id] += (double)tsum;
    };
    auto flush8 = [&](float (&v)[8], int base) {
        const float tsum = wave_transpose_sum8f(v);
        if (lane_id < 8) red[wave_id * 64 + base + lane_id] += (double)tsum;
    };
    static_assert(B::R % OR::PER == 0, "whole table rows per batch");
    const char *vob = reinterpret_cast<const char *>(P.vo);
    const char *xob = reinterpret_cast<const char *>(P.xo);
    constexpr uint32_t RB = B::RB;
    extern __shared__ __align__(16) char rows_lds[];
    __shared__ T ramp[kAmpCross - kAmpRight];
    __shared__ T xamp[kJzCross - kAmpCross], xjz[kAmpBond - kJzCross];
    __shared__ T lamp[LEFT ? kMaxBonds : 1];
    __shared__ uint32_t slots[2];
    {
        const T *A = reinterpret_cast<const T *>(P.amp);
        for (int q = threadIdx.x; q < kAmpBond; q += kThreads) {
            const T v = A[q];
            if (q < kAmpCross)
                ramp[q] = v;
            else if (q < kJzCross)
                xamp[q - kAmpCross] = v;
            else
                xjz[q - kJzCross] = v;
        }
        if constexpr (LEFT)
            for (int q = threadIdx.x; q < kMaxBonds; q += kThreads) lamp[q] = A[kAmpBond + q];
    }
    const T *__restrict__ x = reinterpret_cast<const T *>(P.x);
    T *__restrict__ y = reinterpret_cast<T *>(P.y);
    const int nRq = (P.nR + OR::PER - 1) / OR::PER;
    AheadQueue Q(P.counters, P.xbase, slots);  // its barrier also publishes the LDS above
    BlockCursor blk(P.tbase, P.m_count);
    uint64_t t;
    while (Q.get(t)) {
        int mi;
        uint32_t gl, ch;
        if (P.order) {  // uniform
            const uint32_t e = ro(P.order)[t];
            gl = e >> 8;
            ch = e & 0xFFu;
            mi = 0;
            while (mi + 1 < P.m_count && gl >= P.lbase[mi + 1]) ++mi;
        } else {
            mi = blk(t);
            const uint32_t local = (uint32_t)(t - P.tbase[mi]);
            const uint32_t lq = local / P.nsub[mi];
            ch = local - lq * P.nsub[mi];
            gl = P.lbase[mi] + lq;
        }
        const uint32_t ncols = P.ncols[mi];
        const uint32_t r = ch * kThreads + threadIdx.x;
        const bool active = r < ncols;
        const uint32_t gr = P.rbase[mi] + (active ? r : 0u);
        const uint64_t R = ro(P.runs)[gl];
        // ADJ: the primal row (zero past the run) and this wave's slots
        Acc<T, K> xo;
        if constexpr (ADJ) {
            xo = buf_load<T, K>(rsrc(reinterpret_cast<const T *>(P.xprim) + R * K, ncols * B::RB), r * B::RB);
            red[wave_id * 64 + lane_id] = 0.0;
        }
        auto dotx = [&](const Acc<T, K> &v) -> float {
            float d = 0.f;
#pragma unroll
            for (int c = 0; c < K; ++c) d += (float)xo.v[c] * (float)v.v[c];
            return d;
        };
        const uint32_t lw = ro(P.lwords)[gl];
        const double dl = ro(P.dl)[gl];
        const auto rs = rsrc(x + R * K, ncols * RB);
        const uint32_t rw = P.rwords[gr];
        const double dr = P.dr[gr];
        // table rows of this tile's rows, loaded before anything waits
        uint4 tv0[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            tv0[i] = i < nRq ? *reinterpret_cast<const uint4 *>(vob + ((size_t)i * P.rcount + gr) * 16)
                             : make_uint4(~0u, ~0u, ~0u, ~0u);
        const uint4 xw0 = P.nX > 0 ? *reinterpret_cast<const uint4 *>(xob + (size_t)gr * 16)
                                   : make_uint4(~0u, ~0u, ~0u, ~0u);
        // the tile's window of the run in LDS (when bonds inside the last subsystem exist)
        const bool staged = P.nRloc > 0;
        const uint32_t r0 = ch * kThreads;
        const uint32_t s0 = r0 > P.margin ? r0 - P.margin : 0u;
        const uint32_t s1 = min(ncols, r0 + kThreads + P.margin);
        const uint32_t zero_row = kThreads + 2 * P.margin;
        if (staged) {
            stage_rows<T, K>(rows_lds, x, R, s0, s1, zero_row);
            __syncthreads();
        }
        auto load_xs = [&]() {
            return staged ? lds_row<T, K>(rows_lds, active ? r - s0 : zero_row)
                          : buf_load<T, K>(rs, r * RB);  // past the run: zero
        };
        Acc<T, K> xs;
        if constexpr (!ADJ) xs = load_xs();  // ADJ: after the gathers (registers)
        Acc<T, K> acc;
#pragma unroll
        for (int c = 0; c < K; ++c) acc.v[c] = (T)0;
        // bonds across the cut: B::X per batch
        T diag = (T)(dl + dr);
        uint4 xw = xw0;
        int xw_group = 0;
        float px[kAdjX];  // ADJ: cross-cut hop values
#pragma unroll
        for (int q = 0; q < kAdjX; ++q) px[q] = 0.f;
        for (int x0 = 0; x0 < P.nX; x0 += B::X) {
            Acc<T, K> xv[B::X];
            bool hop[B::X];
#pragma unroll
            for (int u = 0; u < B::X; ++u) {
                const bool ok = x0 + u < P.nX;
                const CrossBond cb = P.xb[ok ? x0 + u : 0];
                const uint32_t bi = (lw >> cb.lbit) & 1u;
                const uint64_t Rx = ok ? ro(P.xl)[(size_t)cb.si * P.count + gl] : ~0ull;
                int mx = mi + (bi ? -1 : 1);
                mx = mx < 0 ? 0 : (mx >= P.m_count ? P.m_count - 1 : mx);
                const bool valid = Rx != ~0ull;
                const auto rx = rsrc(x + (valid ? Rx : 0ull) * K, valid ? P.ncols[mx] * RB : 0u);
                if ((int)(cb.sj / OR::PER) != xw_group) {  // uniform: table row of this site group
                    xw_group = cb.sj / OR::PER;
                    xw = *reinterpret_cast<const uint4 *>(xob + ((size_t)xw_group * P.rcount + gr) * 16);
                }
                const uint32_t xo = OR::get(xw, cb.sj % OR::PER);
                hop[u] = ok && bi != ((rw >> cb.rbit) & 1u);
                if (__builtin_amdgcn_ballot_w64(active && hop[u])) {
                    xv[u] = buf_load<T, K>(rx, hop[u] ? xo * RB : kOob);
                } else {
#pragma unroll
                    for (int c = 0; c < K; ++c) xv[u].v[c] = (T)0;
                }
            }
#pragma unroll
            for (int u = 0; u < B::X; ++u) {
                hx::fma_acc<T, K>(acc, xamp[x0 + u], xv[u]);
                diag += hop[u] ? -xjz[x0 + u] : xjz[x0 + u];
                if constexpr (ADJ) {
#pragma unroll
                    for (int q = 0; q < kAdjX; ++q)
                        if (q == x0 + u) px[q] = dotx(xv[u]);
                }
            }
        }
        if constexpr (ADJ) flush8(px, kAdjR);
        // right family: B::R targets per batch, OR::PER per 16-byte table row; bonds
        // [0, nRloc) from the staged window, the others from the run in HBM.  The
        // first four table rows were loaded at the start of the tile.
        for (int q0 = 0; q0 < nRq * OR::PER; q0 += B::R) {
            uint32_t ov[B::R];
#pragma unroll
            for (int i = 0; i < B::R / OR::PER; ++i) {
                const int qr = q0 / OR::PER + i;
                uint4 tv = make_uint4(~0u, ~0u, ~0u, ~0u);
                if (qr < 4) {
#pragma unroll
                    for (int z = 0; z < 4; ++z)
                        if (z == qr) tv = tv0[z];
                } else if (qr < nRq) {
                    tv = *reinterpret_cast<const uint4 *>(vob + ((size_t)qr * P.rcount + gr) * 16);
                }
#pragma unroll
                for (int u = 0; u < OR::PER; ++u) ov[i * OR::PER + u] = OR::template byte<RB>(OR::get(tv, u));
            }
            // a bond with no hop on any lane of the wave (frequent for bonds inside
            // the first right subsystem, whose hops are shared by runs of rows) is skipped
            Acc<T, K> xv[B::R];
#pragma unroll
            for (int u = 0; u < B::R; ++u) {
                if (q0 + u < P.nRloc) {
                    const uint32_t e = ov[u] / RB;
                    const uint32_t wr = (e < s0 || e >= s1) ? zero_row : e - s0;  // no hop: past s1
                    xv[u] = lds_row<T, K>(rows_lds, wr);
                } else if (__builtin_amdgcn_ballot_w64(active && OR::template hop<RB>(ov[u]))) {
                    xv[u] = buf_load<T, K>(rs, ov[u]);
                } else {
#pragma unroll
                    for (int c = 0; c < K; ++c) xv[u].v[c] = (T)0;
                }
            }
#pragma unroll
            for (int u = 0; u < B::R; ++u) hx::fma_acc<T, K>(acc, ramp[q0 + u], xv[u]);
            if constexpr (ADJ) {  // right-family hop values, 16 (or 8) bonds per flush (bonds < kAdjR)
                if constexpr (B::R >= 16) {
#pragma unroll
                    for (int h = 0; h < B::R; h += 16) {
                        float pv[16];
#pragma unroll
                        for (int u = 0; u < 16; ++u) pv[u] = dotx(xv[h + u]);
                        flush16(pv, q0 + h);
                    }
                } else {
                    float pv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) pv[u] = dotx(xv[u]);
                    flush8(pv, q0);
                }
            }
        }
        if constexpr (LEFT) {
            // left family: B::R target runs per batch (wave-uniform list), row r of each;
            // lanes past the run end read zeros
            const uint32_t q1 = ro(P.lptr)[gl + 1];
            for (uint32_t q0 = ro(P.lptr)[gl]; q0 < q1; q0 += B::R) {
                Acc<T, K> xv[B::R];
                T a[B::R];
#pragma unroll
                for (int u = 0; u < B::R; ++u) {
                    const bool ok = q0 + u < q1;  // uniform
                    const uint64_t e = ro(P.lrun)[ok ? q0 + u : q0];
                    const auto rl = rsrc(x + (e & 0xFFFFFFFFFFFFull) * K, ok ? ncols * RB : 0u);
                    xv[u] = buf_load<T, K>(rl, r * RB);
                    a[u] = ok ? lamp[(e >> 48) & 0xFFu] : (T)0;
                }
#pragma unroll
                for (int u = 0; u < B::R; ++u) hx::fma_acc<T, K>(acc, a[u], xv[u]);
            }
        }
        if constexpr (ADJ) xs = load_xs();
        if (active) {
            T *yr = y + (R + r) * K;
#pragma unroll
            for (int c = 0; c < K; ++c) __builtin_nontemporal_store(acc.v[c] + diag * xs.v[c], yr + c);
        }
        if constexpr (ADJ) {
            // the diagonal values: sum_c x_s,c g_s,c, and its signs by crossing right site
            const float pg = dotx(xs);
            if (P.dots && active) __builtin_nontemporal_store(pg, P.dots + R + r);
            float pd[8];
            pd[0] = pg;
#pragma unroll
            for (int j = 0; j < kAdjJ; ++j) pd[1 + j] = j < P.nJs ? (((rw >> P.jbit[j]) & 1u) ? pg : -pg) : 0.f;
#pragma unroll
            for (int j = 1 + kAdjJ; j < 8; ++j) pd[j] = 0.f;
            flush8(pd, kAdjR + kAdjX);
            // the tile's values: the waves' slots added in wave order, at the tile's
            // place in run order (its run's tiles are consecutive there)
            __syncthreads();
            if ((int)threadIdx.x < kAdjRowValues) {
                double tot = 0.0;
                for (int w = 0; w < kThreads / 64; ++w) tot += red[w * 64 + threadIdx.x];
                const uint64_t tr = P.tbase[mi] + (uint64_t)(gl - P.lbase[mi]) * P.nsub[mi] + ch;
                P.part[(size_t)threadIdx.x * P.part_n + tr] = tot;
            }
        }
        Q.finish();  // its barrier also ends the reads of red
    }
}

// Rows kernel with the run of X staged in LDS (rows of at most 8 bytes and runs
// that fit): one tile = one left configuration's whole run.  The right family
// (and the diagonal) read the staged run; entry ncols of the staged run is
// zero and stands for "no hop".  Bonds across the cut gather from HBM as above.
constexpr uint32_t kRowLdsMax = 112 * 1024;

// Per-lane table data of one chunk of a run (loaded one chunk ahead).
struct ChunkIdx {
    uint4 tv[4];   // right-family targets of the first 32 bonds
    uint4 xw;      // flipped-right-site offsets of the first 8 site slots
    uint32_t rw;   // packed right word
    double dr;     // right diagonal
};

__device__ __forceinline__ ChunkIdx load_chunk_idx(const RowParams &P, int mi, uint32_t r, uint32_t ncols,
                                                   int nRq) {
    ChunkIdx c;
    const uint32_t gr = P.rbase[mi] + (r < ncols ? r : 0u);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        c.tv[i] = i < nRq ? *reinterpret_cast<const uint4 *>(P.vo + ((size_t)i * P.rcount + gr) * 8)
                          : make_uint4(~0u, ~0u, ~0u, ~0u);
    c.xw = P.nX > 0 ? *reinterpret_cast<const uint4 *>(P.xo + (size_t)gr * 8) : make_uint4(~0u, ~0u, ~0u, ~0u);
    c.rw = P.rwords[gr];
    c.dr = P.dr[gr];
    return c;
}

__device__ __forceinline__ uint32_t u16_of(const uint4 &v, uint32_t i) {  // i uniform, < 8
    const uint32_t w = (i >> 1) == 0 ? v.x : ((i >> 1) == 1 ? v.y : ((i >> 1) == 2 ? v.z : v.w));
    return (i & 1u) ? (w >> 16) : (w & 0xFFFFu);
}

// Threads per workgroup of the staged-run pass: 512 for 4-byte rows (three runs
// fit one CU's LDS), 1024 for 8-byte rows (one run per CU, shared by 16 waves).
template <typename T, int K>
constexpr int lds_rows_threads() {
    return K * sizeof(T) == 4 ? 512 : 1024;
}

// ADJ (k = 1): the product is y = H g (x is g); the pass also forms, per run, the
// values of kAdjRowValues (hop sums of right-family and cross-cut bonds with the
// primal vector at the row, and the diagonal sums) and writes them to P.part.
template <typename T, int K, bool ADJ>
__device__ __forceinline__ void rows_lds_body(const RowParams &P) {
    using V = Acc<T, K>;
    constexpr uint32_t RB = K * sizeof(T);
    static_assert(RB <= 8, "staged runs hold rows of at most 8 bytes");
    constexpr int NT = lds_rows_threads<T, K>();
    constexpr int XF = 32;  // bonds across the cut whose gather descriptors are set up once per run
    constexpr int XB = 2;   // of those, gathers in flight per batch (1, 4 and 8 measured slower)
    extern __shared__ __align__(16) char dyn[];
    V *xr = reinterpret_cast<V *>(dyn);
    __shared__ uint4 xinfo[XF];  // per bond across the cut: run base (lo, hi), bytes | bit << 31
    __shared__ uint32_t slots[2];
    __shared__ double red[ADJ ? (NT / 64) * 64 : 1];  // ADJ: per-wave sums of the run's values
    static_assert(!ADJ || K == 1, "the adjoint row pass takes one column");
    const cptr<T> A = ro(reinterpret_cast<const T *>(P.amp));
    const cptr<T> ramp = A + kAmpRight, xamp = A + kAmpCross, xjz = A + kJzCross;
    const T *__restrict__ x = reinterpret_cast<const T *>(P.x);
    T *__restrict__ y = reinterpret_cast<T *>(P.y);
    const int nRq = (P.nR + 7) >> 3;
    AheadQueue Q(P.counters, P.xbase, slots);
    BlockCursor blk(P.tbase, P.m_count);
    uint64_t t;
    while (Q.get(t)) {
        const int mi = blk(t);
        const uint32_t gl = (uint32_t)t;  // tiles enumerate the left configurations
        const uint32_t ncols = P.ncols[mi];
        const uint64_t R = ro(P.runs)[gl];
        const uint32_t lw = ro(P.lwords)[gl];
        const double dl = ro(P.dl)[gl];
        const uint32_t bytes = ncols * RB;
        // gather descriptors of the first XF bonds across the cut, one lane per bond
        const int nXF = P.nX < XF ? P.nX : XF;
        if ((int)threadIdx.x < nXF) {
            const CrossBond cb = P.xb[threadIdx.x];
            const uint32_t b0 = (lw >> cb.lbit) & 1u;
            const uint64_t Rx = ro(P.xl)[(size_t)cb.si * P.count + gl];
            int mx = mi + (b0 ? -1 : 1);
            mx = mx < 0 ? 0 : (mx >= P.m_count ? P.m_count - 1 : mx);
            const bool valid = Rx != ~0ull;
            const uint64_t base = reinterpret_cast<uint64_t>(x + (valid ? Rx : 0ull) * K);
            xinfo[threadIdx.x] = make_uint4((uint32_t)base, (uint32_t)(base >> 32),
                                            (valid ? P.ncols[mx] * RB : 0u) | (b0 << 31), 0u);
        }
        // stage the run: 16-byte pieces, then the last few 4-byte words; entry ncols is zero
        {
            const auto rs = rsrc(x + R * K, bytes);
            uint4 *d16 = reinterpret_cast<uint4 *>(dyn);
            for (uint32_t i = threadIdx.x; i < bytes / 16; i += NT) {
                const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, i * 16u, 0, 0);
                __builtin_memcpy(&d16[i], &v, 16);
            }
            uint32_t *d4 = reinterpret_cast<uint32_t *>(dyn);
            const uint32_t w0 = (bytes / 16) * 4;
            if (threadIdx.x < (bytes / 4) - w0)
                d4[w0 + threadIdx.x] = __builtin_amdgcn_raw_buffer_load_b32(rs, (w0 + threadIdx.x) * 4u, 0, 0);
            if (threadIdx.x == 0) {
#pragma unroll
                for (int c = 0; c < K; ++c) xr[ncols].v[c] = (T)0;
            }
        }
        ChunkIdx cur = load_chunk_idx(P, mi, threadIdx.x, ncols, nRq);
        const T *__restrict__ xp = reinterpret_cast<const T *>(P.xprim);
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        if constexpr (ADJ) red[wave * 64 + lane] = 0.0;  // this wave's slots (one writing lane each)
        // ADJ: the pass's values of 16 at a time, summed over the wave (FP32) and added
        // to the wave's FP64 slots (slot base + i written by lane i)
        auto flush16 = [&](float (&v)[16], int base) {
            const float tsum = wave_transpose_sum16f(v);
            if (lane < 16) red[wave * 64 + base + lane] += (double)tsum;
        };
        __syncthreads();
        for (uint32_t c0 = 0; c0 < ncols; c0 += NT) {
            const uint32_t r = c0 + threadIdx.x;
            const bool active = r < ncols;
            ChunkIdx nxt = cur;  // the adjoint variant loads it at the end of the pass (registers)
            if constexpr (!ADJ)
                if (c0 + NT < ncols) nxt = load_chunk_idx(P, mi, r + NT, ncols, nRq);
            V acc;
#pragma unroll
            for (int c = 0; c < K; ++c) acc.v[c] = (T)0;
            float xo_own = 0.f;  // ADJ: the primal vector at this row (0 past the run)
            if constexpr (ADJ) xo_own = active ? (float)xp[R + r] : 0.f;
            // right family from the staged run
#pragma unroll
            for (int i2 = 0; i2 < 2; ++i2) {
                float pv[16];
#pragma unroll
                for (int i = 2 * i2; i < 2 * i2 + 2; ++i) {
                    const uint32_t wv[4] = {cur.tv[i].x, cur.tv[i].y, cur.tv[i].z, cur.tv[i].w};
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const uint32_t e = (u & 1) ? (wv[u >> 1] >> 16) : (wv[u >> 1] & 0xFFFFu);
                        const V gv = xr[e < ncols ? e : ncols];
                        hx::fma_acc<T, K>(acc, ramp[i * 8 + u], gv);
                        if constexpr (ADJ) pv[(i - 2 * i2) * 8 + u] = xo_own * (float)gv.v[0];
                    }
                }
                if constexpr (ADJ) flush16(pv, 16 * i2);
            }
            if (nRq > 4) {  // more than 32 right-family bonds
                const uint32_t gr = P.rbase[mi] + (active ? r : 0u);
                for (int qr = 4; qr < nRq; ++qr) {
                    const uint4 tv = *reinterpret_cast<const uint4 *>(P.vo + ((size_t)qr * P.rcount + gr) * 8);
                    const uint32_t wv[4] = {tv.x, tv.y, tv.z, tv.w};
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const uint32_t e = (u & 1) ? (wv[u >> 1] >> 16) : (wv[u >> 1] & 0xFFFFu);
                        hx::fma_acc<T, K>(acc, ramp[qr * 8 + u], xr[e < ncols ? e : ncols]);
                    }
                }
            }
            // bonds across the cut
            T diag = (T)(dl + cur.dr);
            float px[16];  // ADJ: cross-cut hop sums, then the diagonal sums
#pragma unroll
            for (int q = 0; q < 16; ++q) px[q] = 0.f;
            if constexpr (ADJ) {  // at most kAdjX bonds, each with its own sum
#pragma unroll
                for (int q = 0; q < kAdjX; ++q) {
                    if (q < P.nX) {  // uniform
                        const CrossBond cb = P.xb[q];
                        const uint4 info = xinfo[q];
                        const uint32_t lo = __builtin_amdgcn_readfirstlane(info.x);
                        const uint32_t hi = __builtin_amdgcn_readfirstlane(info.y);
                        const uint32_t nb = __builtin_amdgcn_readfirstlane(info.z);
                        const auto rr = rsrc(reinterpret_cast<const void *>(((uint64_t)hi << 32) | lo),
                                             nb & 0x7FFFFFFFu);
                        const uint32_t xo = u16_of(cur.xw, cb.sj);
                        const bool h = (nb >> 31) != ((cur.rw >> cb.rbit) & 1u);
                        const V gv = buf_load<T, K>(rr, h && active ? xo * RB : kOob);
                        hx::fma_acc<T, K>(acc, xamp[q], gv);
                        diag += h ? -xjz[q] : xjz[q];
                        px[q] = xo_own * (float)gv.v[0];
                    }
                }
            }
            for (int q0 = 0; q0 < (ADJ ? 0 : nXF); q0 += XB) {
                V xv[XB];
                bool hop[XB];
#pragma unroll
                for (int u = 0; u < XB; ++u) {
                    const bool ok = q0 + u < nXF;
                    const int q = ok ? q0 + u : 0;
                    const CrossBond cb = P.xb[q];
                    const uint4 info = xinfo[q];
                    const uint32_t lo = __builtin_amdgcn_readfirstlane(info.x);
                    const uint32_t hi = __builtin_amdgcn_readfirstlane(info.y);
                    const uint32_t nb = __builtin_amdgcn_readfirstlane(info.z);
                    const auto rr = rsrc(reinterpret_cast<const void *>(((uint64_t)hi << 32) | lo),
                                         nb & 0x7FFFFFFFu);
                    uint32_t xo;
                    if (cb.sj < 8) {
                        xo = u16_of(cur.xw, cb.sj);
                    } else {
                        const uint32_t gr = P.rbase[mi] + (active ? r : 0u);
                        xo = P.xo[((size_t)(cb.sj >> 3) * P.rcount + gr) * 8 + (cb.sj & 7u)];
                    }
                    hop[u] = ok && (nb >> 31) != ((cur.rw >> cb.rbit) & 1u);
                    if (__builtin_amdgcn_ballot_w64(active && hop[u])) {
                        xv[u] = buf_load<T, K>(rr, hop[u] ? xo * RB : kOob);
                    } else {
#pragma unroll
                        for (int c = 0; c < K; ++c) xv[u].v[c] = (T)0;
                    }
                }
#pragma unroll
                for (int u = 0; u < XB; ++u) {
                    if (q0 + u < nXF) {
                        hx::fma_acc<T, K>(acc, xamp[q0 + u], xv[u]);
                        diag += hop[u] ? -xjz[q0 + u] : xjz[q0 + u];
                    }
                }
            }
            for (int q = XF; q < (ADJ ? 0 : P.nX); ++q) {  // more than XF bonds across the cut
                const CrossBond cb = P.xb[q];
                const uint32_t b0 = (lw >> cb.lbit) & 1u;
                const uint64_t Rx = ro(P.xl)[(size_t)cb.si * P.count + gl];
                int mx = mi + (b0 ? -1 : 1);
                mx = mx < 0 ? 0 : (mx >= P.m_count ? P.m_count - 1 : mx);
                const bool valid = Rx != ~0ull;
                const auto rr = rsrc(x + (valid ? Rx : 0ull) * K, valid ? P.ncols[mx] * RB : 0u);
                const uint32_t gr = P.rbase[mi] + (active ? r : 0u);
                const uint32_t xo = P.xo[((size_t)(cb.sj >> 3) * P.rcount + gr) * 8 + (cb.sj & 7u)];
                const bool h = b0 != ((cur.rw >> cb.rbit) & 1u);
                hx::fma_acc<T, K>(acc, xamp[q], buf_load<T, K>(rr, h ? xo * RB : kOob));
                diag += h ? -xjz[q] : xjz[q];
            }
            if (active) {
                const V xs = xr[r];
                T *yr = y + (R + r) * K;
#pragma unroll
                for (int c = 0; c < K; ++c) __builtin_nontemporal_store(acc.v[c] + diag * xs.v[c], yr + c);
            }
            if constexpr (ADJ) {  // the diagonal sums: x_s g_s, and its signs by crossing right site
                const float pg = xo_own * (float)xr[active ? r : ncols].v[0];
                px[kAdjX] = pg;
#pragma unroll
                for (int j = 0; j < kAdjJ; ++j)
                    if (j < P.nJs) px[kAdjX + 1 + j] = ((cur.rw >> P.jbit[j]) & 1u) ? pg : -pg;
                flush16(px, 32);
                if (c0 + NT < ncols) nxt = load_chunk_idx(P, mi, r + NT, ncols, nRq);
            }
            cur = nxt;
        }
        if constexpr (ADJ) {
            // the run's values: the waves' slots added in wave order
            __syncthreads();
            if ((int)threadIdx.x < kAdjRowValues) {
                double tot = 0.0;
                for (int w = 0; w < NT / 64; ++w) tot += red[w * 64 + threadIdx.x];
                P.part[(size_t)threadIdx.x * P.part_n + gl] = tot;
            }
        }
        Q.finish();  // its barrier also ends the reads of the staged run (and of red)
    }
}

template <typename T, int K>
__global__ __launch_bounds__((lds_rows_threads<T, K>())) void split_rows_lds_kernel(const RowParams P_arg) {
    (void)P_arg;
    rows_lds_body<T, K, false>(kernel_arg0<RowParams>());
}

// The adjoint variant (k = 1).
template <typename T>
__global__ __launch_bounds__((lds_rows_threads<T, 1>())) void split_rows_lds_adj_kernel(const RowParams P_arg) {
    (void)P_arg;
    rows_lds_body<T, 1, true>(kernel_arg0<RowParams>());
}

// ------------------------------------------------------------------ block tiles
// Rows pass for rows of 16 bytes and more: one tile = a range of whole n_K blocks
// of one run (RowTiling), staged in LDS, 1024 threads.  Right-family bonds that keep
// the row inside the tile (every bond that does not move a particle into or out of
// P_K, when the tile holds whole n_K blocks) read LDS; the others read the run in
// HBM; bonds across the cut gather from the runs of the flipped left configurations.
// Tiles come from a list ordered by groups of left configurations that differ
// only on the crossing sites, so a tile's cross-cut gathers land in runs that the
// same XCD stages at about the same time.
struct TileParams {
    const void *x;
    void *y;
    const void *amp;  // coupling factors of the compute type (kAmp* layout)
    const uint32_t *lwords, *rwords;
    const uint64_t *runs, *xl;
    const uint16_t *vo, *xo;
    const double *dl, *dr;
    const uint2 *tiles, *pat;
    uint32_t *counters;
    uint64_t xbase[9];
    uint32_t count, rcount;
    int m_count, nR, nX;
    int nRA;  // right-family bonds [0, nRA) keep n_K: inside a tile of whole n_K blocks
    uint32_t pbase[kMaxLeftM], rbase[kMaxLeftM], ncols[kMaxLeftM];
    CrossBond xb[kMaxCross];
};
static_assert(sizeof(TileParams) <= 4096, "kernel arguments are limited to 4 KiB");

constexpr int kTileThreads = 1024;
constexpr int kTileXF = 32;  // bonds across the cut with descriptors in LDS (more: set up per row)

template <typename T, int K>
__global__ __launch_bounds__(kTileThreads) void split_rows_tiled_kernel(const TileParams P_arg) {
    (void)P_arg;
    const TileParams &P = kernel_arg0<TileParams>();
    using V = Acc<T, K>;
    constexpr uint32_t RB = K * sizeof(T);
    static_assert(RB % 16 == 0, "tiles hold rows of whole 16-byte units");
    constexpr int NT = kTileThreads;
    extern __shared__ __align__(16) char dyn[];
    __shared__ uint4 xinfo[kTileXF];  // per bond across the cut: run base (lo, hi), bytes | bit << 31
    __shared__ uint32_t slots[2];
    const cptr<T> A = ro(reinterpret_cast<const T *>(P.amp));
    const cptr<T> ramp = A + kAmpRight, xamp = A + kAmpCross, xjz = A + kJzCross;
    const T *__restrict__ x = reinterpret_cast<const T *>(P.x);
    T *__restrict__ y = reinterpret_cast<T *>(P.y);
    const int nRq = (P.nR + 7) >> 3;
    const int nXF = P.nX < kTileXF ? P.nX : kTileXF;
    AheadQueue Q(P.counters, P.xbase, slots);
    uint64_t t;
    while (Q.get(t)) {
        const cptr<uint32_t> tw = ro(reinterpret_cast<const uint32_t *>(P.tiles));
        const uint32_t gl = __builtin_amdgcn_readfirstlane(tw[2 * t]);
        const uint32_t tb = __builtin_amdgcn_readfirstlane(tw[2 * t + 1]);
        const int mi = (int)(tb & 0xFFu);
        const uint32_t j = tb >> 8;
        const cptr<uint32_t> pw = ro(reinterpret_cast<const uint32_t *>(P.pat));
        const uint32_t sw = __builtin_amdgcn_readfirstlane(pw[2 * (P.pbase[mi] + j)]);
        const uint32_t s0 = sw & 0x7FFFFFFFu;
        const uint32_t len = __builtin_amdgcn_readfirstlane(pw[2 * (P.pbase[mi] + j) + 1]);
        // bonds [0, nA) never leave a tile of whole n_K blocks: LDS only
        const int nA = (sw >> 31) ? 0 : P.nRA;
        const uint32_t ncols = P.ncols[mi];
        const uint64_t R = ro(P.runs)[gl];
        const uint32_t lw = ro(P.lwords)[gl];
        const double dl = ro(P.dl)[gl];
        const auto rs = rsrc(x + R * K, ncols * RB);
        if ((int)threadIdx.x < nXF) {
            const CrossBond cb = P.xb[threadIdx.x];
            const uint32_t b0 = (lw >> cb.lbit) & 1u;
            const uint64_t Rx = ro(P.xl)[(size_t)cb.si * P.count + gl];
            int mx = mi + (b0 ? -1 : 1);
            mx = mx < 0 ? 0 : (mx >= P.m_count ? P.m_count - 1 : mx);
            const bool valid = Rx != ~0ull;
            const uint64_t base = reinterpret_cast<uint64_t>(x + (valid ? Rx : 0ull) * K);
            xinfo[threadIdx.x] = make_uint4((uint32_t)base, (uint32_t)(base >> 32),
                                            (valid ? P.ncols[mx] * RB : 0u) | (b0 << 31), 0u);
        }
        // stage the tile: len rows of RB bytes in 16-byte pieces, then one zero row
        {
            const auto ts = rsrc(x + (R + s0) * K, len * RB);
            uint4 *d16 = reinterpret_cast<uint4 *>(dyn);
            const uint32_t n16 = len * (RB / 16);
            for (uint32_t i = threadIdx.x; i < n16; i += NT) {
                const auto v = __builtin_amdgcn_raw_buffer_load_b128(ts, i * 16u, 0, 0);
                __builtin_memcpy(&d16[i], &v, 16);
            }
            if (threadIdx.x < RB / 16) d16[n16 + threadIdx.x] = make_uint4(0u, 0u, 0u, 0u);
        }
        __syncthreads();
        const V *xr = reinterpret_cast<const V *>(dyn);
        // per-row index data, loaded one pass ahead so its latency overlaps the pass before
        struct RowIdx {
            uint4 tv[4];  // right-family targets of the first 32 bonds
            uint4 xw;     // flipped-right-site offsets of the first 8 site slots
            uint32_t rw;
            double dr;
        };
        auto load_idx = [&](uint32_t rrow) -> RowIdx {
            RowIdx d;
            const uint32_t gr = P.rbase[mi] + s0 + (rrow < len ? rrow : 0u);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                d.tv[i] = i < nRq ? *reinterpret_cast<const uint4 *>(P.vo + ((size_t)i * P.rcount + gr) * 8)
                                  : make_uint4(~0u, ~0u, ~0u, ~0u);
            d.xw = P.nX > 0 ? *reinterpret_cast<const uint4 *>(P.xo + (size_t)gr * 8) : make_uint4(~0u, ~0u, ~0u, ~0u);
            d.rw = P.rwords[gr];
            d.dr = P.dr[gr];
            return d;
        };
        RowIdx cur = load_idx(threadIdx.x);
        for (uint32_t rr = threadIdx.x; rr - threadIdx.x < len; rr += NT) {  // uniform trip count per wave
            const bool active = rr < len;
            const uint32_t r = s0 + (active ? rr : 0u);
            const uint32_t gr = P.rbase[mi] + r;
            RowIdx nxt = cur;
            if (rr - threadIdx.x + NT < len) nxt = load_idx(rr + NT);  // uniform
            V acc;
#pragma unroll
            for (int c = 0; c < K; ++c) acc.v[c] = (T)0;
            auto targets = [&](int qr, uint32_t (&e)[8]) {  // 0xFFFF: no hop
                uint4 tv = make_uint4(~0u, ~0u, ~0u, ~0u);
                if (qr < 4) {
#pragma unroll
                    for (int z = 0; z < 4; ++z)
                        if (z == qr) tv = cur.tv[z];
                } else {
                    tv = *reinterpret_cast<const uint4 *>(P.vo + ((size_t)qr * P.rcount + gr) * 8);
                }
                const uint32_t wv[4] = {tv.x, tv.y, tv.z, tv.w};
#pragma unroll
                for (int u = 0; u < 8; ++u) e[u] = (u & 1) ? (wv[u >> 1] >> 16) : (wv[u >> 1] & 0xFFFFu);
            };
            int q0 = 0;
            // bonds that stay inside the tile: one LDS read each, the zero row where there is no hop
            for (; q0 + 8 <= nA; q0 += 8) {
                uint32_t e[8];
                targets(q0 >> 3, e);
                V xv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) xv[u] = xr[e[u] != 0xFFFFu ? e[u] - s0 : len];
#pragma unroll
                for (int u = 0; u < 8; ++u) hx::fma_acc<T, K>(acc, ramp[q0 + u], xv[u]);
            }
            // the others (and the tail of the first): the tile where the target is inside
            // it, else the run in HBM
            for (; q0 < P.nR; q0 += 8) {
                uint32_t e[8];
                targets(q0 >> 3, e);
                V xv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const bool okb = q0 + u < P.nR;  // uniform
                    const bool hop = okb && e[u] != 0xFFFFu;
                    const uint32_t lr = e[u] - s0;  // row inside the tile (wraps when below it)
                    const bool in = hop && lr < len;
                    const bool out = hop && !in && active;
                    xv[u] = xr[in ? lr : len];
                    if (__builtin_amdgcn_ballot_w64(out)) {
                        const V g = buf_load<T, K>(rs, out ? e[u] * RB : kOob);
#pragma unroll
                        for (int c = 0; c < K; ++c) xv[u].v[c] += g.v[c];
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) hx::fma_acc<T, K>(acc, q0 + u < P.nR ? (T)ramp[q0 + u] : (T)0, xv[u]);
            }
            // bonds across the cut
            T diag = (T)(dl + cur.dr);
            const uint32_t rw = cur.rw;
            for (int q0x = 0; q0x < P.nX; q0x += 2) {
                V xv[2];
                bool hop[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const bool ok = q0x + u < P.nX;  // uniform
                    const int q = ok ? q0x + u : 0;
                    const CrossBond cb = P.xb[q];
                    __amdgpu_buffer_rsrc_t rr2;
                    uint32_t b0;
                    if (q < kTileXF) {
                        const uint4 info = xinfo[q];
                        const uint32_t lo = __builtin_amdgcn_readfirstlane(info.x);
                        const uint32_t hi = __builtin_amdgcn_readfirstlane(info.y);
                        const uint32_t nb = __builtin_amdgcn_readfirstlane(info.z);
                        rr2 = rsrc(reinterpret_cast<const void *>(((uint64_t)hi << 32) | lo), nb & 0x7FFFFFFFu);
                        b0 = nb >> 31;
                    } else {
                        b0 = (lw >> cb.lbit) & 1u;
                        const uint64_t Rx = ro(P.xl)[(size_t)cb.si * P.count + gl];
                        int mx = mi + (b0 ? -1 : 1);
                        mx = mx < 0 ? 0 : (mx >= P.m_count ? P.m_count - 1 : mx);
                        const bool valid = Rx != ~0ull;
                        rr2 = rsrc(x + (valid ? Rx : 0ull) * K, valid ? P.ncols[mx] * RB : 0u);
                    }
                    const uint32_t xo = cb.sj < 8 ? u16_of(cur.xw, cb.sj)
                                                  : P.xo[((size_t)(cb.sj >> 3) * P.rcount + gr) * 8 + (cb.sj & 7u)];
                    hop[u] = ok && b0 != ((rw >> cb.rbit) & 1u);
                    if (__builtin_amdgcn_ballot_w64(active && hop[u])) {
                        xv[u] = buf_load<T, K>(rr2, hop[u] ? xo * RB : kOob);
                    } else {
#pragma unroll
                        for (int c = 0; c < K; ++c) xv[u].v[c] = (T)0;
                    }
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    if (q0x + u < P.nX) {
                        hx::fma_acc<T, K>(acc, xamp[q0x + u], xv[u]);
                        diag += hop[u] ? -xjz[q0x + u] : xjz[q0x + u];
                    }
                }
            }
            if (active) {
                const V xs = xr[rr];
                T *yr = y + (R + r) * K;
#pragma unroll
                for (int c = 0; c < K; ++c) __builtin_nontemporal_store(acc.v[c] + diag * xs.v[c], yr + c);
            }
            cur = nxt;
        }
        Q.finish();  // its barrier also ends the reads of the staged tile and of xinfo
    }
}

// ------------------------------------------------------------------ columns
struct ColParams {
    const void *x;
    void *y;
    const void *amp;  // coupling factors of the compute type (kAmp* layout)
    const uint32_t *lptr;
    const uint64_t *lent, *runs;
    const uint32_t *clstart, *clsize;
    uint32_t *counters;
    uint64_t xbase[9];
    int m_count, nbonds;
    uint32_t ncols[kMaxLeftM], clbase[kMaxLeftM], nclust[kMaxLeftM];
    uint64_t tbase[kMaxLeftM + 1];
    // adjoint (ADJ): xprim is the primal vector; part receives per-tile sums
    // sum_s x_s g_t of every left-family bond, [bond][tile]
    const void *xprim;
    double *part;
    uint64_t part_n;
    uint32_t adj_lds_off;  // ADJ: byte offset of the per-wave sums
};
static_assert(sizeof(ColParams) <= 4096, "kernel arguments are limited to 4 KiB");

constexpr int kColThreads = 1024;  // 16 waves share one staged cluster
constexpr int kColWaves = kColThreads / 64;
constexpr int kColBatch = 4;              // gathers in flight per wave (8 measured slower)
constexpr uint32_t kColLaneBytes = 16;    // bytes of x per lane and gather
constexpr uint32_t kColWaveBytes = 64 * kColLaneBytes;

// One tile = one cluster of left configurations (see SplitRows) at one 1 KiB
// chunk (64 lanes x 16 bytes) of their runs.  The chunk of every run of the cluster
// is first copied to LDS; the targets inside the cluster (bonds inside P_{K-1})
// are then read there, the others from HBM.  Wave w takes the cluster's runs
// w, w + 16, ...: the entries of a run come in one vector load (lane q holds
// entry q), fetched while the wave works on its previous run, so no gather
// waits on a table load; kColBatch gathers are in flight per wave.
// ADJ (FP32): the product is y += (left family) g (x is g); each hop also adds
// sum_c x_s,c g_t,c to its bond's sum (per-wave LDS slots after the staged chunks,
// one writing wave each, added in wave order at the end of the tile into P.part).
template <typename T, int K, bool ADJ = false>
__global__ __launch_bounds__(kColThreads, ADJ ? 8 : 4) void split_cols_kernel(const ColParams P_arg) {
    (void)P_arg;
    const ColParams &P = kernel_arg0<ColParams>();
    constexpr int LB = (int)kColLaneBytes;
    constexpr int V = LB / sizeof(T);
    constexpr uint32_t WB = kColWaveBytes;  // chunk bytes per run
    typedef T vec_t __attribute__((ext_vector_type(V)));
    extern __shared__ __align__(16) char cl_lds[];  // [cluster run][WB]
    __shared__ uint32_t slots[2];
    __shared__ T amp[kMaxBonds];
    for (int q = threadIdx.x; q < kMaxBonds; q += kColThreads)
        amp[q] = reinterpret_cast<const T *>(P.amp)[kAmpBond + q];
    const T *__restrict__ x = reinterpret_cast<const T *>(P.x);
    T *__restrict__ y = reinterpret_cast<T *>(P.y);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    static_assert(!ADJ || sizeof(T) == 4, "the adjoint column pass is FP32");
    double *wacc = reinterpret_cast<double *>(cl_lds + P.adj_lds_off);  // ADJ: [wave][bond]
    const T *__restrict__ xp = reinterpret_cast<const T *>(P.xprim);
    AheadQueue Q(P.counters, P.xbase, slots);
    BlockCursor blk(P.tbase, P.m_count);
    uint64_t t;
    while (Q.get(t)) {
        const int mi = blk(t);
        const uint32_t local = (uint32_t)(t - P.tbase[mi]);
        const uint32_t c = local / P.nclust[mi], cl = P.clbase[mi] + (local - c * P.nclust[mi]);
        const uint32_t g0 = ro(P.clstart)[cl], size = ro(P.clsize)[cl];
        const uint32_t nrec = P.ncols[mi] * (uint32_t)(K * sizeof(T));
        const uint32_t boff = c * WB + lane * (uint32_t)LB;  // byte of the run
        // the last chunk of a run may end inside a lane's bytes: there every
        // value is loaded on its own, so no load straddles the run end
        const bool tail = (c + 1) * WB > nrec;  // uniform
        auto loadv = [&](__amdgpu_buffer_rsrc_t r) -> vec_t {
            vec_t v;
            if (!tail) {
                const auto raw = __builtin_amdgcn_raw_buffer_load_b128(r, boff, 0, 0);
                __builtin_memcpy(&v, &raw, 16);
            } else {
#pragma unroll
                for (int i = 0; i < V; ++i) v[i] = buf_load<T, 1>(r, boff + i * (uint32_t)sizeof(T)).v[0];
            }
            return v;
        };
        if constexpr (ADJ)
            for (int b = (int)lane; b < P.nbonds; b += 64) wacc[wave * P.nbonds + b] = 0.0;
        // the entries of run i: range [qa, qb) of P.lent, entry qa + lane in ev
        auto fetch = [&](uint32_t i, uint32_t &qa, uint32_t &qb, uint64_t &ev) {
            qa = ro(P.lptr)[g0 + i];
            qb = ro(P.lptr)[g0 + i + 1];
            ev = qa + lane < qb ? P.lent[qa + lane] : 0ull;
        };
        uint32_t qa = 0, qb = 0;
        uint64_t ev = 0;
        if (wave < size) fetch(wave, qa, qb, ev);  // in flight with the staging below
        // stage the chunk of every run of the cluster (zeros past a run's end)
        for (uint32_t i = wave; i < size; i += kColWaves) {
            const vec_t v = loadv(rsrc(x + ro(P.runs)[g0 + i] * K, nrec));
            *reinterpret_cast<vec_t *>(cl_lds + (size_t)i * WB + lane * (uint32_t)LB) = v;
        }
        __syncthreads();
        for (uint32_t i = wave; i < size; i += kColWaves) {
            const uint64_t R = ro(P.runs)[g0 + i];
            const auto yr = rsrc(y + R * K, nrec);
            const vec_t yold = loadv(yr);  // in flight with the gathers
            vec_t acc = (vec_t)(T)0;
            vec_t xo4 = (vec_t)(T)0;  // ADJ: the primal vector at this lane's rows
            if constexpr (ADJ) xo4 = loadv(rsrc(xp + R * K, nrec));
            const uint32_t n = qb - qa, base = qa;
            const uint64_t ecur = ev;
            if (i + kColWaves < size) fetch(i + kColWaves, qa, qb, ev);  // the wave's next run
            float pv[8];  // ADJ: x_s g_t of this lane's elements, hops [q0 & ~7, +8) of the run
#pragma unroll
            for (int j = 0; j < 8; ++j) pv[j] = 0.f;
            for (uint32_t q0 = 0; q0 < n; q0 += kColBatch) {
                vec_t v[kColBatch];
                T a[kColBatch];
                uint32_t bnd[kColBatch];
#pragma unroll
                for (int u = 0; u < kColBatch; ++u) {
                    const uint32_t q = q0 + u;
                    const bool ok = q < n;
                    uint64_t ent;
                    if (q < 64) {
                        const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)ecur, ok ? q : 0);
                        const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(ecur >> 32), ok ? q : 0);
                        ent = (uint64_t)hi << 32 | lo;
                    } else {  // entries past the first 64 of a run (dense left families)
                        ent = ro(P.lent)[base + (ok ? q : 0)];
                    }
                    if (ok && (ent >> 63)) {  // uniform: a run of this cluster
                        const uint32_t j = (uint32_t)(ent & 0xFFFFu);
                        v[u] = *reinterpret_cast<const vec_t *>(cl_lds + (size_t)(j < size ? j : 0) * WB +
                                                                lane * (uint32_t)LB);
                    } else {
                        v[u] = loadv(rsrc(x + (ent & 0xFFFFFFFFFFFFull) * K, ok ? nrec : 0u));
                    }
                    bnd[u] = (uint32_t)(ent >> 48) & 0xFFu;
                    a[u] = ok ? amp[bnd[u]] : (T)0;
                }
#pragma unroll
                for (int u = 0; u < kColBatch; ++u) acc += a[u] * v[u];
                if constexpr (ADJ) {
                    // x_s g_t over this lane's elements, one value per hop, 8 hops per
                    // wave sum (FP32), each total added to its bond's slot of this wave
                    static_assert(8 % kColBatch == 0, "whole batches per 8 hops");
                    float f[kColBatch];
#pragma unroll
                    for (int u = 0; u < kColBatch; ++u) {
                        float d = 0.f;
#pragma unroll
                        for (int e = 0; e < V; ++e) d += (float)xo4[e] * (float)v[u][e];
                        f[u] = q0 + u < n ? d : 0.f;
                    }
                    const uint32_t slot = q0 & 7u;  // uniform
#pragma unroll
                    for (int j = 0; j < 8; j += kColBatch)
                        if (slot == (uint32_t)j)
#pragma unroll
                            for (int u = 0; u < kColBatch; ++u) pv[j + u] = f[u];
                    if (slot + kColBatch == 8 || q0 + kColBatch >= n) {  // uniform
                        const float tsum = wave_transpose_sum8f(pv);
                        const uint32_t h = (q0 & ~7u) + lane;  // the hop of this lane's total (lanes < 8)
                        const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(ecur >> 32), (int)(h & 63u));
                        if (lane < 8 && h < n) {
                            const uint32_t b = h < 64 ? (hi >> 16) & 0xFFu
                                                      : (uint32_t)(ro(P.lent)[base + h] >> 48) & 0xFFu;
                            wacc[wave * P.nbonds + b] += (double)tsum;
                        }
#pragma unroll
                        for (int j = 0; j < 8; ++j) pv[j] = 0.f;
                    }
                }
            }
            if (boff < nrec) {
                T *ys = reinterpret_cast<T *>(reinterpret_cast<char *>(y + R * K) + boff);
                if (boff + (uint32_t)LB <= nrec) {
                    __builtin_nontemporal_store(yold + acc, reinterpret_cast<vec_t *>(ys));
                } else {
                    for (int e = 0; e < V; ++e)
                        if (boff + e * (uint32_t)sizeof(T) < nrec) __builtin_nontemporal_store(yold[e] + acc[e], ys + e);
                }
            }
        }
        if constexpr (ADJ) {
            __syncthreads();
            for (int b = (int)threadIdx.x; b < P.nbonds; b += kColThreads) {
                double tot = 0.0;
                for (int w = 0; w < kColWaves; ++w) tot += wacc[w * P.nbonds + b];
                P.part[(size_t)b * P.part_n + t] = tot;
            }
        }
        Q.finish();  // its barrier also ends the reads of the staged chunks (and of wacc)
    }
}

// ------------------------------------------------------------------ launch
// DCS_SPLIT_LDS=0 in the environment (read at every product) keeps the runs out of LDS.
inline bool rows_lds_enabled() {
    const char *e = getenv("DCS_SPLIT_LDS");
    return !(e && e[0] == '0');
}

// DCS_ROW_ORDER=rows (read at every product) launches the tiles of the row pass
// (both the block tiles and the 512-row tiles) in row order instead of by groups
// of left configurations that differ only at the crossing sites.
inline bool rows_group_order() {
    const char *e = getenv("DCS_ROW_ORDER");
    return !(e && e[0] == 'r');
}

// The column pass's block fields and its dynamic LDS bytes (chunk width wb; with
// adj_nbonds > 0 also the adjoint's per-wave sums).
inline size_t col_params(ColParams &P, const LeftInfo &li, const SplitRows &c, uint32_t wb, int adj_nbonds) {
    (void)li;
    size_t lds = (size_t)std::max<uint32_t>(c.max_cluster, 1) * wb;
    P.adj_lds_off = (uint32_t)lds;
    if (adj_nbonds > 0) lds += (size_t)kColWaves * adj_nbonds * sizeof(double);
    return lds;
}

inline int split_grid(const dcs_sector *s, uint64_t tiles) {
    const uint64_t cus = (uint64_t)device_cu_count(s->device);
    uint64_t w = cus * 4;
    const uint64_t cap = ((tiles + 7) / 8) * 8;
    if (w > cap) w = cap;
    w = ((w + 7) / 8) * 8;  // every XCD queue (blockIdx % 8) has workgroups
    return (int)(w ? w : 8);
}

// Variants of the split product: the staged-run rows pass allowed (rows of at
// most 8 bytes whose runs fit LDS), the rows pass from HBM, or the rows pass
// that also applies the left family (no column pass).
constexpr int kSplitStagedOk = 0, kSplitGlobal = 1, kSplitFused = 2, kSplitTiled = 3;

// The diagonal of each side per configuration and the call's coupling factors
// (FP64 table, then FP32 copy) into c.d_diag.
inline int launch_split_diag(dcs_sector *s, const SplitRows &c, const double *jxy, const double *jz,
                             const double *h, int nbonds, hipStream_t stream) {
    const LeftInfo &li = s->left;
    const uint32_t count = (uint32_t)li.count, rcount = (uint32_t)li.rcount;
    DiagParams D;
    memset(&D, 0, sizeof(D));
    D.lwords = (const uint32_t *)li.d_words;
    D.rwords = (const uint32_t *)li.d_rwords;
    D.jxy = jxy;
    D.jz = jz;
    D.h = h;
    D.out = c.d_diag;
    D.amp64 = c.d_diag + (count + rcount + 1) / 2 * 2;
    D.count = count;
    D.rcount = rcount;
    D.nD = c.nD;
    D.nR = c.nR;
    D.nX = c.nX;
    D.nbonds = nbonds;
    memcpy(D.d, c.d, sizeof(D.d));
    memcpy(D.rbond, c.r_bond, sizeof(D.rbond));
    for (int q = 0; q < c.nX; ++q) D.xbond[q] = c.x[q].bond;
    split_diag_kernel<0><<<(count + rcount + 255) / 256, 256, 0, stream>>>(D);
    return check_hip(hipGetLastError(), "split diagonal launch");
}

template <typename T, int K>
int launch_split_t(dcs_sector *s, const SplitRows &c, const void *x, void *y, const double *jxy,
                   const double *jz, const double *h, int nbonds, int variant, hipStream_t stream) {
    const bool staged_ok = variant == kSplitStagedOk, fused = variant == kSplitFused;
    const bool tiled = variant == kSplitTiled;
    const LeftInfo &li = s->left;
    const uint32_t count = (uint32_t)li.count, rcount = (uint32_t)li.rcount;
    double *amp64 = c.d_diag + (count + rcount + 1) / 2 * 2;  // 16-byte aligned after the diagonal
    const void *amp = sizeof(T) == 8 ? (const void *)amp64 : (const void *)(amp64 + kAmpEntries);
    // 1. diagonal per configuration of each side, coupling factors
    if (int r = launch_split_diag(s, c, jxy, jz, h, nbonds, stream)) return r;
    hx::zero_counters<0><<<1, 64, 0, stream>>>(s->dev.counters, 16);
    // 2. right family, bonds across the cut, diagonal: tiles of 512 offsets of one run
    {
        RowParams P;
        memset(&P, 0, sizeof(P));
        P.x = x;
        P.y = y;
        P.amp = amp;
        P.lwords = (const uint32_t *)li.d_words;
        P.rwords = (const uint32_t *)li.d_rwords;
        P.runs = c.d_runs;
        P.xl = c.d_xl;
        P.vo = c.d_vo;
        P.xo = c.d_xo;
        P.dl = c.d_diag;
        P.dr = c.d_diag + count;
        P.counters = s->dev.counters;
        P.count = count;
        P.rcount = rcount;
        P.m_count = li.m_count;
        P.nR = c.nR;
        P.nX = c.nX;
        uint64_t tiles = 0;
        for (int m = 0; m < li.m_count; ++m) {
            P.lbase[m] = li.lbase[m];
            P.rbase[m] = li.rbase[m];
            P.ncols[m] = (uint32_t)li.ncols[m];
            P.nsub[m] = (uint32_t)((li.ncols[m] + kThreads - 1) / kThreads);
            P.tbase[m] = tiles;
            tiles += (uint64_t)li.nleft[m] * P.nsub[m];
        }
        P.tbase[li.m_count] = tiles;
        xcd_ranges(tiles, P.xbase);
        memcpy(P.rbond, c.r_bond, sizeof(P.rbond));
        memcpy(P.xb, c.x, sizeof(P.xb));
        uint64_t max_cols = 0;
        for (int m = 0; m < li.m_count; ++m) max_cols = std::max<uint64_t>(max_cols, li.ncols[m]);
        const size_t lds = ((max_cols + 1) * RowBatch<T, K>::RB + 15) / 16 * 16;
        bool staged = false;
        if constexpr (RowBatch<T, K>::RB <= 8) {
            if (lds <= kRowLdsMax && staged_ok && rows_lds_enabled() && !c.wide_off) {
                // one tile per left configuration
                // one tile per left configuration; the XCD ranges hold equal row counts
                for (int m = 0; m < li.m_count; ++m) P.tbase[m] = li.lbase[m];
                P.tbase[li.m_count] = count;
                {
                    const uint64_t total = s->desc.dim;
                    uint64_t acc = 0, g = 0;
                    P.xbase[0] = 0;
                    for (int xq = 1; xq < 8; ++xq) {
                        const uint64_t want = total * xq / 8;
                        for (int m = 0; m < li.m_count; ++m) {
                            const uint64_t g1 = (uint64_t)li.lbase[m] + li.nleft[m];
                            while (g < g1 && acc + li.ncols[m] <= want) {
                                acc += li.ncols[m];
                                ++g;
                            }
                            if (g < g1) break;
                        }
                        P.xbase[xq] = g;
                    }
                    P.xbase[8] = count;
                }
                auto kern = split_rows_lds_kernel<T, K>;
                if (int r = ensure_lds(kern, lds)) return r;
                int per_cu = 1;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, lds_rows_threads<T, K>(), lds) !=
                        hipSuccess ||
                    per_cu < 1)
                    per_cu = 1;
                int wgs = device_cu_count(s->device) * std::min(per_cu, 4);
                wgs = std::min<int>(wgs, (int)(((uint64_t)count + 7) / 8 * 8));
                wgs = (wgs + 7) / 8 * 8;
                kern<<<wgs, lds_rows_threads<T, K>(), lds, stream>>>(P);
                if (int r = check_hip(hipGetLastError(), "split rows (staged runs) launch")) return r;
                staged = true;
            }
        }
        if constexpr (RowBatch<T, K>::RB >= 16 && RowBatch<T, K>::RB <= 64) {
            constexpr int ti = RowBatch<T, K>::RB == 16 ? 0 : (RowBatch<T, K>::RB == 32 ? 1 : 2);
            const RowTiling &Tl = c.tiling[ti];
            if (tiled && Tl.ntiles && !c.wide_off) {
                TileParams TP;
                memset(&TP, 0, sizeof(TP));
                TP.x = x;
                TP.y = y;
                TP.amp = amp;
                TP.lwords = P.lwords;
                TP.rwords = P.rwords;
                TP.runs = c.d_runs;
                TP.xl = c.d_xl;
                TP.vo = c.d_vo;
                TP.xo = c.d_xo;
                TP.dl = P.dl;
                TP.dr = P.dr;
                TP.tiles = rows_group_order() ? Tl.d_tiles : Tl.d_tiles_canon;
                TP.pat = Tl.d_pat;
                TP.counters = s->dev.counters;
                xcd_ranges(Tl.ntiles, TP.xbase);
                TP.count = count;
                TP.rcount = rcount;
                TP.m_count = li.m_count;
                TP.nR = c.nR;
                TP.nX = c.nX;
                TP.nRA = c.nRA;
                for (int m = 0; m < li.m_count; ++m) {
                    TP.pbase[m] = Tl.pbase[m];
                    TP.rbase[m] = li.rbase[m];
                    TP.ncols[m] = (uint32_t)li.ncols[m];
                }
                memcpy(TP.xb, c.x, sizeof(TP.xb));
                const size_t lds = (size_t)(Tl.max_rows + 1) * RowBatch<T, K>::RB;
                auto kern = split_rows_tiled_kernel<T, K>;
                if (int r = ensure_lds(kern, lds)) return r;
                const int wgs = (int)std::min<uint64_t>((uint64_t)device_cu_count(s->device), (Tl.ntiles + 7) / 8 * 8);
                kern<<<(wgs + 7) / 8 * 8, kTileThreads, lds, stream>>>(TP);
                if (int r = check_hip(hipGetLastError(), "split rows (block tiles) launch")) return r;
                staged = true;
            }
        }
        if (!staged) {
            P.nRloc = c.nRloc;
            P.margin = c.margin;
            P.lptr = c.d_lptr;
            P.lrun = c.d_lrun;
            size_t wl = P.nRloc > 0 ? (size_t)(kThreads + 2 * c.margin + 1) * RowBatch<T, K>::RB : 0;
            if (wl > kRowLdsMax) {  // the window does not fit on chip: every right-family gather from HBM
                P.nRloc = 0;
                P.margin = 0;
                wl = 0;
            }
            // the tile list by crossing groups (DCS_ROW_ORDER=rows: run order)
            if (rows_group_order() && c.d_rorder && c.n_rorder == tiles) P.order = c.d_rorder;
            auto kern = c.wide_off ? (fused ? split_rows_kernel<T, K, true, true> : split_rows_kernel<T, K, false, true>)
                                   : (fused ? split_rows_kernel<T, K, true> : split_rows_kernel<T, K, false>);
            if (int r = ensure_lds(kern, wl)) return r;
            kern<<<split_grid(s, tiles), kThreads, wl, stream>>>(P);
            if (int r = check_hip(hipGetLastError(), "split rows launch")) return r;
        }
    }
    if (fused) return DCS_OK;  // the rows pass applied the left family
    // 3. left family: tiles of one cluster of runs at one 1 KiB chunk, chunk major
    {
        ColParams P;
        memset(&P, 0, sizeof(P));
        P.x = x;
        P.y = y;
        P.amp = amp;
        P.lptr = c.d_lptr;
        P.lent = c.d_lent;
        P.runs = c.d_runs;
        P.clstart = c.d_clstart;
        P.clsize = c.d_clsize;
        P.counters = s->dev.counters + 8;
        P.m_count = li.m_count;
        P.nbonds = nbonds;
        const uint32_t wb = kColWaveBytes;
        uint64_t tiles = 0;
        for (int m = 0; m < li.m_count; ++m) {
            const uint64_t nchunk = (li.ncols[m] * K * sizeof(T) + wb - 1) / wb;
            P.ncols[m] = (uint32_t)li.ncols[m];
            P.clbase[m] = c.clbase[m];
            P.nclust[m] = c.nclust[m];
            P.tbase[m] = tiles;
            tiles += nchunk * c.nclust[m];
        }
        P.tbase[li.m_count] = tiles;
        xcd_ranges(tiles, P.xbase);
        const size_t lds = col_params(P, li, c, wb, 0);
        auto kern = split_cols_kernel<T, K>;
        if (int r = ensure_lds(kern, lds)) return r;
        kern<<<split_grid(s, tiles), kColThreads, lds, stream>>>(P);
        return check_hip(hipGetLastError(), "split columns launch");
    }
}

}  // namespace sp
}  // namespace dcs
