// Matrix-free Y = H X on one sector (Sec. 2.2 and 4.4 of arXiv:2407.14591),
// and its fused adjoint.
//
// Pull formulation: one thread owns one output row.  It decodes its row's
// state (Alg. iii, keeping the subsystem words w_k, lambda_k and the
// contributions c_k), applies the XXZ bond terms, and ranks each reached
// state incrementally: a hop between sites of P_a and P_b (a <= b) changes
// only w_a, w_b and lambda_k for a < k <= b, so by eq. index
//     col = row - sum_{k=a..b} c_k + sum_{k=a..b} C_k[lambda'_k][w'_k]
// i.e. 1 table read for a hop inside one subsystem, b-a+1 otherwise.  The
// paper's workers walk their rows with increment and rank every reached
// state in full (Sec. 2.2, Alg. i-ii); on the GPU each thread decodes its own
// row and only the touched terms are re-read.
//
// Launch shape: persistent workgroups (8 waves) each own one contiguous chunk
// of rows, walked in tiles of 64 consecutive rows per wave; chunks are
// assigned so that the workgroups of one XCD (dispatch order blockIdx % 8)
// cover one contiguous eighth of the rows and share that XCD's L2.  The
// sector tables and the per-bond coefficients sit in LDS.  Bonds are grouped
// on the host into classes (a, b) so the subsystem indices are compile-time
// constants inside the unrolled class loops (no dynamic register indexing).
// Y is written exactly once per element, with no atomics.
#pragma once

#include <algorithm>
#include <cstring>

#include "device_common.h"

namespace dcs {
namespace hx {

constexpr int kHxThreads = 512;
constexpr int kMaxClasses = kMaxSub * (kMaxSub + 1) / 2;

struct HxParams {
    SectorDesc sd;
    const char *blob;
    const void *x;
    void *y;
    const void *g;      // adjoint: upstream gradient
    void *gx;           // adjoint: H g
    double *partials;   // adjoint: [num_wgs][2*nbonds + L]
    const double *jxy, *jz, *h;
    uint64_t tiles;          // ceil(dim / kHxThreads): one tile per workgroup pass
    uint32_t *counters;      // per-XCD tile queues (8), or NULL for a static schedule
    uint64_t per_xcd;        // tiles of one XCD's range
    uint64_t cls_mask;       // bond classes this launch applies (bit class_id)
    int far_below;           // classes (a, b) with a < far_below gather non-temporally
    int nbonds;
    int xcd_groups;          // workgroups per XCD when the grid is a multiple of 8, else 0
    int want_fields;         // adjoint: accumulate the field gradients
    uint16_t cls_beg[kMaxClasses + 1];
    uint32_t pos[kMaxBonds];
};

template <typename T, int K>
struct Acc {
    T v[K];
};

template <typename T, int K>
__device__ __forceinline__ Acc<T, K> gather(const T *__restrict__ x, uint64_t col) {
    Acc<T, K> v;
    const T *p = x + col * K;
    if constexpr (K > 1 && sizeof(T) * K % 16 == 0) {
        constexpr int V = 16 / sizeof(T);
        typedef T vec_t __attribute__((ext_vector_type(16 / sizeof(T))));
#pragma unroll
        for (int c = 0; c < K; c += V) {
            const vec_t u = *reinterpret_cast<const vec_t *>(p + c);
#pragma unroll
            for (int e = 0; e < V; ++e) v.v[c + e] = u[e];
        }
    } else {
#pragma unroll
        for (int c = 0; c < K; ++c) v.v[c] = p[c];
    }
    return v;
}

// Gather for a hop that leaves the sweep window: non-temporal, so the single-use
// line does not push reusable lines of the window out of L2.
template <typename T, int K>
__device__ __forceinline__ Acc<T, K> gather_nt(const T *__restrict__ x, uint64_t col) {
    Acc<T, K> v;
    const T *p = x + col * K;
    if constexpr (K > 1 && sizeof(T) * K % 16 == 0) {
        constexpr int V = 16 / sizeof(T);
        typedef T vec_t __attribute__((ext_vector_type(16 / sizeof(T))));
#pragma unroll
        for (int c = 0; c < K; c += V) {
            const vec_t u = __builtin_nontemporal_load(reinterpret_cast<const vec_t *>(p + c));
#pragma unroll
            for (int e = 0; e < V; ++e) v.v[c + e] = u[e];
        }
    } else {
#pragma unroll
        for (int c = 0; c < K; ++c) v.v[c] = __builtin_nontemporal_load(p + c);
    }
    return v;
}

template <typename T, int K>
__device__ __forceinline__ void fma_acc(Acc<T, K> &acc, T amp, const Acc<T, K> &v) {
#pragma unroll
    for (int c = 0; c < K; ++c) acc.v[c] += amp * v.v[c];
}

template <typename T, int K>
__device__ __forceinline__ void gather_fma(Acc<T, K> &acc, T amp, const T *__restrict__ x,
                                           uint64_t col) {
    fma_acc<T, K>(acc, amp, gather<T, K>(x, col));
}

__device__ __forceinline__ uint32_t xcd_chunk(int xcd_groups) {
    const uint32_t b = blockIdx.x;
    if (!xcd_groups) return b;
    return (b & 7u) * (uint32_t)xcd_groups + (b >> 3);
}

// Tiles of this workgroup.  The tiles are grouped into super-tiles of one
// pass of an XCD's workgroups (xcd_groups tiles); super-tile s goes to XCD
// s % 8 (dispatch order blockIdx % 8) and workgroup j of that XCD takes tile j
// of it.  The whole GPU thus sweeps one narrow window of rows: hops inside a
// super-tile stay in the XCD's L2, and the farther hop targets of all XCDs
// share one small footprint in the Infinity Cache.
struct TileIter {
    uint64_t xcd, j, groups, tiles, m;
    bool linear;
    __device__ __forceinline__ uint64_t tile() const {
        return linear ? blockIdx.x + m * gridDim.x : (8 * m + xcd) * groups + j;
    }
};

__device__ __forceinline__ TileIter my_tiles(uint64_t tiles, int xcd_groups) {
    TileIter it;
    it.tiles = tiles;
    it.m = 0;
    it.linear = xcd_groups == 0;
    it.xcd = blockIdx.x & 7u;
    it.j = blockIdx.x >> 3;
    it.groups = (uint64_t)xcd_groups;
    return it;
}

// Dynamic tile queue per XCD.  XCD x (dispatch order blockIdx % 8) owns the
// contiguous tile range [x * per_xcd, (x+1) * per_xcd); its workgroups take
// the next tile from one counter, so at any time they work inside one narrow
// window of that range and the hop targets near the window stay in the XCD's
// L2 (a static round robin lets the workgroups drift apart over thousands of
// tiles).  The counters are zeroed by zero_counters before the launch.
__device__ __forceinline__ bool next_tile(uint32_t *counters, uint64_t tiles, uint64_t per_xcd,
                                          uint32_t *slot, uint64_t &t) {
    const uint32_t xcd = blockIdx.x & 7u;
    __syncthreads();
    if (threadIdx.x == 0) *slot = atomicAdd(counters + xcd, 1u);
    __syncthreads();
    const uint64_t lt = *slot;
    const uint64_t base = (uint64_t)xcd * per_xcd;
    if (lt >= per_xcd || base + lt >= tiles) return false;
    t = base + lt;
    return true;
}

template <int Unused = 0>
__global__ void zero_counters(uint32_t *c, int n) {
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0u;
}

// Per-row state kept by a thread: subsystem words, the LDS row of C_k[lambda_k],
// and the contributions c_k of the row.
template <typename IdxT, int NMAX>
struct RowState {
    uint32_t w[NMAX];
    uint32_t rb[NMAX];
    IdxT c[NMAX];
    uint64_t s;
};

template <typename IdxT, int NMAX>
__device__ __forceinline__ void decode_row(const SectorDesc &sd, const Tables<IdxT> &T, IdxT row,
                                           RowState<IdxT, NMAX> &r) {
    int lam[NMAX];
    r.s = unrank_state<IdxT, NMAX>(sd, T, row, r.w, lam, r.c);
#pragma unroll
    for (int k = 0; k < NMAX; ++k)
        r.rb[k] = (k < sd.N) ? sd.ctab_row0[k] + (uint32_t)(lam[k] - sd.lam_lo[k]) * sd.ctab_rowlen[k]
                             : 0u;
}

// Column of the state reached by changing w_a -> wa, w_b -> wb and lambda_k by dl
// for a < k <= b (one table row per unit of lambda; the last subsystem has one row).
template <typename IdxT, int NMAX, int A, int B>
__device__ __forceinline__ IdxT hop_col(const SectorDesc &sd, const Tables<IdxT> &T,
                                        const RowState<IdxT, NMAX> &r, IdxT row, uint32_t wa,
                                        uint32_t wb, int dl) {
    if constexpr (A == B) {
        return row - r.c[A] + T.ctab[r.rb[A] + wa];
    } else {
        IdxT col = row - r.c[A] + T.ctab[r.rb[A] + wa];
#pragma unroll
        for (int k = A + 1; k < B; ++k)
            col += T.ctab[r.rb[k] + (uint32_t)(dl * (int)sd.ctab_rowlen[k]) + r.w[k]] - r.c[k];
        col += T.ctab[r.rb[B] + (uint32_t)(dl * (int)sd.ctab_rowlen[B]) + wb] - r.c[B];
        return col;
    }
}

// Q = 2, one bond t of class (A, B), without branches: the diagonal term is
// added to `diag`; the returned column is the reached state's index when the
// two sites differ (a hop) and the row itself otherwise, with `amp` = 0 then.
// For a non-hop the table reads stay inside the current lambda rows, so every
// LDS address is valid whatever the lane's state.
template <typename IdxT, typename T, int NMAX, int A, int B, typename PT>
__device__ __forceinline__ IdxT q2_bond(const PT &P, const SectorDesc &sd, const Tables<IdxT> &Tb,
                                        const RowState<IdxT, NMAX> &r, IdxT row, int t,
                                        const T *bamp, const T *bjz, T &amp, T &diag) {
    const uint32_t pos = P.pos[t];
    const uint32_t pil = pos & 0xFFu, pjl = (pos >> 8) & 0xFFu;
    const uint32_t bi = (r.w[A] >> pil) & 1u, bj = (r.w[B] >> pjl) & 1u;
    const bool hop = bi != bj;
    const T jz = bjz[t];
    diag += hop ? -jz : jz;
    amp = hop ? bamp[t] : (T)0;
    IdxT col;
    if constexpr (A == B) {
        col = hop_col<IdxT, NMAX, A, B>(sd, Tb, r, row, r.w[A] ^ ((1u << pil) | (1u << pjl)), 0, 0);
    } else {
        const int dl = hop ? (bi ? -1 : 1) : 0;
        col = hop_col<IdxT, NMAX, A, B>(sd, Tb, r, row, r.w[A] ^ (1u << pil), r.w[B] ^ (1u << pjl),
                                        dl);
    }
    return hop ? col : row;
}

// One bond class (A, B): applies every bond of the class to the row.  For Q = 2
// the bonds go in batches: all the batch's columns, then all its gathers in
// flight together, then the multiply-adds.
template <typename IdxT, typename T, int K, int NMAX, bool Q2, int A, int B, typename PT>
__device__ __forceinline__ void apply_class(const PT &P, const SectorDesc &sd,
                                            const Tables<IdxT> &Tb, const RowState<IdxT, NMAX> &r,
                                            IdxT row, const T *__restrict__ x, const T *bamp,
                                            const T *bjz, const T *ladder, Acc<T, K> &acc, T &diag) {
    if constexpr (A >= NMAX || B >= NMAX) {
        return;
    } else {
        const int cls = A * NMAX - A * (A - 1) / 2 + (B - A);
        const int beg = P.cls_beg[cls], end = P.cls_beg[cls + 1];
        if constexpr (Q2) {
            // batches of NB bonds; the last batch of a class is cut by a uniform guard,
            // its unused slots gather x[row] with amplitude 0.  NB measured: 4 for FP32
            // and 2 for FP64 rows of one or two values (8 cost up to 13% more)
            constexpr int NB = K <= 2 ? (sizeof(T) == 8 ? 2 : 4) : 4;
            for (int t = beg; t < end; t += NB) {
                T a[NB];
                IdxT c[NB];
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    if (t + u < end) {
                        c[u] = q2_bond<IdxT, T, NMAX, A, B>(P, sd, Tb, r, row, t + u, bamp, bjz, a[u],
                                                            diag);
                    } else {
                        c[u] = row;
                        a[u] = (T)0;
                    }
                }
                Acc<T, K> v[NB];
                if (A < P.far_below) {
#pragma unroll
                    for (int u = 0; u < NB; ++u) v[u] = gather_nt<T, K>(x, (uint64_t)c[u]);
                } else {
#pragma unroll
                    for (int u = 0; u < NB; ++u) v[u] = gather<T, K>(x, (uint64_t)c[u]);
                }
#pragma unroll
                for (int u = 0; u < NB; ++u) fma_acc<T, K>(acc, a[u], v[u]);
            }
        } else {
            for (int t = beg; t < end; ++t) {
                const uint32_t pos = P.pos[t];
                const uint32_t pil = pos & 0xFFu, pjl = (pos >> 8) & 0xFFu;
                const uint32_t dm = (1u << sd.nb) - 1u;
                const int Qm1 = sd.Q - 1;
                const int di = (int)((r.w[A] >> pil) & dm), dj = (int)((r.w[B] >> pjl) & dm);
                const T *up = ladder, *dn = ladder + 16, *mz = ladder + 32;
                diag += bjz[t] * mz[di] * mz[dj];
                if (di < Qm1 && dj > 0) {  // S+_i S-_j
                    const uint32_t wa = r.w[A] + (1u << pil);
                    IdxT col;
                    if constexpr (A == B)
                        col = hop_col<IdxT, NMAX, A, B>(sd, Tb, r, row, wa - (1u << pjl), 0, 0);
                    else
                        col = hop_col<IdxT, NMAX, A, B>(sd, Tb, r, row, wa, r.w[B] - (1u << pjl), 1);
                    gather_fma<T, K>(acc, bamp[t] * up[di] * dn[dj], x, (uint64_t)col);
                }
                if (di > 0 && dj < Qm1) {  // S-_i S+_j
                    const uint32_t wa = r.w[A] - (1u << pil);
                    IdxT col;
                    if constexpr (A == B)
                        col = hop_col<IdxT, NMAX, A, B>(sd, Tb, r, row, wa + (1u << pjl), 0, 0);
                    else
                        col = hop_col<IdxT, NMAX, A, B>(sd, Tb, r, row, wa, r.w[B] + (1u << pjl), -1);
                    gather_fma<T, K>(acc, bamp[t] * dn[di] * up[dj], x, (uint64_t)col);
                }
            }
        }
    }
}

template <typename IdxT, typename T, int K, int NMAX, bool Q2, int A, int B>
struct ClassLoop {
    template <typename PT>
    __device__ __forceinline__ static void run(const PT &P, const SectorDesc &sd,
                                               const Tables<IdxT> &Tb,
                                               const RowState<IdxT, NMAX> &r, IdxT row,
                                               const T *__restrict__ x, const T *bamp,
                                               const T *bjz, const T *ladder, Acc<T, K> &acc,
                                               T &diag) {
        if constexpr (A < NMAX) {
            if constexpr (B < NMAX) {
                if (B < sd.N && ((P.cls_mask >> (A * NMAX - A * (A - 1) / 2 + (B - A))) & 1u))
                    apply_class<IdxT, T, K, NMAX, Q2, A, B>(P, sd, Tb, r, row, x, bamp, bjz, ladder,
                                                            acc, diag);
                ClassLoop<IdxT, T, K, NMAX, Q2, A, B + 1>::run(P, sd, Tb, r, row, x, bamp, bjz,
                                                               ladder, acc, diag);
            } else {
                ClassLoop<IdxT, T, K, NMAX, Q2, A + 1, A + 1>::run(P, sd, Tb, r, row, x, bamp, bjz,
                                                                   ladder, acc, diag);
            }
        }
    }
};

// Stage per-bond coefficients (in plan order) and the ladder factors into LDS.
template <typename T, bool Q2, typename PT>
__device__ __forceinline__ void stage_coefficients(const PT &P, const SectorDesc &sd, T *bamp,
                                                   T *bjz, T *ladder, T *hf) {
    for (int t = threadIdx.x; t < P.nbonds; t += blockDim.x) {
        const int orig = (int)(P.pos[t] >> 16);
        bamp[t] = (T)(0.5 * P.jxy[orig]);
        bjz[t] = Q2 ? (T)(0.25 * P.jz[orig]) : (T)P.jz[orig];
    }
    if (threadIdx.x < 16) {
        const int d = threadIdx.x;
        const double S = 0.5 * (sd.Q - 1), m = d - S;
        ladder[d] = (T)(d < sd.Q ? sqrt(fmax(0.0, S * (S + 1) - m * (m + 1))) : 0.0);
        ladder[16 + d] = (T)(d < sd.Q ? sqrt(fmax(0.0, S * (S + 1) - m * (m - 1))) : 0.0);
        ladder[32 + d] = (T)m;
    }
    if (threadIdx.x < kMaxSites) hf[threadIdx.x] = (P.h && (int)threadIdx.x < sd.L) ? (T)P.h[threadIdx.x] : (T)0;
}

// y[row] = (H x)[row] for the rows of one wave tile [tile, min(tile+64, end)).
template <typename IdxT, typename T, int K, int NMAX, bool Q2, typename PT>
__device__ __forceinline__ void hx_tile(const PT &P, const SectorDesc &sd, const Tables<IdxT> &Tb,
                                        const T *__restrict__ x, T *__restrict__ y, const T *bamp,
                                        const T *bjz, const T *ladder, const T *hf, bool fields,
                                        uint64_t tile, uint64_t end) {
    const int lane = threadIdx.x & 63;
    const uint64_t row64 = tile + lane;
    const bool active = row64 < end;
    const IdxT row = (IdxT)(active ? row64 : tile);
    RowState<IdxT, NMAX> r;
    decode_row<IdxT, NMAX>(sd, Tb, row, r);
    Acc<T, K> acc;
#pragma unroll
    for (int c = 0; c < K; ++c) acc.v[c] = (T)0;
    T diag = (T)0;
    ClassLoop<IdxT, T, K, NMAX, Q2, 0, 0>::run(P, sd, Tb, r, row, x, bamp, bjz, ladder, acc, diag);
    if (fields) {
        const uint32_t dm = (1u << sd.nb) - 1u;
        for (int i = 0; i < sd.L; ++i)
            diag += hf[i] * ladder[32 + (int)((r.s >> (sd.nb * (sd.L - 1 - i))) & dm)];
    }
    if (active) {
        const T *xr = x + (uint64_t)row * K;
        T *yr = y + (uint64_t)row * K;
#pragma unroll
        for (int c = 0; c < K; ++c) __builtin_nontemporal_store(acc.v[c] + diag * xr[c], yr + c);
    }
}

// LDS layout behind the sector tables: bond coefficients, ladder factors, fields.
template <typename T>
struct CoeffLds {
    T *bamp, *bjz, *ladder, *hf;
    __device__ __forceinline__ CoeffLds(char *lds, uint32_t table_bytes) {
        bamp = reinterpret_cast<T *>(lds + table_bytes);
        bjz = bamp + kMaxBonds;
        ladder = bjz + kMaxBonds;
        hf = ladder + 48;
    }
};

// GT: the sector's tables stay in device memory (too large for LDS); LDS holds
// the coefficients only.
template <typename IdxT, typename T, int K, int NMAX, bool Q2, bool GT = false>
__global__ __launch_bounds__(kHxThreads) void hx_kernel(const HxParams P_arg) {
    (void)P_arg;
    const HxParams &P = kernel_arg0<HxParams>();
    extern __shared__ __align__(16) char lds[];
    const SectorDesc &sd = P.sd;
    if constexpr (!GT) stage_blob(lds, P.blob, sd.lay_bytes);
    const CoeffLds<T> C(lds, GT ? 0u : sd.lay_bytes);
    stage_coefficients<T, Q2>(P, sd, C.bamp, C.bjz, C.ladder, C.hf);
    __syncthreads();
    const Tables<IdxT> Tb = tables_at<IdxT>(GT ? P.blob : lds, sd);
    const T *__restrict__ x = reinterpret_cast<const T *>(P.x);
    T *__restrict__ y = reinterpret_cast<T *>(P.y);
    const uint64_t wrow = (uint64_t)(threadIdx.x >> 6) * 64;
    if (P.counters) {
        __shared__ uint32_t slot;
        uint64_t t;
        while (next_tile(P.counters, P.tiles, P.per_xcd, &slot, t)) {
            const uint64_t tile = t * kHxThreads + wrow;
            if (tile < sd.dim)
                hx_tile<IdxT, T, K, NMAX, Q2>(P, sd, Tb, x, y, C.bamp, C.bjz, C.ladder, C.hf,
                                              P.h != nullptr, tile, sd.dim);
        }
        return;
    }
    for (TileIter it = my_tiles(P.tiles, P.xcd_groups); it.tile() < it.tiles; ++it.m) {
        const uint64_t tile = it.tile() * kHxThreads + wrow;
        if (tile < sd.dim)
            hx_tile<IdxT, T, K, NMAX, Q2>(P, sd, Tb, x, y, C.bamp, C.bjz, C.ladder, C.hf,
                                          P.h != nullptr, tile, sd.dim);
    }
}

// ---------------------------------------------------------------- adjoint

// Sum over the 64 lanes of a wave (all lanes active), returned in every lane:
// row shifts by 1, 2, 4, 8 leave each 16-lane row's sum in its last lane, two
// row broadcasts carry it to lane 63, which is read back.  VALU data-parallel
// moves only, in a fixed order (deterministic).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROW_MASK, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_move<0x111, 0xF>(v);  // row_shr:1
    v += dpp_move<0x112, 0xF>(v);  // row_shr:2
    v += dpp_move<0x114, 0xF>(v);  // row_shr:4
    v += dpp_move<0x118, 0xF>(v);  // row_shr:8
    v += dpp_move<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Rows per lane of the adjoint: each lane carries R rows (R tiles of 64 rows
// per wave), so every cross-lane sum covers 64 * R rows.  One row per lane
// keeps the registers (and the occupancy) of the forward pass.
template <typename IdxT, int NMAX>
constexpr int adj_rows() {
    return 1;
}

// Bonds per batch of the adjoint's Q = 2 path (2 sums per bond: 4, 8 or 16 values).
template <int R>
constexpr int adj_batch() {
    return 2;
}

// KC columns (a block [D][KC] of x and g): the sums run over the columns too.
template <typename IdxT, typename T, int NMAX, int R, int KC = 1>
struct AdjRows {
    RowState<IdxT, NMAX> r[R];
    IdxT row[R];
    Acc<T, KC> xr[R], grow[R];
    T hg[R], diag[R];
};

// sum_c a_c b_c in FP64, columns in order.
template <typename T, int KC>
__device__ __forceinline__ double dotd(const Acc<T, KC> &a, const Acc<T, KC> &b) {
    double s = (double)a.v[0] * (double)b.v[0];
#pragma unroll
    for (int c = 1; c < KC; ++c) s += (double)a.v[c] * (double)b.v[c];
    return s;
}

// Row sums of N = 8 or 16 values at once.  Each step pairs every lane with a
// lane of the same 16-lane row that holds the same subset of the values (row
// mirror, half-row mirror, quad mirror); the lane keeps one half of the subset,
// adds its partner's copy of that half and hands over the other half.  After
// log2(N) steps lane i of each row holds the sum over 16 / N * ... lanes of
// v[(i & 15) >> (16 / N - 1)]; a last plain step (N = 8) completes the row.
// About 4 moves and one add per value replace a separate cross-lane sum per
// value; fixed order (deterministic).
template <int N, int H, int CTRL>
__device__ __forceinline__ void half_step(double (&v)[N], bool upper) {
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const double lo = v[k], hi = v[k + H];
        const double keep = upper ? hi : lo, send = upper ? lo : hi;
        v[k] = keep + dpp_move<CTRL, 0xF>(send);
    }
}

template <int N>
__device__ __forceinline__ double row_transpose_sum(double (&v)[N]) {
    static_assert(N == 4 || N == 8 || N == 16, "4, 8 or 16 values");
    const int l = threadIdx.x & 15;
    if constexpr (N == 16) {
        half_step<N, 8, 0x140>(v, l & 8);  // row_mirror: i <-> 15 - i
        half_step<N, 4, 0x141>(v, l & 4);  // row_half_mirror: i <-> 7 - i in each half row
        half_step<N, 2, 0x1B>(v, l & 2);   // quad_perm [3,2,1,0]
        half_step<N, 1, 0xB1>(v, l & 1);   // quad_perm [1,0,3,2]
    } else if constexpr (N == 8) {
        half_step<N, 4, 0x140>(v, l & 8);
        half_step<N, 2, 0x141>(v, l & 4);
        half_step<N, 1, 0x1B>(v, l & 2);
        v[0] += dpp_move<0xB1, 0xF>(v[0]);  // lanes i and i ^ 1 hold the same value
    } else {
        half_step<N, 2, 0x140>(v, l & 8);
        half_step<N, 1, 0x141>(v, l & 4);
        v[0] += dpp_move<0x1B, 0xF>(v[0]);  // the quad holds one value: two plain steps
        v[0] += dpp_move<0xB1, 0xF>(v[0]);
    }
    return v[0];
}

// Wave totals of v[0..N): lane i < 16 holds the total of v[i / (16 / N)]
// (fixed order, the same bits in both lanes of every pair).
template <int N>
__device__ __forceinline__ double wave_transpose_sum(double (&v)[N]) {
    double s = row_transpose_sum<N>(v);
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    return s;
}

// Adds to a wave's accumulator in LDS; every slot has one writing lane for the
// whole launch, so the order of the additions is fixed.
__device__ __forceinline__ void lds_add(double *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One bond class (A, B) of the adjoint for the R rows of every lane.  For Q = 2
// the bonds go in batches of adj_batch() (two): every column of the batch, the
// gathers of g and x, then the batch's bond sums (two per bond) in one
// transposed row sum.
template <typename IdxT, typename T, int NMAX, bool Q2, bool GX, int A, int B, int R, int KC>
__device__ __forceinline__ void adjoint_class(const HxParams &P, const SectorDesc &sd,
                                              const Tables<IdxT> &Tb,
                                              const T *__restrict__ x, const T *__restrict__ g,
                                              const T *bamp, const T *bjz, const T *ladder,
                                              const int *borig, double *wacc,
                                              AdjRows<IdxT, T, NMAX, R, KC> &W) {
    const int cls = A * NMAX - A * (A - 1) / 2 + (B - A);
    const int beg = P.cls_beg[cls], end = P.cls_beg[cls + 1];
    const int lane = threadIdx.x & 63;
    if constexpr (Q2) {
        constexpr int NB = adj_batch<R>();
        constexpr int SH = NB == 8 ? 0 : (NB == 4 ? 1 : 2);  // lane of value j: j << SH
        for (int t = beg; t < end; t += NB) {
            double val[2 * NB];
#pragma unroll
            for (int v = 0; v < 2 * NB; ++v) val[v] = 0.0;
#pragma unroll
            for (int u = 0; u < R; ++u) {
                IdxT c[NB];
                T amp[NB];
#pragma unroll
                for (int v = 0; v < NB; ++v) {
                    if (t + v < end) {  // uniform
                        // diagonal into diag; the column is the row itself for a non-hop
                        c[v] = q2_bond<IdxT, T, NMAX, A, B>(P, sd, Tb, W.r[u], W.row[u], t + v, bamp,
                                                            bjz, amp[v], W.diag[u]);
                    } else {
                        c[v] = W.row[u];
                        amp[v] = (T)0;
                    }
                }
                T gv[NB];
                Acc<T, KC> xv[NB];
                if (A < P.far_below) {  // far targets: streamed past the caches, as in the forward pass
#pragma unroll
                    for (int v = 0; v < NB; ++v) {
                        if constexpr (GX) gv[v] = __builtin_nontemporal_load(g + c[v]);
                        xv[v] = gather_nt<T, KC>(x, c[v]);
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < NB; ++v) {
                        if constexpr (GX) gv[v] = g[c[v]];
                        xv[v] = gather<T, KC>(x, c[v]);
                    }
                }
                const double p = dotd<T, KC>(W.grow[u], W.xr[u]);
#pragma unroll
                for (int v = 0; v < NB; ++v) {
                    const bool hop = c[v] != W.row[u];
                    if constexpr (GX) W.hg[u] += amp[v] * gv[v];
                    if (t + v < end) {
                        val[2 * v] += hop ? 0.5 * dotd<T, KC>(W.grow[u], xv[v]) : 0.0;
                        val[2 * v + 1] += hop ? -0.25 * p : 0.25 * p;
                    }
                }
            }
            // value 2v + k (k = 0: jxy, 1: jz) of bond t + v ends in lane (2v + k) << SH
            const double sum = wave_transpose_sum<2 * NB>(val);
            const int j = lane >> SH, vi = j >> 1;
            if (lane < 16 && (lane & ((1 << SH) - 1)) == 0 && t + vi < end)
                lds_add(wacc + 2 * borig[t + vi] + (j & 1), sum);
        }
    } else {
        for (int t = beg; t < end; ++t) {
            const uint32_t pos = P.pos[t];
            const uint32_t pil = pos & 0xFFu, pjl = (pos >> 8) & 0xFFu;
            double sxy = 0.0, sz = 0.0;  // this lane's share of the bond's two sums
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const RowState<IdxT, NMAX> &r = W.r[u];
                const IdxT row = W.row[u];
                const uint32_t dm = (1u << sd.nb) - 1u;
                const int Qm1 = sd.Q - 1;
                const int di = (int)((r.w[A] >> pil) & dm), dj = (int)((r.w[B] >> pjl) & dm);
                const T *up = ladder, *dn = ladder + 16, *mz = ladder + 32;
                const T zz = mz[di] * mz[dj];
                Acc<T, KC> hop_x;  // sum over hops of (ladder factors / 2) * x[col]
#pragma unroll
                for (int cc = 0; cc < KC; ++cc) hop_x.v[cc] = (T)0;
                if (di < Qm1 && dj > 0) {
                    const uint32_t wa = r.w[A] + (1u << pil);
                    IdxT col;
                    if constexpr (A == B)
                        col = hop_col<IdxT, NMAX, A, B>(sd, Tb, r, row, wa - (1u << pjl), 0, 0);
                    else
                        col = hop_col<IdxT, NMAX, A, B>(sd, Tb, r, row, wa, r.w[B] - (1u << pjl), 1);
                    const T f = (T)0.5 * up[di] * dn[dj];
                    if constexpr (GX) W.hg[u] += (T)2 * bamp[t] * f * g[col];
                    {
                        const Acc<T, KC> xc = gather<T, KC>(x, col);
#pragma unroll
                        for (int cc = 0; cc < KC; ++cc) hop_x.v[cc] += f * xc.v[cc];
                    }
                }
                if (di > 0 && dj < Qm1) {
                    const uint32_t wa = r.w[A] - (1u << pil);
                    IdxT col;
                    if constexpr (A == B)
                        col = hop_col<IdxT, NMAX, A, B>(sd, Tb, r, row, wa + (1u << pjl), 0, 0);
                    else
                        col = hop_col<IdxT, NMAX, A, B>(sd, Tb, r, row, wa, r.w[B] + (1u << pjl), -1);
                    const T f = (T)0.5 * dn[di] * up[dj];
                    if constexpr (GX) W.hg[u] += (T)2 * bamp[t] * f * g[col];
                    {
                        const Acc<T, KC> xc = gather<T, KC>(x, col);
#pragma unroll
                        for (int cc = 0; cc < KC; ++cc) hop_x.v[cc] += f * xc.v[cc];
                    }
                }
                W.diag[u] += bjz[t] * zz;
                sxy += dotd<T, KC>(W.grow[u], hop_x);
                sz += (double)zz * dotd<T, KC>(W.grow[u], W.xr[u]);
            }
            const double vxy = wave_sum(sxy);
            const double vz = wave_sum(sz);
            if (lane == 0) {
                const int orig = (int)(pos >> 16);
                wacc[2 * orig] += vxy;
                wacc[2 * orig + 1] += vz;
            }
        }
    }
}

template <typename IdxT, typename T, int NMAX, bool Q2, bool GX, int A, int B, int R, int KC>
struct AdjLoop {
    __device__ __forceinline__ static void run(const HxParams &P, const SectorDesc &sd,
                                               const Tables<IdxT> &Tb,
                                               const T *__restrict__ x, const T *__restrict__ g,
                                               const T *bamp, const T *bjz, const T *ladder,
                                               const int *borig, double *wacc,
                                               AdjRows<IdxT, T, NMAX, R, KC> &W) {
        if constexpr (A < NMAX) {
            if constexpr (B < NMAX) {
                if (B < sd.N)
                    adjoint_class<IdxT, T, NMAX, Q2, GX, A, B, R, KC>(P, sd, Tb, x, g, bamp, bjz, ladder,
                                                              borig, wacc, W);
                AdjLoop<IdxT, T, NMAX, Q2, GX, A, B + 1, R, KC>::run(P, sd, Tb, x, g, bamp, bjz, ladder,
                                                             borig, wacc, W);
            } else {
                AdjLoop<IdxT, T, NMAX, Q2, GX, A + 1, A + 1, R, KC>::run(P, sd, Tb, x, g, bamp, bjz,
                                                                 ladder, borig, wacc, W);
            }
        }
    }
};

// Each wave keeps its bond and field sums in its own LDS slice, then the
// workgroup adds the slices in wave order and writes one partial row.  A tile is
// kHxThreads * R rows; wave w takes R consecutive 64-row pieces of it.  GX: the
// kernel also computes grad_x = H g (else only the sums: no gathers of g).
// GT: the sector's tables stay in device memory (LDS holds the rest).
template <typename IdxT, typename T, int NMAX, bool Q2, bool GX, int KC = 1, bool GT = false>
__device__ __forceinline__ void adjoint_body(const HxParams &P, char *lds) {
    static_assert(!GX || KC == 1, "grad_x of a block comes from the block product");
    constexpr int R = adj_rows<IdxT, NMAX>();
    const SectorDesc &sd = P.sd;
    if constexpr (!GT) stage_blob(lds, P.blob, sd.lay_bytes);
    T *bamp = reinterpret_cast<T *>(lds + (GT ? 0u : sd.lay_bytes));
    T *bjz = bamp + kMaxBonds;
    T *ladder = bjz + kMaxBonds;
    T *hf = ladder + 48;
    double *wacc_all = reinterpret_cast<double *>(hf + kMaxSites);
    const int nw = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nacc = 2 * P.nbonds + sd.L;
    int *borig = reinterpret_cast<int *>(wacc_all + nw * nacc);  // bond of each plan slot
    stage_coefficients<T, Q2>(P, sd, bamp, bjz, ladder, hf);
    for (int i = threadIdx.x; i < nw * nacc; i += blockDim.x) wacc_all[i] = 0.0;
    for (int t = threadIdx.x; t < P.nbonds; t += blockDim.x) borig[t] = (int)(P.pos[t] >> 16);
    __syncthreads();
    double *wacc = wacc_all + wave * nacc;
    const Tables<IdxT> Tb = tables_at<IdxT>(GT ? P.blob : lds, sd);
    const T *__restrict__ x = reinterpret_cast<const T *>(P.x);
    const T *__restrict__ g = reinterpret_cast<const T *>(P.g);
    T *__restrict__ gx = reinterpret_cast<T *>(P.gx);

    auto tile_rows = [&](uint64_t tile) {
        const uint64_t base = tile * ((uint64_t)kHxThreads * R) + (uint64_t)wave * (64 * R);
        if (base >= sd.dim) return;
        AdjRows<IdxT, T, NMAX, R, KC> W;
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const uint64_t row64 = base + 64 * u + lane;
            const bool active = row64 < sd.dim;
            // a lane past the end decodes a valid row and adds nothing (g = 0)
            W.row[u] = (IdxT)(active ? row64 : base);
            decode_row<IdxT, NMAX>(sd, Tb, W.row[u], W.r[u]);
            W.xr[u] = gather<T, KC>(x, W.row[u]);
            W.grow[u] = gather<T, KC>(g, W.row[u]);
            if (!active) {
#pragma unroll
                for (int cc = 0; cc < KC; ++cc) W.grow[u].v[cc] = (T)0;
            }
            W.hg[u] = (T)0;
            W.diag[u] = (T)0;
        }
        AdjLoop<IdxT, T, NMAX, Q2, GX, 0, 0, R, KC>::run(P, sd, Tb, x, g, bamp, bjz, ladder, borig, wacc,
                                                     W);
        const uint32_t dm = (1u << sd.nb) - 1u;
        if (P.h || P.want_fields) {
            // sites in batches of 8: the field sums of a batch in one transposed sum
            for (int i0 = 0; i0 < sd.L; i0 += 8) {
                double val[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    val[k] = 0.0;
                    const int i = i0 + k;
                    if (i < sd.L) {  // uniform
                        const int sh = sd.nb * (sd.L - 1 - i);
#pragma unroll
                        for (int u = 0; u < R; ++u) {
                            const T mzi = ladder[32 + (int)((W.r[u].s >> sh) & dm)];
                            if (P.h) W.diag[u] += hf[i] * mzi;
                            val[k] += (double)mzi * dotd<T, KC>(W.grow[u], W.xr[u]);
                        }
                    }
                }
                if (P.want_fields) {  // uniform: the cross-lane sums only when asked for
                    // the total of val[k] is in lane 2k
                    const double sum = wave_transpose_sum<8>(val);
                    const int k = lane >> 1;
                    if (lane < 16 && (lane & 1) == 0 && i0 + k < sd.L)
                        lds_add(wacc + 2 * P.nbonds + i0 + k, sum);
                }
            }
        }
        if constexpr (GX) {
#pragma unroll
            for (int u = 0; u < R; ++u)
                if (base + 64 * u + lane < sd.dim) gx[W.row[u]] = W.hg[u] + W.diag[u] * W.grow[u].v[0];
        }
    };
    // a static tile order: which workgroup adds which rows must not depend on timing,
    // so that the partial sums, and the gradients, are reproducible bit for bit
    for (TileIter it = my_tiles(P.tiles, P.xcd_groups); it.tile() < it.tiles; ++it.m)
        tile_rows(it.tile());
    __syncthreads();
    // partials[i][workgroup]: each sum's partials are contiguous for the reduction
    for (int i = threadIdx.x; i < nacc; i += blockDim.x) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += wacc_all[w * nacc + i];
        P.partials[(size_t)i * gridDim.x + blockIdx.x] = s;
    }
}

// The fused adjoint (grad_x and the sums), used where the single pass is the
// faster product, i.e. on sectors whose tables leave room for eight waves per
// SIMD: the register budget is set for that occupancy.
template <typename IdxT, typename T, int NMAX, bool Q2, bool GT = false>
__global__ __launch_bounds__(kHxThreads) __attribute__((amdgpu_waves_per_eu(8))) void
adjoint_kernel(const HxParams P_arg) {
    (void)P_arg;
    extern __shared__ __align__(16) char lds[];
    adjoint_body<IdxT, T, NMAX, Q2, true, 1, GT>(kernel_arg0<HxParams>(), lds);
}

// The sums only (grad_x comes from the split product).
template <typename IdxT, typename T, int NMAX, bool Q2, int KC = 1, bool GT = false>
__global__ __launch_bounds__(kHxThreads) void adjoint_sums_kernel(const HxParams P_arg) {
    (void)P_arg;
    extern __shared__ __align__(16) char lds[];
    adjoint_body<IdxT, T, NMAX, Q2, false, KC, GT>(kernel_arg0<HxParams>(), lds);
}

// Deterministic second stage: one workgroup of kAdjReduceThreads per sum; each
// thread adds a fixed stride of the workgroup partials (coalesced), then the
// wave sums and the four waves are added in a fixed order.
constexpr int kAdjReduceThreads = 256;

template <int Unused = 0>
__global__ __launch_bounds__(kAdjReduceThreads) void adjoint_reduce(
    const double *__restrict__ partials, int nwg, int nbonds, double *gjxy, double *gjz,
    double *gh) {
    __shared__ double part[kAdjReduceThreads / 64];
    const int i = blockIdx.x;
    const double *p = partials + (size_t)i * nwg;
    double s = 0.0;
    for (int w = threadIdx.x; w < nwg; w += kAdjReduceThreads) s += p[w];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x != 0) return;
    double tot = 0.0;
    for (int w = 0; w < kAdjReduceThreads / 64; ++w) tot += part[w];
    if (i < 2 * nbonds) {
        if (i & 1)
            gjz[i >> 1] = tot;
        else
            gjxy[i >> 1] = tot;
    } else if (gh) {
        gh[i - 2 * nbonds] = tot;
    }
}

// ---------------------------------------------------------------- launch

struct Grid {
    int wgs;
    uint64_t tiles;
    int xcd_groups;
};

// rows_per_thread: rows each thread of a tile covers (the adjoint's R).
inline Grid plan_grid(const dcs_sector *s, size_t lds_bytes, int rows_per_thread = 1) {
    const uint64_t dim = s->desc.dim;
    const int cus = device_cu_count(s->device);
    const size_t lds_cu = 160 * 1024;
    int per_cu = (int)(lds_cu / (lds_bytes ? lds_bytes : 1));
    per_cu = per_cu < 1 ? 1 : (per_cu > 4 ? 4 : per_cu);
    Grid g;
    const uint64_t tile_rows = (uint64_t)kHxThreads * rows_per_thread;
    g.tiles = (dim + tile_rows - 1) / tile_rows;
    uint64_t want = (uint64_t)cus * per_cu;
    if (want > g.tiles) want = g.tiles;
    if (want < 1) want = 1;
    g.wgs = (int)want;
    g.xcd_groups = 0;
    if (g.wgs >= 16 && g.tiles >= 64) {
        g.xcd_groups = g.wgs / 8;
        g.wgs = g.xcd_groups * 8;
    }
    return g;
}

inline int fill_params(const dcs_sector *s, const dcs_terms *t, int nmax, const double *jxy,
                       const double *jz, const double *h, HxParams &P, BondPlan *plan_out = nullptr) {
    BondPlan local;
    BondPlan &bp = plan_out ? *plan_out : local;
    if (int r = make_bond_plan(s, t, nmax, &bp)) return r;
    memset(&P, 0, sizeof(P));
    P.sd = s->desc;
    P.blob = (const char *)s->dev.base;
    P.jxy = jxy;
    P.jz = jz;
    P.h = h;
    P.nbonds = bp.nbonds;
    P.cls_mask = ~0ull;
    P.far_below = 0;
    for (int c = 0; c <= bp.nclasses; ++c) P.cls_beg[c] = bp.cls_beg[c];
    for (int b = 0; b < bp.nbonds; ++b) P.pos[b] = bp.pos[b];
    return DCS_OK;
}

template <typename T>
inline size_t coeff_lds_bytes() {
    return (2 * kMaxBonds + 48 + kMaxSites) * sizeof(T);
}

template <typename IdxT, typename T, int K, int NMAX>
int launch_hx_t(const dcs_sector *s, HxParams &P, hipStream_t stream) {
    if (s->gtab) {  // tables in device memory: the one-column pass only
        if constexpr (K == 1) {
            const size_t lds = coeff_lds_bytes<T>();
            const Grid g = plan_grid(s, lds);
            P.tiles = g.tiles;
            P.xcd_groups = g.xcd_groups;
            P.counters = nullptr;
            P.per_xcd = 0;
            if (g.xcd_groups && s->dev.counters) {
                P.counters = s->dev.counters;
                P.per_xcd = (g.tiles + 7) / 8;
                zero_counters<0><<<1, 64, 0, stream>>>(P.counters, 8);
            }
            auto kern = s->desc.Q == 2 ? hx_kernel<IdxT, T, K, NMAX, true, true> : hx_kernel<IdxT, T, K, NMAX, false, true>;
            if (int r = ensure_lds(kern, lds)) return r;
            kern<<<g.wgs, kHxThreads, lds, stream>>>(P);
            return check_hip(hipGetLastError(), "H*x kernel launch (tables in device memory)");
        } else {
            return set_error(DCS_EUNSUPPORTED,
                             "a block of %d columns on a sector whose tables are in device memory needs the split "
                             "product (Q = 2, runs below 65535 rows)", K);
        }
    }
    const size_t lds = s->desc.lay_bytes + coeff_lds_bytes<T>();
    const Grid g = plan_grid(s, lds);
    P.tiles = g.tiles;
    P.xcd_groups = g.xcd_groups;
    P.counters = nullptr;
    P.per_xcd = 0;
    if (g.xcd_groups && s->dev.counters) {
        P.counters = s->dev.counters;
        P.per_xcd = (g.tiles + 7) / 8;
        zero_counters<0><<<1, 64, 0, stream>>>(P.counters, 8);
    }
    if (s->desc.Q == 2) {
        auto kern = hx_kernel<IdxT, T, K, NMAX, true>;
        if (int r = ensure_lds(kern, lds)) return r;
        kern<<<g.wgs, kHxThreads, lds, stream>>>(P);
    } else {
        auto kern = hx_kernel<IdxT, T, K, NMAX, false>;
        if (int r = ensure_lds(kern, lds)) return r;
        kern<<<g.wgs, kHxThreads, lds, stream>>>(P);
    }
    return check_hip(hipGetLastError(), "H*x kernel launch");
}

// LDS of the adjoint kernel: tables, coefficients, one accumulator slice per
// wave, the bond index of every plan slot.
inline size_t adj_lds_bytes(const dcs_sector *s, int nbonds, size_t coeff_bytes) {
    return (s->gtab ? 0 : s->desc.lay_bytes) + coeff_bytes +
           (size_t)(kHxThreads / 64) * (2 * nbonds + s->desc.L) * sizeof(double) +
           (size_t)kMaxBonds * sizeof(int);
}

// KC > 1: the sums of a block of KC columns (P.gx must be NULL: grad_x of a block
// comes from the block product).
template <typename IdxT, typename T, int NMAX, int KC = 1>
int launch_adj_t(const dcs_sector *s, HxParams &P, double *gjxy, double *gjz, double *gh,
                        hipStream_t stream) {
    if (s->gtab && KC > 1)
        return set_error(DCS_EUNSUPPORTED,
                         "the adjoint of a block of %d columns needs the sector's tables in LDS", KC);
    const int nacc = 2 * P.nbonds + s->desc.L;
    const size_t lds = adj_lds_bytes(s, P.nbonds, coeff_lds_bytes<T>());
    const Grid g = plan_grid(s, adj_lds_bytes(s, P.nbonds, coeff_lds_bytes<double>()),
                             adj_rows<IdxT, NMAX>());
    P.tiles = g.tiles;
    P.xcd_groups = g.xcd_groups;
    P.want_fields = gh != nullptr;
    void (*kern)(const HxParams);
    if constexpr (KC == 1) {
        if (s->gtab)
            kern = s->desc.Q == 2 ? (P.gx ? adjoint_kernel<IdxT, T, NMAX, true, true>
                                          : adjoint_sums_kernel<IdxT, T, NMAX, true, 1, true>)
                                  : (P.gx ? adjoint_kernel<IdxT, T, NMAX, false, true>
                                          : adjoint_sums_kernel<IdxT, T, NMAX, false, 1, true>);
        else
            kern = s->desc.Q == 2 ? (P.gx ? adjoint_kernel<IdxT, T, NMAX, true>
                                          : adjoint_sums_kernel<IdxT, T, NMAX, true>)
                                  : (P.gx ? adjoint_kernel<IdxT, T, NMAX, false>
                                          : adjoint_sums_kernel<IdxT, T, NMAX, false>);
    } else {
        if (P.gx) return set_error(DCS_EINVAL, "internal: block adjoint with grad_x in the sums pass");
        kern = s->desc.Q == 2 ? adjoint_sums_kernel<IdxT, T, NMAX, true, KC>
                              : adjoint_sums_kernel<IdxT, T, NMAX, false, KC>;
    }
    if (int r = ensure_lds(kern, lds)) return r;
    kern<<<g.wgs, kHxThreads, lds, stream>>>(P);
    if (int r = check_hip(hipGetLastError(), "adjoint kernel launch")) return r;
    adjoint_reduce<0><<<nacc, kAdjReduceThreads, 0, stream>>>(P.partials, g.wgs, P.nbonds, gjxy,
                                                               gjz, gh);
    return check_hip(hipGetLastError(), "adjoint reduction launch");
}


}  // namespace hx
}  // namespace dcs
