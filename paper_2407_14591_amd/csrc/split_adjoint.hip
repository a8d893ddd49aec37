// Adjoint of y = H(theta) x on the split view, FP32 (the product and its sums in
// the same passes).  For an upstream gradient g:
//   grad_x = H g (H is real symmetric): the split product of g;
//   dL/dJxy_b = g . (A_b x) = 1/2 sum over hops s -> t of g_s x_t = 1/2 sum x_s g_t,
//     the last form from the symmetry of the hop (t -> s is a hop of the same bond):
//     the product's own gathers of g times the primal x at the row;
//   dL/dJz_b = sum_s zz_b(s) x_s g_s and dL/dh_i = sum_s (b_i(s) - 1/2) x_s g_s:
//     zz and the site terms factor over the cut, so per left configuration the sum
//     of x_s g_s over its run (PL) and its signed sums by crossing right site (CJ),
//     and per right configuration the sum over the runs of its block (PR), give them.
// The row pass (runs staged in LDS) writes per run the right-family and cross-cut
// hop sums, PL and CJ; the column pass writes per tile the left-family hop sums;
// a column-sum kernel forms PR in slices of the left configurations, a second adds
// the slices; a final kernel adds each output sum over its values in a fixed order.  No atomics: the result
// is reproducible bit for bit.
#include "split_impl.h"

namespace dcs {
namespace sp {

constexpr int kPrSplit = 32;        // slices of the left configurations in the PR sums
constexpr int kAdjFinalThreads = 256;

struct ColSumParams {
    const float *x, *g;
    const float *dots;  // if not NULL: sum_c x_s,c g_s,c per row (x and g unused)
    const uint64_t *runs;
    double *prp;  // [slice][right configuration]
    uint32_t rcount;
    int m_count;
    int k;  // columns
    uint32_t rbase[kMaxLeftM + 1], lbase[kMaxLeftM], nleft[kMaxLeftM];
};

// PR in slices: thread = right configuration, the left configurations of the slice
// in order (eight loads in flight, then added in order).
template <int Unused = 0>
__global__ __launch_bounds__(256) void adj_colsum_kernel(const ColSumParams P_arg) {
    (void)P_arg;
    const ColSumParams &P = kernel_arg0<ColSumParams>();
    const uint32_t gr = blockIdx.x * 256u + threadIdx.x;
    const uint32_t sl = blockIdx.y;
    if (gr >= P.rcount) return;
    int mi = 0;
    while (mi + 1 < P.m_count && gr >= P.rbase[mi + 1]) ++mi;
    const uint32_t r = gr - P.rbase[mi];
    const uint32_t n = P.nleft[mi];
    const uint32_t a = (uint32_t)((uint64_t)n * sl / kPrSplit), b = (uint32_t)((uint64_t)n * (sl + 1) / kPrSplit);
    const uint64_t *runs = P.runs + P.lbase[mi];
    double acc = 0.0;
    constexpr int U = 8;
    if (P.dots) {
        uint32_t q = a;
        for (; q + U <= b; q += U) {
            float v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = P.dots[runs[q + u] + r];
#pragma unroll
            for (int u = 0; u < U; ++u) acc += (double)v[u];
        }
        for (; q < b; ++q) acc += (double)P.dots[runs[q] + r];
    } else if (P.k == 1) {
        uint32_t q = a;
        for (; q + U <= b; q += U) {
            float xv[U], gv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t row = runs[q + u] + r;
                xv[u] = P.x[row];
                gv[u] = P.g[row];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) acc += (double)xv[u] * (double)gv[u];
        }
        for (; q < b; ++q) acc += (double)P.x[runs[q] + r] * (double)P.g[runs[q] + r];
    } else {
        for (uint32_t q = a; q < b; ++q) {
            const uint64_t row = runs[q] + r;
            for (int c = 0; c < P.k; ++c) acc += (double)P.x[row * P.k + c] * (double)P.g[row * P.k + c];
        }
    }
    P.prp[(size_t)sl * P.rcount + gr] = acc;
}

// PR[r] = sum over the slices in order (one thread per right configuration).
template <int Unused = 0>
__global__ __launch_bounds__(256) void adj_prsum_kernel(const double *__restrict__ prp, double *__restrict__ pr,
                                                       uint32_t rcount) {
    const uint32_t gr = blockIdx.x * 256u + threadIdx.x;
    if (gr >= rcount) return;
    double acc = 0.0;
    for (int sl = 0; sl < kPrSplit; ++sl) acc += prp[(size_t)sl * rcount + gr];
    pr[gr] = acc;
}

struct FinalParams {
    const AdjTask *tasks;
    const double *rowpart, *colpart, *pr;
    const uint32_t *lwords, *rwords;
    double *gjxy, *gjz, *gh;
    uint64_t count, rcount, ncoltiles;
    int nb;
};

__device__ __forceinline__ double task_weight(const AdjTask &k, uint32_t w) {
    const double sa = ((w >> k.ba) & 1u) ? 1.0 : -1.0, sb = ((w >> k.bb) & 1u) ? 1.0 : -1.0;
    switch (k.mode) {
        case 1: return 0.25 * sa * sb;
        case 2: return 0.25 * sa;
        case 3: return ((w >> k.ba) & 1u) ? 0.5 : -0.5;
        default: return 1.0;
    }
}

template <int Unused = 0>
__global__ __launch_bounds__(kAdjFinalThreads) void adj_final_kernel(const FinalParams P_arg) {
    (void)P_arg;
    const FinalParams &P = kernel_arg0<FinalParams>();
    __shared__ double part[kAdjFinalThreads / 64];
    const AdjTask k = P.tasks[blockIdx.x];
    double *out = k.out < P.nb ? P.gjxy + k.out : (k.out < 2 * P.nb ? P.gjz + (k.out - P.nb) : P.gh ? P.gh + (k.out - 2 * P.nb) : nullptr);
    if (!out) return;  // uniform: field sums not asked for
    double acc = 0.0;
    if (k.src == 0) {
        const double *v = P.rowpart + (size_t)k.v * P.count;
        for (uint64_t i = threadIdx.x; i < P.count; i += kAdjFinalThreads) acc += task_weight(k, P.lwords[i]) * v[i];
    } else if (k.src == 1) {
        const double *v = P.colpart + (size_t)k.v * P.ncoltiles;
        for (uint64_t i = threadIdx.x; i < P.ncoltiles; i += kAdjFinalThreads) acc += v[i];
    } else {
        for (uint64_t i = threadIdx.x; i < P.rcount; i += kAdjFinalThreads) acc += task_weight(k, P.rwords[i]) * P.pr[i];
    }
    acc = hx::wave_sum(acc);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < kAdjFinalThreads / 64; ++w) tot += part[w];
        *out = (double)k.scale * tot;
    }
}

// Column tiles of the column pass for FP32 blocks of k columns (as launch_split_t counts them).
inline uint64_t col_tiles(const LeftInfo &li, const SplitRows &c, int k) {
    uint64_t tiles = 0;
    for (int m = 0; m < li.m_count; ++m) {
        const uint64_t nchunk = (li.ncols[m] * k * sizeof(float) + kColWaveBytes - 1) / kColWaveBytes;
        tiles += nchunk * c.nclust[m];
    }
    return tiles;
}

// Row tiles of 512 rows (the row pass of blocks), in run order.
inline uint64_t row_tiles(const LeftInfo &li) {
    uint64_t tiles = 0;
    for (int m = 0; m < li.m_count; ++m) tiles += (uint64_t)li.nleft[m] * ((li.ncols[m] + kSplitRowTile - 1) / kSplitRowTile);
    return tiles;
}

// The run values of the block row pass: the sum of each run's tile values in
// chunk order (one thread per value and left configuration).
struct FoldParams {
    const double *tilepart;
    double *runpart;
    uint64_t ntiles;
    uint32_t count;
    int m_count;
    uint32_t lbase[kMaxLeftM + 1], nsub[kMaxLeftM];
    uint64_t tbase[kMaxLeftM];
};

template <int Unused = 0>
__global__ __launch_bounds__(256) void adj_fold_kernel(const FoldParams P_arg) {
    (void)P_arg;
    const FoldParams &P = kernel_arg0<FoldParams>();
    const uint32_t gl = blockIdx.x * 256u + threadIdx.x;
    const uint32_t v = blockIdx.y;
    if (gl >= P.count) return;
    int mi = 0;
    while (mi + 1 < P.m_count && gl >= P.lbase[mi + 1]) ++mi;
    const uint64_t t0 = P.tbase[mi] + (uint64_t)(gl - P.lbase[mi]) * P.nsub[mi];
    double acc = 0.0;
    for (uint32_t ch = 0; ch < P.nsub[mi]; ++ch) acc += P.tilepart[(size_t)v * P.ntiles + t0 + ch];
    P.runpart[(size_t)v * P.count + gl] = acc;
}

}  // namespace sp

bool split_adjoint_applies(const dcs_sector *s, const SplitRows &c, int dtype, int k) {
    const LeftInfo &li = s->left;
    if (dtype != DCS_F32 || li.K == 0 || c.wide_off) return false;
    if (c.nR > sp::kAdjR || c.nX > sp::kAdjX || c.nJs > sp::kAdjJ) return false;
    if (k != 1) return k == 2 || k == 4 || k == 8;  // the block row pass reads its runs from HBM
    uint64_t max_cols = 0;
    for (int m = 0; m < li.m_count; ++m) max_cols = std::max<uint64_t>(max_cols, li.ncols[m]);
    return (max_cols + 1) * sizeof(float) <= sp::kRowLdsMax;  // the row pass stages whole runs
}

// Workspace of the split adjoint: row values per left configuration, column-pass
// bond sums per column tile (clusters counted as the split tables form them:
// consecutive left configurations of one block with equal words of P_0..P_{K-2},
// at most kMaxClusterRuns), PR slices.
size_t split_adjoint_ws_bytes(const dcs_sector *s, int nbonds, int k) {
    const LeftInfo &li = s->left;
    if (li.K == 0 || li.h_words.empty()) return 0;
    const uint32_t keep = li.K >= 2 ? ((1u << li.word_shift[li.K - 1]) - 1u) : 0u;
    uint64_t tiles = 0;
    for (int m = 0; m < li.m_count; ++m) {
        uint64_t nclust = 0;
        uint32_t start = 0, size = 0;
        for (uint32_t q = 0; q < li.nleft[m]; ++q) {
            const uint32_t g = li.lbase[m] + q;
            if (q == 0 || ((li.h_words[g] ^ li.h_words[start]) & keep) != 0 || size == kMaxClusterRuns) {
                ++nclust;
                start = g;
                size = 0;
            }
            ++size;
        }
        tiles += (li.ncols[m] * k * sizeof(float) + sp::kColWaveBytes - 1) / sp::kColWaveBytes * nclust;
    }
    const size_t rows = (size_t)sp::kAdjRowValues * (li.count + (k > 1 ? sp::row_tiles(li) : 0));
    const size_t cols = (size_t)std::max(nbonds, 1) * tiles;
    const size_t pr = (size_t)(sp::kPrSplit + 1) * li.rcount;
    const size_t dots = k > 1 ? (size_t)s->desc.dim * sizeof(float) : 0;  // blocks: x . g per row
    return (rows + cols + pr) * sizeof(double) + dots;
}

namespace {

// The row pass of a block of K columns: the product's 512-row tiles (in the product's
// tile order) with the adjoint's values per tile in run order (tilepart).
template <int K>
int rows_adj_block(dcs_sector *s, const SplitRows &c, const void *amp, const void *x, const void *g, void *gx,
                   double *tilepart, uint64_t ntiles, float *dots, hipStream_t stream) {
    using namespace sp;
    const LeftInfo &li = s->left;
    const uint32_t count = (uint32_t)li.count, rcount = (uint32_t)li.rcount;
    RowParams P;
    memset(&P, 0, sizeof(P));
    P.x = g;
    P.y = gx;
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
    if (tiles != ntiles) return set_error(DCS_EHIP, "internal: block adjoint row tiles");
    xcd_ranges(tiles, P.xbase);
    memcpy(P.rbond, c.r_bond, sizeof(P.rbond));
    memcpy(P.xb, c.x, sizeof(P.xb));
    P.nRloc = c.nRloc;
    P.margin = c.margin;
    size_t wl = P.nRloc > 0 ? (size_t)(kThreads + 2 * c.margin + 1) * RowBatch<float, K>::RB : 0;
    if (wl > kRowLdsMax) {
        P.nRloc = 0;
        P.margin = 0;
        wl = 0;
    }
    if (rows_group_order() && c.d_rorder && c.n_rorder == tiles) P.order = c.d_rorder;
    P.xprim = x;
    P.part = tilepart;
    P.dots = dots;
    P.part_n = (uint32_t)tiles;
    P.nJs = c.nJs;
    memcpy(P.jbit, c.jbit, sizeof(P.jbit));
    auto kern = split_rows_kernel<float, K, false, false, true>;
    if (int r = ensure_lds(kern, wl)) return r;
    kern<<<split_grid(s, tiles), kThreads, wl, stream>>>(P);
    return check_hip(hipGetLastError(), "split adjoint rows (block) launch");
}

template <int K>
int cols_adj(dcs_sector *s, const SplitRows &c, int nbonds, const void *amp, const void *x, const void *g,
             void *gx, double *colpart, uint64_t ntiles, hipStream_t stream) {
    using namespace sp;
    const LeftInfo &li = s->left;
    ColParams P;
    memset(&P, 0, sizeof(P));
    P.x = g;
    P.y = gx;
    P.amp = amp;
    P.lptr = c.d_lptr;
    P.lent = c.d_lent;
    P.runs = c.d_runs;
    P.clstart = c.d_clstart;
    P.clsize = c.d_clsize;
    P.counters = s->dev.counters + 8;
    P.m_count = li.m_count;
    P.nbonds = nbonds;
    uint64_t tiles = 0;
    for (int m = 0; m < li.m_count; ++m) {
        const uint64_t nchunk = (li.ncols[m] * K * sizeof(float) + kColWaveBytes - 1) / kColWaveBytes;
        P.ncols[m] = (uint32_t)li.ncols[m];
        P.clbase[m] = c.clbase[m];
        P.nclust[m] = c.nclust[m];
        P.tbase[m] = tiles;
        tiles += nchunk * c.nclust[m];
    }
    P.tbase[li.m_count] = tiles;
    if (tiles != ntiles) return set_error(DCS_EHIP, "internal: adjoint column tiles");
    xcd_ranges(tiles, P.xbase);
    P.xprim = x;
    P.part = colpart;
    P.part_n = tiles;
    const size_t lds = col_params(P, li, c, kColWaveBytes, std::max(nbonds, 1));
    auto kern = split_cols_kernel<float, K, true>;
    if (int r = ensure_lds(kern, lds)) return r;
    kern<<<split_grid(s, tiles), kColThreads, lds, stream>>>(P);
    return check_hip(hipGetLastError(), "split adjoint columns launch");
}

}  // namespace

int launch_split_adjoint(dcs_sector *s, const SplitRows &c, const double *jxy, const double *jz,
                         const double *h, int nbonds, int k, const void *x, const void *g, void *gx,
                         double *gjxy, double *gjz, double *gh, void *ws, size_t ws_bytes,
                         hipStream_t stream) {
    using namespace sp;
    const LeftInfo &li = s->left;
    if (!gx || !split_adjoint_applies(s, c, DCS_F32, k)) return DCS_EUNSUPPORTED;
    const uint32_t count = (uint32_t)li.count, rcount = (uint32_t)li.rcount;
    const uint64_t ncoltiles = col_tiles(li, c, k);
    const uint64_t nrowtiles = k > 1 ? row_tiles(li) : 0;
    double *rowpart = (double *)ws;
    double *tilepart = rowpart + (size_t)kAdjRowValues * count;  // blocks: per row tile
    double *colpart = tilepart + (size_t)kAdjRowValues * nrowtiles;
    double *prp = colpart + (size_t)std::max(nbonds, 1) * ncoltiles;
    double *pr = prp + (size_t)kPrSplit * rcount;
    float *dots = k > 1 ? (float *)(pr + rcount) : nullptr;  // blocks: x . g per row
    const size_t need = (size_t)((pr + rcount) - rowpart) * sizeof(double) + (k > 1 ? (size_t)s->desc.dim * sizeof(float) : 0);
    if (need > ws_bytes) return DCS_EUNSUPPORTED;
    double *amp64 = c.d_diag + (count + rcount + 1) / 2 * 2;
    const void *amp = (const void *)(amp64 + kAmpEntries);  // the FP32 factors
    if (int r = launch_split_diag(s, c, jxy, jz, h, nbonds, stream)) return r;
    hx::zero_counters<0><<<1, 64, 0, stream>>>(s->dev.counters, 16);
    // row pass: grad_x for the right family, bonds across the cut and the diagonal,
    // and the run values (blocks: per 512-row tile, then summed per run)
    if (k > 1) {
        int r = k == 2 ? rows_adj_block<2>(s, c, amp, x, g, gx, tilepart, nrowtiles, dots, stream)
                       : (k == 4 ? rows_adj_block<4>(s, c, amp, x, g, gx, tilepart, nrowtiles, dots, stream)
                                 : rows_adj_block<8>(s, c, amp, x, g, gx, tilepart, nrowtiles, dots, stream));
        if (r) return r;
        FoldParams F;
        memset(&F, 0, sizeof(F));
        F.tilepart = tilepart;
        F.runpart = rowpart;
        F.ntiles = nrowtiles;
        F.count = count;
        F.m_count = li.m_count;
        uint64_t tb = 0;
        for (int m = 0; m < li.m_count; ++m) {
            F.lbase[m] = li.lbase[m];
            F.nsub[m] = (uint32_t)((li.ncols[m] + kSplitRowTile - 1) / kSplitRowTile);
            F.tbase[m] = tb;
            tb += (uint64_t)li.nleft[m] * F.nsub[m];
        }
        F.lbase[li.m_count] = count;
        adj_fold_kernel<0><<<dim3((count + 255) / 256, kAdjRowValues), 256, 0, stream>>>(F);
        if (int r2 = check_hip(hipGetLastError(), "split adjoint fold launch")) return r2;
    } else {
        RowParams P;
        memset(&P, 0, sizeof(P));
        P.x = g;
        P.y = gx;
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
        for (int m = 0; m < li.m_count; ++m) {
            P.lbase[m] = li.lbase[m];
            P.rbase[m] = li.rbase[m];
            P.ncols[m] = (uint32_t)li.ncols[m];
            P.tbase[m] = li.lbase[m];  // one tile per left configuration
        }
        P.tbase[li.m_count] = count;
        // XCD ranges of equal row counts (as the staged product)
        {
            const uint64_t total = s->desc.dim;
            uint64_t acc = 0, gq = 0;
            P.xbase[0] = 0;
            for (int xq = 1; xq < 8; ++xq) {
                const uint64_t want = total * xq / 8;
                for (int m = 0; m < li.m_count; ++m) {
                    const uint64_t g1 = (uint64_t)li.lbase[m] + li.nleft[m];
                    while (gq < g1 && acc + li.ncols[m] <= want) {
                        acc += li.ncols[m];
                        ++gq;
                    }
                    if (gq < g1) break;
                }
                P.xbase[xq] = gq;
            }
            P.xbase[8] = count;
        }
        memcpy(P.rbond, c.r_bond, sizeof(P.rbond));
        memcpy(P.xb, c.x, sizeof(P.xb));
        P.xprim = x;
        P.part = rowpart;
        P.part_n = count;
        P.nJs = c.nJs;
        memcpy(P.jbit, c.jbit, sizeof(P.jbit));
        uint64_t max_cols = 0;
        for (int m = 0; m < li.m_count; ++m) max_cols = std::max<uint64_t>(max_cols, li.ncols[m]);
        const size_t lds = ((max_cols + 1) * sizeof(float) + 15) / 16 * 16;
        auto kern = split_rows_lds_adj_kernel<float>;
        if (int r = ensure_lds(kern, lds)) return r;
        int per_cu = 1;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, lds_rows_threads<float, 1>(), lds) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        int wgs = device_cu_count(s->device) * std::min(per_cu, 4);
        wgs = std::min<int>(wgs, (int)(((uint64_t)count + 7) / 8 * 8));
        wgs = (wgs + 7) / 8 * 8;
        kern<<<wgs, lds_rows_threads<float, 1>(), lds, stream>>>(P);
        if (int r = check_hip(hipGetLastError(), "split adjoint rows launch")) return r;
    }
    // column pass: grad_x += left family, and the left-family hop sums per tile
    if (k > 1) {
        int r = k == 2 ? cols_adj<2>(s, c, nbonds, amp, x, g, gx, colpart, ncoltiles, stream)
                       : (k == 4 ? cols_adj<4>(s, c, nbonds, amp, x, g, gx, colpart, ncoltiles, stream)
                                 : cols_adj<8>(s, c, nbonds, amp, x, g, gx, colpart, ncoltiles, stream));
        if (r) return r;
    } else {
        ColParams P;
        memset(&P, 0, sizeof(P));
        P.x = g;
        P.y = gx;
        P.amp = amp;
        P.lptr = c.d_lptr;
        P.lent = c.d_lent;
        P.runs = c.d_runs;
        P.clstart = c.d_clstart;
        P.clsize = c.d_clsize;
        P.counters = s->dev.counters + 8;
        P.m_count = li.m_count;
        P.nbonds = nbonds;
        uint64_t tiles = 0;
        for (int m = 0; m < li.m_count; ++m) {
            const uint64_t nchunk = (li.ncols[m] * sizeof(float) + kColWaveBytes - 1) / kColWaveBytes;
            P.ncols[m] = (uint32_t)li.ncols[m];
            P.clbase[m] = c.clbase[m];
            P.nclust[m] = c.nclust[m];
            P.tbase[m] = tiles;
            tiles += nchunk * c.nclust[m];
        }
        P.tbase[li.m_count] = tiles;
        xcd_ranges(tiles, P.xbase);
        P.xprim = x;
        P.part = colpart;
        P.part_n = tiles;
        const size_t lds = col_params(P, li, c, kColWaveBytes, std::max(nbonds, 1));
        auto kern = split_cols_kernel<float, 1, true>;
        if (int r = ensure_lds(kern, lds)) return r;
        kern<<<split_grid(s, tiles), kColThreads, lds, stream>>>(P);
        if (int r = check_hip(hipGetLastError(), "split adjoint columns launch")) return r;
    }
    // PR: per right configuration, x_s g_s summed over the runs of its block
    {
        ColSumParams P;
        memset(&P, 0, sizeof(P));
        P.x = (const float *)x;
        P.g = (const float *)g;
        P.dots = dots;
        P.runs = c.d_runs;
        P.prp = prp;
        P.rcount = rcount;
        P.m_count = li.m_count;
        for (int m = 0; m < li.m_count; ++m) {
            P.rbase[m] = li.rbase[m];
            P.lbase[m] = li.lbase[m];
            P.nleft[m] = li.nleft[m];
        }
        P.rbase[li.m_count] = rcount;
        P.k = k;
        adj_colsum_kernel<0><<<dim3((rcount + 255) / 256, kPrSplit), 256, 0, stream>>>(P);
        if (int r = check_hip(hipGetLastError(), "split adjoint column sums launch")) return r;
        adj_prsum_kernel<0><<<(rcount + 255) / 256, 256, 0, stream>>>(prp, pr, rcount);
        if (int r = check_hip(hipGetLastError(), "split adjoint column sums launch")) return r;
    }
    // every output sum in a fixed order
    {
        FinalParams P;
        memset(&P, 0, sizeof(P));
        P.tasks = c.d_adjtasks;
        P.rowpart = rowpart;
        P.colpart = colpart;
        P.pr = pr;
        P.lwords = (const uint32_t *)li.d_words;
        P.rwords = (const uint32_t *)li.d_rwords;
        P.gjxy = gjxy;
        P.gjz = gjz;
        P.gh = gh;
        P.count = count;
        P.rcount = rcount;
        P.ncoltiles = ncoltiles;
        P.nb = nbonds;
        adj_final_kernel<0><<<c.n_adjtasks, kAdjFinalThreads, 0, stream>>>(P);
        return check_hip(hipGetLastError(), "split adjoint final sums launch");
    }
}

}  // namespace dcs
