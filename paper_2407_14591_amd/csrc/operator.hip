// Generic number-conserving local operators on one sector (Sec. 4.1, the operator
// class built from operator strings and user-defined local matrices; App. C, the
// terms of one cluster of sites merged into one sparse matrix).
//
// Host: the terms (coef, sites, Q^m x Q^m matrix) are checked to conserve the
// particle number and grouped greedily into clusters of at most `cluster_sites`
// sites (a term joins the first cluster whose site set it can extend within the
// limit, else it opens one); each cluster's sum of embedded terms is stored row by
// row, every entry with the digits of its input state and its value.  Rows are keyed
// by the output state's digits on the cluster's sites packed nb bits each, first
// site most significant (keys holding a digit >= Q are empty rows), and entries
// carry their input digits packed the same way: for a cluster of adjacent sites both
// are the bit field the digits occupy in a packed state.
//
// Device: one thread per row s of the sector (pull form, y_s = sum_t O_st x_t):
// unrank s (keeping each subsystem's word, particles before it and contribution to
// the index), and for each cluster read the key of s on the cluster's sites, walk
// that row's entries, write the entry's digits into s and re-rank only the
// subsystems from the first to the last one the cluster touches (eq. index is a sum
// over subsystems; the particles before the first and after the last are
// unchanged), gather x there.  The operator's arrays are staged in LDS next to the
// sector's tables when they fit; each workgroup derives per cluster the bit
// positions and table rows it needs from the sector's layout, and every lane reads
// them into scalar registers.
#include "device_common.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <type_traits>
#include <vector>

namespace dcs {
namespace op {

constexpr int kOpMaxSites = 8;       // sites of one cluster
constexpr uint32_t kOpMaxLocal = 4096;  // Q^m of one cluster
constexpr int kOpThreads = 256;
constexpr int kOpBatch = 4;  // entries of a cluster row whose gathers are in flight together
constexpr uint64_t kOpLdsMax = 128 * 1024;  // tables + operator arrays staged per workgroup

struct OpCluster {
    uint8_t m;
    uint8_t site[kOpMaxSites];
    uint8_t pad[3];
    uint32_t row0;  // first entry of the cluster's row pointers
};
static_assert(sizeof(OpCluster) == 16, "cluster record");

// The operator's arrays for one compute type, one contiguous blob (16-byte
// aligned segments): clusters | row pointers (offsets into the
// entries, 2^(nb m) + 1 per cluster) | packed input digits of each entry (site j's
// digit at bits nb (m-1-j)) | values.
struct OpParams {
    SectorDesc sd;  // first: read in place in the kernel argument segment
    const char *blob;
    const char *opblob;
    uint32_t op_bytes, off_rp, off_dep, off_val;
    uint32_t lds_tabs;  // LDS bytes of the sector's tables (0: read in device memory)
    uint32_t lds_recs;  // LDS byte offset of the per-cluster records (kOpRecBytes each)
    const void *x;
    void *y;
    int ncl;
};
static_assert(sizeof(OpParams) <= 4096, "kernel arguments are limited to 4 KiB");

// Values and vectors of the compute type T, each real or complex (interleaved
// re, im); a real operator may act on complex vectors.
template <typename T, bool C>
struct OpScalar {
    using type = T;
};
template <typename T>
struct OpScalar<T, true> {
    struct type {
        T re, im;
    };
};
// A row of K real columns as one vector (K > 1).
template <typename T, int K>
struct OpVecK {
    typedef T type __attribute__((ext_vector_type(K)));
};

template <bool VC, bool XC, typename A, typename V>
__device__ __forceinline__ void op_fma(A &acc, const V &v, const A &x) {
    if constexpr (!XC) {
        acc += v * x;  // real value on a real row (one column or K)
    } else if constexpr (!VC) {  // real value, complex vector
        acc.re += v * x.re;
        acc.im += v * x.im;
    } else {  // complex value and vector
        acc.re += v.re * x.re - v.im * x.im;
        acc.im += v.re * x.im + v.im * x.re;
    }
}

// Per cluster one 48-byte record, built once per workgroup from the sector's layout:
//   r0: posA | posB << 8 | bitsB << 16 | nk << 24, the first row pointer,
//       k1 | m << 8 | runs << 16, the key mask 2^(nb m) - 1
//   r1: the bit positions of sites 0..7 (one byte each), then shift | wbits << 8 of the
//       first two touched subsystems (A in bits 0-15, B in bits 16-31)
//   r2: row length and base (row0 - lam_lo * row length) of the fused table rows of A, B
// The sites (in increasing order) fall into runs whose digits lie next to each other
// in the packed state.  With at most two runs, the cluster's packed digits are two bit
// fields: the first run's, whose lowest bit is posA, above the second run's bitsB bits
// at posB (one run: bitsB = 0).  nk = k2 - k1 + 1 subsystems are touched.
constexpr uint32_t kOpRecBytes = 48;

__device__ __forceinline__ void op_fill_record(const SectorDesc &sd, const OpCluster &C, uint32_t *r) {
    int k1 = kMaxSub, k2 = -1;
    uint32_t p03 = 0, p47 = 0;
    int pos_prev = 0, pos = 0, runs = 0, posA = 0, endA = 0;
    for (int j = 0; j < C.m; ++j) {
        const int k = sd.site_sub[C.site[j]];
        k1 = min(k1, k);
        k2 = max(k2, k);
        pos = sd.shift[k] + sd.site_bit[C.site[j]];
        if (j == 0 || pos + sd.nb != pos_prev) ++runs;
        if (runs == 1) {  // the first run ends at site j
            posA = pos;
            endA = j + 1;
        }
        pos_prev = pos;
        if (j < 4) p03 |= (uint32_t)pos << (8 * j);
        else p47 |= (uint32_t)pos << (8 * (j - 4));
    }
    const int nk = k2 - k1 + 1;
    const int kb = nk >= 2 ? k1 + 1 : k1;
    const int bitsB = sd.nb * (C.m - endA);
    const int posB = runs == 2 ? pos : 0;
    r[0] = (uint32_t)posA | ((uint32_t)posB << 8) | ((uint32_t)bitsB << 16) | ((uint32_t)nk << 24);
    r[1] = C.row0;
    r[2] = (uint32_t)k1 | ((uint32_t)C.m << 8) | ((uint32_t)runs << 16);
    r[3] = (uint32_t)((1ull << (sd.nb * C.m)) - 1ull);
    r[4] = p03;
    r[5] = p47;
    r[6] = sd.shift[k1] | (sd.wbits[k1] << 8) | (sd.shift[kb] << 16) | (sd.wbits[kb] << 24);
    r[7] = 0;
    r[8] = sd.ctab_rowlen[k1];
    r[9] = sd.ctab_row0[k1] - (uint32_t)sd.lam_lo[k1] * sd.ctab_rowlen[k1];
    r[10] = sd.ctab_rowlen[kb];
    r[11] = sd.ctab_row0[kb] - (uint32_t)sd.lam_lo[kb] * sd.ctab_rowlen[kb];
}

// K: columns of a block [D][K] of real vectors (one unrank and one rank per target
// serve all K); complex vectors take one column.  EXP: instead of storing (O x)_i,
// sum x_i (O x)_i over the rows (conj(x_i) for complex vectors) in FP64, and write
// the workgroup's sum (K values, or re and im) to P.y at its block index.
template <typename IdxT, typename T, bool VC, bool XC, bool GT, bool OPL, int K, bool EXP = false>
__global__ __launch_bounds__(kOpThreads) void op_kernel(const OpParams P_arg) {
    static_assert(XC || !VC, "a complex operator needs complex vectors");
    static_assert(!XC || K == 1, "complex vectors take one column");
    using V = typename OpScalar<T, VC>::type;
    using X = std::conditional_t<(K > 1), typename OpVecK<T, K>::type, typename OpScalar<T, XC>::type>;
    (void)P_arg;
    const OpParams &P = kernel_arg0<OpParams>();
    const SectorDesc &sd = P.sd;
    extern __shared__ __align__(16) char lds[];
    if constexpr (!GT) stage_blob(lds, P.blob, sd.lay_bytes);
    if constexpr (OPL) stage_blob(lds + P.lds_tabs, P.opblob, P.op_bytes);
    const OpCluster *gcl = reinterpret_cast<const OpCluster *>(P.opblob);
    uint32_t *recs = reinterpret_cast<uint32_t *>(lds + P.lds_recs);  // [cluster][12]
    for (int c = threadIdx.x; c < P.ncl; c += kOpThreads) {
        op_fill_record(sd, gcl[c], recs + c * (kOpRecBytes / 4));
    }
    __syncthreads();
    const Tables<IdxT> Tb = tables_at<IdxT>(GT ? P.blob : lds, sd);
    const char *ob = OPL ? (const char *)(lds + P.lds_tabs) : P.opblob;
    const uint32_t *rowptr = reinterpret_cast<const uint32_t *>(ob + P.off_rp);
    const uint32_t *dep = reinterpret_cast<const uint32_t *>(ob + P.off_dep);
    const V *val = reinterpret_cast<const V *>(ob + P.off_val);
    const X *__restrict__ x = reinterpret_cast<const X *>(P.x);
    X *__restrict__ y = reinterpret_cast<X *>(P.y);
    const uint32_t nb = sd.nb;
    const uint32_t dmask = (1u << nb) - 1u;
    const uint64_t stride = (uint64_t)gridDim.x * kOpThreads;
    constexpr int NV = XC ? 2 : K;  // values an expectation sums
    double part[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) part[c] = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * kOpThreads + threadIdx.x; i < sd.dim; i += stride) {
        uint32_t w[kMaxSub];
        int lam[kMaxSub];
        IdxT cpart[kMaxSub];
        const uint64_t s = unrank_state<IdxT, kMaxSub>(sd, Tb, (IdxT)i, w, lam, cpart);
        // cpre[k]: the index's contributions of the subsystems before k
        IdxT cpre[kMaxSub + 1];
        cpre[0] = 0;
#pragma unroll
        for (int k = 0; k < kMaxSub; ++k) cpre[k + 1] = cpre[k] + (k < sd.N ? cpart[k] : (IdxT)0);
        X acc;
        memset(&acc, 0, sizeof(acc));
        for (int c = 0; c < P.ncl; ++c) {  // uniform
            // the record is the same on every lane: read it once into scalar registers,
            // so that every test on it below is a scalar branch
            const uint4 *rp4 = reinterpret_cast<const uint4 *>(recs + c * (kOpRecBytes / 4));
            const uint4 q0 = rp4[0], q1 = rp4[1], q2 = rp4[2];
            const uint32_t hdr = __builtin_amdgcn_readfirstlane(q0.x);
            const uint32_t row0 = __builtin_amdgcn_readfirstlane(q0.y);
            const uint32_t hdr2 = __builtin_amdgcn_readfirstlane(q0.z);
            const uint32_t fmask = __builtin_amdgcn_readfirstlane(q0.w);
            const uint32_t p03 = __builtin_amdgcn_readfirstlane(q1.x);
            const uint32_t p47 = __builtin_amdgcn_readfirstlane(q1.y);
            const uint32_t shw = __builtin_amdgcn_readfirstlane(q1.z);
            const uint32_t rlA = __builtin_amdgcn_readfirstlane(q2.x);
            const uint32_t baseA = __builtin_amdgcn_readfirstlane(q2.y);
            const uint32_t rlB = __builtin_amdgcn_readfirstlane(q2.z);
            const uint32_t baseB = __builtin_amdgcn_readfirstlane(q2.w);
            const uint32_t posA = hdr & 0xffu, posB = (hdr >> 8) & 0xffu, bitsB = (hdr >> 16) & 0xffu;
            const int nk = (int)(hdr >> 24);
            const int k1 = (int)(hdr2 & 0xffu), m = (int)((hdr2 >> 8) & 0xffu);
            const int runs = (int)(hdr2 >> 16);
            const uint32_t maskA = fmask >> bitsB, maskB = (1u << bitsB) - 1u;
            const uint32_t shA = shw & 0xffu, mA = (1u << ((shw >> 8) & 0xffu)) - 1u;
            const uint32_t shB = (shw >> 16) & 0xffu, mB = (1u << (shw >> 24)) - 1u;
            const uint64_t pp = ((uint64_t)p47 << 32) | p03;
            // the row's packed digits on the cluster's sites (the row key) and the state
            // with those digits cleared
            uint32_t f;
            uint64_t keep;
            if (runs == 1) {
                f = (uint32_t)(s >> posA) & fmask;
                keep = s & ~((uint64_t)fmask << posA);
            } else if (runs == 2) {
                f = (((uint32_t)(s >> posA) & maskA) << bitsB) | ((uint32_t)(s >> posB) & maskB);
                keep = s & ~(((uint64_t)maskA << posA) | ((uint64_t)maskB << posB));
            } else {
                f = 0;
                uint64_t clmask = 0;
                for (int j = 0; j < m; ++j) {
                    const uint32_t pj = (uint32_t)(pp >> (8 * j)) & 0xffu;
                    f = (f << nb) | ((uint32_t)(s >> pj) & dmask);
                    clmask |= (uint64_t)dmask << pj;
                }
                keep = s & ~clmask;
            }
            // the index without the touched subsystems' contributions; particles before k1
            const IdxT base_idx = (IdxT)i - (cpre[k1 + nk] - cpre[k1]);
            const int lam0 = lam[k1];
            const uint32_t rowA = baseA + (uint32_t)lam0 * rlA;
            const uint32_t eb = rowptr[row0 + f], ee = rowptr[row0 + f + 1];
            // kOpBatch entries at a time: their targets first, then their gathers (in flight
            // together), then the products in entry order
            for (uint32_t e0 = eb; e0 < ee; e0 += kOpBatch) {
                uint64_t t[kOpBatch];
#pragma unroll
                for (int u = 0; u < kOpBatch; ++u) {
                    const bool ok = e0 + u < ee;
                    const uint32_t d = dep[ok ? e0 + u : e0];
                    uint64_t s2 = keep;
                    if (runs == 1) {
                        s2 |= (uint64_t)d << posA;
                    } else if (runs == 2) {
                        s2 |= ((uint64_t)(d >> bitsB) << posA) | ((uint64_t)(d & maskB) << posB);
                    } else {
                        uint32_t dd = d;
                        for (int j = m - 1; j >= 0; --j) {
                            s2 |= (uint64_t)(dd & dmask) << ((uint32_t)(pp >> (8 * j)) & 0xffu);
                            dd >>= nb;
                        }
                    }
                    const uint32_t wa = (uint32_t)(s2 >> shA) & mA;
                    IdxT v = base_idx + Tb.ctab[rowA + wa];
                    if (nk >= 2) {
                        int l = lam0 + digit_sum(sd, wa);
                        const uint32_t wb = (uint32_t)(s2 >> shB) & mB;
                        v += Tb.ctab[baseB + (uint32_t)l * rlB + wb];
                        if (nk >= 3) {
                            l += digit_sum(sd, wb);
                            for (int k = k1 + 2; k < k1 + nk; ++k) {
                                const uint32_t wk = sub_word(sd, s2, k);
                                v += Tb.ctab[sd.ctab_row0[k] + (uint32_t)(l - sd.lam_lo[k]) * sd.ctab_rowlen[k] + wk];
                                l += digit_sum(sd, wk);
                            }
                        }
                    }
                    t[u] = ok ? (uint64_t)v : ~0ull;  // no entry: past the sector, reads zero
                }
                X xt[kOpBatch];
#pragma unroll
                for (int u = 0; u < kOpBatch; ++u) {
                    if (t[u] < sd.dim) xt[u] = x[t[u]];
                    else memset(&xt[u], 0, sizeof(X));
                }
#pragma unroll
                for (int u = 0; u < kOpBatch; ++u)
                    if (e0 + u < ee) op_fma<VC, XC>(acc, val[e0 + u], xt[u]);
            }
        }
        if constexpr (EXP) {
            const X xi = x[i];
            if constexpr (XC) {  // conj(x_i) (O x)_i
                part[0] += (double)xi.re * (double)acc.re + (double)xi.im * (double)acc.im;
                part[1] += (double)xi.re * (double)acc.im - (double)xi.im * (double)acc.re;
            } else if constexpr (K > 1) {
#pragma unroll
                for (int c = 0; c < K; ++c) part[c] += (double)xi[c] * (double)acc[c];
            } else {
                part[0] += (double)xi * (double)acc;
            }
        } else {
            y[i] = acc;
        }
    }
    if constexpr (EXP) {  // the workgroup's sums: across each wave, then the waves in order
        __shared__ double red[kOpThreads / 64][NV];
        const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            double v = part[c];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) red[wave][c] = v;
        }
        __syncthreads();
        if (threadIdx.x < NV) {
            double t = 0.0;
            for (int wv = 0; wv < kOpThreads / 64; ++wv) t += red[wv][threadIdx.x];
            reinterpret_cast<double *>(P.y)[(size_t)blockIdx.x * NV + threadIdx.x] = t;
        }
    }
}

// the workgroups' sums added in a fixed order (deterministic): out[c] for c < nv; each
// of 256 threads sums a strided subset in block order, then a fixed tree in LDS
constexpr int kExpFinalThreads = 256;
__global__ __launch_bounds__(kExpFinalThreads) void op_exp_final(const double *__restrict__ part, int nblocks, int nv,
                                                                 double *__restrict__ out) {
    __shared__ double red[kExpFinalThreads];
    for (int c = 0; c < nv; ++c) {
        double t = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += kExpFinalThreads) t += part[(size_t)b * nv + c];
        red[threadIdx.x] = t;
        __syncthreads();
        for (int w = kExpFinalThreads / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[c] = red[0];
        __syncthreads();
    }
}

}  // namespace op
}  // namespace dcs

struct dcs_operator {
    int Q = 0, L = 0, nb = 0, device = 0;  // Q: the largest local dimension
    int qsite[dcs::kMaxSites] = {};        // local dimension of each site
    int ncl = 0, max_sites = 0;
    bool cplx = false;  // complex values (interleaved re, im)
    uint64_t nnz = 0;
    void *d_base = nullptr;
    const char *blob64 = nullptr, *blob32 = nullptr;  // the OpParams layout with FP64 / FP32 values
    uint64_t bytes64 = 0, bytes32 = 0;
    uint32_t off_rp = 0, off_dep = 0, off_val = 0;
};

namespace {

using namespace dcs;
using namespace dcs::op;

// The local index of digits (d_0, ..., d_{m-1}) on m sites of local dimensions
// r_0, ..., r_{m-1} is the mixed-radix number with the first site most significant
// (sum_j d_j Q^(m-1-j) when every r_j = Q).

// digit j of the local index a
inline int local_digit(uint32_t a, int j, int m, const int *r) {
    for (int k = m - 1; k > j; --k) a /= (uint32_t)r[k];
    return (int)(a % (uint32_t)r[j]);
}

inline int digit_sum_local(uint32_t a, int m, const int *r) {
    int s = 0;
    for (int k = m - 1; k >= 0; --k) {
        s += (int)(a % (uint32_t)r[k]);
        a /= (uint32_t)r[k];
    }
    return s;
}

// the digits of the local index a packed nb bits each, the first site most significant
// (the cluster's digits as they lie in a packed state when its sites are adjacent)
inline uint32_t pack_local(uint32_t a, int m, const int *r, int nb) {
    uint32_t d = 0;
    for (int j = 0; j < m; ++j) d |= (uint32_t)local_digit(a, j, m, r) << (nb * (m - 1 - j));
    return d;
}

// the number of digit strings on sites with local dimensions r_0..r_{m-1} (saturating)
inline uint32_t local_size(const int *r, int m) {
    uint64_t v = 1;
    for (int k = 0; k < m; ++k) v = std::min<uint64_t>(v * (uint64_t)r[k], 0xFFFFFFFFull);
    return (uint32_t)v;
}

struct Entry {
    uint32_t row, col;
    std::complex<double> v;
};

}  // namespace

namespace {

// The operator on L sites, site i with qs[i] states (one Q for all, or one per site).
int operator_create(const int *qs, int L, int num_terms, const int32_t *term_nsites, const int32_t *term_sites,
                    const double *term_coefs, const double *term_mats, int complex_mats, int cluster_sites,
                    int device, dcs_operator **out) {
    if (!out) return set_error(DCS_EINVAL, "out is NULL");
    *out = nullptr;
    int Q = 0;
    for (int i = 0; i < L; ++i) {
        if (qs[i] < 2 || qs[i] > 16) return set_error(DCS_EINVAL, "local dimension %d of site %d outside [2, 16]", qs[i], i);
        Q = std::max(Q, qs[i]);
    }
    auto dims_of = [&](const int32_t *sites, int m, int *r) {
        for (int j = 0; j < m; ++j) r[j] = qs[sites[j]];
    };
    if (num_terms < 0) return set_error(DCS_EINVAL, "num_terms %d < 0", num_terms);
    if (num_terms > 0 && (!term_nsites || !term_sites || !term_coefs || !term_mats))
        return set_error(DCS_EINVAL, "NULL term array");
    if (cluster_sites < 1 || cluster_sites > kOpMaxSites)
        return set_error(DCS_EINVAL, "cluster_sites=%d outside [1, %d]", cluster_sites, kOpMaxSites);
    if (complex_mats != 0 && complex_mats != 1) return set_error(DCS_EINVAL, "complex_mats=%d", complex_mats);
    const int nc = complex_mats ? 2 : 1;  // doubles per matrix entry
    using cd = std::complex<double>;
    auto entry = [&](const double *M, size_t k) { return complex_mats ? cd(M[2 * k], M[2 * k + 1]) : cd(M[k], 0.0); };
    // check every term; offsets of its sites and matrix (a term's matrix has one row
    // and one column per digit string on its sites: the product of their dimensions)
    std::vector<size_t> site_off(num_terms + 1, 0), mat_off(num_terms + 1, 0);
    for (int t = 0; t < num_terms; ++t) {
        const int m = term_nsites[t];
        if (m < 1 || m > kOpMaxSites)
            return set_error(DCS_EUNSUPPORTED, "term %d has %d sites (1..%d)", t, m, kOpMaxSites);
        site_off[t + 1] = site_off[t] + (size_t)m;
    }
    for (int t = 0; t < num_terms; ++t) {
        const int m = term_nsites[t];
        const int32_t *st = term_sites + site_off[t];
        for (int j = 0; j < m; ++j) {
            if (st[j] < 0 || st[j] >= L) return set_error(DCS_EINVAL, "term %d: site %d outside [0, %d)", t, st[j], L);
            for (int k = 0; k < j; ++k)
                if (st[k] == st[j]) return set_error(DCS_EINVAL, "term %d lists site %d twice", t, st[j]);
        }
        int r[kOpMaxSites];
        dims_of(st, m, r);
        const uint32_t n = local_size(r, m);
        if (n > kOpMaxLocal)
            return set_error(DCS_EUNSUPPORTED, "term %d: %u digit strings on its sites > %u", t, n, kOpMaxLocal);
        mat_off[t + 1] = mat_off[t] + (size_t)n * n * nc;
        if (!std::isfinite(term_coefs[t])) return set_error(DCS_EINVAL, "term %d: coefficient not finite", t);
        const double *M = term_mats + mat_off[t];
        for (uint32_t b = 0; b < n; ++b)
            for (uint32_t a = 0; a < n; ++a) {
                const cd v = entry(M, (size_t)b * n + a);
                if (!std::isfinite(v.real()) || !std::isfinite(v.imag()))
                    return set_error(DCS_EINVAL, "term %d: matrix entry not finite", t);
            }
    }
    // clusters (App. C): greedy, in the order of the terms
    std::vector<std::vector<int>> cl_sites, cl_terms;
    for (int t = 0; t < num_terms; ++t) {
        const int m = term_nsites[t];
        std::vector<int> S(term_sites + site_off[t], term_sites + site_off[t] + m);
        std::sort(S.begin(), S.end());
        int found = -1;
        for (size_t c = 0; c < cl_sites.size() && found < 0; ++c) {
            std::vector<int> U;
            std::set_union(cl_sites[c].begin(), cl_sites[c].end(), S.begin(), S.end(), std::back_inserter(U));
            int ru[kMaxSites];
            for (size_t j = 0; j < U.size() && j < (size_t)kMaxSites; ++j) ru[j] = qs[U[j]];
            if (U.size() == cl_sites[c].size() ||
                ((int)U.size() <= cluster_sites && local_size(ru, (int)U.size()) <= kOpMaxLocal)) {
                found = (int)c;
                cl_sites[c] = U;
            }
        }
        if (found < 0) {
            cl_sites.push_back(S);
            cl_terms.emplace_back();
            found = (int)cl_sites.size() - 1;
        }
        cl_terms[found].push_back(t);
    }
    // each cluster's matrix, CSR by the packed output digits (see the key loop below)
    const int nb = (Q - 1) > 0 ? 32 - __builtin_clz((unsigned)(Q - 1)) : 1;
    std::vector<OpCluster> hcl(cl_sites.size());
    std::vector<uint32_t> rowptr, dep;
    std::vector<std::complex<double>> val;
    int max_sites = 0;
    for (size_t c = 0; c < cl_sites.size(); ++c) {
        const int m = (int)cl_sites[c].size();
        int rc[kOpMaxSites];  // the cluster's local dimensions
        for (int j = 0; j < m; ++j) rc[j] = qs[cl_sites[c][j]];
        const uint32_t n = local_size(rc, m);
        max_sites = std::max(max_sites, m);
        std::vector<Entry> ents;
        for (int t : cl_terms[c]) {
            const int mt = term_nsites[t];
            const int32_t *st = term_sites + site_off[t];
            int rt[kOpMaxSites];  // the term's local dimensions
            dims_of(st, mt, rt);
            const uint32_t nt = local_size(rt, mt);
            const double *M = term_mats + mat_off[t];
            int p[kOpMaxSites];  // cluster position of term site j
            for (int j = 0; j < mt; ++j)
                p[j] = (int)(std::lower_bound(cl_sites[c].begin(), cl_sites[c].end(), st[j]) - cl_sites[c].begin());
            int da[kOpMaxSites];
            for (uint32_t a = 0; a < n; ++a) {  // input state of the cluster
                for (int j = 0; j < m; ++j) da[j] = local_digit(a, j, m, rc);
                uint32_t at = 0;
                for (int j = 0; j < mt; ++j) at = at * (uint32_t)rt[j] + (uint32_t)da[p[j]];
                for (uint32_t bt = 0; bt < nt; ++bt) {
                    const cd v = entry(M, (size_t)bt * nt + at);
                    if (v == 0.0) continue;
                    int db[kOpMaxSites];
                    std::copy(da, da + m, db);
                    for (int j = 0; j < mt; ++j) db[p[j]] = local_digit(bt, j, mt, rt);
                    uint32_t b = 0;
                    for (int j = 0; j < m; ++j) b = b * (uint32_t)rc[j] + (uint32_t)db[j];
                    ents.push_back({b, a, term_coefs[t] * v});
                }
            }
        }
        std::sort(ents.begin(), ents.end(), [](const Entry &u, const Entry &v) {
            return u.row != v.row ? u.row < v.row : u.col < v.col;
        });
        OpCluster &C = hcl[c];
        C.m = (uint8_t)m;
        for (int j = 0; j < kOpMaxSites; ++j) C.site[j] = j < m ? (uint8_t)cl_sites[c][j] : 0;
        C.row0 = (uint32_t)rowptr.size();
        if (val.size() + ents.size() > 0xFFFFFFF0ull) return set_error(DCS_EUNSUPPORTED, "more than 2^32 entries");
        size_t e = 0;
        // the cluster's sum must conserve the particle number (a single term need not:
        // Sx Sx and Sy Sy on one bond change it, their sum does not); entries that join
        // different digit sums must cancel to rounding, relative to the cluster's largest
        double vmax = 0.0;
        for (const Entry &en : ents) vmax = std::max(vmax, std::abs(en.v));
        // rows keyed by the packed output digits; keys with a digit >= Q stay empty, and
        // the key order is the order of the local index, so the entries are met in turn
        const uint32_t nkeys = 1u << (nb * m);
        for (uint32_t key = 0; key < nkeys; ++key) {
            rowptr.push_back((uint32_t)val.size());
            uint32_t b = 0;
            bool valid = true;
            for (int j = 0; j < m; ++j) {
                const uint32_t dj = (key >> (nb * (m - 1 - j))) & ((1u << nb) - 1u);
                valid = valid && dj < (uint32_t)rc[j];
                b = b * (uint32_t)rc[j] + dj;
            }
            if (!valid) continue;
            while (e < ents.size() && ents[e].row == b) {
                const uint32_t col = ents[e].col;
                cd v = 0.0;
                double vabs = 0.0;  // magnitude of the summed contributions
                while (e < ents.size() && ents[e].row == b && ents[e].col == col) {
                    vabs += std::abs(ents[e].v);
                    v += ents[e++].v;
                }
                if (digit_sum_local(b, m, rc) != digit_sum_local(col, m, rc)) {
                    if (std::abs(v) > 1e-13 * std::max(vabs, vmax))
                        return set_error(DCS_EINVAL,
                                         "the terms on sites of cluster %zu do not conserve the particle number "
                                         "(entry %u, %u)", c, b, col);
                    continue;
                }
                if (v == 0.0) continue;
                dep.push_back(pack_local(col, m, rc, nb));
                val.push_back(v);
            }
        }
        rowptr.push_back((uint32_t)val.size());
    }
    dcs_operator *o = new (std::nothrow) dcs_operator();
    if (!o) return set_error(DCS_ENOMEM, "host allocation failed");
    o->Q = Q;
    for (int i = 0; i < L; ++i) o->qsite[i] = qs[i];
    o->L = L;
    o->nb = nb;
    o->device = device;
    o->ncl = (int)hcl.size();
    o->max_sites = max_sites;
    o->nnz = val.size();
    // complex terms whose sums are real (Sx Sx + Sy Sy) make a real operator
    double vmax_all = 0.0, imax = 0.0;
    for (const cd &v : val) {
        vmax_all = std::max(vmax_all, std::abs(v));
        imax = std::max(imax, std::abs(v.imag()));
    }
    o->cplx = complex_mats != 0 && imax > 1e-13 * vmax_all;
    if (!o->cplx)
        for (cd &v : val) v = cd(v.real(), 0.0);
    // two blobs (FP64 and FP32 values), each clusters | row pointers | digits | values
    auto a16 = [](uint64_t b) { return (b + 15) / 16 * 16; };
    const uint64_t b_cl = a16(std::max<size_t>(hcl.size(), 1) * sizeof(OpCluster));
    const uint64_t b_rp = a16(rowptr.size() * 4), b_dep = a16(dep.size() * 4);
    o->off_rp = (uint32_t)b_cl;
    o->off_dep = (uint32_t)(b_cl + b_rp);
    o->off_val = (uint32_t)(b_cl + b_rp + b_dep);
    const uint64_t vb = o->cplx ? 16 : 8;  // bytes of one FP64 value
    if (b_cl + b_rp + b_dep + a16(val.size() * vb) > 0xFFFFFFF0ull) {
        delete o;
        return set_error(DCS_EUNSUPPORTED, "operator arrays beyond 4 GiB");
    }
    o->bytes64 = o->off_val + a16(std::max<size_t>(val.size(), 1) * vb);
    o->bytes32 = o->off_val + a16(std::max<size_t>(val.size(), 1) * vb / 2);
    const uint64_t at32 = (o->bytes64 + 255) / 256 * 256;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        delete o;
        return set_error(DCS_EINVAL, "device %d not present", device);
    }
    DeviceGuard g(device);
    char *base = nullptr;
    if (hipMalloc((void **)&base, at32 + o->bytes32) != hipSuccess) {
        (void)hipGetLastError();
        delete o;
        return set_error(DCS_ENOMEM, "device allocation of %llu bytes failed", (unsigned long long)(at32 + o->bytes32));
    }
    o->d_base = base;
    o->blob64 = base;
    o->blob32 = base + at32;
    std::vector<char> h64(o->bytes64, 0), h32(o->bytes32, 0);
    for (std::vector<char> *h : {&h64, &h32}) {
        if (!hcl.empty()) memcpy(h->data(), hcl.data(), hcl.size() * sizeof(OpCluster));
        if (!rowptr.empty()) memcpy(h->data() + o->off_rp, rowptr.data(), rowptr.size() * 4);
        if (!dep.empty()) memcpy(h->data() + o->off_dep, dep.data(), dep.size() * 4);
    }
    for (size_t e = 0; e < val.size(); ++e) {
        const double d2[2] = {val[e].real(), val[e].imag()};
        const float f2[2] = {(float)d2[0], (float)d2[1]};
        memcpy(h64.data() + o->off_val + e * vb, d2, vb);
        memcpy(h32.data() + o->off_val + e * vb / 2, f2, vb / 2);
    }
    int r = check_hip(hipMemcpy(base, h64.data(), h64.size(), hipMemcpyHostToDevice), "operator upload");
    if (!r) r = check_hip(hipMemcpy(base + at32, h32.data(), h32.size(), hipMemcpyHostToDevice), "operator upload");
    if (r) {
        (void)hipFree(base);
        delete o;
        return r;
    }
    *out = o;
    return DCS_OK;
}

}  // namespace

extern "C" int dcs_operator_create(int Q, int L, int num_terms, const int32_t *term_nsites,
                                   const int32_t *term_sites, const double *term_coefs,
                                   const double *term_mats, int complex_mats, int cluster_sites,
                                   int device, dcs_operator **out) {
    clear_error();
    if (Q < 2 || Q > 16) return set_error(DCS_EINVAL, "Q=%d outside [2, 16]", Q);
    if (L < 1 || L > kMaxSites) return set_error(DCS_EINVAL, "L=%d outside [1, %d]", L, kMaxSites);
    int qs[kMaxSites];
    for (int i = 0; i < L; ++i) qs[i] = Q;
    return operator_create(qs, L, num_terms, term_nsites, term_sites, term_coefs, term_mats, complex_mats,
                           cluster_sites, device, out);
}

extern "C" int dcs_operator_create_mixed(int L, const int32_t *local_dims, int num_terms,
                                         const int32_t *term_nsites, const int32_t *term_sites,
                                         const double *term_coefs, const double *term_mats, int complex_mats,
                                         int cluster_sites, int device, dcs_operator **out) {
    clear_error();
    if (!local_dims) return set_error(DCS_EINVAL, "local_dims is NULL");
    if (L < 1 || L > kMaxSites) return set_error(DCS_EINVAL, "L=%d outside [1, %d]", L, kMaxSites);
    int qs[kMaxSites];
    for (int i = 0; i < L; ++i) qs[i] = local_dims[i];
    return operator_create(qs, L, num_terms, term_nsites, term_sites, term_coefs, term_mats, complex_mats,
                           cluster_sites, device, out);
}

extern "C" int dcs_operator_destroy(dcs_operator *o) {
    clear_error();
    if (!o) return DCS_OK;
    int r = DCS_OK;
    if (o->d_base) {
        DeviceGuard g(o->device);
        r = check_hip(hipFree(o->d_base), "operator free");
    }
    delete o;
    return r;
}

extern "C" int dcs_operator_info(const dcs_operator *o, int *num_clusters, uint64_t *nnz, int *max_cluster_sites,
                                 int *is_complex) {
    clear_error();
    if (!o) return set_error(DCS_EINVAL, "operator is NULL");
    if (is_complex) *is_complex = o->cplx ? 1 : 0;
    if (num_clusters) *num_clusters = o->ncl;
    if (nnz) *nnz = o->nnz;
    if (max_cluster_sites) *max_cluster_sites = o->max_sites;
    return DCS_OK;
}

namespace dcs {

using namespace op;

int operator_check(const dcs_sector *s, const dcs_operator *o, int dtype, int k) {
    if (!s || !o) return set_error(DCS_EINVAL, "NULL sector or operator");
    for (int i = 0; i < o->L && o->L == s->desc.L; ++i)
        if (o->qsite[i] != s->qsite[i])
            return set_error(DCS_EINVAL, "site %d: local dimension %d in the operator, %d in the sector", i,
                             o->qsite[i], s->qsite[i]);
    if (o->Q != s->desc.Q || o->L != s->desc.L)
        return set_error(DCS_EINVAL, "operator of Q=%d, L=%d on a sector of Q=%d, L=%d", o->Q, o->L, s->desc.Q,
                         s->desc.L);
    if (o->device != s->device)
        return set_error(DCS_EINVAL, "operator on device %d, sector on device %d", o->device, s->device);
    if (dtype != DCS_F32 && dtype != DCS_F64 && dtype != DCS_C64 && dtype != DCS_C128)
        return set_error(DCS_EINVAL, "dtype %d", dtype);
    const bool xc = dtype == DCS_C64 || dtype == DCS_C128;
    if (o->cplx && !xc) return set_error(DCS_EINVAL, "a complex operator needs complex vectors (DCS_C64 / DCS_C128)");
    if (k != 1 && k != 2 && k != 4 && k != 8) return set_error(DCS_EINVAL, "k=%d not in {1,2,4,8}", k);
    if (xc && k != 1) return set_error(DCS_EUNSUPPORTED, "complex vectors take one column (k=%d)", k);
    return DCS_OK;
}

// workgroups of an operator launch on the sector (the expectation's partial sums)
static int op_grid(const dcs_sector *s) {
    const uint64_t blocks = (s->desc.dim + kOpThreads - 1) / kOpThreads;
    const uint64_t cap = (uint64_t)device_cu_count(s->device) * 8;
    return (int)std::max<uint64_t>(1, std::min(blocks, cap));
}

// EXP: y is the workspace of the workgroups' sums, out the expectation (device)
template <bool EXP>
static int launch_operator_t(const dcs_sector *s, const dcs_operator *o, int dtype, int k, const void *x, void *y,
                             double *out, hipStream_t stream) {
    const bool xc = dtype == DCS_C64 || dtype == DCS_C128;
    const bool single = dtype == DCS_F32 || dtype == DCS_C64;
    DeviceGuard g(s->device);
    OpParams P;
    memset(&P, 0, sizeof(P));
    P.sd = s->desc;
    P.blob = (const char *)s->dev.base;
    P.opblob = single ? o->blob32 : o->blob64;
    P.op_bytes = (uint32_t)(single ? o->bytes32 : o->bytes64);
    P.off_rp = o->off_rp;
    P.off_dep = o->off_dep;
    P.off_val = o->off_val;
    P.lds_tabs = s->gtab ? 0u : (uint32_t)s->desc.lay_bytes;  // a multiple of 16
    P.x = x;
    P.y = y;
    P.ncl = o->ncl;
    // the operator's arrays go to LDS beside the tables when both fit the budget
    const bool opl = (uint64_t)P.lds_tabs + P.op_bytes + (uint64_t)kOpRecBytes * o->ncl <= kOpLdsMax;
    P.lds_recs = P.lds_tabs + (opl ? P.op_bytes : 0u);
    const size_t lds = (size_t)P.lds_recs + kOpRecBytes * (size_t)std::max(o->ncl, 1);
    if (lds > 160 * 1024) return set_error(DCS_EUNSUPPORTED, "operator of %d clusters beyond the LDS budget", o->ncl);
    const int grid = op_grid(s);
    hipStream_t st = stream;
    auto go = [&](auto kern) -> int {
        if (int r = ensure_lds(kern, lds)) return r;
        kern<<<grid, kOpThreads, lds, st>>>(P);
        if (int r = check_hip(hipGetLastError(), "operator kernel launch")) return r;
        if constexpr (EXP) {
            op_exp_final<<<1, kExpFinalThreads, 0, st>>>(reinterpret_cast<const double *>(y), grid, xc ? 2 : k, out);
            return check_hip(hipGetLastError(), "expectation sum launch");
        }
        return DCS_OK;
    };
    auto pick_k = [&](auto tag, auto vc, auto xcc, auto kk) -> int {
        using T = decltype(tag);
        constexpr bool VC = decltype(vc)::value, XC = decltype(xcc)::value;
        constexpr int K = decltype(kk)::value;
        if (s->wide) {
            if (s->gtab)
                return opl ? go(op_kernel<uint64_t, T, VC, XC, true, true, K, EXP>)
                           : go(op_kernel<uint64_t, T, VC, XC, true, false, K, EXP>);
            return opl ? go(op_kernel<uint64_t, T, VC, XC, false, true, K, EXP>)
                       : go(op_kernel<uint64_t, T, VC, XC, false, false, K, EXP>);
        }
        if (s->gtab)
            return opl ? go(op_kernel<uint32_t, T, VC, XC, true, true, K, EXP>)
                       : go(op_kernel<uint32_t, T, VC, XC, true, false, K, EXP>);
        return opl ? go(op_kernel<uint32_t, T, VC, XC, false, true, K, EXP>)
                   : go(op_kernel<uint32_t, T, VC, XC, false, false, K, EXP>);
    };
    auto pick = [&](auto tag, auto vc, auto xcc) -> int {
        if constexpr (decltype(xcc)::value) {
            return pick_k(tag, vc, xcc, std::integral_constant<int, 1>{});
        } else {
            switch (k) {
                case 2: return pick_k(tag, vc, xcc, std::integral_constant<int, 2>{});
                case 4: return pick_k(tag, vc, xcc, std::integral_constant<int, 4>{});
                case 8: return pick_k(tag, vc, xcc, std::integral_constant<int, 8>{});
                default: return pick_k(tag, vc, xcc, std::integral_constant<int, 1>{});
            }
        }
    };
    using F = std::false_type;
    using Tt = std::true_type;
    if (!xc) return single ? pick(0.0f, F{}, F{}) : pick(0.0, F{}, F{});
    if (!o->cplx) return single ? pick(0.0f, F{}, Tt{}) : pick(0.0, F{}, Tt{});
    return single ? pick(0.0f, Tt{}, Tt{}) : pick(0.0, Tt{}, Tt{});
}

int launch_operator(const dcs_sector *s, const dcs_operator *o, int dtype, int k, const void *x, void *y,
                    hipStream_t stream) {
    return launch_operator_t<false>(s, o, dtype, k, x, y, nullptr, stream);
}

}  // namespace dcs

extern "C" int dcs_operator_apply(const dcs_sector *s, const dcs_operator *o, int dtype, int k, const void *x,
                                  void *y, void *stream) {
    clear_error();
    if (int r = operator_check(s, o, dtype, k)) return r;
    if (!x || !y) return set_error(DCS_EINVAL, "NULL vector");
    const bool xc = dtype == DCS_C64 || dtype == DCS_C128;
    const bool single = dtype == DCS_F32 || dtype == DCS_C64;
    const size_t bytes = (size_t)s->desc.dim * (single ? 4 : 8) * (xc ? 2 : 1) * (size_t)k;
    if ((const char *)y < (const char *)x + bytes && (const char *)x < (const char *)y + bytes)
        return set_error(DCS_EINVAL, "y overlaps x");
    return launch_operator(s, o, dtype, k, x, y, (hipStream_t)stream);
}

extern "C" int dcs_operator_expectation_workspace_size(const dcs_sector *s, const dcs_operator *o, int k,
                                                       size_t *bytes) {
    clear_error();
    if (!s || !o || !bytes) return set_error(DCS_EINVAL, "NULL argument");
    if (k != 1 && k != 2 && k != 4 && k != 8) return set_error(DCS_EINVAL, "k=%d not in {1,2,4,8}", k);
    *bytes = (size_t)op_grid(s) * (size_t)std::max(k, 2) * sizeof(double);
    return DCS_OK;
}

extern "C" int dcs_operator_expectation(const dcs_sector *s, const dcs_operator *o, int dtype, int k, const void *x,
                                        double *out, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    if (int r = operator_check(s, o, dtype, k)) return r;
    if (!x || !out || !ws) return set_error(DCS_EINVAL, "NULL argument");
    const bool xc = dtype == DCS_C64 || dtype == DCS_C128;
    const size_t need = (size_t)op_grid(s) * (size_t)(xc ? 2 : k) * sizeof(double);
    if (ws_bytes < need) return set_error(DCS_EINVAL, "workspace of %zu bytes < %zu", ws_bytes, need);
    return launch_operator_t<true>(s, o, dtype, k, x, ws, out, (hipStream_t)stream);
}
