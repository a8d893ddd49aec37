// Device-side helpers shared by the index and H*x kernels: table views,
// staging of a sector's tables into LDS, digit sums, rank and unrank.
#pragma once

#include "dcs_internal.h"

namespace dcs {

template <typename IdxT>
struct Tables {
    const IdxT *ctab;       // fused contributions C_k[lambda][w]
    const IdxT *doff;       // offset_k(m, lambda), rows of mk+1
    const IdxT *dstr;       // stride_k(m, lambda)
    const float *drcp;      // 1 / stride (float)
    const uint32_t *invs;   // start of the words of digit sum m of P_k in inv
    const uint16_t *inv;    // words by (digit sum, local index)
};

// A kernel's first (by-value) argument, read where it lies in the kernel
// argument segment (constant memory; the first argument starts at offset 0).
// Uniform field reads then become scalar loads.  Without this, the compiler
// makes a per-lane copy of a large argument block in scratch memory when the
// kernel body is large (the single pass with more than four subsystems), and
// spills scalar registers in others.
template <typename P>
__device__ __forceinline__ const P &kernel_arg0() {
    return *(const P *)__builtin_amdgcn_kernarg_segment_ptr();
}

template <typename IdxT>
__device__ __forceinline__ Tables<IdxT> tables_at(const char *base, const SectorDesc &sd) {
    Tables<IdxT> t;
    t.ctab = reinterpret_cast<const IdxT *>(base + sd.lay_ctab);
    t.doff = reinterpret_cast<const IdxT *>(base + sd.lay_doff);
    t.dstr = reinterpret_cast<const IdxT *>(base + sd.lay_dstr);
    t.drcp = reinterpret_cast<const float *>(base + sd.lay_drcp);
    t.invs = reinterpret_cast<const uint32_t *>(base + sd.lay_invs);
    t.inv = reinterpret_cast<const uint16_t *>(base + sd.lay_inv);
    return t;
}

// Copy the sector's table blob (lay_bytes, a multiple of 16) into LDS.
__device__ __forceinline__ void stage_blob(void *lds, const void *gbase, uint32_t bytes) {
    const uint4 *src = reinterpret_cast<const uint4 *>(gbase);
    uint4 *dst = reinterpret_cast<uint4 *>(lds);
    const uint32_t n16 = bytes / 16;
    for (uint32_t i = threadIdx.x; i < n16; i += blockDim.x) dst[i] = src[i];
}

// Digit sum of a subsystem word: sum over bit planes t of 2^t * popcount.
__device__ __forceinline__ int digit_sum(const SectorDesc &sd, uint32_t w) {
    if (sd.nb == 1) return __popc(w);
    int s = 0;
    for (int t = 0; t < sd.nb; ++t) s += __popc(w & sd.field_mask[t]) << t;
    return s;
}

__device__ __forceinline__ uint32_t sub_word(const SectorDesc &sd, uint64_t s, int k) {
    return (uint32_t)(s >> sd.shift[k]) & ((1u << sd.wbits[k]) - 1u);
}

// Alg. i with the fused table: index = sum_k C_k[lambda_k][w_k].  With kCheck,
// returns the sentinel for states outside the sector.
template <typename IdxT, bool kCheck>
__device__ __forceinline__ IdxT rank_state(const SectorDesc &sd, const Tables<IdxT> &T,
                                           uint64_t s) {
    if (kCheck && sd.total_bits < 64 && (s >> sd.total_bits)) return Bad<IdxT>::value;
    IdxT idx = 0;
    int lam = 0;
    for (int k = 0; k < sd.N; ++k) {
        const uint32_t w = sub_word(sd, s, k);
        if (kCheck && (lam < sd.lam_lo[k] || lam > sd.lam_hi[k])) return Bad<IdxT>::value;
        const IdxT c = T.ctab[sd.ctab_row0[k] + (uint32_t)(lam - sd.lam_lo[k]) * sd.ctab_rowlen[k] + w];
        if (kCheck && c == Bad<IdxT>::value) return Bad<IdxT>::value;
        idx += c;
        lam += digit_sum(sd, w);
    }
    if (kCheck && lam != sd.n) return Bad<IdxT>::value;
    return idx;
}

// Exact idx / str for a quotient below 2^14: float estimate, one-step correction.
template <typename IdxT>
__device__ __forceinline__ uint32_t small_quotient(IdxT rem, IdxT str, float rcp, IdxT &prod) {
    uint32_t q = (uint32_t)((float)rem * rcp);
    IdxT qs = (IdxT)q * str;
    if (qs > rem) {
        --q;
        qs -= str;
    } else if (rem - qs >= str) {
        ++q;
        qs += str;
    }
    prod = qs;
    return q;
}

// Alg. iii: for each P_k (k < N-1) find n_k with offset(n_k) <= rem < offset(n_k+1),
// peel off the offset and stride*index_k, read the word from the inverse table;
// the last subsystem takes the remainder.  idx must be < dim.
// Also returns, per subsystem, the word, lambda_k and the contribution c_k.
// COUNT: find each particle count by counting the offsets at or below the
// remainder (every entry of the row read, independent loads) instead of a scan
// that stops at the first larger one (fewer reads, each waiting on the last);
// the batched unrank is faster with the count, the H*x decode with the scan.
template <typename IdxT, int NMAX, bool COUNT = false>
__device__ __forceinline__ uint64_t unrank_state(const SectorDesc &sd, const Tables<IdxT> &T,
                                                 IdxT idx, uint32_t *w_out, int *lam_out,
                                                 IdxT *c_out) {
    uint64_t s = 0;
    int lam = 0;
    IdxT rem = idx;
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
        if (k < sd.N - 1) {
            const int lo = max(0, sd.n - lam - sd.rest_max[k]);
            const int hi = min(sd.mk[k], sd.n - lam);
            const uint32_t row = sd.dec_row0[k] + (uint32_t)(lam - sd.lam_lo[k]) * (sd.mk[k] + 1);
            int m = lo;
            if constexpr (COUNT) {  // the offsets rise with m: m - lo = entries of [lo, hi) <= rem
                const int mk = sd.mk[k];
#pragma unroll 4
                for (int i = 0; i < mk; ++i) m += (i >= lo && i < hi && rem >= T.doff[row + i + 1]) ? 1 : 0;
            } else {
                while (m < hi && rem >= T.doff[row + m + 1]) ++m;
            }
            const IdxT off = T.doff[row + m];
            rem -= off;
            IdxT prod;
            const uint32_t q = small_quotient<IdxT>(rem, T.dstr[row + m], T.drcp[row + m], prod);
            rem -= prod;
            const uint32_t w = T.inv[T.invs[sd.inv_start0[k] + m] + q];
            s |= (uint64_t)w << sd.shift[k];
            if (w_out) {
                w_out[k] = w;
                lam_out[k] = lam;
                c_out[k] = off + prod;
            }
            lam += m;
        } else if (k == sd.N - 1) {
            const int m = sd.n - lam;
            const uint32_t w = T.inv[T.invs[sd.inv_start0[k] + m] + (uint32_t)rem];
            s |= (uint64_t)w << sd.shift[k];
            if (w_out) {
                w_out[k] = w;
                lam_out[k] = lam;
                c_out[k] = rem;
            }
        }
    }
    return s;
}

}  // namespace dcs
