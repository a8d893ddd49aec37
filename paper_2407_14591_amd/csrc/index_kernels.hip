// Batched rank (Alg. i), unrank (Alg. iii) and enumeration of a sector.
//
// Persistent grid-stride kernels: every workgroup stages the sector's tables
// into LDS once (GT: tables too large for LDS are read in device memory), then
// each thread handles one item per iteration.  Invalid
// items are counted with one atomic per wavefront (ballot + popcount).
#include "device_common.h"

namespace dcs {
namespace {

constexpr int kThreads = 1024;  // two workgroups fill a CU under the tables' LDS (256: 0.13 / 0.23 ms at 2^24 states)

__device__ __forceinline__ void count_bad(uint64_t *nbad, bool bad) {
    if (!nbad) return;
    const uint64_t mask = __ballot(bad);
    if (mask && (threadIdx.x % warpSize) == 0) atomicAdd((unsigned long long *)nbad, (unsigned long long)__popcll(mask));
}

template <typename IdxT, bool GT>
__global__ __launch_bounds__(kThreads) void rank_kernel(SectorDesc sd_arg, const char *blob,
                                                        const uint64_t *__restrict__ st,
                                                        uint64_t *__restrict__ out, size_t count,
                                                        uint64_t *nbad) {
    (void)sd_arg;
    const SectorDesc &sd = kernel_arg0<SectorDesc>();
    extern __shared__ __align__(16) char lds[];
    if constexpr (!GT) {
        stage_blob(lds, blob, sd.lay_bytes);
        __syncthreads();
    }
    const Tables<IdxT> T = tables_at<IdxT>(GT ? blob : lds, sd);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t base = (size_t)blockIdx.x * blockDim.x; base < count; base += stride) {
        const size_t i = base + threadIdx.x;
        bool bad = false;
        if (i < count) {
            const IdxT r = rank_state<IdxT, true>(sd, T, st[i]);
            bad = r == Bad<IdxT>::value;
            out[i] = bad ? DCS_INVALID_INDEX : (uint64_t)r;
        }
        count_bad(nbad, bad);
    }
}

// Container (ii) of Sec. 4.2: each subsystem's local index from a search among the
// valid words of its digit sum in lexicographic (numeric) order -- the inverse
// table, a sorted list -- instead of the dense table indexed by the word; then
// c_k = offset_k(m, lambda) + stride_k(m, lambda) * index (eq. ck), the last
// subsystem contributing its index.  Words with a digit >= Q are not in the list.
template <typename IdxT, bool GT>
__global__ __launch_bounds__(kThreads) void rank_search_kernel(SectorDesc sd_arg, const char *blob,
                                                               const uint64_t *__restrict__ st,
                                                               uint64_t *__restrict__ out, size_t count,
                                                               uint64_t *nbad) {
    (void)sd_arg;
    const SectorDesc &sd = kernel_arg0<SectorDesc>();
    extern __shared__ __align__(16) char lds[];
    if constexpr (!GT) {
        stage_blob(lds, blob, sd.lay_bytes);
        __syncthreads();
    }
    const Tables<IdxT> T = tables_at<IdxT>(GT ? blob : lds, sd);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t base = (size_t)blockIdx.x * blockDim.x; base < count; base += stride) {
        const size_t i = base + threadIdx.x;
        bool bad = false;
        if (i < count) {
            const uint64_t s = st[i];
            bad = sd.total_bits < 64 && (s >> sd.total_bits) != 0;
            IdxT idx = 0;
            int lam = 0;
            for (int k = 0; k < sd.N && !bad; ++k) {
                const uint32_t w = sub_word(sd, s, k);
                const int m = digit_sum(sd, w);
                if (m > sd.mk[k] || lam < sd.lam_lo[k] || lam > sd.lam_hi[k]) {
                    bad = true;
                    break;
                }
                const uint32_t b = T.invs[sd.inv_start0[k] + m], e = T.invs[sd.inv_start0[k] + m + 1];
                uint32_t lo = b, hi = e;
                while (lo < hi) {  // first entry >= w
                    const uint32_t mid = (lo + hi) >> 1;
                    if ((uint32_t)T.inv[mid] < w) lo = mid + 1;
                    else hi = mid;
                }
                if (lo == e || (uint32_t)T.inv[lo] != w) {
                    bad = true;
                    break;
                }
                const IdxT sigma = (IdxT)(lo - b);
                if (k < sd.N - 1) {
                    const uint32_t row = sd.dec_row0[k] + (uint32_t)(lam - sd.lam_lo[k]) * (sd.mk[k] + 1) + m;
                    const IdxT str = T.dstr[row];
                    if (str == 0) {  // no completion of this prefix has n particles
                        bad = true;
                        break;
                    }
                    idx += T.doff[row] + str * sigma;
                } else {
                    idx += sigma;
                }
                lam += m;
            }
            bad = bad || lam != sd.n;
            out[i] = bad ? DCS_INVALID_INDEX : (uint64_t)idx;
        }
        count_bad(nbad, bad);
    }
}

template <typename IdxT, bool GT>
__global__ __launch_bounds__(kThreads) void unrank_kernel(SectorDesc sd_arg, const char *blob,
                                                          const uint64_t *__restrict__ idx,
                                                          uint64_t *__restrict__ out, size_t count,
                                                          uint64_t first, int use_first,
                                                          uint64_t *nbad) {
    (void)sd_arg;
    const SectorDesc &sd = kernel_arg0<SectorDesc>();
    extern __shared__ __align__(16) char lds[];
    if constexpr (!GT) {
        stage_blob(lds, blob, sd.lay_bytes);
        __syncthreads();
    }
    const Tables<IdxT> T = tables_at<IdxT>(GT ? blob : lds, sd);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t base = (size_t)blockIdx.x * blockDim.x; base < count; base += stride) {
        const size_t i = base + threadIdx.x;
        bool bad = false;
        if (i < count) {
            const uint64_t v = use_first ? first + i : idx[i];
            bad = v >= sd.dim;
            out[i] = bad ? DCS_INVALID_INDEX
                         : unrank_state<IdxT, kMaxSub, true>(sd, T, (IdxT)v, nullptr, nullptr, nullptr);
        }
        count_bad(nbad, bad);
    }
}

int grid_for(const dcs_sector *s, size_t count) {
    const size_t blocks = (count + kThreads - 1) / kThreads;
    const size_t cap = (size_t)device_cu_count(s->device) * 4;
    return (int)(blocks < cap ? blocks : cap);
}

}  // namespace

int launch_rank(const dcs_sector *s, const uint64_t *st, uint64_t *idx, size_t count,
                uint64_t *nbad, hipStream_t stream) {
    DeviceGuard g(s->device);
    const int grid = grid_for(s, count);
    const char *blob = (const char *)s->dev.base;
    const size_t lds = s->gtab ? 0 : s->desc.lay_bytes;  // tables in LDS or in device memory
    auto go = [&](auto kern) -> int {
        if (int r = ensure_lds(kern, lds)) return r;
        kern<<<grid, kThreads, lds, stream>>>(s->desc, blob, st, idx, count, nbad);
        return check_hip(hipGetLastError(), "rank kernel launch");
    };
    if (s->wide) return s->gtab ? go(rank_kernel<uint64_t, true>) : go(rank_kernel<uint64_t, false>);
    return s->gtab ? go(rank_kernel<uint32_t, true>) : go(rank_kernel<uint32_t, false>);
}

int launch_rank_search(const dcs_sector *s, const uint64_t *st, uint64_t *idx, size_t count,
                       uint64_t *nbad, hipStream_t stream) {
    DeviceGuard g(s->device);
    const int grid = grid_for(s, count);
    const char *blob = (const char *)s->dev.base;
    const size_t lds = s->gtab ? 0 : s->desc.lay_bytes;
    auto go = [&](auto kern) -> int {
        if (int r = ensure_lds(kern, lds)) return r;
        kern<<<grid, kThreads, lds, stream>>>(s->desc, blob, st, idx, count, nbad);
        return check_hip(hipGetLastError(), "rank (search) kernel launch");
    };
    if (s->wide) return s->gtab ? go(rank_search_kernel<uint64_t, true>) : go(rank_search_kernel<uint64_t, false>);
    return s->gtab ? go(rank_search_kernel<uint32_t, true>) : go(rank_search_kernel<uint32_t, false>);
}

// unrank of idx[0..count) (use_first = 0) or of first, first + 1, ... (enumerate)
static int launch_unrank_any(const dcs_sector *s, const uint64_t *idx, uint64_t *st, size_t count,
                             uint64_t first, int use_first, uint64_t *nbad, hipStream_t stream,
                             const char *what) {
    DeviceGuard g(s->device);
    const int grid = grid_for(s, count);
    const char *blob = (const char *)s->dev.base;
    const size_t lds = s->gtab ? 0 : s->desc.lay_bytes;
    auto go = [&](auto kern) -> int {
        if (int r = ensure_lds(kern, lds)) return r;
        kern<<<grid, kThreads, lds, stream>>>(s->desc, blob, idx, st, count, first, use_first, nbad);
        return check_hip(hipGetLastError(), what);
    };
    if (s->wide) return s->gtab ? go(unrank_kernel<uint64_t, true>) : go(unrank_kernel<uint64_t, false>);
    return s->gtab ? go(unrank_kernel<uint32_t, true>) : go(unrank_kernel<uint32_t, false>);
}

int launch_unrank(const dcs_sector *s, const uint64_t *idx, uint64_t *st, size_t count,
                  uint64_t *nbad, hipStream_t stream) {
    return launch_unrank_any(s, idx, st, count, 0, 0, nbad, stream, "unrank kernel launch");
}

int launch_enumerate(const dcs_sector *s, uint64_t first, size_t count, uint64_t *st,
                     hipStream_t stream) {
    return launch_unrank_any(s, nullptr, st, count, first, 1, nullptr, stream, "enumerate kernel launch");
}

}  // namespace dcs
