// Rank and unrank without tables: the canonical order of a spin-1/2 sector cut
// into L single-site subsystems (eq. N=L), which is the lexicographic order of
// the site strings, site 0 first.  Alg. on-the-fly sums, over the sites, the
// number of completions with a smaller digit there; for Q = 2 that is, over the
// occupied sites i, D_2(L-1-i, n - lambda_i) = C(L-1-i, n - lambda_i).  No
// table: each thread steps one binomial coefficient along the sites by exact
// integer updates (C(p+1, r) = C(p, r) (p+1) / (p+1-r) and
// C(p, r+1) = C(p, r) (p-r) / (r+1)), so the products stay below 2^64 for every
// sector the host admits (checked there).
#include "dcs_internal.h"

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void count_bad(uint64_t *nbad, bool bad) {
    if (!nbad) return;
    const uint64_t mask = __ballot(bad);
    if (mask && (threadIdx.x % warpSize) == 0) atomicAdd((unsigned long long *)nbad, (unsigned long long)__popcll(mask));
}

// rank = sum over occupied sites, taken from the last site (p = 0, p = L-1-i) to
// the first, of C(p, t + 1) with t the occupied sites after it.  c tracks
// C(p, t + 1) as p grows (and t with it).
__global__ __launch_bounds__(kThreads) void lex_rank_kernel(int L, int n, const uint64_t *__restrict__ st,
                                                            uint64_t *__restrict__ out, size_t count,
                                                            uint64_t *nbad) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t base = (size_t)blockIdx.x * blockDim.x; base < count; base += stride) {
        const size_t k = base + threadIdx.x;
        bool bad = false;
        if (k < count) {
            const uint64_t s = st[k];
            bad = (L < 64 && (s >> L) != 0) || __popcll(s) != n;
            uint64_t idx = 0;
            if (!bad) {
                uint64_t c = 0;  // C(p, t + 1), zero while p < t + 1
                int t = 0;
                for (int p = 0; p < L; ++p) {
                    // c = C(p, t + 1) here
                    if ((s >> p) & 1u) {
                        idx += c;
                        // t -> t + 1: C(p, t + 2) = C(p, t + 1) (p - t - 1) / (t + 2)
                        c = p - t - 1 > 0 ? c * (uint64_t)(p - t - 1) / (uint64_t)(t + 2) : 0;
                        ++t;
                    }
                    // p -> p + 1: C(p + 1, t + 1) = C(p, t + 1) (p + 1) / (p - t), or 1 when p + 1 == t + 1
                    c = p + 1 == t + 1 ? 1 : (p - t > 0 ? c * (uint64_t)(p + 1) / (uint64_t)(p - t) : 0);
                }
            }
            out[k] = bad ? DCS_INVALID_INDEX : idx;
        }
        count_bad(nbad, bad);
    }
}

// unrank: from site 0 on, with rem particles left for the g = L-1-i sites after
// site i, C(g, rem) completions put a 0 at site i; c tracks C(g, rem).
__global__ __launch_bounds__(kThreads) void lex_unrank_kernel(int L, int n, uint64_t dim, const uint64_t *__restrict__ ix,
                                                              uint64_t *__restrict__ out, size_t count, uint64_t c0,
                                                              uint64_t *nbad) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t base = (size_t)blockIdx.x * blockDim.x; base < count; base += stride) {
        const size_t k = base + threadIdx.x;
        bool bad = false;
        if (k < count) {
            uint64_t idx = ix[k];
            bad = idx >= dim;
            uint64_t s = 0;
            if (!bad) {
                uint64_t c = c0;  // C(L - 1, n)
                int rem = n;
                for (int i = 0; i < L; ++i) {
                    const int g = L - 1 - i;  // sites after i; c = C(g, rem)
                    if (rem > 0 && idx >= c) {  // a 1 here
                        idx -= c;
                        s |= 1ull << g;
                        // C(g - 1, rem - 1) = C(g, rem) rem / g
                        c = g > 0 ? c * (uint64_t)rem / (uint64_t)g : 0;
                        --rem;
                    } else if (g > 0) {
                        // C(g - 1, rem) = C(g, rem) (g - rem) / g
                        c = c * (uint64_t)(g - rem) / (uint64_t)g;
                    }
                }
            }
            out[k] = bad ? DCS_INVALID_INDEX : s;
        }
        count_bad(nbad, bad);
    }
}

// C(a, b) exactly (host, 128-bit), and the largest product the kernels form
unsigned __int128 binom(int a, int b) {
    if (b < 0 || b > a) return 0;
    unsigned __int128 c = 1;
    for (int i = 1; i <= b; ++i) c = c * (unsigned __int128)(a - b + i) / (unsigned __int128)i;
    return c;
}

int check_args(int L, int n, uint64_t *dim_out) {
    if (L < 1 || L > 64) return dcs::set_error(DCS_EINVAL, "L=%d outside [1, 64]", L);
    if (n < 0 || n > L) return dcs::set_error(DCS_EINVAL, "n_particles %d outside [0, %d]", n, L);
    // the coefficients the kernels form: C(p, r) with at most L - n empty sites
    // among the p, so r >= p - (L - n) - 1
    unsigned __int128 worst = 0;
    for (int p = 0; p <= L; ++p)
        for (int r = std::max(0, p - (L - n) - 1); r <= n + 1 && r <= p + 1; ++r) {
            const unsigned __int128 v = binom(p, r) * (unsigned __int128)(p + 1);
            if (v > worst) worst = v;
        }
    if (worst >> 64) return dcs::set_error(DCS_EUNSUPPORTED, "L=%d, n=%d: the on-the-fly coefficients pass 2^64", L, n);
    *dim_out = (uint64_t)binom(L, n);
    return DCS_OK;
}

int grid(size_t count) {
    const size_t blocks = (count + kThreads - 1) / kThreads;
    return (int)(blocks < 4096 ? blocks : 4096);
}

}  // namespace

using namespace dcs;

extern "C" int dcs_lex_rank(int L, int n, const uint64_t *st, uint64_t *idx, size_t count, uint64_t *nbad,
                            void *stream) {
    clear_error();
    uint64_t dim = 0;
    if (int r = check_args(L, n, &dim)) return r;
    if (count == 0) return DCS_OK;
    if (!st || !idx) return set_error(DCS_EINVAL, "NULL array");
    lex_rank_kernel<<<grid(count), kThreads, 0, (hipStream_t)stream>>>(L, n, st, idx, count, nbad);
    return check_hip(hipGetLastError(), "lex rank launch");
}

extern "C" int dcs_lex_unrank(int L, int n, const uint64_t *idx, uint64_t *st, size_t count, uint64_t *nbad,
                              void *stream) {
    clear_error();
    uint64_t dim = 0;
    if (int r = check_args(L, n, &dim)) return r;
    if (count == 0) return DCS_OK;
    if (!st || !idx) return set_error(DCS_EINVAL, "NULL array");
    const uint64_t c0 = (uint64_t)binom(L - 1, n);
    lex_unrank_kernel<<<grid(count), kThreads, 0, (hipStream_t)stream>>>(L, n, dim, idx, st, count, c0, nbad);
    return check_hip(hipGetLastError(), "lex unrank launch");
}
