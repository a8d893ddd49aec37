// Rank and unrank without tables of states (eq. N=L, Alg. on-the-fly): the canonical
// order of a sector cut into L single-site subsystems is the lexicographic order of the
// digit strings, site 0 first, and the rank is the sum over the sites i of the number of
// completions that put a smaller digit at site i, sum_{k < q_i} D(L-1-i, n - lambda_i - k).
// The counts D(g, m) (g < L, m <= n; binomials for Q = 2) are not stored anywhere: every
// workgroup derives them in LDS by App. A's recurrence before serving its states, for
// one Q or a local dimension per site.
#include "dcs_internal.h"

#include <algorithm>
#include <vector>

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void count_bad(uint64_t *nbad, bool bad) {
    if (!nbad) return;
    const uint64_t mask = __ballot(bad);
    if (mask && (threadIdx.x % warpSize) == 0) atomicAdd((unsigned long long *)nbad, (unsigned long long)__popcll(mask));
}

// Any Q (eq. N=L with D_Q): the rank is the sum over the sites i of
// sum_{k < q_i} D_Q(L-1-i, n - lambda_i - k), the number of completions that put a
// smaller digit at site i.  D_Q(g, m) for g < L and m <= n is a small count table,
// not a table of states: every workgroup builds it in LDS by App. A's recurrence
// D(g, m) = sum_{d < Q} D(g-1, m-d), one row per step, and then serves its states.
// The host checks that every entry stays below 2^64.  Sites may have their own local
// dimensions (Sec. 5): row g then counts strings on the last g sites, the step to g
// adding site L-g with its own q.
struct SiteDims {
    uint8_t q[64];  // local dimension of each site
};

__device__ void build_counts(uint64_t *Dt, int L, int n, const SiteDims &qs) {
    const int W = n + 1;
    for (int m = threadIdx.x; m <= n; m += blockDim.x) Dt[m] = m == 0 ? 1u : 0u;
    __syncthreads();
    for (int g = 1; g < L; ++g) {
        const int Q = qs.q[L - g];
        for (int m = threadIdx.x; m <= n; m += blockDim.x) {
            uint64_t acc = 0;
            for (int d = 0; d < Q && d <= m; ++d) acc += Dt[(g - 1) * W + m - d];
            Dt[g * W + m] = acc;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kThreads) void lexq_rank_kernel(int L, int n, SiteDims qs, int nb,
                                                             const uint64_t *__restrict__ st, uint64_t *__restrict__ out,
                                                             size_t count, uint64_t *nbad) {
    extern __shared__ uint64_t Dt[];  // [L][n + 1]
    build_counts(Dt, L, n, qs);
    const int W = n + 1;
    const uint64_t dmask = (1ull << nb) - 1ull;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t base = (size_t)blockIdx.x * blockDim.x; base < count; base += stride) {
        const size_t t = base + threadIdx.x;
        bool bad = false;
        if (t < count) {
            const uint64_t s = st[t];
            bad = L * nb < 64 && (s >> (L * nb)) != 0;
            uint64_t idx = 0;
            int lam = 0;
            for (int i = 0; i < L && !bad; ++i) {
                const int g = L - 1 - i;
                const int q = (int)((s >> (nb * g)) & dmask);
                bad = q >= qs.q[i] || lam + q > n;
                for (int k = 0; k < q && !bad; ++k) {
                    const int m = n - lam - k;  // in [0, n]: lam + q <= n
                    idx += Dt[g * W + m];
                }
                lam += q;
            }
            bad = bad || lam != n;
            out[t] = bad ? DCS_INVALID_INDEX : idx;
        }
        count_bad(nbad, bad);
    }
}

__global__ __launch_bounds__(kThreads) void lexq_unrank_kernel(int L, int n, SiteDims qs, int nb, uint64_t dim,
                                                               const uint64_t *__restrict__ ix, uint64_t *__restrict__ out,
                                                               size_t count, uint64_t *nbad) {
    extern __shared__ uint64_t Dt[];  // [L][n + 1]
    build_counts(Dt, L, n, qs);
    const int W = n + 1;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t base = (size_t)blockIdx.x * blockDim.x; base < count; base += stride) {
        const size_t t = base + threadIdx.x;
        bool bad = false;
        if (t < count) {
            uint64_t idx = ix[t];
            bad = idx >= dim;
            uint64_t s = 0;
            int rem = n;
            for (int i = 0; i < L && !bad; ++i) {
                const int g = L - 1 - i;
                // the digit: skip the completions of every smaller digit
                int d = 0;
                for (; d < qs.q[i] - 1 && d <= rem; ++d) {
                    const uint64_t c = Dt[g * W + rem - d];
                    if (idx < c) break;
                    idx -= c;
                }
                s |= (uint64_t)d << (nb * g);
                rem -= d;
            }
            bad = bad || rem != 0;
            out[t] = bad ? DCS_INVALID_INDEX : s;
        }
        count_bad(nbad, bad);
    }
}

// the checks of the any-Q calls (qs: the local dimension of every site, L entries); the
// dimension and the LDS bytes of the count table
int check_args_q(int L, int n, const int *qs, SiteDims *dims, int *nb_out, uint64_t *dim_out, size_t *lds_out) {
    if (L < 1 || L > 64) return dcs::set_error(DCS_EINVAL, "L=%d outside [1, 64]", L);
    int Q = 0, nmax = 0;
    for (int i = 0; i < L; ++i) {
        if (qs[i] < 2 || qs[i] > 16) return dcs::set_error(DCS_EINVAL, "local dimension %d of site %d outside [2, 16]", qs[i], i);
        Q = std::max(Q, qs[i]);
        nmax += qs[i] - 1;
        dims->q[i] = (uint8_t)qs[i];
    }
    int nb = 0;
    while ((1 << nb) < Q) ++nb;
    if (L * nb > 64) return dcs::set_error(DCS_EINVAL, "L=%d needs %d bits > 64", L, L * nb);
    if (n < 0 || n > nmax) return dcs::set_error(DCS_EINVAL, "n_particles %d outside [0, %d]", n, nmax);
    // D_Q(g, m) for g <= L, m <= n in 128 bits: every entry the kernels hold (g < L) and
    // the dimension D_Q(L, n) must stay below 2^64
    std::vector<unsigned __int128> prev(n + 1, 0), cur(n + 1, 0);
    prev[0] = 1;
    for (int g = 1; g <= L; ++g) {
        const int q = qs[L - g];
        for (int m = 0; m <= n; ++m) {
            unsigned __int128 acc = 0;
            for (int d = 0; d < q && d <= m; ++d) acc += prev[m - d];
            if (acc >> 64) return dcs::set_error(DCS_EUNSUPPORTED, "L=%d, n=%d, Q=%d: counts pass 2^64", L, n, Q);
            cur[m] = acc;
        }
        std::swap(prev, cur);
    }
    *nb_out = nb;
    *dim_out = (uint64_t)prev[n];
    *lds_out = (size_t)L * (size_t)(n + 1) * sizeof(uint64_t);
    if (*lds_out > 64 * 1024) return dcs::set_error(DCS_EUNSUPPORTED, "count table of %zu bytes", *lds_out);
    return DCS_OK;
}

int grid(size_t count) {
    const size_t blocks = (count + kThreads - 1) / kThreads;
    return (int)(blocks < 4096 ? blocks : 4096);
}

}  // namespace

using namespace dcs;

namespace {

int lexq_launch(bool rank, int L, int n, const int *qs, const uint64_t *in, uint64_t *out, size_t count, uint64_t *nbad,
                void *stream) {
    SiteDims dims{};
    int nb = 0;
    uint64_t dim = 0;
    size_t lds = 0;
    if (int r = check_args_q(L, n, qs, &dims, &nb, &dim, &lds)) return r;
    if (count == 0) return DCS_OK;
    if (!in || !out) return set_error(DCS_EINVAL, "NULL array");
    if (rank)
        lexq_rank_kernel<<<grid(count), kThreads, lds, (hipStream_t)stream>>>(L, n, dims, nb, in, out, count, nbad);
    else
        lexq_unrank_kernel<<<grid(count), kThreads, lds, (hipStream_t)stream>>>(L, n, dims, nb, dim, in, out, count, nbad);
    return check_hip(hipGetLastError(), rank ? "lex rank launch" : "lex unrank launch");
}

int uniform_dims(int L, int Q, int *qs) {
    if (Q < 2 || Q > 16) return set_error(DCS_EINVAL, "Q=%d outside [2, 16]", Q);
    if (L < 1 || L > 64) return set_error(DCS_EINVAL, "L=%d outside [1, 64]", L);
    for (int i = 0; i < L; ++i) qs[i] = Q;
    return DCS_OK;
}

int copy_dims(int L, const int32_t *local_dims, int *qs) {
    if (!local_dims) return set_error(DCS_EINVAL, "local_dims is NULL");
    if (L < 1 || L > 64) return set_error(DCS_EINVAL, "L=%d outside [1, 64]", L);
    for (int i = 0; i < L; ++i) qs[i] = local_dims[i];
    return DCS_OK;
}

}  // namespace

extern "C" int dcs_lex_rank_q(int L, int n, int Q, const uint64_t *st, uint64_t *idx, size_t count, uint64_t *nbad,
                              void *stream) {
    clear_error();
    int qs[64];
    if (int r = uniform_dims(L, Q, qs)) return r;
    return lexq_launch(true, L, n, qs, st, idx, count, nbad, stream);
}

extern "C" int dcs_lex_unrank_q(int L, int n, int Q, const uint64_t *idx, uint64_t *st, size_t count, uint64_t *nbad,
                                void *stream) {
    clear_error();
    int qs[64];
    if (int r = uniform_dims(L, Q, qs)) return r;
    return lexq_launch(false, L, n, qs, idx, st, count, nbad, stream);
}

extern "C" int dcs_lex_rank_mixed(int L, int n, const int32_t *local_dims, const uint64_t *st, uint64_t *idx,
                                  size_t count, uint64_t *nbad, void *stream) {
    clear_error();
    int qs[64];
    if (int r = copy_dims(L, local_dims, qs)) return r;
    return lexq_launch(true, L, n, qs, st, idx, count, nbad, stream);
}

extern "C" int dcs_lex_unrank_mixed(int L, int n, const int32_t *local_dims, const uint64_t *idx, uint64_t *st,
                                    size_t count, uint64_t *nbad, void *stream) {
    clear_error();
    int qs[64];
    if (int r = copy_dims(L, local_dims, qs)) return r;
    return lexq_launch(false, L, n, qs, idx, st, count, nbad, stream);
}

extern "C" int dcs_lex_rank(int L, int n, const uint64_t *st, uint64_t *idx, size_t count, uint64_t *nbad,
                            void *stream) {
    return dcs_lex_rank_q(L, n, 2, st, idx, count, nbad, stream);
}

extern "C" int dcs_lex_unrank(int L, int n, const uint64_t *idx, uint64_t *st, size_t count, uint64_t *nbad,
                              void *stream) {
    return dcs_lex_unrank_q(L, n, 2, idx, st, count, nbad, stream);
}
