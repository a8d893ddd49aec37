// Generic number-conserving local operators on one sector (Sec. 4.1, the operator
// class built from operator strings and user-defined local matrices; App. C, the
// terms of one cluster of sites merged into one sparse matrix).
//
// Host: the terms (coef, sites, Q^m x Q^m matrix) are checked to conserve the
// particle number and grouped greedily into clusters of at most `cluster_sites`
// sites (a term joins the first cluster whose site set it can extend within the
// limit, else it opens one); each cluster's sum of embedded terms is stored row by
// row (CSR over the cluster's local index of the output state), every entry with
// the packed digits of its input state and its value.
//
// Device: one thread per row s of the sector (pull form, y_s = sum_t O_st x_t):
// unrank s, and for each cluster read the local index of s on the cluster's sites,
// walk that row's entries, write the entry's digits into s, rank the result with the
// fused tables (a diagonal entry keeps s and its index), gather x there.
#include "device_common.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace dcs {
namespace op {

constexpr int kOpMaxSites = 8;       // sites of one cluster
constexpr uint32_t kOpMaxLocal = 4096;  // Q^m of one cluster
constexpr int kOpThreads = 256;

struct OpCluster {
    uint8_t m;
    uint8_t site[kOpMaxSites];
    uint8_t pad[3];
    uint32_t row0;  // first entry of the cluster's row pointers
};
static_assert(sizeof(OpCluster) == 16, "cluster record");

struct OpParams {
    SectorDesc sd;  // first: read in place in the kernel argument segment
    const char *blob;
    const OpCluster *cl;
    const uint32_t *rowptr;  // per cluster Q^m + 1 offsets into the entries
    const uint32_t *dep;     // input digits of each entry: site j's digit at bits nb * j
    const void *val;         // entry values in the compute type
    const void *x;
    void *y;
    int ncl;
};
static_assert(sizeof(OpParams) <= 4096, "kernel arguments are limited to 4 KiB");

template <typename IdxT, typename T, bool GT>
__global__ __launch_bounds__(kOpThreads) void op_kernel(const OpParams P_arg) {
    (void)P_arg;
    const OpParams &P = kernel_arg0<OpParams>();
    const SectorDesc &sd = P.sd;
    extern __shared__ __align__(16) char lds[];
    if constexpr (!GT) {
        stage_blob(lds, P.blob, sd.lay_bytes);
        __syncthreads();
    }
    const Tables<IdxT> Tb = tables_at<IdxT>(GT ? P.blob : lds, sd);
    const T *__restrict__ x = reinterpret_cast<const T *>(P.x);
    T *__restrict__ y = reinterpret_cast<T *>(P.y);
    const T *__restrict__ val = reinterpret_cast<const T *>(P.val);
    const uint64_t dmask = (1ull << sd.nb) - 1ull;
    const uint64_t stride = (uint64_t)gridDim.x * kOpThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kOpThreads + threadIdx.x; i < sd.dim; i += stride) {
        const uint64_t s = unrank_state<IdxT, kMaxSub>(sd, Tb, (IdxT)i, nullptr, nullptr, nullptr);
        T acc = (T)0;
        for (int c = 0; c < P.ncl; ++c) {  // uniform
            const OpCluster C = P.cl[c];
            int pos[kOpMaxSites];
            uint64_t clmask = 0;
            uint32_t a = 0;
#pragma unroll
            for (int j = 0; j < kOpMaxSites; ++j) {
                if (j < C.m) {
                    const int site = C.site[j];
                    pos[j] = sd.shift[sd.site_sub[site]] + sd.site_bit[site];
                    a = a * (uint32_t)sd.Q + (uint32_t)((s >> pos[j]) & dmask);
                    clmask |= dmask << pos[j];
                } else {
                    pos[j] = 0;
                }
            }
            const uint64_t keep = s & ~clmask;
            const uint32_t e1 = P.rowptr[C.row0 + a + 1];
            for (uint32_t e = P.rowptr[C.row0 + a]; e < e1; ++e) {
                const uint32_t d = P.dep[e];
                uint64_t s2 = keep;
#pragma unroll
                for (int j = 0; j < kOpMaxSites; ++j)
                    if (j < C.m) s2 |= (uint64_t)((d >> (sd.nb * j)) & (uint32_t)dmask) << pos[j];
                const uint64_t t = s2 == s ? i : (uint64_t)rank_state<IdxT, false>(sd, Tb, s2);
                acc += val[e] * (t < sd.dim ? x[t] : (T)0);
            }
        }
        y[i] = acc;
    }
}

}  // namespace op
}  // namespace dcs

struct dcs_operator {
    int Q = 0, L = 0, nb = 0, device = 0;
    int ncl = 0, max_sites = 0;
    uint64_t nnz = 0;
    void *d_base = nullptr;
    const dcs::op::OpCluster *d_cl = nullptr;
    const uint32_t *d_rowptr = nullptr, *d_dep = nullptr;
    const double *d_val = nullptr;
    const float *d_valf = nullptr;
};

namespace {

using namespace dcs;
using namespace dcs::op;

// digit j (first site most significant) of the local index a over m sites
inline int local_digit(uint32_t a, int j, int m, int Q) {
    for (int k = m - 1; k > j; --k) a /= (uint32_t)Q;
    return (int)(a % (uint32_t)Q);
}

inline int digit_sum_local(uint32_t a, int m, int Q) {
    int s = 0;
    for (int k = 0; k < m; ++k) {
        s += (int)(a % (uint32_t)Q);
        a /= (uint32_t)Q;
    }
    return s;
}

inline uint32_t ipow(int Q, int m) {
    uint64_t v = 1;
    for (int k = 0; k < m; ++k) v *= (uint64_t)Q;
    return v > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)v;
}

struct Entry {
    uint32_t row, col;
    double v;
};

}  // namespace

extern "C" int dcs_operator_create(int Q, int L, int num_terms, const int32_t *term_nsites,
                                   const int32_t *term_sites, const double *term_coefs,
                                   const double *term_mats, int cluster_sites, int device,
                                   dcs_operator **out) {
    clear_error();
    if (!out) return set_error(DCS_EINVAL, "out is NULL");
    *out = nullptr;
    if (Q < 2 || Q > 16) return set_error(DCS_EINVAL, "Q=%d outside [2, 16]", Q);
    if (L < 1 || L > kMaxSites) return set_error(DCS_EINVAL, "L=%d outside [1, %d]", L, kMaxSites);
    if (num_terms < 0) return set_error(DCS_EINVAL, "num_terms %d < 0", num_terms);
    if (num_terms > 0 && (!term_nsites || !term_sites || !term_coefs || !term_mats))
        return set_error(DCS_EINVAL, "NULL term array");
    if (cluster_sites < 1 || cluster_sites > kOpMaxSites)
        return set_error(DCS_EINVAL, "cluster_sites=%d outside [1, %d]", cluster_sites, kOpMaxSites);
    // check every term; offsets of its sites and matrix
    std::vector<size_t> site_off(num_terms + 1, 0), mat_off(num_terms + 1, 0);
    for (int t = 0; t < num_terms; ++t) {
        const int m = term_nsites[t];
        if (m < 1 || m > kOpMaxSites)
            return set_error(DCS_EUNSUPPORTED, "term %d has %d sites (1..%d)", t, m, kOpMaxSites);
        const uint32_t n = ipow(Q, m);
        if (n > kOpMaxLocal) return set_error(DCS_EUNSUPPORTED, "term %d: Q^m = %u > %u", t, n, kOpMaxLocal);
        site_off[t + 1] = site_off[t] + (size_t)m;
        mat_off[t + 1] = mat_off[t] + (size_t)n * n;
    }
    for (int t = 0; t < num_terms; ++t) {
        const int m = term_nsites[t];
        const int32_t *st = term_sites + site_off[t];
        for (int j = 0; j < m; ++j) {
            if (st[j] < 0 || st[j] >= L) return set_error(DCS_EINVAL, "term %d: site %d outside [0, %d)", t, st[j], L);
            for (int k = 0; k < j; ++k)
                if (st[k] == st[j]) return set_error(DCS_EINVAL, "term %d lists site %d twice", t, st[j]);
        }
        if (!std::isfinite(term_coefs[t])) return set_error(DCS_EINVAL, "term %d: coefficient not finite", t);
        const uint32_t n = ipow(Q, m);
        const double *M = term_mats + mat_off[t];
        for (uint32_t b = 0; b < n; ++b)
            for (uint32_t a = 0; a < n; ++a) {
                const double v = M[(size_t)b * n + a];
                if (!std::isfinite(v)) return set_error(DCS_EINVAL, "term %d: matrix entry not finite", t);
                if (v != 0.0 && digit_sum_local(b, m, Q) != digit_sum_local(a, m, Q))
                    return set_error(DCS_EINVAL,
                                     "term %d does not conserve the particle number (entry %u, %u)", t, b, a);
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
            if (U.size() == cl_sites[c].size() ||
                ((int)U.size() <= cluster_sites && ipow(Q, (int)U.size()) <= kOpMaxLocal)) {
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
    // each cluster's matrix, CSR by output local index
    const int nb = (Q - 1) > 0 ? 32 - __builtin_clz((unsigned)(Q - 1)) : 1;
    std::vector<OpCluster> hcl(cl_sites.size());
    std::vector<uint32_t> rowptr, dep;
    std::vector<double> val;
    int max_sites = 0;
    for (size_t c = 0; c < cl_sites.size(); ++c) {
        const int m = (int)cl_sites[c].size();
        const uint32_t n = ipow(Q, m);
        max_sites = std::max(max_sites, m);
        std::vector<Entry> ents;
        for (int t : cl_terms[c]) {
            const int mt = term_nsites[t];
            const int32_t *st = term_sites + site_off[t];
            const uint32_t nt = ipow(Q, mt);
            const double *M = term_mats + mat_off[t];
            int p[kOpMaxSites];  // cluster position of term site j
            for (int j = 0; j < mt; ++j)
                p[j] = (int)(std::lower_bound(cl_sites[c].begin(), cl_sites[c].end(), st[j]) - cl_sites[c].begin());
            int da[kOpMaxSites];
            for (uint32_t a = 0; a < n; ++a) {  // input state of the cluster
                for (int j = 0; j < m; ++j) da[j] = local_digit(a, j, m, Q);
                uint32_t at = 0;
                for (int j = 0; j < mt; ++j) at = at * (uint32_t)Q + (uint32_t)da[p[j]];
                for (uint32_t bt = 0; bt < nt; ++bt) {
                    const double v = M[(size_t)bt * nt + at];
                    if (v == 0.0) continue;
                    int db[kOpMaxSites];
                    std::copy(da, da + m, db);
                    for (int j = 0; j < mt; ++j) db[p[j]] = local_digit(bt, j, mt, Q);
                    uint32_t b = 0;
                    for (int j = 0; j < m; ++j) b = b * (uint32_t)Q + (uint32_t)db[j];
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
        for (uint32_t b = 0; b < n; ++b) {
            rowptr.push_back((uint32_t)val.size());
            while (e < ents.size() && ents[e].row == b) {
                const uint32_t col = ents[e].col;
                double v = 0.0;
                while (e < ents.size() && ents[e].row == b && ents[e].col == col) v += ents[e++].v;
                if (v == 0.0) continue;
                uint32_t d = 0;
                for (int j = 0; j < m; ++j) d |= (uint32_t)local_digit(col, j, m, Q) << (nb * j);
                dep.push_back(d);
                val.push_back(v);
            }
        }
        rowptr.push_back((uint32_t)val.size());
    }
    dcs_operator *o = new (std::nothrow) dcs_operator();
    if (!o) return set_error(DCS_ENOMEM, "host allocation failed");
    o->Q = Q;
    o->L = L;
    o->nb = nb;
    o->device = device;
    o->ncl = (int)hcl.size();
    o->max_sites = max_sites;
    o->nnz = val.size();
    // one device allocation: clusters | row pointers | digits | FP64 values | FP32 values
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t b_cl = al(std::max<size_t>(hcl.size(), 1) * sizeof(OpCluster));
    const size_t b_rp = al(std::max<size_t>(rowptr.size(), 1) * 4);
    const size_t b_dep = al(std::max<size_t>(dep.size(), 1) * 4);
    const size_t b_val = al(std::max<size_t>(val.size(), 1) * 8);
    const size_t b_valf = al(std::max<size_t>(val.size(), 1) * 4);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        delete o;
        return set_error(DCS_EINVAL, "device %d not present", device);
    }
    DeviceGuard g(device);
    char *base = nullptr;
    if (hipMalloc((void **)&base, b_cl + b_rp + b_dep + b_val + b_valf) != hipSuccess) {
        (void)hipGetLastError();
        delete o;
        return set_error(DCS_ENOMEM, "device allocation of %zu bytes failed", b_cl + b_rp + b_dep + b_val + b_valf);
    }
    o->d_base = base;
    o->d_cl = (const OpCluster *)base;
    o->d_rowptr = (const uint32_t *)(base + b_cl);
    o->d_dep = (const uint32_t *)(base + b_cl + b_rp);
    o->d_val = (const double *)(base + b_cl + b_rp + b_dep);
    o->d_valf = (const float *)(base + b_cl + b_rp + b_dep + b_val);
    std::vector<float> valf(val.begin(), val.end());
    int r = DCS_OK;
    if (!hcl.empty()) r = check_hip(hipMemcpy((void *)o->d_cl, hcl.data(), hcl.size() * sizeof(OpCluster), hipMemcpyHostToDevice), "operator upload");
    if (!r && !rowptr.empty()) r = check_hip(hipMemcpy((void *)o->d_rowptr, rowptr.data(), rowptr.size() * 4, hipMemcpyHostToDevice), "operator upload");
    if (!r && !dep.empty()) r = check_hip(hipMemcpy((void *)o->d_dep, dep.data(), dep.size() * 4, hipMemcpyHostToDevice), "operator upload");
    if (!r && !val.empty()) r = check_hip(hipMemcpy((void *)o->d_val, val.data(), val.size() * 8, hipMemcpyHostToDevice), "operator upload");
    if (!r && !val.empty()) r = check_hip(hipMemcpy((void *)o->d_valf, valf.data(), valf.size() * 4, hipMemcpyHostToDevice), "operator upload");
    if (r) {
        (void)hipFree(base);
        delete o;
        return r;
    }
    *out = o;
    return DCS_OK;
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

extern "C" int dcs_operator_info(const dcs_operator *o, int *num_clusters, uint64_t *nnz, int *max_cluster_sites) {
    clear_error();
    if (!o) return set_error(DCS_EINVAL, "operator is NULL");
    if (num_clusters) *num_clusters = o->ncl;
    if (nnz) *nnz = o->nnz;
    if (max_cluster_sites) *max_cluster_sites = o->max_sites;
    return DCS_OK;
}

extern "C" int dcs_operator_apply(const dcs_sector *s, const dcs_operator *o, int dtype, const void *x, void *y,
                                  void *stream) {
    clear_error();
    if (!s || !o) return set_error(DCS_EINVAL, "NULL sector or operator");
    if (o->Q != s->desc.Q || o->L != s->desc.L)
        return set_error(DCS_EINVAL, "operator of Q=%d, L=%d on a sector of Q=%d, L=%d", o->Q, o->L, s->desc.Q,
                         s->desc.L);
    if (o->device != s->device)
        return set_error(DCS_EINVAL, "operator on device %d, sector on device %d", o->device, s->device);
    if (dtype != DCS_F32 && dtype != DCS_F64) return set_error(DCS_EINVAL, "dtype %d", dtype);
    if (!x || !y) return set_error(DCS_EINVAL, "NULL vector");
    const size_t bytes = (size_t)s->desc.dim * (dtype == DCS_F32 ? 4 : 8);
    if ((const char *)y < (const char *)x + bytes && (const char *)x < (const char *)y + bytes)
        return set_error(DCS_EINVAL, "y overlaps x");
    DeviceGuard g(s->device);
    OpParams P;
    memset(&P, 0, sizeof(P));
    P.sd = s->desc;
    P.blob = (const char *)s->dev.base;
    P.cl = o->d_cl;
    P.rowptr = o->d_rowptr;
    P.dep = o->d_dep;
    P.val = dtype == DCS_F32 ? (const void *)o->d_valf : (const void *)o->d_val;
    P.x = x;
    P.y = y;
    P.ncl = o->ncl;
    const size_t lds = s->gtab ? 0 : s->desc.lay_bytes;
    const uint64_t blocks = (s->desc.dim + kOpThreads - 1) / kOpThreads;
    const uint64_t cap = (uint64_t)device_cu_count(s->device) * 8;
    const int grid = (int)std::max<uint64_t>(1, std::min(blocks, cap));
    hipStream_t st = (hipStream_t)stream;
    auto go = [&](auto kern) -> int {
        if (int r = ensure_lds(kern, lds)) return r;
        kern<<<grid, kOpThreads, lds, st>>>(P);
        return check_hip(hipGetLastError(), "operator kernel launch");
    };
    if (dtype == DCS_F32) {
        if (s->wide) return s->gtab ? go(op_kernel<uint64_t, float, true>) : go(op_kernel<uint64_t, float, false>);
        return s->gtab ? go(op_kernel<uint32_t, float, true>) : go(op_kernel<uint32_t, float, false>);
    }
    if (s->wide) return s->gtab ? go(op_kernel<uint64_t, double, true>) : go(op_kernel<uint64_t, double, false>);
    return s->gtab ? go(op_kernel<uint32_t, double, true>) : go(op_kernel<uint32_t, double, false>);
}
