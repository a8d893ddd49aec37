// Host-side sector planner: dimensions, offsets, strides and the device tables
// of the divide-and-conquer index (Sec. 3.2 and 4.2 of arXiv:2407.14591).
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "dcs_internal.h"

namespace dcs {
namespace {

typedef unsigned __int128 u128;

// get(l, m): the number of digit strings on the last l sites with digit sum m, for
// 0 <= l <= L, by the recurrence D(l, m) = sum_{d < q} D(l-1, m-d) with q the local
// dimension of the site that the l-th step adds: the coefficients of the product of
// (1 + x + ... + x^{q_i - 1}) over those sites (App. A; with one Q, D_Q(l, m)).
// Values must stay below 2^63; returns false on overflow.
struct DimTable {
    int L = 0, mmax = 0;
    std::vector<uint64_t> v;
    bool build(const int *qs, int L_) {
        L = L_;
        mmax = 0;
        for (int i = 0; i < L; ++i) mmax += qs[i] - 1;
        v.assign((size_t)(L + 1) * (mmax + 1), 0);
        v[0] = 1;
        int cap = 0;
        for (int l = 1; l <= L; ++l) {
            const int q = qs[L - l];
            cap += q - 1;
            for (int m = 0; m <= cap; ++m) {
                u128 acc = 0;
                for (int d = 0; d < q && d <= m; ++d) acc += get(l - 1, m - d);
                if (acc >> 63) return false;
                v[(size_t)l * (mmax + 1) + m] = (uint64_t)acc;
            }
        }
        return true;
    }
    uint64_t get(int l, int m) const {
        if (l < 0 || l > L || m < 0 || m > mmax) return 0;
        return v[(size_t)l * (mmax + 1) + m];
    }
};

// the largest digit sum of sites [a, b)
inline int max_sum(const int *qs, int a, int b) {
    int t = 0;
    for (int i = a; i < b; ++i) t += qs[i] - 1;
    return t;
}

template <typename IdxT>
struct HostTables {
    std::vector<IdxT> ctab, dec_off, dec_str;
    std::vector<float> dec_rcp;
    std::vector<uint16_t> inv;
    std::vector<uint32_t> inv_start;
};

template <typename IdxT>
int build_tables(const DimTable &Dt, SectorDesc &sd, const int *split, const int *qs, HostTables<IdxT> &ht) {
    const int n = sd.n, L = sd.L;
    int start = 0;
    uint32_t ctab_pos = 0, dec_pos = 0, inv_pos = 0, invs_pos = 0;
    for (int k = 0; k < sd.N; ++k) {
        const int Lk = split[k];
        const int mk = max_sum(qs, start, start + Lk);
        const int g = L - start - Lk;
        const uint32_t W = 1u << sd.wbits[k];
        sd.rest_max[k] = max_sum(qs, start + Lk, L);
        sd.mk[k] = mk;
        sd.lam_lo[k] = std::max(0, n - max_sum(qs, start, L));
        sd.lam_hi[k] = std::min(n, max_sum(qs, 0, start));
        // local tables: digit sum and lexicographic index of every word
        std::vector<int> sum(W);
        std::vector<uint32_t> lidx(W);
        std::vector<uint32_t> cnt(mk + 1, 0);
        for (uint32_t w = 0; w < W; ++w) {
            int s = 0;
            bool ok = true;
            for (int i = 0; i < Lk; ++i) {
                int d = (int)((w >> (sd.nb * i)) & ((1u << sd.nb) - 1));
                ok = ok && d < qs[start + Lk - 1 - i];  // bits nb i hold the site's digit Lk-1-i
                s += d;
            }
            sum[w] = ok ? s : -1;
            if (ok) lidx[w] = cnt[s]++;
        }
        sd.inv_start0[k] = invs_pos;
        uint32_t acc = inv_pos;
        for (int m = 0; m <= mk; ++m) {
            ht.inv_start.push_back(acc);
            acc += cnt[m];
        }
        ht.inv_start.push_back(acc);
        invs_pos += mk + 2;
        ht.inv.resize(acc);
        for (uint32_t w = 0; w < W; ++w)
            if (sum[w] >= 0) ht.inv[ht.inv_start[sd.inv_start0[k] + sum[w]] + lidx[w]] = (uint16_t)w;
        inv_pos = acc;
        // offsets / strides per feasible lambda, and the fused c-table rows
        sd.ctab_row0[k] = ctab_pos;
        sd.dec_row0[k] = dec_pos;
        const bool last = k == sd.N - 1;
        sd.ctab_rowlen[k] = last ? 0u : W;
        if (last) {  // offset 0, stride 1: one row holding the local index
            for (uint32_t w = 0; w < W; ++w)
                ht.ctab.push_back(sum[w] < 0 ? Bad<IdxT>::value : (IdxT)lidx[w]);
            ctab_pos += W;
        }
        for (int lam = sd.lam_lo[k]; lam <= sd.lam_hi[k]; ++lam) {
            const int lo = std::max(0, n - lam - sd.rest_max[k]);
            const int hi = std::min(mk, n - lam);
            std::vector<u128> off(mk + 1, 0), str(mk + 1, 0);
            u128 run = 0;
            for (int m = 0; m <= mk; ++m) {
                off[m] = run;
                str[m] = (m >= lo && m <= hi) ? Dt.get(g, n - lam - m) : 0;
                if (m >= lo && m <= hi) run += (u128)cnt[m] * Dt.get(g, n - lam - m);
            }
            for (int m = 0; m <= mk; ++m) {
                ht.dec_off.push_back((IdxT)off[m]);
                ht.dec_str.push_back((IdxT)str[m]);
                ht.dec_rcp.push_back(str[m] ? (float)(1.0 / (double)str[m]) : 0.f);
            }
            dec_pos += mk + 1;
            if (last) continue;
            for (uint32_t w = 0; w < W; ++w) {
                int m = sum[w];
                if (m < lo || m > hi) {
                    ht.ctab.push_back(Bad<IdxT>::value);
                } else {
                    u128 c = off[m] + str[m] * (u128)lidx[w];
                    ht.ctab.push_back((IdxT)c);
                }
            }
            ctab_pos += W;
        }
        start += Lk;
    }
    sd.ctab_entries = ctab_pos;
    sd.dec_entries = dec_pos;
    sd.inv_entries = inv_pos;
    sd.inv_start_entries = invs_pos;
    return DCS_OK;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

template <typename IdxT>
int upload(dcs_sector *s, HostTables<IdxT> &ht) {
    SectorDev &d = s->dev;
    size_t pos = 0;
    d.ctab_off = pos;
    pos = align_up(pos + ht.ctab.size() * sizeof(IdxT), 16);
    d.dec_off_off = pos;
    pos = align_up(pos + ht.dec_off.size() * sizeof(IdxT), 16);
    d.dec_str_off = pos;
    pos = align_up(pos + ht.dec_str.size() * sizeof(IdxT), 16);
    d.dec_rcp_off = pos;
    pos = align_up(pos + ht.dec_rcp.size() * sizeof(float), 16);
    d.inv_start_off = pos;
    pos = align_up(pos + ht.inv_start.size() * sizeof(uint32_t), 16);
    d.inv_off = pos;
    pos = align_up(pos + ht.inv.size() * sizeof(uint16_t), 16);
    d.bytes = pos;
    d.lds_bytes = pos;
    SectorDesc &sd = s->desc;
    sd.lay_ctab = (uint32_t)d.ctab_off;
    sd.lay_doff = (uint32_t)d.dec_off_off;
    sd.lay_dstr = (uint32_t)d.dec_str_off;
    sd.lay_drcp = (uint32_t)d.dec_rcp_off;
    sd.lay_invs = (uint32_t)d.inv_start_off;
    sd.lay_inv = (uint32_t)d.inv_off;
    sd.lay_bytes = (uint32_t)pos;
    std::vector<char> host(pos, 0);
    memcpy(host.data() + d.ctab_off, ht.ctab.data(), ht.ctab.size() * sizeof(IdxT));
    memcpy(host.data() + d.dec_off_off, ht.dec_off.data(), ht.dec_off.size() * sizeof(IdxT));
    memcpy(host.data() + d.dec_str_off, ht.dec_str.data(), ht.dec_str.size() * sizeof(IdxT));
    memcpy(host.data() + d.dec_rcp_off, ht.dec_rcp.data(), ht.dec_rcp.size() * sizeof(float));
    memcpy(host.data() + d.inv_start_off, ht.inv_start.data(),
           ht.inv_start.size() * sizeof(uint32_t));
    memcpy(host.data() + d.inv_off, ht.inv.data(), ht.inv.size() * sizeof(uint16_t));
    int prev = 0;
    if (int r = check_hip(hipGetDevice(&prev), "hipGetDevice")) return r;
    if (int r = check_hip(hipSetDevice(s->device), "hipSetDevice")) return r;
    hipError_t e = hipMalloc(&d.base, pos);
    if (e != hipSuccess) {
        hipSetDevice(prev);
        d.base = nullptr;
        return set_error(DCS_ENOMEM, "hipMalloc of %zu bytes of sector tables failed: %s", pos,
                         hipGetErrorString(e));
    }
    e = hipMemcpy(d.base, host.data(), pos, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&d.counters, kNumCounters * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(d.counters, 0, kNumCounters * sizeof(uint32_t));
    hipSetDevice(prev);
    return check_hip(e, "sector tables and counters");
}

// Left configurations of the split product (see LeftInfo): for every left
// particle number m, the configurations (w_0..w_{K-1}) with digit sum m in
// canonical order, with the first row of their run, sum_k C_k[lambda_k][w_k].
constexpr uint64_t kSplitMinDim = 1ull << 20;
constexpr size_t kMaxLeftConfigs = 1u << 22;

template <typename IdxT>
int build_left(const DimTable &Dt, dcs_sector *s, const HostTables<IdxT> &ht, const int *split) {
    SectorDesc &sd = s->desc;
    LeftInfo &li = s->left;
    li.K = 0;
    uint64_t min_dim = kSplitMinDim;
    if (const char *e = getenv("DCS_SPLIT_MIN_DIM")) min_dim = strtoull(e, nullptr, 10);
    if (sd.N < 2 || sd.Q != 2 || s->mixed || sd.dim < min_dim) return DCS_OK;
    const int K = sd.N / 2;
    int L_left = 0, bits = 0;
    for (int k = 0; k < K; ++k) {
        li.word_shift[k] = (uint32_t)bits;
        L_left += split[k];
        bits += sd.wbits[k];
    }
    const int Q = sd.Q, n = sd.n;
    const int m_lo = std::max(0, n - (Q - 1) * (sd.L - L_left));
    const int m_hi = std::min(n, (Q - 1) * L_left);
    if (bits > 32 || m_hi - m_lo + 1 > kMaxLeftM) return DCS_OK;
    uint64_t total = 0;
    for (int m = m_lo; m <= m_hi; ++m) total += Dt.get(L_left, m);
    if (total > kMaxLeftConfigs) return DCS_OK;
    std::vector<uint32_t> words;
    std::vector<IdxT> runs;
    words.reserve(total);
    runs.reserve(total);
    uint32_t w[kMaxSub];
    int lam[kMaxSub];
    // nested loops over the left subsystems: digit sums in increasing order, then words
    // in increasing (lexicographic) order, the last left subsystem taking what remains
    auto rec = [&](auto &&self, int k, int rem) -> void {
        if (k == K) {
            if (rem != 0) return;
            uint32_t pw = 0;
            u128 start = 0;
            for (int j = 0; j < K; ++j) {
                pw |= w[j] << li.word_shift[j];
                start += ht.ctab[sd.ctab_row0[j] + (uint32_t)(lam[j] - sd.lam_lo[j]) * sd.ctab_rowlen[j] + w[j]];
            }
            words.push_back(pw);
            runs.push_back((IdxT)start);
            return;
        }
        int rest_sites = 0;
        for (int j = k + 1; j < K; ++j) rest_sites += split[j];
        const int lo = std::max(0, rem - (Q - 1) * rest_sites);
        const int hi = std::min(sd.mk[k], rem);
        const int base = lam[k];
        for (int nk = lo; nk <= hi; ++nk) {
            const uint32_t b = ht.inv_start[sd.inv_start0[k] + nk];
            const uint32_t e = ht.inv_start[sd.inv_start0[k] + nk + 1];
            for (uint32_t i = b; i < e; ++i) {
                w[k] = ht.inv[i];
                if (k + 1 < K) lam[k + 1] = base + nk;
                self(self, k + 1, rem - nk);
            }
        }
    };
    for (int m = m_lo; m <= m_hi; ++m) {
        li.lbase[m - m_lo] = (uint32_t)words.size();
        lam[0] = 0;
        rec(rec, 0, m);
        li.nleft[m - m_lo] = (uint32_t)(words.size() - li.lbase[m - m_lo]);
        li.ncols[m - m_lo] = Dt.get(sd.L - L_left, n - m);
    }
    // right configurations of every block in offset order, checked against the
    // fused table: offset = sum_{k>=K} C_k[lambda_k][w_k]
    int rbits = 0;
    for (int k = K; k < sd.N; ++k) {
        li.word_shift[k] = (uint32_t)rbits;
        rbits += sd.wbits[k];
    }
    if (rbits > 32) return DCS_OK;
    std::vector<uint32_t> rwords;
    auto rrec = [&](auto &&self, int k, int rem, uint32_t acc) -> void {
        if (k == sd.N) {
            if (rem == 0) rwords.push_back(acc);
            return;
        }
        int rest_sites = 0;
        for (int j = k + 1; j < sd.N; ++j) rest_sites += split[j];
        const int lo = std::max(0, rem - (Q - 1) * rest_sites);
        const int hi = std::min(sd.mk[k], rem);
        for (int nk = lo; nk <= hi; ++nk) {
            const uint32_t b = ht.inv_start[sd.inv_start0[k] + nk];
            const uint32_t e = ht.inv_start[sd.inv_start0[k] + nk + 1];
            for (uint32_t i = b; i < e; ++i)
                self(self, k + 1, rem - nk, acc | ((uint32_t)ht.inv[i] << li.word_shift[k]));
        }
    };
    for (int m = m_lo; m <= m_hi; ++m) {
        li.rbase[m - m_lo] = (uint32_t)rwords.size();
        rrec(rrec, K, n - m, 0u);
        if (rwords.size() - li.rbase[m - m_lo] != li.ncols[m - m_lo])
            return set_error(DCS_EHIP, "internal: right configurations of block %d", m);
    }
    DeviceGuard g(s->device);
    if (int r = check_hip(hipMalloc(&li.d_rwords, rwords.size() * sizeof(uint32_t)), "hipMalloc right words"))
        return r;
    if (int r = check_hip(hipMemcpy(li.d_rwords, rwords.data(), rwords.size() * sizeof(uint32_t),
                                    hipMemcpyHostToDevice), "copy right words"))
        return r;
    if (int r = check_hip(hipMalloc(&li.d_words, words.size() * sizeof(uint32_t)), "hipMalloc left words"))
        return r;
    if (int r = check_hip(hipMalloc(&li.d_runs, runs.size() * sizeof(IdxT)), "hipMalloc left runs"))
        return r;
    if (int r = check_hip(hipMemcpy(li.d_words, words.data(), words.size() * sizeof(uint32_t),
                                    hipMemcpyHostToDevice), "copy left words"))
        return r;
    if (int r = check_hip(hipMemcpy(li.d_runs, runs.data(), runs.size() * sizeof(IdxT),
                                    hipMemcpyHostToDevice), "copy left runs"))
        return r;
    li.K = K;
    li.L_left = L_left;
    li.m_lo = m_lo;
    li.m_count = m_hi - m_lo + 1;
    li.count = words.size();
    li.rcount = rwords.size();
    li.h_words = std::move(words);
    li.h_rwords = std::move(rwords);
    li.h_runs.assign(runs.begin(), runs.end());
    li.h_ctab.assign(ht.ctab.begin(), ht.ctab.end());
    return DCS_OK;
}

}  // namespace

void free_rows(SplitRows &c) {
    hipFree(c.d_lptr);
    hipFree(c.d_lent);
    hipFree(c.d_vo);
    hipFree(c.d_xl);
    hipFree(c.d_xo);
    hipFree(c.d_runs);
    hipFree(c.d_clstart);
    hipFree(c.d_clsize);
    hipFree(c.d_lrun);
    hipFree(c.d_rorder);
    hipFree(c.d_diag);
    for (int i = 0; i < kRowTilings; ++i) {
        hipFree(c.tiling[i].d_tiles);
        hipFree(c.tiling[i].d_tiles_canon);
        hipFree(c.tiling[i].d_pat);
    }
    hipFree(c.d_adjtasks);
    for (int i = 0; i < c.nuse; ++i) hipEventDestroy(c.use_event[i]);
    c = SplitRows();
}

void free_split(dcs_sector *s) {
    LeftInfo &li = s->left;
    hipFree(li.d_words);
    hipFree(li.d_runs);
    hipFree(li.d_rwords);
    li.d_words = li.d_runs = li.d_rwords = nullptr;
    for (int i = 0; i < kMaxSplitCache; ++i) free_rows(li.rows[i]);
}

int make_bond_plan(const dcs_sector *s, const dcs_terms *t, int nmax, BondPlan *p) {
    const SectorDesc &sd = s->desc;
    if (s->mixed)
        return set_error(DCS_EUNSUPPORTED, "the XXZ products take one local dimension on every site");
    if (t->max_site >= sd.L)
        return set_error(DCS_EINVAL, "bond site %d outside the sector's %d sites", t->max_site,
                         sd.L);
    const int ncls = nmax * (nmax + 1) / 2;
    p->nbonds = t->num_bonds;
    p->nclasses = ncls;
    std::vector<int> cls(t->num_bonds);
    std::vector<int> count(ncls + 1, 0);
    for (int b = 0; b < t->num_bonds; ++b) {
        int i = t->si[b], j = t->sj[b];
        int a = sd.site_sub[i], c = sd.site_sub[j];
        if (a > c || (a == c && sd.site_bit[i] < sd.site_bit[j])) {
            std::swap(i, j);
            std::swap(a, c);
        }
        cls[b] = class_id(a, c, nmax);
        count[cls[b] + 1]++;
    }
    for (int c = 0; c < ncls; ++c) count[c + 1] += count[c];
    for (int c = 0; c <= ncls; ++c) p->cls_beg[c] = (uint16_t)count[c];
    std::vector<int> fill(count.begin(), count.end() - 1);
    for (int b = 0; b < t->num_bonds; ++b) {
        int i = t->si[b], j = t->sj[b];
        int a = sd.site_sub[i], c = sd.site_sub[j];
        if (a > c || (a == c && sd.site_bit[i] < sd.site_bit[j])) std::swap(i, j);
        int slot = fill[cls[b]]++;
        p->pos[slot] = (uint32_t)sd.site_bit[i] | ((uint32_t)sd.site_bit[j] << 8) |
                       ((uint32_t)b << 16);
        p->site_i[slot] = (int16_t)i;
        p->site_j[slot] = (int16_t)j;
    }
    return DCS_OK;
}

}  // namespace dcs

using namespace dcs;

namespace {

// The sector of n particles on L sites, site i with qs[i] states (one Q for all
// sites, or a local dimension per site: Sec. 5 names this generalisation; every
// count becomes a product over the sites' own (1 + x + ... + x^{q_i - 1})).
int sector_create(int L, int n, const int *qs, int N, const int *sizes, int device, dcs_sector **out) {
    if (!out) return set_error(DCS_EINVAL, "out is NULL");
    *out = nullptr;
    if (L < 1 || L > kMaxSites) return set_error(DCS_EINVAL, "L=%d outside [1, %d]", L, kMaxSites);
    int Q = 0;
    bool mixed = false;
    for (int i = 0; i < L; ++i) {
        if (qs[i] < 2 || qs[i] > 16) return set_error(DCS_EINVAL, "local_dim %d of site %d outside [2, 16]", qs[i], i);
        Q = std::max(Q, qs[i]);
        mixed = mixed || qs[i] != qs[0];
    }
    int nb = 0;
    while ((1 << nb) < Q) ++nb;
    if (L * nb > 64) return set_error(DCS_EINVAL, "L=%d needs %d bits > 64", L, L * nb);
    const int nmax = max_sum(qs, 0, L);
    if (n < 0 || n > nmax) return set_error(DCS_EINVAL, "n_particles %d outside [0, %d]", n, nmax);
    int split[kMaxSub];
    if (sizes == nullptr) {
        int per = std::max(1, 9 / nb);
        N = (L + per - 1) / per;
        if (N > kMaxSub) return set_error(DCS_EUNSUPPORTED, "default split needs %d > %d parts", N, kMaxSub);
        int base = L / N, extra = L % N;
        for (int k = 0; k < N; ++k) split[k] = base + (k >= N - extra ? 1 : 0);
    } else {
        if (N < 1) return set_error(DCS_EINVAL, "num_subsystems %d < 1", N);
        if (N > kMaxSub)
            return set_error(DCS_EUNSUPPORTED, "num_subsystems %d > %d", N, kMaxSub);
        int tot = 0;
        for (int k = 0; k < N; ++k) {
            if (sizes[k] < 1) return set_error(DCS_EINVAL, "subsystem %d has size %d", k, sizes[k]);
            split[k] = sizes[k];
            tot += sizes[k];
        }
        if (tot != L) return set_error(DCS_EINVAL, "subsystem sizes sum to %d, not L=%d", tot, L);
    }
    for (int k = 0; k < N; ++k)
        if (split[k] * nb > kMaxWordBits)
            return set_error(DCS_EUNSUPPORTED, "subsystem %d word has %d bits > %d", k,
                             split[k] * nb, kMaxWordBits);
    int ndev = 0;
    if (int r = check_hip(hipGetDeviceCount(&ndev), "hipGetDeviceCount")) return r;
    if (device < 0 || device >= ndev)
        return set_error(DCS_EINVAL, "device %d outside [0, %d)", device, ndev);

    DimTable Dt;
    if (!Dt.build(qs, L)) return set_error(DCS_EUNSUPPORTED, "sector dimensions exceed 2^63");
    for (int k = 0, start = 0; k < N; start += split[k++]) {
        DimTable Dk;  // the words of subsystem k alone
        Dk.build(qs + start, split[k]);
        for (int m = 0; m <= Dk.mmax; ++m)
            if (Dk.get(split[k], m) > kMaxClassWords)
                return set_error(DCS_EUNSUPPORTED, "subsystem %d has %llu words of digit sum %d > %llu", k,
                                 (unsigned long long)Dk.get(split[k], m), m,
                                 (unsigned long long)kMaxClassWords);
    }
    dcs_sector *s = new (std::nothrow) dcs_sector();
    if (!s) return set_error(DCS_ENOMEM, "host allocation failed");
    s->device = device;
    s->mixed = mixed;
    for (int i = 0; i < L; ++i) s->qsite[i] = qs[i];
    SectorDesc &sd = s->desc;
    memset(&sd, 0, sizeof(sd));
    sd.Q = Q;
    sd.nb = nb;
    sd.L = L;
    sd.n = n;
    sd.N = N;
    sd.total_bits = nb * L;
    sd.dim = Dt.get(L, n);
    for (int t = 0; t < 4; ++t) {
        uint32_t m = 0;
        if (t < nb)
            for (int f = 0; f * nb < 32; ++f) m |= 1u << (f * nb + t);
        sd.field_mask[t] = m;
    }
    int start = 0;
    for (int k = 0; k < N; ++k) {
        s->split[k] = split[k];
        sd.wbits[k] = nb * split[k];
        sd.shift[k] = nb * (L - start - split[k]);
        for (int i = 0; i < split[k]; ++i) {
            sd.site_sub[start + i] = (uint8_t)k;
            sd.site_bit[start + i] = (uint8_t)(nb * (split[k] - 1 - i));
        }
        start += split[k];
    }
    // 64-bit index arithmetic for dim >= 2^32 - 1 (the 32-bit sentinel), or on request
    // (environment DCS_INDEX_BITS=64, used to test the 64-bit kernels on small sectors)
    const char *bits = getenv("DCS_INDEX_BITS");
    s->wide = sd.dim >= 0xFFFFFFFFull || (bits && strcmp(bits, "64") == 0);
    int r;
    if (s->wide) {
        HostTables<uint64_t> ht;
        r = build_tables(Dt, sd, split, qs, ht);
        if (!r) r = upload(s, ht);
        if (!r) r = build_left(Dt, s, ht, split);
    } else {
        HostTables<uint32_t> ht;
        r = build_tables(Dt, sd, split, qs, ht);
        if (!r) r = upload(s, ht);
        if (!r) r = build_left(Dt, s, ht, split);
    }
    // tables beyond the on-chip budget (or DCS_GLOBAL_TABLES=1) stay in device memory
    const char *gt = getenv("DCS_GLOBAL_TABLES");
    s->gtab = s->dev.lds_bytes > kLdsTableBudget || (gt && gt[0] == '1');
    if (r) {
        if (s->dev.base) hipFree(s->dev.base);
        if (s->dev.counters) hipFree(s->dev.counters);
        free_split(s);
        delete s;
        return r;
    }
    *out = s;
    return DCS_OK;
}

}  // namespace

extern "C" int dcs_sector_create(int L, int n, int Q, int N, const int *sizes, int device,
                                 dcs_sector **out) {
    clear_error();
    if (Q < 2 || Q > 16) return set_error(DCS_EINVAL, "local_dim %d outside [2, 16]", Q);
    if (L < 1 || L > kMaxSites) return set_error(DCS_EINVAL, "L=%d outside [1, %d]", L, kMaxSites);
    int qs[kMaxSites];
    for (int i = 0; i < L; ++i) qs[i] = Q;
    return sector_create(L, n, qs, N, sizes, device, out);
}

extern "C" int dcs_sector_create_mixed(int L, int n, const int32_t *local_dims, int N, const int *sizes,
                                       int device, dcs_sector **out) {
    clear_error();
    if (!local_dims) return set_error(DCS_EINVAL, "local_dims is NULL");
    if (L < 1 || L > kMaxSites) return set_error(DCS_EINVAL, "L=%d outside [1, %d]", L, kMaxSites);
    int qs[kMaxSites];
    for (int i = 0; i < L; ++i) qs[i] = local_dims[i];
    return sector_create(L, n, qs, N, sizes, device, out);
}

extern "C" int dcs_sector_local_dims(const dcs_sector *s, int32_t *local_dims) {
    clear_error();
    if (!s || !local_dims) return set_error(DCS_EINVAL, "NULL argument");
    for (int i = 0; i < s->desc.L; ++i) local_dims[i] = s->qsite[i];
    return DCS_OK;
}

extern "C" int dcs_sector_destroy(dcs_sector *s) {
    clear_error();
    if (!s) return DCS_OK;
    int r = DCS_OK;
    if (s->dev.base) {
        int prev = 0;
        hipGetDevice(&prev);
        hipSetDevice(s->device);
        r = check_hip(hipFree(s->dev.base), "hipFree of sector tables");
        if (s->dev.counters) hipFree(s->dev.counters);
        free_split(s);
        hipSetDevice(prev);
    }
    delete s;
    return r;
}

extern "C" int dcs_sector_dim(const dcs_sector *s, uint64_t *dim) {
    clear_error();
    if (!s || !dim) return set_error(DCS_EINVAL, "NULL argument");
    *dim = s->desc.dim;
    return DCS_OK;
}

extern "C" int dcs_sector_tables(const dcs_sector *s, int *in_device_memory, size_t *bytes) {
    clear_error();
    if (!s) return set_error(DCS_EINVAL, "sector is NULL");
    if (in_device_memory) *in_device_memory = s->gtab ? 1 : 0;
    if (bytes) *bytes = s->dev.lds_bytes;
    return DCS_OK;
}

extern "C" int dcs_sector_split(const dcs_sector *s, int *num, int *sizes) {
    clear_error();
    if (!s || !num) return set_error(DCS_EINVAL, "NULL argument");
    *num = s->desc.N;
    if (sizes)
        for (int k = 0; k < s->desc.N; ++k) sizes[k] = s->split[k];
    return DCS_OK;
}

extern "C" int dcs_terms_create(int num_bonds, const int32_t *si, const int32_t *sj,
                                dcs_terms **out) {
    clear_error();
    if (!out) return set_error(DCS_EINVAL, "out is NULL");
    *out = nullptr;
    if (num_bonds < 0) return set_error(DCS_EINVAL, "num_bonds %d < 0", num_bonds);
    if (num_bonds > kMaxBonds)
        return set_error(DCS_EUNSUPPORTED, "num_bonds %d > %d", num_bonds, kMaxBonds);
    if (num_bonds > 0 && (!si || !sj)) return set_error(DCS_EINVAL, "NULL site arrays");
    dcs_terms *t = new (std::nothrow) dcs_terms();
    if (!t) return set_error(DCS_ENOMEM, "host allocation failed");
    static std::atomic<uint64_t> next_id{1};
    t->id = next_id++;
    t->num_bonds = num_bonds;
    t->max_site = -1;
    for (int b = 0; b < num_bonds; ++b) {
        if (si[b] < 0 || sj[b] < 0 || si[b] == sj[b]) {
            delete t;
            return set_error(DCS_EINVAL, "bond %d joins sites %d and %d", b, si[b], sj[b]);
        }
        if (si[b] >= kMaxSites || sj[b] >= kMaxSites) {
            delete t;
            return set_error(DCS_EUNSUPPORTED, "bond %d site >= %d", b, kMaxSites);
        }
        t->si[b] = si[b];
        t->sj[b] = sj[b];
        t->max_site = std::max(t->max_site, (int)std::max(si[b], sj[b]));
    }
    *out = t;
    return DCS_OK;
}

extern "C" int dcs_terms_destroy(dcs_terms *t) {
    clear_error();
    delete t;
    return DCS_OK;
}
