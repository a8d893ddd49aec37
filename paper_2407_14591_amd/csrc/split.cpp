// Sparse rows of the bond families left and right of the cut of a sector's
// split view (LeftInfo): built on the host from the fused contribution table,
// once per (sector, terms) pair, and cached in the sector.
#include <algorithm>
#include <vector>

#include "dcs_internal.h"

namespace dcs {

namespace {

struct FamilyBond {
    int a, b;        // subsystems of the two sites, a <= b
    uint32_t pil, pjl;  // bits of the sites inside their subsystem words
    uint32_t t;      // position in the bond plan
};

}  // namespace

SplitCsr *split_csr(dcs_sector *s, const dcs_terms *t, const BondPlan &plan, int nmax) {
    LeftInfo &li = s->left;
    const SectorDesc &sd = s->desc;
    if (li.K == 0 || sd.Q != 2 || li.h_rwords.empty()) return nullptr;
    for (int i = 0; i < kMaxSplitCache; ++i)
        if (li.csr[i].terms_id == t->id && li.csr[i].nmax == nmax) return &li.csr[i];
    const int K = li.K, N = sd.N;
    std::vector<FamilyBond> left, right;
    for (int a = 0; a < nmax; ++a)
        for (int b = a; b < nmax; ++b) {
            const int cls = class_id(a, b, nmax);
            for (int q = plan.cls_beg[cls]; q < plan.cls_beg[cls + 1]; ++q) {
                FamilyBond fb{a, b, plan.pos[q] & 0xFFu, (plan.pos[q] >> 8) & 0xFFu, (uint32_t)q};
                if (b < K)
                    left.push_back(fb);
                else if (a >= K)
                    right.push_back(fb);
            }
        }
    auto cval = [&](int k, int lam, uint32_t w) -> uint64_t {
        return li.h_ctab[sd.ctab_row0[k] + (uint32_t)(lam - sd.lam_lo[k]) * sd.ctab_rowlen[k] + w];
    };
    auto unpack = [&](uint32_t pw, int k) -> uint32_t {
        return (pw >> li.word_shift[k]) & ((1u << sd.wbits[k]) - 1u);
    };
    // a hop of bond fb on the words w (lambda prefix lam): new words and lambda shift
    auto hop = [&](const FamilyBond &fb, const uint32_t *w, uint32_t *w2, int *dl) -> bool {
        const uint32_t bi = (w[fb.a] >> fb.pil) & 1u, bj = (w[fb.b] >> fb.pjl) & 1u;
        if (bi == bj) return false;
        for (int k = 0; k < N; ++k) w2[k] = w[k];
        w2[fb.a] ^= 1u << fb.pil;
        w2[fb.b] ^= 1u << fb.pjl;
        *dl = bi ? -1 : 1;  // site i (in P_a) loses or gains the particle
        return true;
    };
    SplitCsr c;
    c.terms_id = t->id;
    c.nmax = nmax;
    std::vector<uint32_t> lptr(li.count + 1), rptr(li.rcount + 1);
    std::vector<uint64_t> lent;
    std::vector<uint32_t> rent;
    uint32_t w[kMaxSub] = {0}, w2[kMaxSub];
    int lam[kMaxSub + 1];
    // every left target must be the run start of a left configuration with the
    // same particle count (so the target row shares the offset's run length)
    std::vector<std::pair<uint64_t, int>> run_block(li.count);
    for (int mi = 0; mi < li.m_count; ++mi)
        for (uint32_t q = 0; q < li.nleft[mi]; ++q)
            run_block[li.lbase[mi] + q] = {li.h_runs[li.lbase[mi] + q], mi};
    std::sort(run_block.begin(), run_block.end());
    auto block_of_run = [&](uint64_t run) -> int {
        auto it = std::lower_bound(run_block.begin(), run_block.end(), std::make_pair(run, -1));
        return (it != run_block.end() && it->first == run) ? it->second : -1;
    };
    int gmi = 0;
    for (size_t g = 0; g < li.count; ++g) {
        while (gmi + 1 < li.m_count && g >= li.lbase[gmi + 1]) ++gmi;
        lptr[g] = (uint32_t)lent.size();
        lam[0] = 0;
        for (int k = 0; k < K; ++k) {
            w[k] = unpack(li.h_words[g], k);
            lam[k + 1] = lam[k] + __builtin_popcount(w[k]);
        }
        for (const FamilyBond &fb : left) {
            int dl;
            if (!hop(fb, w, w2, &dl)) continue;
            uint64_t run = 0;
            for (int k = 0; k < K; ++k) run += cval(k, lam[k] + ((k > fb.a && k <= fb.b) ? dl : 0), w2[k]);
            if (run >= (1ull << 48) || block_of_run(run) != gmi)
                return set_error(DCS_EHIP, "internal: left target is not a run of the same block"), nullptr;
            lent.push_back(run | ((uint64_t)fb.t << 48));
        }
    }
    lptr[li.count] = (uint32_t)lent.size();
    for (int mi = 0; mi < li.m_count; ++mi) {
        const int m = li.m_lo + mi;
        for (uint64_t r = 0; r < li.ncols[mi]; ++r) {
            const size_t g = li.rbase[mi] + r;
            rptr[g] = (uint32_t)rent.size();
            lam[K] = m;
            for (int k = K; k < N; ++k) {
                w[k] = unpack(li.h_rwords[g], k);
                lam[k + 1] = lam[k] + __builtin_popcount(w[k]);
            }
            for (const FamilyBond &fb : right) {
                int dl;
                if (!hop(fb, w, w2, &dl)) continue;
                uint64_t off = 0;
                for (int k = K; k < N; ++k)
                    off += cval(k, lam[k] + ((k > fb.a && k <= fb.b) ? dl : 0), w2[k]);
                if (off >= li.ncols[mi] || off >= (1u << 24))
                    return set_error(DCS_EHIP, "internal: right offset out of its run"), nullptr;
                rent.push_back((uint32_t)off | (fb.t << 24));
            }
        }
    }
    rptr[li.rcount] = (uint32_t)rent.size();
    c.lnnz = lent.size();
    c.rnnz = rent.size();
    DeviceGuard dg(s->device);
    auto up = [&](void **dst, const void *src, size_t bytes) -> bool {
        if (check_hip(hipMalloc(dst, bytes ? bytes : 8), "hipMalloc sparse rows")) return false;
        if (bytes && check_hip(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice), "copy sparse rows"))
            return false;
        return true;
    };
    bool ok = up((void **)&c.d_lptr, lptr.data(), lptr.size() * sizeof(uint32_t)) &&
              up((void **)&c.d_lent, lent.data(), lent.size() * sizeof(uint64_t)) &&
              up((void **)&c.d_rptr, rptr.data(), rptr.size() * sizeof(uint32_t)) &&
              up((void **)&c.d_rent, rent.data(), rent.size() * sizeof(uint32_t)) &&
              check_hip(hipMalloc(&c.d_diag, (li.count + li.rcount) * sizeof(double)),
                        "hipMalloc split diagonal") == DCS_OK;
    if (!ok) {
        free_csr(c);
        return nullptr;
    }
    SplitCsr &slot = li.csr[li.next_slot];
    li.next_slot = (li.next_slot + 1) % kMaxSplitCache;
    if (slot.terms_id) (void)hipDeviceSynchronize();  // the evicted rows may still be in use
    free_csr(slot);
    slot = c;
    return &slot;
}

}  // namespace dcs
