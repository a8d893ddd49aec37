// Target tables of the split product (LeftInfo): built on the host from the
// fused contribution table, once per (sector, terms) pair, and cached in the
// sector.  Every target is the rank of eq. index of a configuration that one
// bond reaches, evaluated per side of the cut.
#include <algorithm>
#include <cstring>
#include <vector>

#include "dcs_internal.h"

namespace dcs {

namespace {

struct SideBond {
    int a, b;             // subsystems of the two sites
    uint32_t pi, pj;      // bits of the sites inside their subsystem words
    uint16_t bond;        // index in the terms
};

}  // namespace

SplitRows *split_rows(dcs_sector *s, const dcs_terms *t) {
    LeftInfo &li = s->left;
    const SectorDesc &sd = s->desc;
    if (li.K == 0 || sd.Q != 2 || li.h_rwords.empty()) return nullptr;
    std::lock_guard<std::mutex> guard(*li.rows_lock);  // concurrent first calls build the tables once
    for (int i = 0; i < kMaxSplitCache; ++i)
        if (li.rows[i].terms_id == t->id) return &li.rows[i];
    const int K = li.K, N = sd.N;
    bool wide = false;  // 32-bit target offsets for runs of 65,535 rows or more
    for (int mi = 0; mi < li.m_count; ++mi) {
        if (li.ncols[mi] >= 0xFFFFu) wide = true;
        if (li.ncols[mi] >= (1u << 25)) return nullptr;  // byte offsets of rows of up to 64 B stay below 2^31
    }
    auto packed_bit = [&](int site) -> uint8_t {
        return (uint8_t)(li.word_shift[sd.site_sub[site]] + sd.site_bit[site]);
    };
    SplitRows c;
    c.terms_id = t->id;
    c.wide_off = wide;
    std::vector<SideBond> left, right;
    std::vector<int> lsites, rsites;  // crossing sites per slot
    for (int q = 0; q < t->num_bonds; ++q) {
        int i = t->si[q], j = t->sj[q];
        int a = sd.site_sub[i], b = sd.site_sub[j];
        if (a > b) {
            std::swap(i, j);
            std::swap(a, b);
        }
        if (b < K || a >= K) {
            SideBond fb{a, b, sd.site_bit[i], sd.site_bit[j], (uint16_t)q};
            (b < K ? left : right).push_back(fb);
            c.d[c.nD++] = DiagTerm{(uint8_t)(b < K ? 0 : 1), packed_bit(i), packed_bit(j), 0,
                                   (uint16_t)q, 0};
            continue;
        }
        if (c.nX == kMaxCross) return nullptr;
        auto slot = [](std::vector<int> &v, int site) -> int {
            auto it = std::find(v.begin(), v.end(), site);
            if (it != v.end()) return (int)(it - v.begin());
            v.push_back(site);
            return (int)v.size() - 1;
        };
        const int si = slot(lsites, i), sj = slot(rsites, j);
        if (si >= kMaxCrossSites || sj >= kMaxCrossSites) return nullptr;
        c.x[c.nX++] = CrossBond{(uint8_t)si, (uint8_t)sj, packed_bit(i), packed_bit(j), (uint16_t)q, 0};
    }
    for (int i = 0; i < sd.L; ++i)
        c.d[c.nD++] = DiagTerm{(uint8_t)(sd.site_sub[i] < K ? 0 : 1), packed_bit(i), 0, 1, (uint16_t)i, 0};
    // bonds that keep the particle number of P_K first (both sites in P_K or both
    // beyond it: their targets stay in the row's n_K block), the others after them;
    // among the first, the bonds inside the last subsystem lead: their targets
    // share the row's words of P_K..P_{N-2}, i.e. lie within `margin` rows of it
    auto keeps_nK = [&](const SideBond &fb) { return (fb.a == K) == (fb.b == K); };
    std::stable_partition(right.begin(), right.end(), keeps_nK);
    std::stable_partition(right.begin(), right.end(),
                          [&](const SideBond &fb) { return fb.a == N - 1 && fb.b == N - 1; });
    for (const SideBond &fb : right) c.nRloc += (fb.a == N - 1 && fb.b == N - 1) ? 1 : 0;
    for (const SideBond &fb : right) c.nRA += keeps_nK(fb) ? 1 : 0;
    {
        const int l = sd.wbits[N - 1];  // sites of the last subsystem (Q = 2)
        uint64_t best = 1;
        for (int m = 0; m <= l; ++m) {
            uint64_t b = 1;
            for (int i = 0; i < m; ++i) b = b * (uint64_t)(l - i) / (uint64_t)(i + 1);
            best = std::max(best, b);
        }
        c.margin = (uint32_t)best;
    }
    c.nR = (int)right.size();
    c.nIs = (int)lsites.size();
    c.nJs = (int)rsites.size();
    for (int b = 0; b < c.nR; ++b) c.r_bond[b] = right[b].bond;

    auto cval = [&](int k, int lam, uint32_t w) -> uint64_t {
        return li.h_ctab[sd.ctab_row0[k] + (uint32_t)(lam - sd.lam_lo[k]) * sd.ctab_rowlen[k] + w];
    };
    auto unpack = [&](uint32_t pw, int k) -> uint32_t {
        return (pw >> li.word_shift[k]) & ((1u << sd.wbits[k]) - 1u);
    };
    // sum of C_k[lambda_k][w_k] over subsystems k0..k1-1, lambda starting at lam0
    auto rank_part = [&](const uint32_t *w, int k0, int k1, int lam0) -> uint64_t {
        uint64_t v = 0;
        int lam = lam0;
        for (int k = k0; k < k1; ++k) {
            v += cval(k, lam, w[k]);
            lam += __builtin_popcount(w[k]);
        }
        return v;
    };
    auto in_block = [&](int m) { return m >= li.m_lo && m < li.m_lo + li.m_count; };
    // every left target must be the run start of a left configuration of the
    // expected block (so the target's run has the offset's length)
    std::vector<std::pair<uint64_t, int>> run_block(li.count);
    for (int mi = 0; mi < li.m_count; ++mi)
        for (uint32_t q = 0; q < li.nleft[mi]; ++q)
            run_block[li.lbase[mi] + q] = {li.h_runs[li.lbase[mi] + q], mi};
    std::sort(run_block.begin(), run_block.end());
    auto block_of_run = [&](uint64_t run) -> int {
        auto it = std::lower_bound(run_block.begin(), run_block.end(), std::make_pair(run, -1));
        return (it != run_block.end() && it->first == run) ? it->second : -1;
    };

    // clusters: consecutive left configurations of one block with equal words of
    // P_0..P_{K-2} (the bonds inside P_{K-1} keep them), split at kMaxClusterRuns
    std::vector<uint32_t> clstart, clsize, cl_of(li.count);
    {
        const uint32_t keep = K >= 2 ? ((1u << li.word_shift[K - 1]) - 1u) : 0u;  // bits of P_0..P_{K-2}
        for (int mi = 0; mi < li.m_count; ++mi) {
            c.clbase[mi] = (uint32_t)clstart.size();
            for (uint32_t q = 0; q < li.nleft[mi]; ++q) {
                const uint32_t g = li.lbase[mi] + q;
                const bool fresh = clstart.empty() || q == 0 ||
                                   ((li.h_words[g] ^ li.h_words[clstart.back()]) & keep) != 0 ||
                                   clsize.back() == kMaxClusterRuns;
                if (fresh) {
                    clstart.push_back(g);
                    clsize.push_back(0);
                }
                cl_of[g] = (uint32_t)clstart.size() - 1;
                ++clsize.back();
            }
            c.nclust[mi] = (uint32_t)clstart.size() - c.clbase[mi];
        }
        for (uint32_t z : clsize) c.max_cluster = std::max(c.max_cluster, z);
    }
    // left family rows and crossing left flips
    std::vector<uint32_t> lptr(li.count + 1);
    std::vector<uint64_t> lent;
    std::vector<uint64_t> xl((size_t)c.nIs * li.count, ~0ull);
    uint32_t w[kMaxSub] = {0}, w2[kMaxSub];
    for (int mi = 0; mi < li.m_count; ++mi) {
        const int m = li.m_lo + mi;
        for (uint32_t q = 0; q < li.nleft[mi]; ++q) {
            const size_t g = li.lbase[mi] + q;
            lptr[g] = (uint32_t)lent.size();
            for (int k = 0; k < K; ++k) w[k] = unpack(li.h_words[g], k);
            for (const SideBond &fb : left) {
                if (((w[fb.a] >> fb.pi) & 1u) == ((w[fb.b] >> fb.pj) & 1u)) continue;
                std::copy(w, w + K, w2);
                w2[fb.a] ^= 1u << fb.pi;
                w2[fb.b] ^= 1u << fb.pj;
                const uint64_t run = rank_part(w2, 0, K, 0);
                if (run >= (1ull << 48) || block_of_run(run) != mi)
                    return set_error(DCS_EHIP, "internal: left target is not a run of the same block"),
                           nullptr;
                // the target's left configuration (runs of one block are in configuration order)
                const auto it = std::lower_bound(li.h_runs.begin() + li.lbase[mi],
                                                 li.h_runs.begin() + li.lbase[mi] + li.nleft[mi], run);
                const uint32_t g2 = (uint32_t)(it - li.h_runs.begin());
                if (it == li.h_runs.begin() + li.lbase[mi] + li.nleft[mi] || *it != run)
                    return set_error(DCS_EHIP, "internal: left target configuration"), nullptr;
                if (cl_of[g2] == cl_of[g])
                    lent.push_back((1ull << 63) | ((uint64_t)fb.bond << 48) | (g2 - clstart[cl_of[g]]));
                else
                    lent.push_back(run | ((uint64_t)fb.bond << 48));
            }
            for (int si = 0; si < c.nIs; ++si) {
                const int site = lsites[si], k = sd.site_sub[site];
                const uint32_t bit = 1u << sd.site_bit[site];
                const int m2 = m + ((w[k] & bit) ? -1 : 1);
                if (!in_block(m2)) continue;
                std::copy(w, w + K, w2);
                w2[k] ^= bit;
                const uint64_t run = rank_part(w2, 0, K, 0);
                if (block_of_run(run) != m2 - li.m_lo)
                    return set_error(DCS_EHIP, "internal: flipped left configuration"), nullptr;
                xl[(size_t)si * li.count + g] = run;
            }
        }
    }
    lptr[li.count] = (uint32_t)lent.size();
    c.lnnz = lent.size();

    // right family targets and crossing right flips: 16-byte rows of eight 16-bit
    // offsets, or of four 32-bit ones for runs of 65,535 rows or more
    const int per = wide ? 4 : 8;
    const uint32_t nohop = wide ? 0xFFFFFFFFu : 0xFFFFu;
    const int nRq = (c.nR + per - 1) / per;
    const int nJq = (c.nJs + per - 1) / per;
    std::vector<uint32_t> vo((size_t)nRq * li.rcount * per, nohop);
    std::vector<uint32_t> xo((size_t)nJq * li.rcount * per, nohop);
    for (int mi = 0; mi < li.m_count; ++mi) {
        const int m = li.m_lo + mi;
        for (uint64_t r = 0; r < li.ncols[mi]; ++r) {
            const size_t g = li.rbase[mi] + r;
            for (int k = K; k < N; ++k) w[k] = unpack(li.h_rwords[g], k);
            if (rank_part(w, K, N, m) != r)
                return set_error(DCS_EHIP, "internal: right configuration order"), nullptr;
            for (int b = 0; b < c.nR; ++b) {
                const SideBond &fb = right[b];
                if (((w[fb.a] >> fb.pi) & 1u) == ((w[fb.b] >> fb.pj) & 1u)) continue;
                std::copy(w, w + N, w2);
                w2[fb.a] ^= 1u << fb.pi;
                w2[fb.b] ^= 1u << fb.pj;
                const uint64_t off = rank_part(w2, K, N, m);
                if (off >= li.ncols[mi])
                    return set_error(DCS_EHIP, "internal: right offset out of its run"), nullptr;
                vo[((size_t)(b / per) * li.rcount + g) * per + b % per] = (uint32_t)off;
            }
            for (int sj = 0; sj < c.nJs; ++sj) {
                const int site = rsites[sj], k = sd.site_sub[site];
                const uint32_t bit = 1u << sd.site_bit[site];
                // the particle moves to (+1 on the left) or from (-1) the other side
                const int m2 = m + ((w[k] & bit) ? 1 : -1);
                if (!in_block(m2)) continue;
                std::copy(w, w + N, w2);
                w2[k] ^= bit;
                const uint64_t off = rank_part(w2, K, N, m2);
                if (off >= li.ncols[m2 - li.m_lo])
                    return set_error(DCS_EHIP, "internal: flipped right configuration"), nullptr;
                xo[((size_t)(sj / per) * li.rcount + g) * per + sj % per] = (uint32_t)off;
            }
        }
    }
    // block tiles of the row pass for rows of 16, 32 and 64 bytes
    {
        uint32_t cross_mask = 0;
        for (int si = 0; si < c.nIs; ++si) cross_mask |= 1u << packed_bit(lsites[si]);
        const uint32_t maskK = (1u << sd.wbits[K]) - 1u;  // P_K's word: the low bits of a right word
        std::vector<uint32_t> order(li.count);
        for (uint32_t g = 0; g < li.count; ++g) order[g] = g;
        std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
            return (li.h_words[a] & ~cross_mask) < (li.h_words[b] & ~cross_mask);
        });
        std::vector<int> block_of(li.count);
        for (int mi = 0; mi < li.m_count; ++mi)
            for (uint32_t q = 0; q < li.nleft[mi]; ++q) block_of[li.lbase[mi] + q] = mi;
        // tiles of kSplitRowTile rows: each group of left configurations that differ
        // only at the crossing sites (closed under every crossing bond) together,
        // their runs interleaved at equal fractions of their lengths, so that the
        // crossing targets of the tiles in flight lie in runs being read.  An entry
        // keeps the chunk in 8 bits: runs of more than 256 tiles keep the run order.
        uint64_t max_nsub = 0;
        for (int mi = 0; mi < li.m_count; ++mi)
            max_nsub = std::max<uint64_t>(max_nsub, (li.ncols[mi] + kSplitRowTile - 1) / kSplitRowTile);
        if (max_nsub <= 256 && li.count < (1u << 24)) {
            std::vector<std::pair<double, uint32_t>> grp;
            for (size_t a = 0; a < order.size();) {
                size_t b = a + 1;
                const uint32_t key = li.h_words[order[a]] & ~cross_mask;
                while (b < order.size() && (li.h_words[order[b]] & ~cross_mask) == key) ++b;
                grp.clear();
                for (size_t q = a; q < b; ++q) {
                    const uint32_t g = order[q];
                    const uint32_t nsub = (uint32_t)((li.ncols[block_of[g]] + kSplitRowTile - 1) / kSplitRowTile);
                    for (uint32_t j = 0; j < nsub; ++j)
                        grp.emplace_back((j + 0.5) / nsub, (g << 8) | j);
                }
                std::stable_sort(grp.begin(), grp.end(),
                                 [](const std::pair<double, uint32_t> &u, const std::pair<double, uint32_t> &v) {
                                     return u.first < v.first;
                                 });
                for (const auto &e : grp) c.h_rorder.push_back(e.second);
                a = b;
            }
        }
        for (int ti = 0; ti < kRowTilings; ++ti) {
            RowTiling &T = c.tiling[ti];
            const uint32_t rb = 16u << ti;
            const uint32_t maxrows = (kTileLdsTotal - kTileLdsStatic) / rb - 1;  // one zero row after the tile
            std::vector<uint2> pat;
            bool ok = true;
            for (int mi = 0; mi < li.m_count && ok; ++mi) {
                T.pbase[mi] = (uint32_t)pat.size();
                const uint32_t *rw = li.h_rwords.data() + li.rbase[mi];
                const uint32_t ncols = (uint32_t)li.ncols[mi];
                uint32_t cur0 = 0, cur = 0;
                // (first offset | 1 << 31 for a tile that holds part of an n_K block, rows)
                auto flush = [&](bool part = false) {
                    if (cur) pat.push_back(make_uint2(cur0 | (part ? 0x80000000u : 0u), cur));
                    cur = 0;
                };
                uint32_t g0 = 0;
                while (g0 < ncols) {  // n_K blocks
                    uint32_t g1 = g0 + 1;
                    while (g1 < ncols && __builtin_popcount(rw[g1] & maskK) == __builtin_popcount(rw[g0] & maskK)) ++g1;
                    const uint32_t glen = g1 - g0;
                    if (glen <= maxrows) {
                        if (cur + glen > maxrows) flush();
                        if (!cur) cur0 = g0;
                        cur += glen;
                    } else {  // whole sub-runs of equal P_K word
                        flush();
                        uint32_t u0 = g0;
                        while (u0 < g1) {
                            uint32_t u1 = u0 + 1;
                            while (u1 < g1 && (rw[u1] & maskK) == (rw[u0] & maskK)) ++u1;
                            for (uint32_t a = u0; a < u1;) {
                                const uint32_t take = std::min(u1 - a, maxrows);
                                if (cur + take > maxrows) flush(true);
                                if (!cur) cur0 = a;
                                cur += take;
                                a += take;
                            }
                            u0 = u1;
                        }
                        flush(true);
                    }
                    g0 = g1;
                }
                flush();
                T.ntile[mi] = (uint32_t)pat.size() - T.pbase[mi];
                if (T.ntile[mi] > (uint32_t)kMaxRunTiles) ok = false;
            }
            if (!ok) continue;  // no tiling for this row size: the launcher keeps the other row passes
            uint32_t maxt = 0;
            for (const uint2 &p : pat) T.max_rows = std::max(T.max_rows, p.y);
            for (int mi = 0; mi < li.m_count; ++mi) maxt = std::max(maxt, T.ntile[mi]);
            std::vector<uint2> tiles, canon;
            for (uint32_t g = 0; g < li.count; ++g)
                for (uint32_t j = 0; j < T.ntile[block_of[g]]; ++j)
                    canon.push_back(make_uint2(g, (uint32_t)block_of[g] | (j << 8)));
            for (size_t a = 0; a < order.size();) {
                size_t b = a + 1;
                const uint32_t key = li.h_words[order[a]] & ~cross_mask;
                while (b < order.size() && (li.h_words[order[b]] & ~cross_mask) == key) ++b;
                for (uint32_t j = 0; j < maxt; ++j)
                    for (size_t q = a; q < b; ++q) {
                        const uint32_t g = order[q];
                        if (j < T.ntile[block_of[g]]) tiles.push_back(make_uint2(g, (uint32_t)block_of[g] | (j << 8)));
                    }
                a = b;
            }
            T.ntiles = tiles.size();
            T.h_pat = std::move(pat);
            T.h_tiles = std::move(tiles);
            T.h_canon = std::move(canon);
        }
    }
    // the adjoint's output sums (see split_adjoint.hip for the values they read)
    std::vector<AdjTask> tasks;
    {
        const int nb = t->num_bonds;
        for (int q = 0; q < c.nR; ++q) {
            const SideBond &fb = right[q];
            const uint8_t bi = (uint8_t)(li.word_shift[fb.a] + fb.pi), bj = (uint8_t)(li.word_shift[fb.b] + fb.pj);
            tasks.push_back(AdjTask{fb.bond, 0, 0, 0, 0, (uint16_t)q, 0.5f});
            tasks.push_back(AdjTask{(uint16_t)(nb + fb.bond), 2, 1, bi, bj, 0, 1.0f});
        }
        for (int q = 0; q < c.nX; ++q) {
            const CrossBond &cb = c.x[q];
            tasks.push_back(AdjTask{cb.bond, 0, 0, 0, 0, (uint16_t)(32 + q), 0.5f});
            tasks.push_back(AdjTask{(uint16_t)(nb + cb.bond), 0, 2, cb.lbit, 0, (uint16_t)(41 + cb.sj), 1.0f});
        }
        for (const SideBond &fb : left) {
            const uint8_t bi = (uint8_t)(li.word_shift[fb.a] + fb.pi), bj = (uint8_t)(li.word_shift[fb.b] + fb.pj);
            tasks.push_back(AdjTask{fb.bond, 1, 0, 0, 0, fb.bond, 0.5f});
            tasks.push_back(AdjTask{(uint16_t)(nb + fb.bond), 0, 1, bi, bj, 40, 1.0f});
        }
        for (int i = 0; i < sd.L; ++i) {
            const bool lft = sd.site_sub[i] < K;
            tasks.push_back(AdjTask{(uint16_t)(2 * nb + i), (uint8_t)(lft ? 0 : 2), 3, packed_bit(i), 0,
                                    (uint16_t)(lft ? 40 : 0), 1.0f});
        }
        c.n_adjtasks = (int)tasks.size();
        for (int j = 0; j < c.nJs && j < 8; ++j) c.jbit[j] = packed_bit(rsites[j]);
    }
    DeviceGuard dg(s->device);
    // the left family with every target as a run start (bond << 48 | run), for the
    // rows pass that applies the left family itself
    std::vector<uint64_t> lrun(lent.size());
    for (uint32_t g = 0; g < li.count; ++g)
        for (uint32_t q = lptr[g]; q < lptr[g + 1]; ++q) {
            const uint64_t e = lent[q];
            lrun[q] = (e >> 63) ? ((e & (0xFFull << 48)) | li.h_runs[clstart[cl_of[g]] + (uint32_t)(e & 0xFFFFu)])
                                : e;
        }
    // the offset tables in their device width (16 or 32 bits per entry)
    auto narrow = [&](const std::vector<uint32_t> &v) {
        std::vector<char> out(v.size() * (wide ? 4 : 2));
        for (size_t i = 0; i < v.size(); ++i) {
            if (wide) {
                memcpy(out.data() + 4 * i, &v[i], 4);
            } else {
                const uint16_t h = (uint16_t)v[i];
                memcpy(out.data() + 2 * i, &h, 2);
            }
        }
        return out;
    };
    const std::vector<char> vo_dev = narrow(vo), xo_dev = narrow(xo);
    auto up = [&](void **dst, const void *src, size_t bytes) -> bool {
        if (check_hip(hipMalloc(dst, bytes ? bytes : 16), "hipMalloc split tables")) return false;
        if (bytes && check_hip(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice), "copy split tables"))
            return false;
        return true;
    };
    bool ok = up((void **)&c.d_lptr, lptr.data(), lptr.size() * sizeof(uint32_t)) &&
              up((void **)&c.d_lent, lent.data(), lent.size() * sizeof(uint64_t)) &&
              up((void **)&c.d_vo, vo_dev.data(), vo_dev.size()) &&
              up((void **)&c.d_xl, xl.data(), xl.size() * sizeof(uint64_t)) &&
              up((void **)&c.d_xo, xo_dev.data(), xo_dev.size()) &&
              up((void **)&c.d_runs, li.h_runs.data(), li.h_runs.size() * sizeof(uint64_t)) &&
              up((void **)&c.d_clstart, clstart.data(), clstart.size() * sizeof(uint32_t)) &&
              up((void **)&c.d_clsize, clsize.data(), clsize.size() * sizeof(uint32_t)) &&
              up((void **)&c.d_lrun, lrun.data(), lrun.size() * sizeof(uint64_t)) &&
              up((void **)&c.d_rorder, c.h_rorder.data(), c.h_rorder.size() * sizeof(uint32_t)) &&
              // diagonal of both sides, then the per-call coupling factors (1024 doubles + 1024 floats)
              check_hip(hipMalloc(&c.d_diag, ((li.count + li.rcount + 1) / 2 * 2 + 1536) * sizeof(double)),
                        "hipMalloc split diagonal") == DCS_OK;
    ok = ok && up((void **)&c.d_adjtasks, tasks.data(), tasks.size() * sizeof(AdjTask));
    for (int ti = 0; ti < kRowTilings && ok; ++ti) {
        RowTiling &T = c.tiling[ti];
        if (!T.ntiles) continue;
        ok = up((void **)&T.d_tiles, T.h_tiles.data(), T.h_tiles.size() * sizeof(uint2)) &&
             up((void **)&T.d_tiles_canon, T.h_canon.data(), T.h_canon.size() * sizeof(uint2)) &&
             up((void **)&T.d_pat, T.h_pat.data(), T.h_pat.size() * sizeof(uint2));
        T.h_tiles.clear();
        T.h_tiles.shrink_to_fit();
        T.h_canon.clear();
        T.h_canon.shrink_to_fit();
    }
    c.n_rorder = c.h_rorder.size();
    c.h_rorder.clear();
    c.h_rorder.shrink_to_fit();
    if (!ok) {
        free_rows(c);
        return nullptr;
    }
    SplitRows &slot = li.rows[li.next_slot];
    li.next_slot = (li.next_slot + 1) % kMaxSplitCache;
    if (slot.terms_id) {  // the evicted tables may still be in use on the streams that ran them
        if (slot.use_overflow) {
            (void)hipDeviceSynchronize();
        } else {
            for (int i = 0; i < slot.nuse; ++i) (void)hipEventSynchronize(slot.use_event[i]);
        }
    }
    free_rows(slot);
    slot = c;
    return &slot;
}

void note_split_use(dcs_sector *s, SplitRows &c, hipStream_t stream) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    std::lock_guard<std::mutex> guard(*s->left.rows_lock);
    int i = 0;
    while (i < c.nuse && c.use_stream[i] != stream) ++i;
    if (i == c.nuse) {
        if (c.nuse == SplitRows::kUseStreams ||
            hipEventCreateWithFlags(&c.use_event[i], hipEventDisableTiming) != hipSuccess) {
            c.use_overflow = true;
            return;
        }
        c.use_stream[i] = stream;
        ++c.nuse;
    }
    if (hipEventRecord(c.use_event[i], stream) != hipSuccess) c.use_overflow = true;
}

}  // namespace dcs
