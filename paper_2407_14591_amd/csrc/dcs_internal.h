// Internal declarations of the dcs library (not part of the ABI).
//
// Device data of a sector, built on the host by sector.cpp:
//
//  * fused contribution table ("c-table"), one row per (subsystem k, lambda):
//      C_k[lambda][w] = offset_k(n(w), lambda) + stride_k(n(w), lambda) * index_k(w)
//    for every word w of P_k (eq. ck with eq. offset / eq. stride), or the
//    sentinel kBad when w has a digit >= Q or its digit sum n(w) cannot occur
//    with lambda particles to the left.  The last subsystem has offset 0 and
//    stride 1 (its digit sum is fixed by lambda), so it keeps a single row with
//    the local index; rank checks its digit sum separately.  The paper keeps offsets, strides and
//    the local table apart and multiplies at lookup time; for two subsystems
//    it folds c_0 into P_0's table (Sec. 3.3.1).  Adding lambda as a table
//    dimension applies that folding to every subsystem: a rank becomes N
//    table reads and N-1 adds, index(s) = sum_k C_k[lambda_k][w_k].  The rows
//    cover only the feasible lambda of each subsystem; for the workloads here
//    the whole table is 9..64 KiB and is staged in LDS.
//  * decode table per (k, lambda, m): offset_k(m, lambda), stride_k(m, lambda)
//    and a float reciprocal of the stride (the quotient index_k is below
//    2^14, so one float multiply plus a one-step correction is exact);
//  * inverse local tables: the words of P_k listed by (digit sum, index).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "dcs.h"

namespace dcs {

constexpr int kMaxSub = DCS_MAX_SUBSYSTEMS;
constexpr int kMaxSites = DCS_MAX_SITES;
constexpr int kMaxBonds = DCS_MAX_BONDS;
constexpr int kMaxWordBits = 16;       // inverse tables hold words in 16 bits
constexpr uint64_t kMaxClassWords = 1u << 14;  // decode: the quotient index_k stays below 2^14
constexpr size_t kLdsTableBudget = 112 * 1024;
constexpr int kMaxDevices = 64;

template <typename IdxT>
struct Bad;
template <>
struct Bad<uint32_t> {
    static constexpr uint32_t value = 0xFFFFFFFFu;
};
template <>
struct Bad<uint64_t> {
    static constexpr uint64_t value = ~0ull;
};

// Everything a kernel needs to know about a sector; passed by value.
struct SectorDesc {
    uint64_t dim;
    int Q, nb, L, n, N;             // Q: the largest local dimension (sets nb)
    int total_bits;                 // nb * L
    int shift[kMaxSub];             // bit position of P_k's word in the state
    int wbits[kMaxSub];             // nb * L_k
    int rest_max[kMaxSub];          // largest digit sum of the sites to the right of P_k
    int mk[kMaxSub];                // largest digit sum of P_k's sites ((Q-1) L_k for one Q)
    int lam_lo[kMaxSub], lam_hi[kMaxSub];
    uint32_t ctab_row0[kMaxSub];    // entry of C_k[lam_lo[k]][0]
    uint32_t ctab_rowlen[kMaxSub];  // entries per lambda row: 2^wbits, 0 for the last subsystem
    uint32_t ctab_entries;
    uint32_t dec_row0[kMaxSub];     // entry of (k, lam_lo[k], m=0); rows of mk[k]+1
    uint32_t dec_entries;
    uint32_t inv_start0[kMaxSub];   // entry of inv_start for (k, m=0); mk[k]+2 per k
    uint32_t inv_start_entries;
    uint32_t inv_entries;
    uint32_t field_mask[4];         // bit t of every site field of a word (digit sums)
    // byte offsets of the table arrays inside the sector's device blob
    uint32_t lay_ctab, lay_doff, lay_dstr, lay_drcp, lay_invs, lay_inv, lay_bytes;
    uint8_t site_sub[kMaxSites];    // subsystem of each site
    uint8_t site_bit[kMaxSites];    // bit of the site's field inside its subsystem word
};

// Device-side arrays of one sector (one allocation, see sector.cpp for layout).
struct SectorDev {
    void *base = nullptr;
    size_t bytes = 0;
    size_t ctab_off = 0, dec_off_off = 0, dec_str_off = 0, dec_rcp_off = 0, inv_off = 0,
           inv_start_off = 0;
    // bytes the H*x kernels stage in LDS (c-table + decode + inverse tables)
    size_t lds_bytes = 0;
    // work-queue counters of the H*x launches (8 per pass, zeroed by a kernel
    // before each launch); calls on one sector must therefore not overlap
    uint32_t *counters = nullptr;
};
constexpr int kNumCounters = 32;

// Left/right view of a sector for the split product.  Cut the subsystems at
// K: for a fixed number m of particles in P_0..P_{K-1} ("left"), every left
// configuration (w_0..w_{K-1}) owns one contiguous run of rows of the same
// length, one row per right configuration (w_K..w_{N-1}) (the rank of eq. index
// is a sum over subsystems, so row = run start + offset).  A bond with both
// sites left of the cut maps a row to the same offset of another run; a bond
// with both sites right of it stays inside the run; a bond across the cut
// flips one site on each side.  All three act on small sub-sectors (2^16
// configurations per side at L = 32), so their targets are tabulated once per
// (sector, terms) pair, like the paper's cluster matrices (App. C).
constexpr int kMaxLeftM = 40;
constexpr int kMaxSplitCache = 4;
constexpr int kMaxCross = 96;       // bonds across the cut
constexpr int kMaxCrossSites = 32;  // distinct sites of those bonds on either side
constexpr uint32_t kMaxClusterRuns = 70;  // left configurations per cluster of the column pass

struct CrossBond {
    uint8_t si, sj;      // slot of the left / right site in the flip tables
    uint8_t lbit, rbit;  // bit of the left / right site in the packed left / right word
    uint16_t bond;       // index in the terms
    uint16_t pad;
};

// Bond or field entry of the per-configuration diagonal (one side of the cut).
struct DiagTerm {
    uint8_t side;        // 0 left, 1 right
    uint8_t bi, bj;      // bits in the packed word of that side (bj unused for a field)
    uint8_t is_field;
    uint16_t index;      // bond index in the terms, or site for a field
    uint16_t pad;
};

// Tiles of the row pass that stages whole blocks of a run in LDS (one tiling per
// row size class RB = 16, 32, 64 bytes).  The rows of a run with equal particle
// number on P_K (the first right subsystem) are contiguous ("n_K blocks"); a
// tile is a contiguous range of whole n_K blocks of one run that fits the LDS
// budget, or, for an n_K block larger than that, a range of whole sub-runs of
// equal P_K word.  Bonds that keep n_K then read the tile in LDS.
constexpr int kRowTilings = 3;             // RB = 16, 32, 64
constexpr uint32_t kTileLdsTotal = 160 * 1024;  // LDS of one workgroup of the block-tiled row pass
constexpr uint32_t kTileLdsStatic = 1024;       // its static LDS and slack
constexpr int kMaxRunTiles = 64;           // tiles of one run
constexpr uint32_t kSplitRowTile = 512;    // rows of one tile of the row pass (one per thread)
struct RowTiling {
    uint2 *d_tiles = nullptr;              // (left configuration, block | tile-in-run << 8), in launch order:
                                           // groups of left configurations that differ only on the
                                           // sites of bonds across the cut, tile index, configuration
    uint2 *d_tiles_canon = nullptr;        // the same tiles in row order
    uint2 *d_pat = nullptr;                // (first offset, rows) of tile j of block m: pat[pbase[m] + j]
    uint64_t ntiles = 0;
    uint32_t max_rows = 0;                 // rows of the largest tile
    uint32_t pbase[kMaxLeftM] = {};
    uint32_t ntile[kMaxLeftM] = {};
    std::vector<uint2> h_pat, h_tiles, h_canon;  // host copies while building
};

// One output sum of the adjoint on the split view: a weighted sum over the
// per-tile values the passes wrote (see split_adjoint.hip).
struct AdjTask {
    uint16_t out;     // [0, nb) d/dJxy, [nb, 2 nb) d/dJz, [2 nb, 2 nb + L) d/dh
    uint8_t src;      // 0: row-pass value v per left configuration, 1: column-pass bond v per
                      // column tile, 2: right-configuration sum of x_s g_s
    uint8_t mode;     // weight from the entry's word: 0: 1, 1: s_a s_b / 4, 2: s_a / 4, 3: bit_a - 1/2
    uint8_t ba, bb;   // bits a, b of the packed left (src 0) or right (src 2) word (s = 2 bit - 1)
    uint16_t v;
    float scale;
};

struct SplitRows {
    uint64_t terms_id = 0;           // 0: empty slot
    uint32_t *d_lptr = nullptr;      // left family: entry range of every left configuration
    uint64_t *d_lent = nullptr;      // target run start (low 48 bits) | bond << 48, or, for a target
                                     // in the own cluster, 1 << 63 | bond << 48 | index in the cluster
    bool wide_off = false;           // runs of 65,535 rows or more: 32-bit entries in vo / xo,
                                     // four per 16-byte row ([group][r][4]), 0xFFFFFFFF = no hop
    uint16_t *d_vo = nullptr;        // right family: [bond group][right configuration][8] target
                                     // offset in the run, 0xFFFF where the bond does not hop
    uint64_t *d_xl = nullptr;        // crossing: [left site slot][left configuration] run start of
                                     // the configuration with that site flipped, ~0 if none
    uint16_t *d_xo = nullptr;        // crossing: [group of 8 right site slots][right configuration][8]
                                     // offset of the configuration with that site flipped in its
                                     // block, 0xFFFF if none
    uint64_t *d_runs = nullptr;      // run start of every left configuration
    // clusters of the left family: consecutive left configurations (one block)
    // with equal words of P_0..P_{K-2}, at most kMaxClusterRuns each; bonds
    // inside P_{K-1} map a cluster onto itself
    uint32_t *d_clstart = nullptr;   // first left configuration of every cluster
    uint32_t *d_clsize = nullptr;    // its number of left configurations
    uint64_t *d_lrun = nullptr;      // the left family entries with run starts only: bond << 48 | run
    uint32_t *d_rorder = nullptr;    // tiles of the row pass (left configuration << 8 | chunk) by
                                     // groups of equal words outside the crossing sites
    uint64_t n_rorder = 0;
    std::vector<uint32_t> h_rorder;  // (host, while building)
    uint32_t clbase[kMaxLeftM];      // first cluster of block m - m_lo
    uint32_t nclust[kMaxLeftM];
    uint32_t max_cluster = 0;
    double *d_diag = nullptr;        // per call: left | right configuration diagonals, coupling factors
    int nR = 0, nX = 0, nIs = 0, nJs = 0, nD = 0;
    int nRloc = 0;                   // right-family bonds inside the last subsystem (listed first)
    int nRA = 0;                     // right-family bonds keeping n_K (listed before the others)
    uint32_t margin = 0;             // rows of the largest run of equal P_K..P_{N-2} words
    uint64_t lnnz = 0;
    uint16_t r_bond[kMaxBonds];      // bond index of every right-family bond
    RowTiling tiling[kRowTilings];   // block tiles of the row pass, by row size
    AdjTask *d_adjtasks = nullptr;   // the adjoint's output sums (2 per bond, 1 per site)
    int n_adjtasks = 0;
    uint8_t jbit[8] = {};            // packed right bit of crossing right-site slot j (j < 8)
    CrossBond x[kMaxCross];
    DiagTerm d[kMaxBonds + kMaxSites];
    // streams that have run products on these tables, with an event recorded
    // after the last one on each; evicting the set waits for those events only
    static constexpr int kUseStreams = 8;
    hipStream_t use_stream[kUseStreams] = {};
    hipEvent_t use_event[kUseStreams] = {};
    int nuse = 0;
    bool use_overflow = false;  // more streams than slots: eviction synchronises the device
};

struct LeftInfo {
    int K = 0;                 // 0: no split view
    int L_left = 0;
    int m_lo = 0, m_count = 0; // left particle numbers with rows
    uint32_t lbase[kMaxLeftM]; // first left configuration of block m - m_lo
    uint32_t nleft[kMaxLeftM];
    uint64_t ncols[kMaxLeftM]; // run length R(m)
    uint32_t rbase[kMaxLeftM]; // first right configuration of block m - m_lo
    uint32_t word_shift[kMaxSub];  // bit of P_k's word inside a packed left / right word
    void *d_words = nullptr;   // uint32 packed left words, all blocks in order
    void *d_runs = nullptr;    // run start (IdxT) of every left configuration
    void *d_rwords = nullptr;  // uint32 packed right words, all blocks in order
    size_t count = 0, rcount = 0;
    std::vector<uint32_t> h_words, h_rwords;
    std::vector<uint64_t> h_runs;
    std::vector<uint64_t> h_ctab;  // host copy of the fused contribution table
    SplitRows rows[kMaxSplitCache];
    int next_slot = 0;
    std::unique_ptr<std::mutex> rows_lock{new std::mutex};  // guards rows[], next_slot, tuned
    std::map<uint64_t, int> tuned;  // autotuned launch form per (terms id, dtype, k)
};

}  // namespace dcs

struct dcs_sector {
    int device;
    int split[dcs::kMaxSub];
    bool wide;  // 64-bit indices (dim >= 2^32)
    bool gtab;  // tables beyond the LDS budget: kernels read them in device memory
    bool mixed;  // local dimensions differ between sites (qsite); XXZ products refuse it
    int qsite[dcs::kMaxSites];  // local dimension of each site
    dcs::SectorDesc desc;
    dcs::SectorDev dev;
    dcs::LeftInfo left;
};

struct dcs_terms {
    uint64_t id;  // unique per created object (keys the per-sector sparse rows)
    int num_bonds;
    int max_site;
    int32_t si[dcs::kMaxBonds];
    int32_t sj[dcs::kMaxBonds];
};

namespace dcs {

// error state (capi.cpp)
int set_error(int code, const char *fmt, ...);
int check_hip(hipError_t e, const char *what);
void clear_error();

// the XXZ products, their adjoint, expectation values and plans assume one local
// dimension on every site: DCS_EUNSUPPORTED for a sector with several
inline int refuse_mixed(const dcs_sector *s) {
    if (s && s->mixed) return set_error(DCS_EUNSUPPORTED, "the XXZ products take one local dimension on every site");
    return DCS_OK;
}

// Bond plan of one (sector, terms) pair: bonds sorted into classes (a, b) of
// the subsystems of their two sites, a <= b, with i in P_a and j in P_b.
struct BondPlan {
    int nbonds;
    int nclasses;                  // kMaxSub * (kMaxSub + 1) / 2
    uint16_t cls_beg[kMaxSub * (kMaxSub + 1) / 2 + 1];
    uint32_t pos[kMaxBonds];       // site_bit(i) | site_bit(j) << 8 | orig << 16
    int16_t site_i[kMaxBonds];     // for the kernels that need sites
    int16_t site_j[kMaxBonds];
};

inline int class_id(int a, int b, int nmax) {  // a <= b < nmax
    return a * nmax - a * (a - 1) / 2 + (b - a);
}

int make_bond_plan(const dcs_sector *s, const dcs_terms *t, int nmax, BondPlan *plan);
void free_split(dcs_sector *s);
void free_rows(SplitRows &c);
// Target tables of the split product of (s, t) (built on first use, cached per
// terms object); NULL if s has no split view or the tables do not apply (an
// error is set only for a failure).
SplitRows *split_rows(dcs_sector *s, const dcs_terms *t);
// Records that work using c was enqueued on `stream` (nothing inside stream capture).
void note_split_use(dcs_sector *s, SplitRows &c, hipStream_t stream);

// kernels launchers (index_kernels.hip, hx_kernels.hip, lanczos.hip)
int launch_rank(const dcs_sector *s, const uint64_t *st, uint64_t *idx, size_t count,
                uint64_t *nbad, hipStream_t stream);
int launch_rank_search(const dcs_sector *s, const uint64_t *st, uint64_t *idx, size_t count,
                       uint64_t *nbad, hipStream_t stream);
// generic operators (operator.hip): argument checks, and y = O x (no checks) on a stream
int operator_check(const dcs_sector *s, const dcs_operator *o, int dtype, int k);
int launch_operator(const dcs_sector *s, const dcs_operator *o, int dtype, int k, const void *x, void *y,
                    hipStream_t stream);
int launch_unrank(const dcs_sector *s, const uint64_t *idx, uint64_t *st, size_t count,
                  uint64_t *nbad, hipStream_t stream);
int launch_enumerate(const dcs_sector *s, uint64_t first, size_t count, uint64_t *st,
                     hipStream_t stream);
int launch_hx(const dcs_sector *s, const dcs_terms *t, const double *jxy, const double *jz,
              const double *h, int dtype, int k, const void *x, void *y, hipStream_t stream);
int hx_form(const dcs_sector *s, const dcs_terms *t, int dtype, int k);
size_t adjoint_ws_bytes(const dcs_sector *s, const dcs_terms *t, int k = 1);  // blocks of k columns
size_t adjoint_single_ws_bytes(const dcs_sector *s, const dcs_terms *t);  // the fused single pass
// The adjoint on the split view for FP32 blocks of k columns (sums formed inside
// the split product of g); DCS_EUNSUPPORTED (no error message) where it does not apply.
int launch_split_adjoint(dcs_sector *s, const SplitRows &c, const double *jxy, const double *jz,
                         const double *h, int nbonds, int k, const void *x, const void *g, void *gx,
                         double *gjxy, double *gjz, double *gh, void *ws, size_t ws_bytes,
                         hipStream_t stream);
size_t split_adjoint_ws_bytes(const dcs_sector *s, int nbonds, int k = 1);
bool split_adjoint_applies(const dcs_sector *s, const SplitRows &c, int dtype, int k = 1);
// The adjoint in one fused pass over the rows (no split tables, no autotuner, no
// allocation): workspace partials only.
int launch_adjoint_single(const dcs_sector *s, const dcs_terms *t, const double *jxy,
                          const double *jz, const double *h, int dtype, const void *x,
                          const void *g, void *gx, double *gjxy, double *gjz, double *gh,
                          void *ws, hipStream_t stream);
int launch_adjoint(const dcs_sector *s, const dcs_terms *t, const double *jxy, const double *jz,
                   const double *h, int dtype, int k, const void *x, const void *g, void *gx,
                   double *gjxy, double *gjz, double *gh, void *ws, size_t ws_bytes,
                   hipStream_t stream);

int device_cu_count(int device);

// Allow a kernel more than the default 64 KiB of dynamic LDS when it needs it.
template <typename KernelT>
inline int ensure_lds(KernelT kernel, size_t bytes) {
    if (bytes <= 64 * 1024) return DCS_OK;
    return check_hip(hipFuncSetAttribute((const void *)kernel,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes),
                     "hipFuncSetAttribute(max dynamic LDS)");
}

// Makes `dev` current for the lifetime of the object and restores the caller's device.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace dcs
