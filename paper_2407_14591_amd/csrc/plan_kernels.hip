// Many sectors in one persistent launch: y_s = H_s x_s for every sector s of a plan.
//
// The rows of all sectors are cut into tiles of kHxThreads rows that never
// cross a sector boundary, listed sector by sector.  The tiles go out in
// chunks of kPlanChunk consecutive tiles, dealt round robin to the 8 XCDs; the
// workgroups of an XCD (dispatch order blockIdx % 8) take the next tile of
// their XCD's sequence from one counter, claimed one tile ahead, so sectors of
// unequal cost per row (spin 1 against spin 1/2) spread evenly over the chip.
// When a workgroup's tile moves to another sector it re-stages that sector's
// tables and bond coefficients into LDS.  Sectors may differ in L, n, Q and
// split; each tile takes the Q=2 or general-Q bond code by a uniform branch.
// Each row is written by one thread, so the result does not depend on which
// workgroup took which tile.
#include <algorithm>
#include <vector>

#include "hx_impl.h"

namespace dcs {
namespace hx {

// Per-sector parameters, resident in device memory.
struct PlanSector {
    SectorDesc sd;
    const char *blob;
    const double *jxy, *jz, *h;
    int nbonds;
    int q2;
    uint64_t cls_mask;
    int far_below;
    uint16_t cls_beg[kMaxClasses + 1];
    uint32_t pos[kMaxBonds];
};

struct PlanIO {
    const void *x;
    void *y;
};
static_assert(sizeof(PlanIO) == 2 * sizeof(void *), "PlanIO is read as two pointers");
static_assert(sizeof(uint2) == 2 * sizeof(uint32_t), "tiles are read as two words");

struct PlanArgs {
    const PlanSector *secs;
    const PlanIO *io;
    const uint2 *tiles;  // (sector, first row)
    uint32_t ntiles;
    uint32_t *counters;  // one per XCD, zero at launch
};

constexpr uint32_t kPlanChunk = 256;

// The plan's device arrays are read-only during a launch: read them through the
// constant address space, so that wave-uniform reads become scalar loads.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *const_view(const T *p) {
    return (const __attribute__((address_space(4))) T *)p;
}

// Tile of position i in XCD x's sequence (chunks dealt round robin).
__device__ __forceinline__ uint32_t plan_tile(uint32_t i, uint32_t x) {
    return ((i / kPlanChunk) * 8u + x) * kPlanChunk + i % kPlanChunk;
}

template <typename IdxT, typename T, int NMAX>
__global__ __launch_bounds__(kHxThreads) void plan_kernel(const PlanArgs A) {
    extern __shared__ __align__(16) char lds[];
    __shared__ uint32_t slot[2];
    const uint32_t xcd = blockIdx.x & 7u;
    const int wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) slot[0] = atomicAdd(A.counters + xcd, 1u);
    __syncthreads();
    uint32_t cur_slot = slot[0];
    int b = 0;
    int cur = -1;
    // an XCD's sequence is increasing in the tile index: the first position past
    // the list ends the workgroup
    for (uint32_t t = plan_tile(cur_slot, xcd); t < A.ntiles; t = plan_tile(cur_slot, xcd)) {
        if (threadIdx.x == 0) slot[b ^ 1] = atomicAdd(A.counters + xcd, 1u);  // the next, ahead
        const uint32_t *tw = reinterpret_cast<const uint32_t *>(A.tiles);
        const int sid = (int)const_view(tw)[2 * t];
        const uint32_t row0 = const_view(tw)[2 * t + 1];
        const PlanSector &ps = *(const PlanSector *)(const_view(A.secs) + sid);
        const CoeffLds<T> C(lds, ps.sd.lay_bytes);
        if (sid != cur) {
            __syncthreads();
            stage_blob(lds, ps.blob, ps.sd.lay_bytes);
            if (ps.q2)
                stage_coefficients<T, true>(ps, ps.sd, C.bamp, C.bjz, C.ladder, C.hf);
            else
                stage_coefficients<T, false>(ps, ps.sd, C.bamp, C.bjz, C.ladder, C.hf);
            __syncthreads();
            cur = sid;
        }
        const Tables<IdxT> Tb = tables_at<IdxT>(lds, ps.sd);
        const void *const *io = reinterpret_cast<const void *const *>(A.io);  // (x, y) per sector
        const T *__restrict__ x = reinterpret_cast<const T *>(const_view(io)[2 * sid]);
        T *__restrict__ y = reinterpret_cast<T *>(const_cast<void *>(const_view(io)[2 * sid + 1]));
        const uint64_t end = min((uint64_t)row0 + kHxThreads, ps.sd.dim);
        const uint64_t tile = (uint64_t)row0 + (uint64_t)wave * 64;
        if (tile < end) {
            if (ps.q2)
                hx_tile<IdxT, T, 1, NMAX, true>(ps, ps.sd, Tb, x, y, C.bamp, C.bjz, C.ladder, C.hf,
                                                false, tile, end);
            else
                hx_tile<IdxT, T, 1, NMAX, false>(ps, ps.sd, Tb, x, y, C.bamp, C.bjz, C.ladder, C.hf,
                                                 false, tile, end);
        }
        __syncthreads();  // slot[b ^ 1] is written; slot[b] is free for the claim after next
        b ^= 1;
        cur_slot = slot[b];
    }
}

}  // namespace hx
}  // namespace dcs

using namespace dcs;
using namespace dcs::hx;

struct dcs_plan {
    int device = 0;
    int nsec = 0;
    int nmax = 4;
    uint32_t ntiles = 0;
    size_t lds_bytes = 0;
    PlanSector *d_secs = nullptr;
    PlanIO *d_io = nullptr;
    uint2 *d_tiles = nullptr;
    PlanIO *h_io = nullptr;  // pinned staging of the vector pointers
    hipEvent_t io_copied = nullptr;
    bool io_pending = false;
    std::vector<uint64_t> dims;
    uint32_t *d_counters = nullptr;  // the tile queue's per-XCD counters
    // sectors that run their own product (own_product) after or beside the launch,
    // in the form the autotuner keeps for them
    struct Own {
        int index;
        dcs_sector *sector;
        const dcs_terms *terms;
        const double *jxy, *jz;
        int side;  // side stream; every product of one sector goes to the same one
    };
    std::vector<Own> own;
    // After the first apply of a dtype (whose products the autotuner times on the
    // caller's stream), the own products run on kSideStreams more streams beside
    // it, forked and joined with events, so that their launch tails overlap.
    static constexpr int kSideStreams = 3;
    hipStream_t side[kSideStreams] = {};
    hipEvent_t fork = nullptr, join[kSideStreams] = {};
    bool applied[2] = {false, false};  // per dtype (F32, F64)
};

static void plan_free(dcs_plan *p) {
    if (!p) return;
    DeviceGuard g(p->device);
    if (p->io_copied) {
        hipEventSynchronize(p->io_copied);
        hipEventDestroy(p->io_copied);
    }
    hipFree(p->d_secs);
    hipFree(p->d_io);
    hipFree(p->d_tiles);
    hipFree(p->d_counters);
    hipHostFree(p->h_io);
    for (int i = 0; i < dcs_plan::kSideStreams; ++i) {
        if (p->side[i]) {
            hipStreamSynchronize(p->side[i]);
            hipStreamDestroy(p->side[i]);
        }
        if (p->join[i]) hipEventDestroy(p->join[i]);
    }
    if (p->fork) hipEventDestroy(p->fork);
    delete p;
}

// Whether a sector runs its own product beside the launch instead of inside it:
// only sectors with a split view (Q = 2, the split product) can, and they do when
// their tables are in device memory (the launch stages tables in LDS) or when
// DCS_PLAN_HYBRID=1 (read at plan creation).  By default every other sector is in
// the one launch: for the 101 sectors of L = 20..26 and spin-1 L = 12..16 that
// is 2.33 ms against 2.39 ms with the 18 largest on their own split products.
static bool own_product(const dcs_sector *sec, bool hybrid) {
    return sec->left.K > 0 && sec->desc.Q == 2 && (hybrid || sec->gtab);
}

extern "C" int dcs_plan_create(int nsec, dcs_sector *const *secs, dcs_terms *const *terms,
                               const double *const *jxy, const double *const *jz, dcs_plan **out) {
    clear_error();
    if (!out) return set_error(DCS_EINVAL, "out is NULL");
    *out = nullptr;
    if (nsec < 1 || !secs || !terms || !jxy || !jz) return set_error(DCS_EINVAL, "empty plan");
    const int device = secs[0] ? secs[0]->device : 0;
    const char *hy = getenv("DCS_PLAN_HYBRID");
    const bool hybrid = hy && hy[0] == '1';
    int nmax = 4;
    size_t lds = 0;
    std::vector<PlanSector> hs(nsec);
    std::vector<uint2> tiles;
    for (int s = 0; s < nsec; ++s) {
        const dcs_sector *sec = secs[s];
        const dcs_terms *t = terms[s];
        if (!sec || !t) return set_error(DCS_EINVAL, "NULL sector or terms at %d", s);
        if (int r = refuse_mixed(sec)) return r;
        if (sec->device != device) return set_error(DCS_EINVAL, "sectors on different devices");
        if (sec->wide) return set_error(DCS_EUNSUPPORTED, "plan sectors need dimension < 2^32");
        if (t->num_bonds > 0 && (!jxy[s] || !jz[s]))
            return set_error(DCS_EINVAL, "NULL couplings at %d", s);
        if (sec->desc.N > 4) nmax = 8;
        if (own_product(sec, hybrid)) continue;  // a product of its own, outside the launch
        if (sec->gtab)
            return set_error(DCS_EUNSUPPORTED, "plan sector %d: tables in device memory and no split view", s);
        lds = std::max(lds, (size_t)sec->desc.lay_bytes + coeff_lds_bytes<double>());
    }
    for (int s = 0; s < nsec; ++s) {
        BondPlan bp;
        if (int r = make_bond_plan(secs[s], terms[s], nmax, &bp)) return r;
        PlanSector &ps = hs[s];
        memset(&ps, 0, sizeof(ps));
        ps.sd = secs[s]->desc;
        ps.blob = (const char *)secs[s]->dev.base;
        ps.jxy = jxy[s];
        ps.jz = jz[s];
        ps.h = nullptr;
        ps.nbonds = bp.nbonds;
        ps.q2 = secs[s]->desc.Q == 2;
        ps.cls_mask = ~0ull;
        ps.far_below = ps.sd.dim >= (1ull << 22) ? ps.sd.N / 2 : 0;  // as for one sector
        for (int c = 0; c <= bp.nclasses; ++c) ps.cls_beg[c] = bp.cls_beg[c];
        for (int b = 0; b < bp.nbonds; ++b) ps.pos[b] = bp.pos[b];
        if (own_product(secs[s], hybrid)) continue;  // a product of its own
        for (uint64_t r0 = 0; r0 < ps.sd.dim; r0 += kHxThreads) tiles.push_back(make_uint2(s, (uint32_t)r0));
    }
    dcs_plan *p = new (std::nothrow) dcs_plan();
    if (!p) return set_error(DCS_ENOMEM, "host allocation failed");
    p->device = device;
    p->nsec = nsec;
    p->nmax = nmax;
    p->ntiles = (uint32_t)tiles.size();
    p->lds_bytes = lds;
    // A sector listed more than once (other terms or couplings) shares its tile
    // counters, cached tables and diagonal buffer between its products, so those
    // products must not overlap: they all go to the side stream of the sector's
    // first appearance, in plan order.
    int distinct = 0;
    for (int s = 0; s < nsec; ++s) {
        p->dims.push_back(secs[s]->desc.dim);
        if (own_product(secs[s], hybrid)) {
            int side = -1;
            for (const auto &o : p->own)
                if (o.sector == secs[s]) side = o.side;
            if (side < 0) side = distinct++ % dcs_plan::kSideStreams;
            p->own.push_back(dcs_plan::Own{s, secs[s], terms[s], jxy[s], jz[s], side});
        }
    }
    DeviceGuard g(device);
    int r = check_hip(hipMalloc(&p->d_secs, nsec * sizeof(PlanSector)), "hipMalloc plan");
    if (!r) r = check_hip(hipMalloc(&p->d_io, nsec * sizeof(PlanIO)), "hipMalloc plan io");
    if (!r) r = check_hip(hipMalloc(&p->d_tiles, std::max<size_t>(tiles.size(), 1) * sizeof(uint2)),
                          "hipMalloc tiles");
    if (!r) r = check_hip(hipHostMalloc(&p->h_io, nsec * sizeof(PlanIO)), "hipHostMalloc");
    if (!r) r = check_hip(hipMalloc(&p->d_counters, 8 * sizeof(uint32_t)), "hipMalloc plan counters");
    if (!r) r = check_hip(hipEventCreateWithFlags(&p->io_copied, hipEventDisableTiming), "event");
    if (!r && p->own.size() > 1) {  // default priority, not synchronising with the null stream
        r = check_hip(hipEventCreateWithFlags(&p->fork, hipEventDisableTiming), "event");
        for (int i = 0; i < dcs_plan::kSideStreams && !r; ++i) {
            r = check_hip(hipStreamCreateWithFlags(&p->side[i], hipStreamNonBlocking), "plan stream");
            if (!r) r = check_hip(hipEventCreateWithFlags(&p->join[i], hipEventDisableTiming), "event");
        }
    }
    if (!r)
        r = check_hip(hipMemcpy(p->d_secs, hs.data(), nsec * sizeof(PlanSector), hipMemcpyHostToDevice),
                      "copy plan");
    if (!r && !tiles.empty())
        r = check_hip(hipMemcpy(p->d_tiles, tiles.data(), tiles.size() * sizeof(uint2),
                                hipMemcpyHostToDevice),
                      "copy tiles");
    if (r) {
        plan_free(p);
        return r;
    }
    *out = p;
    return DCS_OK;
}

extern "C" int dcs_plan_destroy(dcs_plan *p) {
    clear_error();
    plan_free(p);
    return DCS_OK;
}

template <typename T, int NMAX>
static int launch_plan(dcs_plan *p, hipStream_t stream) {
    const uint2 *tiles = p->d_tiles;
    const uint32_t ntiles = p->ntiles;
    const int cus = device_cu_count(p->device);
    int per_cu = (int)((160 * 1024) / p->lds_bytes);
    per_cu = per_cu < 1 ? 1 : (per_cu > 4 ? 4 : per_cu);
    // a multiple of 8 workgroups, so that every XCD's tile sequence has workers
    uint64_t wgs = std::min<uint64_t>((uint64_t)cus * per_cu, ntiles);
    wgs = std::max<uint64_t>(8, (wgs + 7) / 8 * 8);
    PlanArgs A;
    A.secs = p->d_secs;
    A.io = p->d_io;
    A.tiles = tiles;
    A.ntiles = ntiles;
    A.counters = p->d_counters;
    zero_counters<0><<<1, 64, 0, stream>>>(p->d_counters, 8);
    auto kern = plan_kernel<uint32_t, T, NMAX>;
    if (int r = ensure_lds(kern, p->lds_bytes)) return r;
    kern<<<(unsigned)wgs, kHxThreads, p->lds_bytes, stream>>>(A);
    return check_hip(hipGetLastError(), "plan kernel launch");
}

extern "C" int dcs_plan_apply(const dcs_plan *pc, int dtype, const void *const *xs,
                              void *const *ys, void *stream_v) {
    clear_error();
    dcs_plan *p = const_cast<dcs_plan *>(pc);
    if (!p || !xs || !ys) return set_error(DCS_EINVAL, "NULL argument");
    if (dtype != DCS_F32 && dtype != DCS_F64) return set_error(DCS_EINVAL, "dtype %d", dtype);
    const size_t es = dtype == DCS_F32 ? 4 : 8;
    for (int s = 0; s < p->nsec; ++s) {
        if (!xs[s] || !ys[s]) return set_error(DCS_EINVAL, "NULL vector for sector %d", s);
        const char *xb = (const char *)xs[s], *yb = (const char *)ys[s];
        const size_t bytes = p->dims[s] * es;
        if (xb < yb + bytes && yb < xb + bytes)
            return set_error(DCS_EINVAL, "x and y of sector %d overlap", s);
    }
    hipStream_t stream = (hipStream_t)stream_v;
    DeviceGuard g(p->device);
    // the pinned staging buffer may still feed the previous call's copy
    if (p->io_pending)
        if (int r = check_hip(hipEventSynchronize(p->io_copied), "wait for plan io copy")) return r;
    for (int s = 0; s < p->nsec; ++s) p->h_io[s] = PlanIO{xs[s], ys[s]};
    if (int r = check_hip(hipMemcpyAsync(p->d_io, p->h_io, p->nsec * sizeof(PlanIO),
                                         hipMemcpyHostToDevice, stream),
                          "copy plan io"))
        return r;
    if (int r = check_hip(hipEventRecord(p->io_copied, stream), "record plan io event")) return r;
    p->io_pending = true;
    auto launch_core = [&]() -> int {
        if (p->ntiles == 0) return DCS_OK;
        return dtype == DCS_F32
                   ? (p->nmax == 4 ? launch_plan<float, 4>(p, stream) : launch_plan<float, 8>(p, stream))
                   : (p->nmax == 4 ? launch_plan<double, 4>(p, stream) : launch_plan<double, 8>(p, stream));
    };
    const int di = dtype == DCS_F32 ? 0 : 1;
    if (!p->applied[di] || !p->fork) {  // the first apply of a dtype: one stream (autotuner timing)
        if (int r = launch_core()) return r;
        for (const auto &o : p->own)
            if (int r = launch_hx(o.sector, o.terms, o.jxy, o.jz, nullptr, dtype, 1, xs[o.index], ys[o.index], stream))
                return r;
        p->applied[di] = true;
        return DCS_OK;
    }
    // fork: the side streams wait for the work queued so far on the caller's stream
    if (int r = check_hip(hipEventRecord(p->fork, stream), "plan fork")) return r;
    for (int i = 0; i < dcs_plan::kSideStreams; ++i)
        if (int r = check_hip(hipStreamWaitEvent(p->side[i], p->fork, 0), "plan fork wait")) return r;
    // the one launch on the caller's stream, the own products on the side streams
    // (distinct sectors have their own counters and tables, so they may run
    // together; repeated sectors are serialised on one stream)
    int r = launch_core();
    for (size_t q = 0; q < p->own.size() && !r; ++q) {
        const auto &o = p->own[q];
        r = launch_hx(o.sector, o.terms, o.jxy, o.jz, nullptr, dtype, 1, xs[o.index], ys[o.index],
                      p->side[o.side]);
    }
    // join, also after a failed launch, so that no side stream is left behind
    for (int i = 0; i < dcs_plan::kSideStreams; ++i) {
        const int rr = check_hip(hipEventRecord(p->join[i], p->side[i]), "plan join");
        const int rw = rr ? rr : check_hip(hipStreamWaitEvent(stream, p->join[i], 0), "plan join wait");
        if (!r) r = rw;
    }
    return r;
}
