// Many sectors in one persistent launch: y_s = H_s x_s for every sector s of a plan.
//
// The rows of all sectors are cut into tiles of kHxThreads rows that never
// cross a sector boundary, listed sector by sector.  Each workgroup owns a
// contiguous range of tiles (XCD-aware, as for one sector); when its tile
// moves to another sector it re-stages that sector's tables and bond
// coefficients into LDS.  Sectors may differ in L, n, Q and split; each tile
// takes the Q=2 or general-Q bond code by a uniform branch.
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

struct PlanArgs {
    const PlanSector *secs;
    const PlanIO *io;
    const uint2 *tiles;  // (sector, first row)
    uint32_t ntiles;
    uint32_t tiles_per_wg;
    int xcd_groups;
};

template <typename IdxT, typename T, int NMAX>
__global__ __launch_bounds__(kHxThreads) void plan_kernel(const PlanArgs A) {
    extern __shared__ __align__(16) char lds[];
    const uint32_t g = xcd_chunk(A.xcd_groups);
    const uint32_t t0 = g * A.tiles_per_wg;
    const uint32_t t1 = min(t0 + A.tiles_per_wg, A.ntiles);
    const int wave = threadIdx.x >> 6;
    int cur = -1;
    for (uint32_t t = t0; t < t1; ++t) {
        const uint2 tl = A.tiles[t];
        const int sid = (int)tl.x;
        const PlanSector &ps = A.secs[sid];
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
        const T *__restrict__ x = reinterpret_cast<const T *>(A.io[sid].x);
        T *__restrict__ y = reinterpret_cast<T *>(A.io[sid].y);
        const uint64_t end = min((uint64_t)tl.y + kHxThreads, ps.sd.dim);
        const uint64_t tile = (uint64_t)tl.y + (uint64_t)wave * 64;
        if (tile < end) {
            if (ps.q2)
                hx_tile<IdxT, T, 1, NMAX, true>(ps, ps.sd, Tb, x, y, C.bamp, C.bjz, C.ladder, C.hf,
                                                false, tile, end);
            else
                hx_tile<IdxT, T, 1, NMAX, false>(ps, ps.sd, Tb, x, y, C.bamp, C.bjz, C.ladder, C.hf,
                                                 false, tile, end);
        }
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
    // sectors with a split view run their own split product after the launch
    struct Own {
        int index;
        dcs_sector *sector;
        const dcs_terms *terms;
        const double *jxy, *jz;
    };
    std::vector<Own> own;
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
    hipHostFree(p->h_io);
    delete p;
}

extern "C" int dcs_plan_create(int nsec, dcs_sector *const *secs, dcs_terms *const *terms,
                               const double *const *jxy, const double *const *jz, dcs_plan **out) {
    clear_error();
    if (!out) return set_error(DCS_EINVAL, "out is NULL");
    *out = nullptr;
    if (nsec < 1 || !secs || !terms || !jxy || !jz) return set_error(DCS_EINVAL, "empty plan");
    const int device = secs[0] ? secs[0]->device : 0;
    int nmax = 4;
    size_t lds = 0;
    std::vector<PlanSector> hs(nsec);
    std::vector<uint2> tiles;
    for (int s = 0; s < nsec; ++s) {
        const dcs_sector *sec = secs[s];
        const dcs_terms *t = terms[s];
        if (!sec || !t) return set_error(DCS_EINVAL, "NULL sector or terms at %d", s);
        if (sec->device != device) return set_error(DCS_EINVAL, "sectors on different devices");
        if (sec->wide) return set_error(DCS_EUNSUPPORTED, "plan sectors need dimension < 2^32");
        if (t->num_bonds > 0 && (!jxy[s] || !jz[s]))
            return set_error(DCS_EINVAL, "NULL couplings at %d", s);
        if (sec->desc.N > 4) nmax = 8;
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
        ps.far_below = 0;
        for (int c = 0; c <= bp.nclasses; ++c) ps.cls_beg[c] = bp.cls_beg[c];
        for (int b = 0; b < bp.nbonds; ++b) ps.pos[b] = bp.pos[b];
        if (secs[s]->left.K > 0 && secs[s]->desc.Q == 2) continue;  // split product of its own
        for (uint64_t r0 = 0; r0 < ps.sd.dim; r0 += kHxThreads) tiles.push_back(make_uint2(s, (uint32_t)r0));
    }
    dcs_plan *p = new (std::nothrow) dcs_plan();
    if (!p) return set_error(DCS_ENOMEM, "host allocation failed");
    p->device = device;
    p->nsec = nsec;
    p->nmax = nmax;
    p->ntiles = (uint32_t)tiles.size();
    p->lds_bytes = lds;
    for (int s = 0; s < nsec; ++s) {
        p->dims.push_back(secs[s]->desc.dim);
        if (secs[s]->left.K > 0 && secs[s]->desc.Q == 2)
            p->own.push_back(dcs_plan::Own{s, secs[s], terms[s], jxy[s], jz[s]});
    }
    DeviceGuard g(device);
    int r = check_hip(hipMalloc(&p->d_secs, nsec * sizeof(PlanSector)), "hipMalloc plan");
    if (!r) r = check_hip(hipMalloc(&p->d_io, nsec * sizeof(PlanIO)), "hipMalloc plan io");
    if (!r) r = check_hip(hipMalloc(&p->d_tiles, std::max<size_t>(tiles.size(), 1) * sizeof(uint2)),
                          "hipMalloc tiles");
    if (!r) r = check_hip(hipHostMalloc(&p->h_io, nsec * sizeof(PlanIO)), "hipHostMalloc");
    if (!r) r = check_hip(hipEventCreateWithFlags(&p->io_copied, hipEventDisableTiming), "event");
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
    const int cus = device_cu_count(p->device);
    int per_cu = (int)((160 * 1024) / p->lds_bytes);
    per_cu = per_cu < 1 ? 1 : (per_cu > 4 ? 4 : per_cu);
    uint32_t wgs = (uint32_t)std::min<uint64_t>((uint64_t)cus * per_cu, p->ntiles);
    PlanArgs A;
    A.secs = p->d_secs;
    A.io = p->d_io;
    A.tiles = p->d_tiles;
    A.ntiles = p->ntiles;
    A.xcd_groups = 0;
    if (wgs >= 16) {
        wgs = (wgs + 7) / 8 * 8;
        A.xcd_groups = (int)(wgs / 8);
    }
    A.tiles_per_wg = (p->ntiles + wgs - 1) / wgs;
    auto kern = plan_kernel<uint32_t, T, NMAX>;
    if (int r = ensure_lds(kern, p->lds_bytes)) return r;
    kern<<<wgs, kHxThreads, p->lds_bytes, stream>>>(A);
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
    if (p->ntiles > 0) {
        const int r = dtype == DCS_F32
                          ? (p->nmax == 4 ? launch_plan<float, 4>(p, stream) : launch_plan<float, 8>(p, stream))
                          : (p->nmax == 4 ? launch_plan<double, 4>(p, stream) : launch_plan<double, 8>(p, stream));
        if (r) return r;
    }
    for (const auto &o : p->own)
        if (int r = launch_hx(o.sector, o.terms, o.jxy, o.jz, nullptr, dtype, 1, xs[o.index], ys[o.index], stream))
            return r;
    return DCS_OK;
}
