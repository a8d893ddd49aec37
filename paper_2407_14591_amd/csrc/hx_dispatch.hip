// Dispatch of the matrix-free H*x and adjoint launchers by index type, value type,
// column count and subsystem bound; the instantiations live in hx_f*_k*.hip and
// hx_adjoint_f*.hip so they compile in parallel.
#include <cstdlib>
#include <mutex>

#include "split_impl.h"

namespace dcs {
namespace sp {
#define DCS_SPLIT_EXTERN(T, K)                                                                   \
    extern template int launch_split_t<T, K>(dcs_sector *, const SplitRows &, const void *, void *, \
                                             const double *, const double *, const double *, int,   \
                                             int, hipStream_t);
DCS_SPLIT_EXTERN(float, 1)
DCS_SPLIT_EXTERN(float, 2)
DCS_SPLIT_EXTERN(float, 4)
DCS_SPLIT_EXTERN(float, 8)
DCS_SPLIT_EXTERN(double, 1)
DCS_SPLIT_EXTERN(double, 2)
DCS_SPLIT_EXTERN(double, 4)
DCS_SPLIT_EXTERN(double, 8)
}  // namespace sp
namespace hx {
#define DCS_HX_EXTERN(IDX, T, K, NMAX)                                                          \
    extern template int launch_hx_t<IDX, T, K, NMAX>(const dcs_sector *, HxParams &, hipStream_t);
#define DCS_HX_EXTERN_ALL(T, K)           \
    DCS_HX_EXTERN(uint32_t, T, K, 4)      \
    DCS_HX_EXTERN(uint32_t, T, K, 8)      \
    DCS_HX_EXTERN(uint64_t, T, K, 4)      \
    DCS_HX_EXTERN(uint64_t, T, K, 8)
DCS_HX_EXTERN_ALL(float, 1)
DCS_HX_EXTERN_ALL(float, 2)
DCS_HX_EXTERN_ALL(float, 4)
DCS_HX_EXTERN_ALL(float, 8)
DCS_HX_EXTERN_ALL(double, 1)
DCS_HX_EXTERN_ALL(double, 2)
DCS_HX_EXTERN_ALL(double, 4)
DCS_HX_EXTERN_ALL(double, 8)
#define DCS_ADJ_EXTERN(IDX, T, NMAX)                                                         \
    extern template int launch_adj_t<IDX, T, NMAX>(const dcs_sector *, HxParams &, double *, \
                                                   double *, double *, hipStream_t);
DCS_ADJ_EXTERN(uint32_t, float, 4)
DCS_ADJ_EXTERN(uint32_t, float, 8)
DCS_ADJ_EXTERN(uint64_t, float, 4)
DCS_ADJ_EXTERN(uint64_t, float, 8)
DCS_ADJ_EXTERN(uint32_t, double, 4)
DCS_ADJ_EXTERN(uint32_t, double, 8)
DCS_ADJ_EXTERN(uint64_t, double, 4)
DCS_ADJ_EXTERN(uint64_t, double, 8)
#define DCS_ADJK_EXTERN(T, KC)                                                                        \
    extern template int launch_adj_t<uint32_t, T, 4, KC>(const dcs_sector *, HxParams &, double *,   \
                                                         double *, double *, hipStream_t);           \
    extern template int launch_adj_t<uint32_t, T, 8, KC>(const dcs_sector *, HxParams &, double *,   \
                                                         double *, double *, hipStream_t);           \
    extern template int launch_adj_t<uint64_t, T, 4, KC>(const dcs_sector *, HxParams &, double *,   \
                                                         double *, double *, hipStream_t);           \
    extern template int launch_adj_t<uint64_t, T, 8, KC>(const dcs_sector *, HxParams &, double *,   \
                                                         double *, double *, hipStream_t);
DCS_ADJK_EXTERN(float, 2)
DCS_ADJK_EXTERN(float, 4)
DCS_ADJK_EXTERN(float, 8)
DCS_ADJK_EXTERN(double, 2)
DCS_ADJK_EXTERN(double, 4)
DCS_ADJK_EXTERN(double, 8)

namespace {

// The split form (LeftInfo) for Q = 2 sectors that have a split view.
// DCS_SPLIT=0 in the environment (read at every product) selects the single pass.
inline bool split_enabled() {
    const char *e = getenv("DCS_SPLIT");
    return !(e && e[0] == '0');
}

template <typename IdxT, typename T, int K, int NMAX>
int launch_one(const dcs_sector *s, HxParams &P, hipStream_t stream) {
    // the bonds touching the first half of the subsystems jump far
    P.far_below = s->desc.dim >= (1ull << 22) ? s->desc.N / 2 : 0;
    return launch_hx_t<IdxT, T, K, NMAX>(s, P, stream);
}

template <typename IdxT, typename T, int NMAX>
int launch_hx_k(const dcs_sector *s, HxParams &P, int k, hipStream_t stream) {
    switch (k) {
        case 1: return launch_one<IdxT, T, 1, NMAX>(s, P, stream);
        case 2: return launch_one<IdxT, T, 2, NMAX>(s, P, stream);
        case 4: return launch_one<IdxT, T, 4, NMAX>(s, P, stream);
        default: return launch_one<IdxT, T, 8, NMAX>(s, P, stream);
    }
}

template <typename IdxT, int NMAX>
int launch_hx_d(const dcs_sector *s, HxParams &P, int dtype, int k, hipStream_t stream) {
    if (dtype == DCS_F32) return launch_hx_k<IdxT, float, NMAX>(s, P, k, stream);
    return launch_hx_k<IdxT, double, NMAX>(s, P, k, stream);
}

template <typename T>
int launch_split_k(dcs_sector *s, const SplitRows &c, const void *x, void *y, const double *jxy,
                   const double *jz, const double *h, int nbonds, int k, int variant,
                   hipStream_t stream) {
    switch (k) {
        case 1: return sp::launch_split_t<T, 1>(s, c, x, y, jxy, jz, h, nbonds, variant, stream);
        case 2: return sp::launch_split_t<T, 2>(s, c, x, y, jxy, jz, h, nbonds, variant, stream);
        case 4: return sp::launch_split_t<T, 4>(s, c, x, y, jxy, jz, h, nbonds, variant, stream);
        default: return sp::launch_split_t<T, 8>(s, c, x, y, jxy, jz, h, nbonds, variant, stream);
    }
}

int pick_nmax(const dcs_sector *s) { return s->desc.N <= 4 ? 4 : 8; }

}  // namespace
}  // namespace hx

using namespace hx;

namespace {

int launch_single(const dcs_sector *s, const dcs_terms *t, const double *jxy, const double *jz,
                  const double *h, int dtype, int k, const void *x, void *y, hipStream_t stream) {
    const int nmax = pick_nmax(s);
    HxParams P;
    if (int r = fill_params(s, t, nmax, jxy, jz, h, P)) return r;
    P.x = x;
    P.y = y;
    if (s->wide)
        return nmax == 4 ? launch_hx_d<uint64_t, 4>(s, P, dtype, k, stream)
                         : launch_hx_d<uint64_t, 8>(s, P, dtype, k, stream);
    return nmax == 4 ? launch_hx_d<uint32_t, 4>(s, P, dtype, k, stream)
                     : launch_hx_d<uint32_t, 8>(s, P, dtype, k, stream);
}

// Launch forms of a product on a sector with a split view: the split product
// with runs staged in LDS where they fit, without, with the left family applied
// by the row pass (no column pass), and the single pass.
enum Form {
    kFormSplitStaged = 0,
    kFormSplitGlobal = 1,
    kFormSplitFused = 2,
    kFormSingle = 3,
    kFormSplitTiled = 4,
    kNumForms = 5
};

// The block-tiled row pass exists for rows of 16 to 64 bytes with a tiling.
bool tiled_applies(const SplitRows &c, int dtype, int k) {
    const int rb = k * (dtype == DCS_F32 ? 4 : 8);
    if (rb < 16 || rb > 64 || c.wide_off) return false;  // the tiled pass reads 16-bit offsets
    return c.tiling[rb == 16 ? 0 : (rb == 32 ? 1 : 2)].ntiles > 0;
}

int launch_form(dcs_sector *s, const dcs_terms *t, const SplitRows &c, int form, const double *jxy,
                const double *jz, const double *h, int dtype, int k, const void *x, void *y,
                hipStream_t stream) {
    if (form == kFormSingle) return launch_single(s, t, jxy, jz, h, dtype, k, x, y, stream);
    const int variant = form == kFormSplitStaged  ? sp::kSplitStagedOk
                        : form == kFormSplitGlobal ? sp::kSplitGlobal
                        : form == kFormSplitTiled  ? sp::kSplitTiled
                                                   : sp::kSplitFused;
    return dtype == DCS_F32 ? launch_split_k<float>(s, c, x, y, jxy, jz, h, t->num_bonds, k, variant, stream)
                            : launch_split_k<double>(s, c, x, y, jxy, jz, h, t->num_bonds, k, variant, stream);
}

// DCS_AUTOTUNE=0 in the environment (read at every call) keeps the default form.
bool autotune_enabled() {
    const char *e = getenv("DCS_AUTOTUNE");
    return !(e && e[0] == '0');
}

// The default form: the staged split, or (DCS_SPLIT_FUSED=1, read at every call)
// the split form whose rows pass also applies the left family.
int default_form() {
    const char *e = getenv("DCS_SPLIT_FUSED");
    if (e && e[0] == '1') return kFormSplitFused;
    const char *t = getenv("DCS_SPLIT_TILED");
    return (t && t[0] == '1') ? kFormSplitTiled : kFormSplitStaged;
}

// Autotuner: the first product of a (terms, dtype, k) on a split sector times
// every launch form twice (HIP events on the caller's stream, second run
// counted) and keeps the fastest for that key in the sector.  Every form
// writes the same Y (up to rounding order), so the call's result is valid
// whichever form ran last; the fastest runs last.
inline uint64_t tuned_key(const dcs_terms *t, int dtype, int k) {
    return (t->id << 8) | ((uint64_t)dtype << 4) | (uint64_t)k;
}

int tuned_form(dcs_sector *s, const dcs_terms *t, const SplitRows &c, const double *jxy,
               const double *jz, const double *h, int dtype, int k, const void *x, void *y,
               hipStream_t stream, bool *ran) {
    *ran = false;
    const uint64_t key = tuned_key(t, dtype, k);
    LeftInfo &li = s->left;
    {
        std::lock_guard<std::mutex> g(*li.rows_lock);
        auto it = li.tuned.find(key);
        if (it != li.tuned.end()) return it->second;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (!autotune_enabled() || hipStreamIsCapturing(stream, &cs) != hipSuccess ||
        cs != hipStreamCaptureStatusNone)
        return default_form();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (check_hip(hipEventCreate(&e0), "autotune event") || check_hip(hipEventCreate(&e1), "autotune event")) {
        if (e0) hipEventDestroy(e0);
        return -1;
    }
    float best_ms = 0.f;
    int best = kFormSplitStaged;
    int r = DCS_OK;
    int last = -1;
    for (int f = 0; f < kNumForms && !r; ++f) {
        if (f == kFormSplitTiled && !tiled_applies(c, dtype, k)) continue;
        if (f == kFormSingle && s->gtab && k > 1) continue;  // no one-pass block kernel without LDS tables
        last = f;
        float ms = 0.f;
        for (int rep = 0; rep < 2 && !r; ++rep) {
            r = check_hip(hipEventRecord(e0, stream), "autotune record");
            if (!r) r = launch_form(s, t, c, f, jxy, jz, h, dtype, k, x, y, stream);
            if (!r) r = check_hip(hipEventRecord(e1, stream), "autotune record");
            if (!r) r = check_hip(hipEventSynchronize(e1), "autotune synchronise");
            if (!r) r = check_hip(hipEventElapsedTime(&ms, e0, e1), "autotune time");
        }
        if (!r && (f == 0 || ms < best_ms)) {
            best_ms = ms;
            best = f;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (r) return -1;
    {
        std::lock_guard<std::mutex> g(*li.rows_lock);
        li.tuned[key] = best;
    }
    *ran = best == last;  // the fastest form was the last one timed: Y is its output
    return best;
}

}  // namespace

int hx_form(const dcs_sector *s, const dcs_terms *t, int dtype, int k) {
    static_assert(kFormSplitStaged == DCS_FORM_SPLIT_STAGED && kFormSplitGlobal == DCS_FORM_SPLIT_GLOBAL &&
                      kFormSplitFused == DCS_FORM_SPLIT_FUSED && kFormSingle == DCS_FORM_SINGLE &&
                      kFormSplitTiled == DCS_FORM_SPLIT_TILED,
                  "form codes of the ABI");
    if (!(s->left.K > 0 && s->desc.Q == 2 && split_enabled())) return kFormSingle;
    for (int m = 0; m < s->left.m_count; ++m)
        if (s->left.ncols[m] >= (1u << 25)) return kFormSingle;  // no split tables for such runs
    if (!autotune_enabled()) return default_form();
    std::lock_guard<std::mutex> g(*s->left.rows_lock);
    auto it = s->left.tuned.find(tuned_key(t, dtype, k));
    return it == s->left.tuned.end() ? DCS_FORM_UNTUNED : it->second;
}

int launch_hx(const dcs_sector *s, const dcs_terms *t, const double *jxy, const double *jz,
              const double *h, int dtype, int k, const void *x, void *y, hipStream_t stream) {
    DeviceGuard dg(s->device);
    if (s->left.K > 0 && s->desc.Q == 2 && split_enabled()) {
        if (t->max_site >= s->desc.L)
            return set_error(DCS_EINVAL, "bond site %d outside the sector's %d sites", t->max_site,
                             s->desc.L);
        clear_error();
        dcs_sector *sm = const_cast<dcs_sector *>(s);
        SplitRows *c = split_rows(sm, t);
        if (c) {
            bool ran = false;
            const int form = tuned_form(sm, t, *c, jxy, jz, h, dtype, k, x, y, stream, &ran);
            if (form < 0) return DCS_EHIP;
            const int r = ran ? DCS_OK : launch_form(sm, t, *c, form, jxy, jz, h, dtype, k, x, y, stream);
            if (!r) note_split_use(sm, *c, stream);
            return r;
        }
        if (dcs_last_error()[0]) return DCS_EHIP;
    }
    return launch_single(s, t, jxy, jz, h, dtype, k, x, y, stream);
}

// An upper bound: the adjoint's tiles of several rows per thread need at most as many
// workgroups as tiles of one row per thread.
size_t adjoint_single_ws_bytes(const dcs_sector *s, const dcs_terms *t) {
    const Grid g = plan_grid(s, adj_lds_bytes(s, t->num_bonds, coeff_lds_bytes<double>()));
    return (size_t)g.wgs * (2 * t->num_bonds + s->desc.L) * sizeof(double);
}

size_t adjoint_ws_bytes(const dcs_sector *s, const dcs_terms *t, int k) {
    return std::max(adjoint_single_ws_bytes(s, t), split_adjoint_ws_bytes(s, t->num_bonds, k));
}

namespace {

// The adjoint pass (the fused kernel when gx is given, else the sums only).
int adjoint_pass(const dcs_sector *s, const dcs_terms *t, const double *jxy, const double *jz,
                 const double *h, int dtype, const void *x, const void *g, void *gx, double *gjxy,
                 double *gjz, double *gh, void *ws, hipStream_t stream) {
    const int nmax = pick_nmax(s);
    HxParams P;
    if (int r = fill_params(s, t, nmax, jxy, jz, h, P)) return r;
    P.x = x;
    P.g = g;
    P.gx = gx;
    P.far_below = s->desc.dim >= (1ull << 22) ? s->desc.N / 2 : 0;
    P.partials = (double *)ws;
    if (s->wide) {
        if (dtype == DCS_F32)
            return nmax == 4 ? launch_adj_t<uint64_t, float, 4>(s, P, gjxy, gjz, gh, stream)
                             : launch_adj_t<uint64_t, float, 8>(s, P, gjxy, gjz, gh, stream);
        return nmax == 4 ? launch_adj_t<uint64_t, double, 4>(s, P, gjxy, gjz, gh, stream)
                         : launch_adj_t<uint64_t, double, 8>(s, P, gjxy, gjz, gh, stream);
    }
    if (dtype == DCS_F32)
        return nmax == 4 ? launch_adj_t<uint32_t, float, 4>(s, P, gjxy, gjz, gh, stream)
                         : launch_adj_t<uint32_t, float, 8>(s, P, gjxy, gjz, gh, stream);
    return nmax == 4 ? launch_adj_t<uint32_t, double, 4>(s, P, gjxy, gjz, gh, stream)
                     : launch_adj_t<uint32_t, double, 8>(s, P, gjxy, gjz, gh, stream);
}

template <int KC>
int adjoint_block_pass_k(const dcs_sector *s, HxParams &P, int dtype, int nmax, double *gjxy, double *gjz,
                         double *gh, hipStream_t stream) {
    if (s->wide) {
        if (dtype == DCS_F32)
            return nmax == 4 ? launch_adj_t<uint64_t, float, 4, KC>(s, P, gjxy, gjz, gh, stream)
                             : launch_adj_t<uint64_t, float, 8, KC>(s, P, gjxy, gjz, gh, stream);
        return nmax == 4 ? launch_adj_t<uint64_t, double, 4, KC>(s, P, gjxy, gjz, gh, stream)
                         : launch_adj_t<uint64_t, double, 8, KC>(s, P, gjxy, gjz, gh, stream);
    }
    if (dtype == DCS_F32)
        return nmax == 4 ? launch_adj_t<uint32_t, float, 4, KC>(s, P, gjxy, gjz, gh, stream)
                         : launch_adj_t<uint32_t, float, 8, KC>(s, P, gjxy, gjz, gh, stream);
    return nmax == 4 ? launch_adj_t<uint32_t, double, 4, KC>(s, P, gjxy, gjz, gh, stream)
                     : launch_adj_t<uint32_t, double, 8, KC>(s, P, gjxy, gjz, gh, stream);
}

// The sums of a block of k columns in one pass (decode and rank per row, the k
// columns of x and g dotted at every hop); grad_x is not formed here.
int adjoint_block_pass(const dcs_sector *s, const dcs_terms *t, const double *jxy, const double *jz,
                       const double *h, int dtype, int k, const void *x, const void *g, double *gjxy,
                       double *gjz, double *gh, void *ws, hipStream_t stream) {
    const int nmax = pick_nmax(s);
    HxParams P;
    if (int r = fill_params(s, t, nmax, jxy, jz, h, P)) return r;
    P.x = x;
    P.g = g;
    P.gx = nullptr;
    P.far_below = s->desc.dim >= (1ull << 22) ? s->desc.N / 2 : 0;
    P.partials = (double *)ws;
    switch (k) {
        case 2: return adjoint_block_pass_k<2>(s, P, dtype, nmax, gjxy, gjz, gh, stream);
        case 4: return adjoint_block_pass_k<4>(s, P, dtype, nmax, gjxy, gjz, gh, stream);
        default: return adjoint_block_pass_k<8>(s, P, dtype, nmax, gjxy, gjz, gh, stream);
    }
}

// Milliseconds of one run of fn on the stream (HIP events, synchronising); -1 on error.
template <typename F>
float time_on_stream(F &&fn, hipStream_t stream) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return -1.f;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return -1.f;
    }
    float ms = -1.f;
    if (hipEventRecord(e0, stream) == hipSuccess && fn() == DCS_OK &&
        hipEventRecord(e1, stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        ms = -1.f;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return ms;
}

}  // namespace

int launch_adjoint_single(const dcs_sector *s, const dcs_terms *t, const double *jxy,
                          const double *jz, const double *h, int dtype, const void *x,
                          const void *g, void *gx, double *gjxy, double *gjz, double *gh,
                          void *ws, hipStream_t stream) {
    DeviceGuard dg(s->device);
    return adjoint_pass(s, t, jxy, jz, h, dtype, x, g, gx, gjxy, gjz, gh, ws, stream);
}

int launch_adjoint(const dcs_sector *s, const dcs_terms *t, const double *jxy, const double *jz,
                   const double *h, int dtype, int k, const void *x, const void *g, void *gx,
                   double *gjxy, double *gjz, double *gh, void *ws, size_t ws_bytes,
                   hipStream_t stream) {
    DeviceGuard dg(s->device);
    if (k > 1) {
        // a block: (1) grad_x = H G by the block product and the sums in one pass over
        // the rows, or, for FP32 on the split tables, (2) the sums formed inside the
        // split product of G; the first call for a (terms, dtype, k) times both
        auto way1 = [&]() -> int {
            if (gx)
                if (int r = launch_hx(s, t, jxy, jz, h, dtype, k, g, gx, stream)) return r;
            return adjoint_block_pass(s, t, jxy, jz, h, dtype, k, x, g, gjxy, gjz, gh, ws, stream);
        };
        if (!(gx && s->left.K > 0 && s->desc.Q == 2 && split_enabled() && dtype == DCS_F32)) return way1();
        if (t->max_site >= s->desc.L)
            return set_error(DCS_EINVAL, "bond site %d outside the sector's %d sites", t->max_site, s->desc.L);
        clear_error();
        dcs_sector *sm = const_cast<dcs_sector *>(s);
        SplitRows *c = split_rows(sm, t);
        if (!c) return dcs_last_error()[0] ? DCS_EHIP : way1();
        if (!(split_adjoint_applies(s, *c, dtype, k) && ws_bytes >= split_adjoint_ws_bytes(s, t->num_bonds, k)))
            return way1();
        auto way2 = [&]() -> int {
            return launch_split_adjoint(sm, *c, jxy, jz, h, t->num_bonds, k, x, g, gx, gjxy, gjz, gh, ws, ws_bytes,
                                        stream);
        };
        const uint64_t key = tuned_key(t, dtype, k) | (1ull << 62);  // the block adjoint's entry
        int way = -1;
        if (const char *e = getenv("DCS_ADJOINT_WAY")) {
            way = e[0] - '0';
            if (way != 1 && way != 2) way = -1;
        }
        if (way < 0) {
            std::lock_guard<std::mutex> lk(*sm->left.rows_lock);
            auto it = sm->left.tuned.find(key);
            if (it != sm->left.tuned.end()) way = it->second;
        }
        if (way < 0) {
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            if (!autotune_enabled() || hipStreamIsCapturing(stream, &cs) != hipSuccess ||
                cs != hipStreamCaptureStatusNone) {
                way = 2;
            } else {
                float best = 0.f;
                for (int w = 1; w <= 2; ++w) {
                    float ms = 0.f;
                    for (int rep = 0; rep < 2; ++rep) {
                        ms = time_on_stream([&]() { return w == 1 ? way1() : way2(); }, stream);
                        if (ms < 0.f)
                            return dcs_last_error()[0] ? DCS_EHIP : set_error(DCS_EHIP, "adjoint autotune timing");
                    }
                    if (w == 1 || ms < best) {
                        best = ms;
                        way = w;
                    }
                }
                std::lock_guard<std::mutex> lk(*sm->left.rows_lock);
                sm->left.tuned[key] = way;
            }
        }
        const int r = way == 1 ? way1() : way2();
        if (!r) note_split_use(sm, *c, stream);
        return r;
    }
    auto fused = [&]() {
        return adjoint_pass(s, t, jxy, jz, h, dtype, x, g, gx, gjxy, gjz, gh, ws, stream);
    };
    // grad_x = H g is a product (H is real symmetric).  Where the sector's
    // products run on the split tables, that product can compute it, and the
    // adjoint pass then forms only the coupling and field sums (it gathers x, not
    // g).  Which of the two ways is faster depends on the sector: the autotuner
    // times both on the first call for a (terms, dtype) and keeps the faster.
    if (!(gx && s->left.K > 0 && s->desc.Q == 2 && split_enabled())) return fused();
    if (t->max_site >= s->desc.L)
        return set_error(DCS_EINVAL, "bond site %d outside the sector's %d sites", t->max_site,
                         s->desc.L);
    clear_error();
    dcs_sector *sm = const_cast<dcs_sector *>(s);
    SplitRows *c = split_rows(sm, t);
    if (!c) return dcs_last_error()[0] ? DCS_EHIP : fused();
    bool ran = false;
    const int form = tuned_form(sm, t, *c, jxy, jz, h, dtype, 1, g, gx, stream, &ran);
    if (form < 0) return DCS_EHIP;
    if (form == kFormSingle) return fused();
    auto split_way = [&]() {
        if (int r = launch_form(sm, t, *c, form, jxy, jz, h, dtype, 1, g, gx, stream)) return r;
        return adjoint_pass(s, t, jxy, jz, h, dtype, x, g, nullptr, gjxy, gjz, gh, ws, stream);
    };
    // the adjoint on the split view with its sums formed inside the product (FP32)
    const bool adj_ok = split_adjoint_applies(s, *c, dtype, 1) && ws_bytes >= split_adjoint_ws_bytes(s, t->num_bonds, 1);
    auto split_adj = [&]() {
        return launch_split_adjoint(sm, *c, jxy, jz, h, t->num_bonds, 1, x, g, gx, gjxy, gjz, gh, ws, ws_bytes, stream);
    };
    auto run_way = [&](int w) { return w == 0 ? fused() : (w == 1 ? split_way() : split_adj()); };
    const uint64_t key = tuned_key(t, dtype, 0);  // k = 0: the adjoint's entry
    LeftInfo &li = sm->left;
    int way = -1;
    if (const char *e = getenv("DCS_ADJOINT_WAY")) {  // 0 fused pass, 1 product + sums pass, 2 sums in the product
        way = e[0] - '0';
        if (way < 0 || way > 2 || (way == 2 && !adj_ok)) way = -1;
    }
    if (way < 0) {
        std::lock_guard<std::mutex> lk(*li.rows_lock);
        auto it = li.tuned.find(key);
        if (it != li.tuned.end()) way = it->second;
    }
    if (way < 0) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (!autotune_enabled() || hipStreamIsCapturing(stream, &cs) != hipSuccess ||
            cs != hipStreamCaptureStatusNone) {
            const int r = run_way(adj_ok ? 2 : 1);
            if (!r) note_split_use(sm, *c, stream);
            return r;
        }
        float best = 0.f;
        for (int w = 0; w < (adj_ok ? 3 : 2); ++w) {
            float ms = 0.f;
            for (int rep = 0; rep < 2; ++rep) {
                ms = time_on_stream([&]() { return run_way(w); }, stream);
                if (ms < 0.f) return dcs_last_error()[0] ? DCS_EHIP : set_error(DCS_EHIP, "adjoint autotune timing");
            }
            if (w == 0 || ms < best) {
                best = ms;
                way = w;
            }
        }
        std::lock_guard<std::mutex> lk(*li.rows_lock);
        li.tuned[key] = way;
    }
    const int r = run_way(way);
    if (!r) note_split_use(sm, *c, stream);
    return r;
}

}  // namespace dcs
