// C ABI entry points that only validate and forward to the kernel launchers,
// plus the per-thread error state.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "dcs_internal.h"

namespace dcs {

static thread_local char g_err[512] = "";

int set_error(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = 0; }

int check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return DCS_OK;
    return set_error(DCS_EHIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

int device_cu_count(int device) {
    static int cache[64] = {0};
    if (device < 0 || device >= 64) return 256;
    if (!cache[device]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
            v <= 0)
            v = 256;
        cache[device] = v;
    }
    return cache[device];
}

}  // namespace dcs

using namespace dcs;

extern "C" const char *dcs_last_error(void) { return g_err; }

extern "C" int dcs_version(void) { return 100; }

extern "C" int dcs_rank(const dcs_sector *s, const uint64_t *st, uint64_t *idx, size_t count,
                        uint64_t *nbad, void *stream) {
    clear_error();
    if (!s) return set_error(DCS_EINVAL, "sector is NULL");
    if (count == 0) return DCS_OK;
    if (!st || !idx) return set_error(DCS_EINVAL, "NULL array");
    return launch_rank(s, st, idx, count, nbad, (hipStream_t)stream);
}

extern "C" int dcs_rank_search(const dcs_sector *s, const uint64_t *st, uint64_t *idx, size_t count,
                               uint64_t *nbad, void *stream) {
    clear_error();
    if (!s) return set_error(DCS_EINVAL, "sector is NULL");
    if (count == 0) return DCS_OK;
    if (!st || !idx) return set_error(DCS_EINVAL, "NULL array");
    return launch_rank_search(s, st, idx, count, nbad, (hipStream_t)stream);
}

extern "C" int dcs_unrank(const dcs_sector *s, const uint64_t *idx, uint64_t *st, size_t count,
                          uint64_t *nbad, void *stream) {
    clear_error();
    if (!s) return set_error(DCS_EINVAL, "sector is NULL");
    if (count == 0) return DCS_OK;
    if (!st || !idx) return set_error(DCS_EINVAL, "NULL array");
    return launch_unrank(s, idx, st, count, nbad, (hipStream_t)stream);
}

extern "C" int dcs_enumerate(const dcs_sector *s, uint64_t first, size_t count, uint64_t *st,
                             void *stream) {
    clear_error();
    if (!s) return set_error(DCS_EINVAL, "sector is NULL");
    if (first > s->desc.dim || count > s->desc.dim - first)
        return set_error(DCS_ERANGE, "range [%llu, +%zu) passes the sector dimension %llu",
                         (unsigned long long)first, count, (unsigned long long)s->desc.dim);
    if (count == 0) return DCS_OK;
    if (!st) return set_error(DCS_EINVAL, "NULL array");
    return launch_enumerate(s, first, count, st, (hipStream_t)stream);
}

static int check_apply_args(const dcs_sector *s, const dcs_terms *t, const double *jxy,
                            const double *jz, int dtype) {
    if (!s || !t) return set_error(DCS_EINVAL, "sector or terms is NULL");
    if (int r = refuse_mixed(s)) return r;
    if (dtype != DCS_F32 && dtype != DCS_F64) return set_error(DCS_EINVAL, "dtype %d", dtype);
    if (t->num_bonds > 0 && (!jxy || !jz)) return set_error(DCS_EINVAL, "NULL couplings");
    if (t->max_site >= s->desc.L)
        return set_error(DCS_EINVAL, "bond site %d outside the sector's %d sites", t->max_site,
                         s->desc.L);
    return DCS_OK;
}

extern "C" int dcs_hamiltonian_apply(const dcs_sector *s, const dcs_terms *t, const double *jxy,
                                     const double *jz, const double *h, int dtype, int k,
                                     const void *x, void *y, void *stream) {
    clear_error();
    if (int r = check_apply_args(s, t, jxy, jz, dtype)) return r;
    if (k != 1 && k != 2 && k != 4 && k != 8) return set_error(DCS_EINVAL, "k=%d not in {1,2,4,8}", k);
    if (!x || !y) return set_error(DCS_EINVAL, "NULL vector");
    size_t es = dtype == DCS_F32 ? 4 : 8;
    size_t bytes = (size_t)s->desc.dim * k * es;
    const char *xb = (const char *)x, *yb = (const char *)y;
    if (xb < yb + bytes && yb < xb + bytes) return set_error(DCS_EINVAL, "x and y overlap");
    return launch_hx(s, t, jxy, jz, h, dtype, k, x, y, (hipStream_t)stream);
}

extern "C" int dcs_hamiltonian_form(const dcs_sector *s, const dcs_terms *t, int dtype, int k,
                                    int *form) {
    clear_error();
    if (!s || !t || !form) return set_error(DCS_EINVAL, "NULL argument");
    if (int r = refuse_mixed(s)) return r;
    if (dtype != DCS_F32 && dtype != DCS_F64) return set_error(DCS_EINVAL, "dtype %d", dtype);
    if (k != 1 && k != 2 && k != 4 && k != 8) return set_error(DCS_EINVAL, "k=%d not in {1,2,4,8}", k);
    *form = hx_form(s, t, dtype, k);
    return DCS_OK;
}

extern "C" int dcs_adjoint_workspace_size(const dcs_sector *s, const dcs_terms *t, int k,
                                          size_t *bytes) {
    clear_error();
    if (!s || !t || !bytes) return set_error(DCS_EINVAL, "NULL argument");
    if (int r = refuse_mixed(s)) return r;
    if (k != 1 && k != 2 && k != 4 && k != 8) return set_error(DCS_EINVAL, "k=%d not in {1,2,4,8}", k);
    *bytes = adjoint_ws_bytes(s, t, k);
    return DCS_OK;
}

extern "C" int dcs_hamiltonian_apply_adjoint(const dcs_sector *s, const dcs_terms *t,
                                             const double *jxy, const double *jz,
                                             const double *h, int dtype, int k, const void *x,
                                             const void *g, void *gx, double *gjxy, double *gjz,
                                             double *gh, void *ws, size_t ws_bytes,
                                             void *stream) {
    clear_error();
    if (int r = check_apply_args(s, t, jxy, jz, dtype)) return r;
    if (k != 1 && k != 2 && k != 4 && k != 8) return set_error(DCS_EINVAL, "k=%d not in {1,2,4,8}", k);
    if (!x || !g) return set_error(DCS_EINVAL, "NULL vector");
    if (gx) {
        const size_t bytes = (size_t)s->desc.dim * k * (dtype == DCS_F32 ? 4 : 8);
        const char *a = (const char *)gx;
        for (const char *b : {(const char *)x, (const char *)g})
            if (a < b + bytes && b < a + bytes) return set_error(DCS_EINVAL, "grad_x overlaps x or g");
    }
    if (t->num_bonds > 0 && (!gjxy || !gjz)) return set_error(DCS_EINVAL, "NULL coupling gradients");
    size_t need = adjoint_ws_bytes(s, t);
    if (!ws || ws_bytes < need)
        return set_error(DCS_EINVAL, "workspace of %zu bytes < %zu needed", ws_bytes, need);
    return launch_adjoint(s, t, jxy, jz, h, dtype, k, x, g, gx, gjxy, gjz, gh, ws, ws_bytes,
                          (hipStream_t)stream);
}
