// The adjoint of y = H(theta) x for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc): the per-workgroup partial sums live in a fixed device array of
// this library instead of a caller workspace, and the product runs as the fused
// single pass (no split tables are built and the autotuner times nothing).
#include <mutex>

#include "dcs_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(4) << 20;  // 4 MiB per device

// The partials of the adjoint's workgroups.  Each GPU the library runs on holds
// its own copy until the process ends.  In host code `scratch` is only a
// stand-in for the symbol: its device address comes from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_scratch_lock;
void *g_scratch_ptr[dcs::kMaxDevices] = {};

// Device address of this device's scratch array, looked up once per device with
// that device current (the caller's DeviceGuard).
int scratch_address(int device, void **out) {
    std::lock_guard<std::mutex> lk(g_scratch_lock);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        if (int r = dcs::check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
                                   "hipGetSymbolAddress(scratch)"))
            return r;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return DCS_OK;
}

}  // namespace

using namespace dcs;

extern "C" int dcs_hamiltonian_apply_adjoint_noalloc(const dcs_sector *s, const dcs_terms *t,
                                                     const double *jxy, const double *jz,
                                                     const double *h, int dtype, const void *x,
                                                     const void *g, void *gx, double *gjxy,
                                                     double *gjz, double *gh, void *stream) {
    clear_error();
    if (!s || !t) return set_error(DCS_EINVAL, "sector or terms is NULL");
    if (int r = refuse_mixed(s)) return r;
    if (dtype != DCS_F32 && dtype != DCS_F64) return set_error(DCS_EINVAL, "dtype %d", dtype);
    if (t->num_bonds > 0 && (!jxy || !jz)) return set_error(DCS_EINVAL, "NULL couplings");
    if (t->max_site >= s->desc.L)
        return set_error(DCS_EINVAL, "bond site %d outside the sector's %d sites", t->max_site,
                         s->desc.L);
    if (!x || !g) return set_error(DCS_EINVAL, "NULL vector");
    if (t->num_bonds > 0 && (!gjxy || !gjz)) return set_error(DCS_EINVAL, "NULL coupling gradients");
    if (s->device < 0 || s->device >= kMaxDevices)
        return set_error(DCS_EUNSUPPORTED, "device %d beyond the %d devices of the scratch table",
                         s->device, kMaxDevices);
    const size_t need = adjoint_single_ws_bytes(s, t);
    if (need > kScratchBytes)
        return set_error(DCS_EUNSUPPORTED,
                         "the adjoint needs %zu bytes of partial sums here, more than the %zu of the "
                         "fixed scratch array; use dcs_hamiltonian_apply_adjoint with a workspace",
                         need, kScratchBytes);
    DeviceGuard dg(s->device);
    void *ws = nullptr;
    if (int r = scratch_address(s->device, &ws)) return r;
    return launch_adjoint_single(s, t, jxy, jz, h, dtype, x, g, gx, gjxy, gjz, gh, ws,
                                 (hipStream_t)stream);
}
