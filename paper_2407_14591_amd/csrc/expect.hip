// Expectation values of the terms of H in given states (the observables of
// App. D).  For a real state psi and a real symmetric term M,
// psi^T M psi is the adjoint's coupling sum for that term with g = x = psi, so
// this runs the adjoint's sums-only pass once per state.
#include "dcs_internal.h"

namespace {

__global__ void fill_ones(double *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 1.0;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

using namespace dcs;

extern "C" int dcs_expectation_workspace_size(const dcs_sector *s, const dcs_terms *t,
                                              size_t *bytes) {
    clear_error();
    if (!s || !t || !bytes) return set_error(DCS_EINVAL, "NULL argument");
    if (int r = refuse_mixed(s)) return r;
    *bytes = align256(adjoint_ws_bytes(s, t)) + align256((size_t)std::max(t->num_bonds, 1) * sizeof(double));
    return DCS_OK;
}

extern "C" int dcs_expectation_values(const dcs_sector *s, const dcs_terms *t, int dtype, int num,
                                      const void *psi, double *exy, double *ez, double *esz,
                                      void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    if (!s || !t) return set_error(DCS_EINVAL, "sector or terms is NULL");
    if (int r = refuse_mixed(s)) return r;
    if (dtype != DCS_F32 && dtype != DCS_F64) return set_error(DCS_EINVAL, "dtype %d", dtype);
    if (num < 0) return set_error(DCS_EINVAL, "num %d", num);
    if (num == 0) return DCS_OK;
    if (!psi) return set_error(DCS_EINVAL, "NULL states");
    if (t->max_site >= s->desc.L)
        return set_error(DCS_EINVAL, "bond site %d outside the sector's %d sites", t->max_site,
                         s->desc.L);
    if (t->num_bonds > 0 && (!exy || !ez)) return set_error(DCS_EINVAL, "NULL bond outputs");
    const size_t adj = align256(adjoint_ws_bytes(s, t));
    const size_t need = adj + align256((size_t)std::max(t->num_bonds, 1) * sizeof(double));
    if (!ws || ws_bytes < need)
        return set_error(DCS_EINVAL, "workspace of %zu bytes < %zu needed", ws_bytes, need);
    DeviceGuard dg(s->device);
    hipStream_t q = (hipStream_t)stream;
    // the sums do not depend on the couplings; the pass reads unit ones
    double *ones = (double *)((char *)ws + adj);
    const int nb = std::max(t->num_bonds, 1);
    fill_ones<<<(nb + 255) / 256, 256, 0, q>>>(ones, nb);
    if (int r = check_hip(hipGetLastError(), "fill couplings")) return r;
    const size_t es = dtype == DCS_F32 ? 4 : 8;
    for (int e = 0; e < num; ++e) {
        const void *v = (const char *)psi + (size_t)e * s->desc.dim * es;
        if (int r = launch_adjoint(s, t, ones, ones, nullptr, dtype, 1, v, v, nullptr,
                                   exy ? exy + (size_t)e * t->num_bonds : nullptr,
                                   ez ? ez + (size_t)e * t->num_bonds : nullptr,
                                   esz ? esz + (size_t)e * s->desc.L : nullptr, ws, adj, q))
            return r;
    }
    return DCS_OK;
}
