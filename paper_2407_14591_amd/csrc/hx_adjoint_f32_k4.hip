// Instantiations of the adjoint sums launcher for blocks of 4 float columns.
#include "hx_impl.h"

namespace dcs {
namespace hx {
template int launch_adj_t<uint32_t, float, 4, 4>(const dcs_sector *, HxParams &, double *, double *,
                                                  double *, hipStream_t);
template int launch_adj_t<uint32_t, float, 8, 4>(const dcs_sector *, HxParams &, double *, double *,
                                                  double *, hipStream_t);
template int launch_adj_t<uint64_t, float, 4, 4>(const dcs_sector *, HxParams &, double *, double *,
                                                  double *, hipStream_t);
template int launch_adj_t<uint64_t, float, 8, 4>(const dcs_sector *, HxParams &, double *, double *,
                                                  double *, hipStream_t);
}  // namespace hx
}  // namespace dcs
