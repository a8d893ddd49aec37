// Instantiations of the H*x launchers (one pass and split) for double vectors with k=1 columns.
#include "split_impl.h"

namespace dcs {
namespace hx {
template int launch_hx_t<uint32_t, double, 1, 4>(const dcs_sector *, HxParams &, hipStream_t);
template int launch_hx_t<uint32_t, double, 1, 8>(const dcs_sector *, HxParams &, hipStream_t);
template int launch_hx_t<uint64_t, double, 1, 4>(const dcs_sector *, HxParams &, hipStream_t);
template int launch_hx_t<uint64_t, double, 1, 8>(const dcs_sector *, HxParams &, hipStream_t);
}  // namespace hx
namespace sp {
template int launch_split_t<double, 1>(dcs_sector *, const SplitRows &, const void *, void *,
                                     const double *, const double *, const double *, int, int,
                                     hipStream_t);
}  // namespace sp
}  // namespace dcs
