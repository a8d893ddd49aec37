// Instantiations of the H*x launchers (one pass and split) for float vectors with k=2 columns.
#include "hx_impl.h"

namespace dcs {
namespace hx {
template int launch_hx_t<uint32_t, float, 2, 4>(const dcs_sector *, HxParams &, hipStream_t);
template int launch_hx_t<uint32_t, float, 2, 8>(const dcs_sector *, HxParams &, hipStream_t);
template int launch_hx_t<uint64_t, float, 2, 4>(const dcs_sector *, HxParams &, hipStream_t);
template int launch_hx_t<uint64_t, float, 2, 8>(const dcs_sector *, HxParams &, hipStream_t);
template int launch_split_t<uint32_t, float, 2, 4>(dcs_sector *, const HxParams &, const SplitCsr &,
                                                   hipStream_t);
template int launch_split_t<uint32_t, float, 2, 8>(dcs_sector *, const HxParams &, const SplitCsr &,
                                                   hipStream_t);
template int launch_split_t<uint64_t, float, 2, 4>(dcs_sector *, const HxParams &, const SplitCsr &,
                                                   hipStream_t);
template int launch_split_t<uint64_t, float, 2, 8>(dcs_sector *, const HxParams &, const SplitCsr &,
                                                   hipStream_t);
}  // namespace hx
}  // namespace dcs
