// Tangent-pass adjoint, FP64 network.
#include "k_tangent_adj_impl.h"

namespace pn {
template size_t tangent_adj_arena_elems<double>(const Dims&, int);
template size_t tangent_adj_lds_bytes<double>(const Dims&, int, bool);
template void launch_net_tangent_adj<double>(const pn_ctx*, hipStream_t, int64_t, const double*, const double*, char*,
                                             const WsLayout&);
}  // namespace pn
