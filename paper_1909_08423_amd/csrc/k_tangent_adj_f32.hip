// Tangent-pass adjoint, FP32 network (also the BF16-operand form, whose
// adjoint products run in FP32).
#include "k_tangent_adj_impl.h"

namespace pn {
template size_t tangent_adj_arena_elems<float>(const Dims&, int);
template size_t tangent_adj_lds_bytes<float>(const Dims&, int, bool);
template void launch_net_tangent_adj<float>(const pn_ctx*, hipStream_t, int64_t, const double*, const float*, char*,
                                            const WsLayout&);
}  // namespace pn
