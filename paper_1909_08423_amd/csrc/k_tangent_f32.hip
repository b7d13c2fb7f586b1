// Network tangent pass, FP32 network (also the BF16-operand form).
#include "k_tangent_impl.h"

namespace pn {
template void launch_net_tangent<float>(const pn_ctx*, hipStream_t, int64_t, const double*, const float*, char*,
                                        const WsLayout&, bool, float*);
}  // namespace pn
