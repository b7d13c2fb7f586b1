// Parameter conversion to the network precision.
#include "pn_internal.h"

namespace pn {
namespace {
__global__ __launch_bounds__(kThreads) void k_convert(int64_t n, const double* __restrict__ src,
                                                      float* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}
}  // namespace

void launch_convert_params(hipStream_t s, int64_t n, const double* src, float* dst) {
  int64_t nb = std::min<int64_t>((n + kThreads - 1) / kThreads, 4096);
  hipLaunchKernelGGL(k_convert, dim3((unsigned)nb), dim3(kThreads), 0, s, n, src, dst);
}
}  // namespace pn
