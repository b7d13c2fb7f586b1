// Parameter conversion to the network precision; zero fill.
#include "pn_internal.h"

namespace pn {
namespace {
__global__ __launch_bounds__(kThreads) void k_convert(int64_t n, const double* __restrict__ src,
                                                      float* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}
__global__ __launch_bounds__(kThreads) void k_fill(int64_t n, double* __restrict__ dst, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = v;
}
}  // namespace

// fills by a kernel (they stay kernel nodes if the caller captures the stream)
void launch_fill(hipStream_t s, int64_t n, double* dst, double v) {
  int64_t nb = std::max<int64_t>(1, std::min<int64_t>((n + kThreads - 1) / kThreads, 1024));
  hipLaunchKernelGGL(k_fill, dim3((unsigned)nb), dim3(kThreads), 0, s, n, dst, v);
}
void launch_fill0(hipStream_t s, int64_t n, double* dst) { launch_fill(s, n, dst, 0.0); }

void launch_convert_params(hipStream_t s, int64_t n, const double* src, float* dst) {
  int64_t nb = std::min<int64_t>((n + kThreads - 1) / kThreads, 4096);
  hipLaunchKernelGGL(k_convert, dim3((unsigned)nb), dim3(kThreads), 0, s, n, src, dst);
}
}  // namespace pn
