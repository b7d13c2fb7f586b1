// Small dense products used inside the fused network kernels:
//   Y[rows][O] (+)= X[rows][I] * W[I][O]
// X and Y live in LDS, W (a parameter block, shared by every workgroup)
// is read through the L1/L2 caches.  All threads of the block take part;
// the caller places __syncthreads() around the call.
#pragma once

#include <hip/hip_runtime.h>

namespace pn {

// Round-to-nearest-even to bfloat16 precision, kept in a float.
__device__ __forceinline__ float round_bf16(float x) {
  unsigned u = __float_as_uint(x);
  unsigned lsb = (u >> 16) & 1u;
  u = (u + 0x7fffu + lsb) & 0xffff0000u;
  return __uint_as_float(u);
}

template <typename T>
__device__ __forceinline__ T maybe_bf16(T x, bool bf16) {
  return x;
}
template <>
__device__ __forceinline__ float maybe_bf16<float>(float x, bool bf16) {
  return bf16 ? round_bf16(x) : x;
}

// Each thread owns RB rows x 1 column of the output.
template <typename T, int RB = 4>
__device__ __forceinline__ void gemm_xw(const T* X, int ldx, int rows, int I, const T* __restrict__ W, int O,
                                        T* Y, int ldy, bool accumulate, bool bf16 = false) {
  const int nrb = (rows + RB - 1) / RB;
  for (int t = threadIdx.x; t < nrb * O; t += blockDim.x) {
    const int o = t % O, r0 = (t / O) * RB;
    const T* xr[RB];
    T acc[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      int rr = min(r0 + q, rows - 1);
      xr[q] = X + (size_t)rr * ldx;
      acc[q] = (accumulate && r0 + q < rows) ? Y[(size_t)(r0 + q) * ldy + o] : T(0);
    }
    for (int k = 0; k < I; ++k) {
      T w = maybe_bf16(W[(size_t)k * O + o], bf16);
#pragma unroll
      for (int q = 0; q < RB; ++q) acc[q] += maybe_bf16(xr[q][k], bf16) * w;
    }
#pragma unroll
    for (int q = 0; q < RB; ++q)
      if (r0 + q < rows) Y[(size_t)(r0 + q) * ldy + o] = acc[q];
  }
}

}  // namespace pn
