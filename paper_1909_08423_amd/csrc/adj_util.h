// Helpers of the adjoint kernels: parameter-gradient outer products summed
// over rows (into a block's private gradient slot) and derivatives of the
// shifted softplus.
#pragma once
#include "mfma_gemm.h"
#include "pn_internal.h"

namespace pn {

// first three derivatives of ssp: s, s (1 - s), s (1 - s) (1 - 2 s), s = sigmoid(u)
template <typename TN>
__device__ __forceinline__ TN sig(TN u) {
  return sigmoid_d(u);
}
template <typename TN>
__device__ __forceinline__ TN ssp2(TN u) {
  const TN s = sigmoid_d(u);
  return s * (TN(1) - s);
}
template <typename TN>
__device__ __forceinline__ TN ssp3(TN u) {
  const TN s = sigmoid_d(u);
  return s * (TN(1) - s) * (TN(1) - TN(2) * s);
}


// slot[a*B + b] (+)= sum_r X[r][a] Y[r][b]
template <typename TN>
__device__ void outer_acc(const TN* X, int ldx, int A, const TN* Y, int ldy, int B, int rows, TN* slot, bool first) {
  for (int q = threadIdx.x; q < A * B; q += blockDim.x) {
    const int a = q / B, b = q % B;
    TN s = 0;
    for (int r = 0; r < rows; ++r) s += X[(size_t)r * ldx + a] * Y[(size_t)r * ldy + b];
    slot[q] = first ? s : slot[q] + s;
  }
}
// same with X replaced by ssp(U) (recomputed on the fly)
template <typename TN>
__device__ void outer_acc_ssp(const TN* U, int ldu, int A, const TN* Y, int ldy, int B, int rows, TN* slot,
                              bool first) {
  for (int q = threadIdx.x; q < A * B; q += blockDim.x) {
    const int a = q / B, b = q % B;
    TN s = 0;
    for (int r = 0; r < rows; ++r) s += ssp(U[(size_t)r * ldu + a]) * Y[(size_t)r * ldy + b];
    slot[q] = first ? s : slot[q] + s;
  }
}
// slot[a*B + b] (+)= sum_r f(X[r][a]) Y[r][b] on the matrix cores (f = identity
// or ssp); A and B multiples of 16.  Rows are reduced in chunks of 32: lane
// group g takes rows g*8 .. g*8+7 of a chunk, rows past `rows` read as zero.
template <typename TN, bool SSP>
__device__ void outer_mfma(const TN* X, int ldx, int A, const TN* Y, int ldy, int B, int rows, TN* slot, bool first) {
  typedef typename MfmaTile<TN>::acc_t acc_t;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  const int nbt = B / 16, nt = (A / 16) * nbt;
  for (int tt = wv; tt < nt; tt += nwv) {
    const int a0 = (tt / nbt) * 16, b0 = (tt % nbt) * 16;
    acc_t c;
#pragma unroll
    for (int v = 0; v < 4; ++v) c[v] = 0;
    for (int r0 = 0; r0 < rows; r0 += 32) {
      TN af[8], bf[8];
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2) {
        const int r = r0 + g * 8 + s2;
        const bool ok = r < rows;
        const TN xv = ok ? X[(size_t)r * ldx + a0 + c16] : TN(0);
        af[s2] = SSP ? (ok ? ssp(xv) : TN(0)) : xv;
        bf[s2] = ok ? Y[(size_t)r * ldy + b0 + c16] : TN(0);
      }
      c = MfmaChain<TN, 8>::run(af, bf, c, false);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const size_t q = (size_t)(a0 + MfmaTile<TN>::row_of(lane, v)) * B + b0 + c16;
      slot[q] = first ? c[v] : slot[q] + c[v];
    }
  }
}

// slot[b] (+)= sum_r Y[r][b]
template <typename TN>
__device__ void colsum_acc(const TN* Y, int ldy, int B, int rows, TN* slot, bool first) {
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    TN s = 0;
    for (int r = 0; r < rows; ++r) s += Y[(size_t)r * ldy + b];
    slot[b] = first ? s : slot[b] + s;
  }
}

}  // namespace pn
