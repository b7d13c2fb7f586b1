// Dense products on the CDNA4 matrix cores, for the fused network kernels:
//
//   Y[rows][O] (+)= X[rows][I] * W[I][O]
//
// X and Y live in LDS (row strides ldx, ldy), W is a parameter block in
// global memory ([I][O] row-major, shared by every workgroup, read through
// L1/L2).  The output is cut into 16 x 16 tiles; each wavefront of the
// block keeps one 16-column slab of W in registers and walks row tiles.
//
// Instructions (wave64):
//   FP64           v_mfma_f64_16x16x4_f64     (one k per lane and step)
//   FP32           v_mfma_f32_16x16x4_f32
//   BF16 operands  v_mfma_f32_16x16x32_bf16   (I % 32 == 0) or
//                  v_mfma_f32_16x16x16_bf16   (I % 16 == 0), FP32 accumulate
//
// The reduction index is split so that lane group g = lane / 16 covers a
// contiguous range of I / 4 values of k: each lane then reads its A operand
// as contiguous LDS words, and every step still sums over distinct k.
//
// Output layout of the 16 x 16 result (checked on gfx950): lane l, element
// v holds row 4 (l / 16) + v (FP32 and BF16 forms) or row 4 v + l / 16
// (FP64 form), column l % 16.
//
// Requirements: O % 16 == 0; I in {16, 32, 64, 128}; rows >= 1.  Rows past `rows` read a clamped row and are not stored.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace pn {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ short bf16_bits(float x) {
  // round to nearest even
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

template <typename TN>
struct MfmaTile;

template <>
struct MfmaTile<double> {
  typedef v4d acc_t;
  __device__ static int row_of(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <>
struct MfmaTile<float> {
  typedef v4f acc_t;
  __device__ static int row_of(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// Output epilogue: called as epi(row_tile, column, acc) on each 16 x 16
// result just before it is stored (this lane's four elements of `column`,
// layout as above).  NoEpi stores the product as is.
struct NoEpi {
  template <typename A>
  __device__ void operator()(int, int, A&) const {}
};
// An epilogue with `static constexpr bool kOwnStore = true` also stores the
// tile itself (epi.store(row_tile, column, acc)) in a layout of its own; the
// product then writes nothing to Y and must not accumulate.
template <typename E, typename = void>
struct EpiOwnsStore : std::false_type {};
template <typename E>
struct EpiOwnsStore<E, std::void_t<decltype(E::kOwnStore)>> : std::integral_constant<bool, E::kOwnStore> {};

// One wavefront: C += A_tile(16 x I) * B_slab(I x 16), operands in registers
// (afrag[s] = X[row][g*KQ + s], bfrag[s] = W[g*KQ + s][col]).
template <typename TN, int KQ>
struct MfmaChain;

template <int KQ>
struct MfmaChain<double, KQ> {
  __device__ static v4d run(const double* a, const double* b, v4d c, bool) {
#pragma unroll
    for (int s = 0; s < KQ; ++s) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], c, 0, 0, 0);
    return c;
  }
};

template <int KQ>
struct MfmaChain<float, KQ> {
  __device__ static v4f run(const float* a, const float* b, v4f c, bool bf16) {
    if (!bf16) {
#pragma unroll
      for (int s = 0; s < KQ; ++s) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], c, 0, 0, 0);
      return c;
    }
    if constexpr ((KQ % 8) == 0) {
#pragma unroll
      for (int s = 0; s < KQ; s += 8) {
        v8bf av, bv;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          av[q] = __builtin_bit_cast(__bf16, bf16_bits(a[s + q]));
          bv[q] = __builtin_bit_cast(__bf16, bf16_bits(b[s + q]));
        }
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int s = 0; s < KQ; s += 4) {
        v4s av, bv;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          av[q] = bf16_bits(a[s + q]);
          bv[q] = bf16_bits(b[s + q]);
        }
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, c, 0, 0, 0);
      }
    }
    return c;
  }
};

// WIN: a row window.  Only output rows [lo, lo + n) receive a product, and
// their A rows are X[row - lo]; tiles that miss the window are skipped.  The
// tile-to-wave assignment depends only on rows and O, so a windowed product
// and a full one over the same output share it: each output element is
// updated by the same wave in both, and the two need no barrier between them.
// PAIR (FP32 and BF16 forms): whole row tiles are taken two at a time and
// without per-element bounds tests (more registers, half the exposed LDS
// latency).
// DUAL: a second product on a row window, X2[row - lo] * W2 for output rows
// [lo, lo + n), summed into the same tiles as the full product X * W (its
// weight slab is read together with the first one).
template <typename TN, int KQ, bool WT = false, bool WIN = false, bool PAIR = false, bool DUAL = false,
          typename EPI = NoEpi>
__device__ __forceinline__ void gemm_mfma_k(const TN* X, int ldx, int rows, const TN* __restrict__ W, int ldw, int O,
                                            int ncol, TN* Y, int ldy, bool accumulate, bool bf16, int lo = 0,
                                            int n = 0, const TN* X2 = nullptr, int ldx2 = 0,
                                            const TN* __restrict__ W2 = nullptr, EPI epi = EPI()) {
  typedef typename MfmaTile<TN>::acc_t acc_t;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  const int n_rt = (rows + 15) >> 4, n_ct = O >> 4;
  int ct0, ct_step, rt0, rt_step;
  if (n_ct >= nwv || (nwv % n_ct) != 0) {
    ct0 = wv;
    ct_step = nwv;
    rt0 = 0;
    rt_step = 1;
  } else {
    ct0 = wv % n_ct;
    ct_step = O;  // a single slab per wave
    rt0 = wv / n_ct;
    rt_step = nwv / n_ct;
  }
  constexpr bool kPair = PAIR && !WIN && sizeof(TN) == 4;
  constexpr bool kEpi = !std::is_same<EPI, NoEpi>::value;
  constexpr bool kOwn = EpiOwnsStore<EPI>::value;
  // A fragment of row tile rt: 16-byte reads, so each group of 8 lanes
  // covers every LDS bank once (rows are padded by 16 bytes); element-wise
  // reads of the same rows hit each bank up to four times.  Rows and
  // lane-group offsets are 16-byte aligned for every caller (row strides
  // from ld_pad, KQ * size a multiple of 16 bytes).
  auto load_a = [&](int rt, TN* afrag) {
    const int rw = (rt << 4) + c16 - lo;
    const bool inw = !WIN || (rw >= 0 && rw < n);
    const int r = WIN ? (inw ? rw : 0) : min((rt << 4) + c16, rows - 1);
    const TN* xr = X + r * ldx + g * KQ;
    if constexpr ((KQ * sizeof(TN)) % 16 == 0) {
      constexpr int NV = (int)(KQ * sizeof(TN) / 16), PV = (int)(16 / sizeof(TN));
      const uint4* xv = reinterpret_cast<const uint4*>(xr);
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const uint4 q = xv[k];
        __builtin_memcpy(&afrag[k * PV], &q, 16);
      }
    } else {
#pragma unroll
      for (int s = 0; s < KQ; ++s) afrag[s] = xr[s];
    }
    if constexpr (WIN) {
#pragma unroll
      for (int s = 0; s < KQ; ++s) afrag[s] = inw ? afrag[s] : TN(0);
    }
  };
  // the second product's A fragment (window rows, zero elsewhere)
  auto load_a2 = [&](int rt, TN* af) {
    const int rw = (rt << 4) + c16 - lo;
    const bool inw = rw >= 0 && rw < n;
    const TN* xr = X2 + (inw ? rw : 0) * ldx2 + g * KQ;
    if constexpr ((KQ * sizeof(TN)) % 16 == 0) {
      constexpr int NV = (int)(KQ * sizeof(TN) / 16), PV = (int)(16 / sizeof(TN));
      const uint4* xv = reinterpret_cast<const uint4*>(xr);
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const uint4 q = xv[k];
        __builtin_memcpy(&af[k * PV], &q, 16);
      }
    } else {
#pragma unroll
      for (int s = 0; s < KQ; ++s) af[s] = xr[s];
    }
#pragma unroll
    for (int s = 0; s < KQ; ++s) af[s] = inw ? af[s] : TN(0);
  };
  auto meets = [&](int rt) { return (rt << 4) < lo + n && (rt << 4) + 16 > lo; };  // wave-uniform
  for (int ct = ct0; ct < n_ct; ct += ct_step) {
    const int col = (ct << 4) + c16;
    const bool colok = col < ncol;
    const bool colfull = (ct << 4) + 16 <= ncol;  // wave-uniform
    TN bfrag[KQ];
#pragma unroll
    for (int s = 0; s < KQ; ++s)
      bfrag[s] = colok ? (WT ? W[col * ldw + g * KQ + s] : W[(g * KQ + s) * ldw + col]) : TN(0);
    TN bfrag2[DUAL ? KQ : 1];
    if constexpr (DUAL) {
#pragma unroll
      for (int s = 0; s < KQ; ++s) bfrag2[s] = colok ? W2[(g * KQ + s) * ldw + col] : TN(0);
    }
    auto second = [&](int rt, acc_t c) -> acc_t {
      if constexpr (DUAL) {
        if (meets(rt)) {
          TN a2[KQ];
          load_a2(rt, a2);
          c = MfmaChain<TN, KQ>::run(a2, bfrag2, c, bf16);
        }
      }
      return c;
    };
    int rt = rt0;
    // Pairs of whole tiles: both tiles' operand and output reads are issued
    // before the two (independent) MFMA chains, and no element needs a
    // bounds test.
    if constexpr (kPair) {
      for (; colfull && rt + rt_step < n_rt && ((rt + rt_step) << 4) + 16 <= rows; rt += 2 * rt_step) {
        const int rtb = rt + rt_step;
        TN afa[KQ], afb[KQ];
        load_a(rt, afa);
        load_a(rtb, afb);
        acc_t ca, cb;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = MfmaTile<TN>::row_of(lane, v);
          ca[v] = accumulate ? Y[((rt << 4) + row) * ldy + col] : TN(0);
          cb[v] = accumulate ? Y[((rtb << 4) + row) * ldy + col] : TN(0);
        }
        ca = MfmaChain<TN, KQ>::run(afa, bfrag, ca, bf16);
        cb = MfmaChain<TN, KQ>::run(afb, bfrag, cb, bf16);
        ca = second(rt, ca);
        cb = second(rtb, cb);
        if constexpr (kEpi) {
          epi(rt, col, ca);
          epi(rtb, col, cb);
        }
        if constexpr (kOwn) {
          epi.store(rt, col, ca);
          epi.store(rtb, col, cb);
          continue;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = MfmaTile<TN>::row_of(lane, v);
          Y[((rt << 4) + row) * ldy + col] = ca[v];
          Y[((rtb << 4) + row) * ldy + col] = cb[v];
        }
      }
    }
    for (; rt < n_rt; rt += rt_step) {
      if (WIN && ((rt << 4) >= lo + n || (rt << 4) + 16 <= lo)) continue;  // wave-uniform
      TN afrag[KQ];
      load_a(rt, afrag);
      acc_t c;
      if (kPair && colfull && (rt << 4) + 16 <= rows) {  // whole tile: no per-element tests
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = (rt << 4) + MfmaTile<TN>::row_of(lane, v);
          c[v] = accumulate ? Y[row * ldy + col] : TN(0);
        }
        c = MfmaChain<TN, KQ>::run(afrag, bfrag, c, bf16);
        c = second(rt, c);
        if constexpr (kEpi) epi(rt, col, c);
        if constexpr (kOwn) {
          epi.store(rt, col, c);
          continue;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = (rt << 4) + MfmaTile<TN>::row_of(lane, v);
          Y[row * ldy + col] = c[v];
        }
        continue;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = (rt << 4) + MfmaTile<TN>::row_of(lane, v);
        c[v] = (accumulate && row < rows && colok) ? Y[row * ldy + col] : TN(0);
      }
      c = MfmaChain<TN, KQ>::run(afrag, bfrag, c, bf16);
      c = second(rt, c);
      if constexpr (kEpi) epi(rt, col, c);
      if constexpr (kOwn) {
        if (colok) epi.store(rt, col, c);  // the epilogue tests its rows
        continue;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = (rt << 4) + MfmaTile<TN>::row_of(lane, v);
        if (row < rows && colok) Y[row * ldy + col] = c[v];
      }
    }
  }
}

// Whole-block product; every thread of the block must call it.  I must be
// one of 16, 32, 64, 128 (128 runs as two accumulated halves of 64, which
// keeps at most 16 operand fragments live per lane); O a multiple of 16.
// The caller separates the halves' read and write of Y with nothing: each
// output element is owned by one lane in both halves.
// Narrow output: W is [I][ncol] (row stride ncol), the product is computed
// on ceil(ncol / 16) column tiles and only the ncol valid columns are
// stored (used for the backflow output layer, ncol = number of orbitals).
template <typename TN>
__device__ __forceinline__ void gemm_mfma_cols(const TN* X, int ldx, int rows, int I, const TN* __restrict__ W,
                                               int ncol, TN* Y, int ldy, bool accumulate, bool bf16) {
  const int O = (ncol + 15) & ~15;
  switch (I) {
    case 16: gemm_mfma_k<TN, 4>(X, ldx, rows, W, ncol, O, ncol, Y, ldy, accumulate, bf16); break;
    case 32: gemm_mfma_k<TN, 8>(X, ldx, rows, W, ncol, O, ncol, Y, ldy, accumulate, bf16); break;
    case 64: gemm_mfma_k<TN, 16>(X, ldx, rows, W, ncol, O, ncol, Y, ldy, accumulate, bf16); break;
    default:
      gemm_mfma_k<TN, 16>(X, ldx, rows, W, ncol, O, ncol, Y, ldy, accumulate, bf16);
      gemm_mfma_k<TN, 16>(X + 64, ldx, rows, W + (size_t)64 * ncol, ncol, O, ncol, Y, ldy, true, bf16);
      break;
  }
}

template <typename TN, bool PAIR = false, typename EPI = NoEpi>
__device__ __forceinline__ void gemm_mfma(const TN* X, int ldx, int rows, int I, const TN* __restrict__ W, int O,
                                          TN* Y, int ldy, bool accumulate, bool bf16, EPI epi = EPI()) {
  switch (I) {
    case 16:
      gemm_mfma_k<TN, 4, false, false, PAIR, false, EPI>(X, ldx, rows, W, O, O, O, Y, ldy, accumulate, bf16, 0, 0,
                                                           nullptr, 0, nullptr, epi);
      break;
    case 32:
      gemm_mfma_k<TN, 8, false, false, PAIR, false, EPI>(X, ldx, rows, W, O, O, O, Y, ldy, accumulate, bf16, 0, 0,
                                                           nullptr, 0, nullptr, epi);
      break;
    case 64:
      gemm_mfma_k<TN, 16, false, false, PAIR, false, EPI>(X, ldx, rows, W, O, O, O, Y, ldy, accumulate, bf16, 0, 0,
                                                            nullptr, 0, nullptr, epi);
      break;
    default:  // the epilogue acts on the sum of both halves
      if constexpr (sizeof(TN) == 4) {  // both halves on each tile: one slab wait, one pass over Y
        gemm_mfma_k<TN, 16, false, false, PAIR, true, EPI>(X, ldx, rows, W, O, O, O, Y, ldy, accumulate, bf16, 0,
                                                             rows, X + 64, ldx, W + (size_t)64 * O, epi);
      } else {  // FP64: the halves one after the other (two slabs would spill)
        gemm_mfma_k<TN, 16, false, false, PAIR>(X, ldx, rows, W, O, O, O, Y, ldy, accumulate, bf16);
        gemm_mfma_k<TN, 16, false, false, PAIR, false, EPI>(X + 64, ldx, rows, W + (size_t)64 * O, O, O, O, Y, ldy,
                                                              true, bf16, 0, 0, nullptr, 0, nullptr, epi);
      }
      break;
  }
}

// Y[rows][O] += X * W + (rows lo .. lo + n) X2[row - lo] * W2, the two with
// the same I (16, 32, 64 or 128) and O: one pass over the output tiles, and
// both weight slabs read up front.
template <typename TN, bool PAIR = false>
__device__ __forceinline__ void gemm_mfma_dual(const TN* X, int ldx, int rows, int I, const TN* __restrict__ W,
                                               int O, TN* Y, int ldy, const TN* X2, int ldx2, int lo, int n,
                                               const TN* __restrict__ W2, bool bf16) {
  switch (I) {
    case 16:
      gemm_mfma_k<TN, 4, false, false, PAIR, true>(X, ldx, rows, W, O, O, O, Y, ldy, true, bf16, lo, n, X2, ldx2, W2);
      break;
    case 32:
      gemm_mfma_k<TN, 8, false, false, PAIR, true>(X, ldx, rows, W, O, O, O, Y, ldy, true, bf16, lo, n, X2, ldx2, W2);
      break;
    case 64:
      gemm_mfma_k<TN, 16, false, false, PAIR, true>(X, ldx, rows, W, O, O, O, Y, ldy, true, bf16, lo, n, X2, ldx2, W2);
      break;
    default:
      gemm_mfma_k<TN, 16, false, false, PAIR, true>(X, ldx, rows, W, O, O, O, Y, ldy, true, bf16, lo, n, X2, ldx2, W2);
      gemm_mfma_k<TN, 16, false, false, PAIR, true>(X + 64, ldx, rows, W + (size_t)64 * O, O, O, O, Y, ldy, true,
                                                    bf16, lo, n, X2 + 64, ldx2, W2 + (size_t)64 * O);
      break;
  }
}

// Y[lo + r][O] += X[r][I] * W for r < n, as the windowed form above: it may
// follow a gemm_mfma over the same Y, rows and O without a barrier.
template <typename TN>
__device__ __forceinline__ void gemm_mfma_window(const TN* X, int ldx, int rows, int lo, int n, int I,
                                                 const TN* __restrict__ W, int O, TN* Y, int ldy, bool bf16) {
  switch (I) {
    case 16: gemm_mfma_k<TN, 4, false, true>(X, ldx, rows, W, O, O, O, Y, ldy, true, bf16, lo, n); break;
    case 32: gemm_mfma_k<TN, 8, false, true>(X, ldx, rows, W, O, O, O, Y, ldy, true, bf16, lo, n); break;
    case 64: gemm_mfma_k<TN, 16, false, true>(X, ldx, rows, W, O, O, O, Y, ldy, true, bf16, lo, n); break;
    default:
      gemm_mfma_k<TN, 16, false, true>(X, ldx, rows, W, O, O, O, Y, ldy, true, bf16, lo, n);
      gemm_mfma_k<TN, 16, false, true>(X + 64, ldx, rows, W + (size_t)64 * O, O, O, O, Y, ldy, true, bf16, lo, n);
      break;
  }
}

// Y[rows][O] (+)= X[rows][I] * W^T with W stored [O][I] row-major (the
// transposed products of the adjoint pass).  I in {16, 32, 64, 128}.
template <typename TN>
__device__ __forceinline__ void gemm_mfma_wt(const TN* X, int ldx, int rows, int I, const TN* __restrict__ W, int O,
                                             TN* Y, int ldy, bool accumulate) {
  switch (I) {
    case 16: gemm_mfma_k<TN, 4, true>(X, ldx, rows, W, I, O, O, Y, ldy, accumulate, false); break;
    case 32: gemm_mfma_k<TN, 8, true>(X, ldx, rows, W, I, O, O, Y, ldy, accumulate, false); break;
    case 64: gemm_mfma_k<TN, 16, true>(X, ldx, rows, W, I, O, O, Y, ldy, accumulate, false); break;
    default:
      gemm_mfma_k<TN, 16, true>(X, ldx, rows, W, I, O, O, Y, ldy, accumulate, false);
      gemm_mfma_k<TN, 16, true>(X + 64, ldx, rows, W + 64, I, O, O, Y, ldy, true, false);
      break;
  }
}

}  // namespace pn
