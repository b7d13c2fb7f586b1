// Distance features and filter networks w^(n,c) for every pair, as radial
// jets (value, derivative / distance, second derivative).
//
// e_k(d) = d^2 exp(-d - (d - mu_k)^2 / sigma_k^2)   (Methods, featurisation)
// w(d)   = ssp(e(d) W1 + b1) W2 + b2                 (two-layer filter, one per
//                                                     layer n and channel c)
// With e' and e'' the jets propagate through the first Linear unchanged,
// through ssp as  y' = ssp'(u) u',  y'' = ssp'(u) u'' + ssp''(u) u'^2,  and
// through the second Linear unchanged (bias on the value only).  The first
// derivative is carried divided by d (w'/d), which stays finite as d -> 0.
//
// Rows of a block are (walker, pair) of one channel; pairs of a channel are
// contiguous in the unified pair list (same-spin ee, opposite-spin ee, e-n).
// A block takes its rows through every layer: distances and feature jets are
// computed once, and the per-layer weights of one 16-column tile stay in the
// registers of the wave that owns the tile.  The first product's three jet
// tiles of the same rows and columns meet in one lane, so the ssp jets are
// formed from the accumulators; the second product goes from its tiles to the
// table.
#include "gemm_lds.h"
#include "mfma_gemm.h"
#include "pn_internal.h"

namespace pn {
namespace {

// One lane's operand fragment: KQ consecutive elements from 16-byte aligned
// LDS (rows padded by 16 bytes, lane-group offsets multiples of 16 bytes).
template <typename TN, int KQ>
__device__ __forceinline__ void load_frag(const TN* x, TN* f) {
  constexpr int NV = (int)(KQ * sizeof(TN) / 16), PV = (int)(16 / sizeof(TN));
  static_assert((KQ * sizeof(TN)) % 16 == 0, "fragment of whole 16-byte units");
  const uint4* xv = reinterpret_cast<const uint4*>(x);
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const uint4 q = xv[k];
    __builtin_memcpy(&f[k * PV], &q, 16);
  }
}

// KQ1 = K / 4 (features), KQ2 = DZ / 4 (filter width).
template <typename TN, int KQ1, int KQ2>
__global__ __launch_bounds__(kThreads) void k_filters(Dims d, DevTables t, int64_t nw, const double* __restrict__ r,
                                                      const TN* __restrict__ P, ParamLayout pl, TN* __restrict__ filt,
                                                      int PT, int n_same, bool bf16) {
  typedef typename MfmaTile<TN>::acc_t acc_t;
  constexpr int K = 4 * KQ1, DZ = 4 * KQ2, LDK = ld_pad<TN>(K), LDZ = ld_pad<TN>(DZ);
  extern __shared__ __align__(16) char smem[];
  const int ch = blockIdx.y;
  const int p_lo = ch == 0 ? 0 : (ch == 1 ? n_same : d.n_ee);
  const int p_hi = ch == 0 ? n_same : (ch == 1 ? d.n_ee : d.n_pairs);
  const int np = p_hi - p_lo;
  const int64_t nrows = nw * np;
  const int64_t row0 = (int64_t)blockIdx.x * PT;
  if (np == 0 || row0 >= nrows) return;
  const int rows = (int)min((int64_t)PT, nrows - row0);
  double* dd = reinterpret_cast<double*>(smem);       // [PT] distances
  int64_t* doff = reinterpret_cast<int64_t*>(dd + PT);  // [PT] table offset of each row (layer 0)
  TN* E = reinterpret_cast<TN*>(doff + PT);           // [3][PT][LDK] feature jets
  TN* U = E + 3 * PT * LDK;                           // [3][PT][LDZ] ssp jets
  const int64_t lstride = (int64_t)3 * d.n_pairs * DZ, jstride = (int64_t)d.n_pairs * DZ;

  // --- distances (padding rows of a partial tile: 0) ---
  for (int q = threadIdx.x; q < PT; q += blockDim.x) {
    if (q >= rows) {
      dd[q] = 0.0;
      doff[q] = 0;
      continue;
    }
    int64_t g = row0 + q;
    int64_t w = g / np;
    int p = p_lo + (int)(g % np);
    const double* rw = r + w * d.N * 3;
    double x, y, z;
    if (p < d.n_ee) {
      int i = t.pair_ij[2 * p], j = t.pair_ij[2 * p + 1];
      x = rw[3 * i] - rw[3 * j];
      y = rw[3 * i + 1] - rw[3 * j + 1];
      z = rw[3 * i + 2] - rw[3 * j + 2];
    } else {
      int q2 = p - d.n_ee, i = q2 / d.NN, I = q2 % d.NN;
      x = rw[3 * i] - t.nuc_xyz[3 * I];
      y = rw[3 * i + 1] - t.nuc_xyz[3 * I + 1];
      z = rw[3 * i + 2] - t.nuc_xyz[3 * I + 2];
    }
    dd[q] = sqrt(x * x + y * y + z * z);
    doff[q] = w * (int64_t)d.L * lstride + (int64_t)p * DZ;
  }
  __syncthreads();
  // --- feature jets (computed in FP64, stored in the network type) ---
  for (int q = threadIdx.x; q < PT * K; q += blockDim.x) {
    int row = q / K, k = q % K;
    if (row >= rows) {  // padding rows: zero features
      E[(0 * PT + row) * LDK + k] = E[(1 * PT + row) * LDK + k] = E[(2 * PT + row) * LDK + k] = TN(0);
      continue;
    }
    double dv = dd[row];
    double dm = dv - t.feat_mu[k], s = t.feat_sig2inv[k];
    double eg = exp(-dv - dm * dm * s);
    double g1 = -1.0 - 2.0 * dm * s, g2 = -2.0 * s;
    E[(0 * PT + row) * LDK + k] = (TN)(dv * dv * eg);
    E[(1 * PT + row) * LDK + k] = (TN)((2.0 + dv * g1) * eg);                                  // e'/d
    E[(2 * PT + row) * LDK + k] = (TN)((2.0 + 4.0 * dv * g1 + dv * dv * (g1 * g1 + g2)) * eg);  // e''
  }
  __syncthreads();

  // Tile ownership: each wave takes column tiles ct0, ct0 + ct_step, ... and,
  // of each, the row groups rg0, rg0 + rg_step, ... (16 rows per group).
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  constexpr int n_ct = DZ / 16;
  const int n_rg = PT / 16;
  int ct0, ct_step, rg0, rg_step;
  if (n_ct >= nwv) {
    ct0 = wv;
    ct_step = nwv;
    rg0 = 0;
    rg_step = 1;
  } else {  // n_ct divides the wave count (both powers of two)
    ct0 = wv % n_ct;
    ct_step = n_ct;
    rg0 = wv / n_ct;
    rg_step = nwv / n_ct;
  }

  for (int layer = 0; layer < d.L; ++layer) {
    const ParamLayout::Layer& Lp = pl.layer[layer];
    const TN* __restrict__ W1 = P + Lp.w1W[ch];
    const TN* __restrict__ W2 = P + Lp.w2W[ch];
    // --- first Linear on the three jets, ssp jets from the accumulators
    // (bias on the value; y' = ssp'(u) u', y'' = ssp'(u) u'' + ssp''(u) u'^2
    // with u' = d * (u'/d)) ---
    for (int ct = ct0; ct < n_ct; ct += ct_step) {
      const int col = (ct << 4) + c16;
      TN b[KQ1];
#pragma unroll
      for (int s = 0; s < KQ1; ++s) b[s] = W1[(g * KQ1 + s) * DZ + col];
      const TN b1 = P[Lp.w1b[ch] + col];
      for (int rg = rg0; rg < n_rg; rg += rg_step) {
        acc_t c[3];
#pragma unroll
        for (int jet = 0; jet < 3; ++jet) {
          TN a[KQ1];
          load_frag<TN, KQ1>(E + (jet * PT + (rg << 4) + c16) * LDK + g * KQ1, a);
          acc_t z;
#pragma unroll
          for (int v = 0; v < 4; ++v) z[v] = TN(0);
          c[jet] = MfmaChain<TN, KQ1>::run(a, b, z, bf16);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = (rg << 4) + MfmaTile<TN>::row_of(lane, v);
          const TN u = c[0][v] + b1, ud = c[1][v], u2 = c[2][v];
          const TN sg = sigmoid_d(u);
          const TN up = (TN)dd[row] * ud;
          TN* u0 = U + row * LDZ + col;
          u0[0] = ssp(u);
          u0[PT * LDZ] = sg * ud;
          u0[2 * PT * LDZ] = sg * u2 + sg * (TN(1) - sg) * up * up;
        }
      }
    }
    __syncthreads();
    // --- second Linear over the stacked jets, tiles stored to the table
    // [walker][layer][jet][pair][DZ]; bias on the value ---
    for (int ct = ct0; ct < n_ct; ct += ct_step) {
      const int col = (ct << 4) + c16;
      TN b[KQ2];
#pragma unroll
      for (int s = 0; s < KQ2; ++s) b[s] = W2[(g * KQ2 + s) * DZ + col];
      const TN b2 = P[Lp.w2b[ch] + col];
      for (int rg = rg0; rg < n_rg; rg += rg_step) {
#pragma unroll
        for (int jet = 0; jet < 3; ++jet) {
          TN a[KQ2];
          load_frag<TN, KQ2>(U + (jet * PT + (rg << 4) + c16) * LDZ + g * KQ2, a);
          acc_t c;
#pragma unroll
          for (int v = 0; v < 4; ++v) c[v] = TN(0);
          c = MfmaChain<TN, KQ2>::run(a, b, c, bf16);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = (rg << 4) + MfmaTile<TN>::row_of(lane, v);
            TN val = c[v];
            if (jet == 0) val += b2;
            if (row < rows) filt[doff[row] + layer * lstride + jet * jstride + col] = val;
          }
        }
      }
    }
    __syncthreads();  // the next layer rewrites U
  }
}

}  // namespace

template <typename TN>
size_t filter_lds_bytes(const Dims& d, int PT) {
  return PT * (sizeof(double) + sizeof(int64_t)) + (size_t)3 * PT * (ld_pad<TN>(d.K) + ld_pad<TN>(d.DZ)) * sizeof(TN);
}
template size_t filter_lds_bytes<double>(const Dims&, int);
template size_t filter_lds_bytes<float>(const Dims&, int);

template <typename TN>
void launch_filters(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const TN* P, char* ws,
                    const WsLayout& L, bool bf16) {
  const Dims& d = c->d;
  const int PT = L.filt_rows;
  int n_same = 0;
  // same-spin ee pairs: n_up(n_up-1)/2 + n_dn(n_dn-1)/2
  n_same = d.n_up * (d.n_up - 1) / 2 + d.n_dn * (d.n_dn - 1) / 2;
  int64_t max_np = std::max<int64_t>(std::max(n_same, d.n_ee - n_same), (int64_t)d.N * d.NN);
  int64_t nbx = (nw * max_np + PT - 1) / PT;
  size_t lds = filter_lds_bytes<TN>(d, PT);
  const dim3 grid((unsigned)nbx, 3), block(kThreads);
  TN* filt = reinterpret_cast<TN*>(ws + L.filt);
#define PN_FILT(KQ1, KQ2)                                                                                         \
  hipLaunchKernelGGL((k_filters<TN, KQ1, KQ2>), grid, block, lds, s, d, c->t, nw, r, P, c->pl, filt, PT, n_same, \
                     bf16)
#define PN_FILT_Z(KQ1)          \
  switch (d.DZ) {               \
    case 16: PN_FILT(KQ1, 4); break;  \
    case 32: PN_FILT(KQ1, 8); break;  \
    case 64: PN_FILT(KQ1, 16); break; \
    default: PN_FILT(KQ1, 32); break; \
  }
  switch (d.K) {  // feature and filter widths are checked at context creation
    case 16: PN_FILT_Z(4); break;
    case 32: PN_FILT_Z(8); break;
    default: PN_FILT_Z(16); break;
  }
#undef PN_FILT_Z
#undef PN_FILT
}

template void launch_filters<double>(const pn_ctx*, hipStream_t, int64_t, const double*, const double*, char*,
                                     const WsLayout&, bool);
template void launch_filters<float>(const pn_ctx*, hipStream_t, int64_t, const double*, const float*, char*,
                                    const WsLayout&, bool);

}  // namespace pn
