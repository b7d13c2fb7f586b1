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
#include "gemm_lds.h"
#include "mfma_gemm.h"
#include "pn_internal.h"

namespace pn {
namespace {

template <typename TN>
__global__ __launch_bounds__(kThreads) void k_filters(Dims d, DevTables t, int64_t nw, const double* __restrict__ r,
                                                      const TN* __restrict__ P, ParamLayout pl, TN* __restrict__ filt,
                                                      int PT, int n_same, bool bf16) {
  extern __shared__ __align__(16) char smem[];
  const int layer = blockIdx.y / 3, ch = blockIdx.y % 3;
  const int p_lo = ch == 0 ? 0 : (ch == 1 ? n_same : d.n_ee);
  const int p_hi = ch == 0 ? n_same : (ch == 1 ? d.n_ee : d.n_pairs);
  const int np = p_hi - p_lo;
  const int64_t nrows = nw * np;
  const int64_t row0 = (int64_t)blockIdx.x * PT;
  if (np == 0 || row0 >= nrows) return;
  const int rows = (int)min((int64_t)PT, nrows - row0);
  const int K = d.K, DZ = d.DZ;
  const int LDK = ld_pad<TN>(K), LDZ = ld_pad<TN>(DZ);
  double* dd = reinterpret_cast<double*>(smem);       // [PT] distances
  int64_t* doff = reinterpret_cast<int64_t*>(dd + PT);  // [PT] output offset of each row
  TN* E = reinterpret_cast<TN*>(doff + PT);           // [3][PT][max(LDK, LDZ)]
  TN* U = E + 3 * PT * max(LDK, LDZ);                 // [3][PT][LDZ]
  TN* O = E;                                          // [3][PT][LDZ], over E once E is consumed
  const int64_t lstride = (int64_t)3 * d.n_pairs * DZ;

  // --- distances ---
  for (int q = threadIdx.x; q < rows; q += blockDim.x) {
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
    doff[q] = w * (int64_t)d.L * lstride + layer * lstride + (int64_t)p * DZ;
  }
  __syncthreads();
  // --- feature jets (computed in FP64, stored in the network type) ---
  for (int q = threadIdx.x; q < PT * K; q += blockDim.x) {
    int row = q / K, k = q % K;
    if (row >= rows) {  // padding rows of a partial tile: zero features
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
  const ParamLayout::Layer& Lp = pl.layer[layer];
  // --- first Linear on the three jets: one product over the 3 PT rows (the
  // jets are stacked with equal strides; rows past `rows` are zero features) ---
  gemm_mfma<TN>(E, LDK, 3 * PT, K, P + Lp.w1W[ch], DZ, U, LDZ, false, bf16);
  __syncthreads();
  // --- ssp jets, in place; bias on the value ---
  for (int q = threadIdx.x; q < rows * DZ; q += blockDim.x) {
    int row = q / DZ, z = q % DZ;
    TN* u0 = U + row * LDZ + z;
    TN u = u0[0] + P[Lp.w1b[ch] + z];
    TN ud = u0[PT * LDZ];
    TN u2 = u0[2 * PT * LDZ];
    TN sg = sigmoid_d(u);
    TN up = (TN)dd[row] * ud;
    u0[0] = ssp(u);
    u0[PT * LDZ] = sg * ud;
    u0[2 * PT * LDZ] = sg * u2 + sg * (TN(1) - sg) * up * up;
  }
  __syncthreads();
  // --- second Linear, again over the stacked jets ---
  gemm_mfma<TN>(U, LDZ, 3 * PT, DZ, P + Lp.w2W[ch], DZ, O, LDZ, false, bf16);
  __syncthreads();
  // --- store as [walker][layer][jet][pair][DZ] in 16-byte units; bias on
  // the value ---
  constexpr int V = 16 / sizeof(TN);
  const int DV = DZ / V;
  for (int q = threadIdx.x; q < 3 * rows * DV; q += blockDim.x) {
    const int jet = q / (rows * DV), rem = q % (rows * DV), row = rem / DV, o = (rem % DV) * V;
    TN v[V];
    __builtin_memcpy(v, O + (jet * PT + row) * LDZ + o, 16);
    if (jet == 0)
#pragma unroll
      for (int e = 0; e < V; ++e) v[e] += P[Lp.w2b[ch] + o + e];
    __builtin_memcpy(filt + doff[row] + (int64_t)jet * d.n_pairs * DZ + o, v, 16);
  }
}

}  // namespace

template <typename TN>
size_t filter_lds_bytes(const Dims& d, int PT) {
  return PT * (sizeof(double) + sizeof(int64_t)) +
         (size_t)3 * PT * (std::max(ld_pad<TN>(d.K), ld_pad<TN>(d.DZ)) + ld_pad<TN>(d.DZ)) * sizeof(TN);
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
  hipLaunchKernelGGL(k_filters<TN>, dim3((unsigned)nbx, 3 * d.L), dim3(kThreads), lds, s, d, c->t, nw, r, P,
                     c->pl, reinterpret_cast<TN*>(ws + L.filt), PT, n_same, bf16);
}

template void launch_filters<double>(const pn_ctx*, hipStream_t, int64_t, const double*, const double*, char*,
                                     const WsLayout&, bool);
template void launch_filters<float>(const pn_ctx*, hipStream_t, int64_t, const double*, const float*, char*,
                                    const WsLayout&, bool);

}  // namespace pn
