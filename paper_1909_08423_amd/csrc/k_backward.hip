// Value-path adjoint: grad_theta += sum_w ct_w d ln|psi_w| / d theta.
//
// The Hermitian gradient estimator (Methods, eq. "trainig") needs only the
// parameter gradient of ln|psi| weighted per walker by 2 (E_loc - L) / B,
// which is this adjoint with ct_w = that weight.  ln|psi| = gamma + J +
// ln|Psi_d| depends on theta through J and through the backflow f inside
// the determinants:
//   d ln|Psi_d| / d A_p^s[k][i] = w_p (A_p^s)^{-1}[i][k],  w_p = c_p D_p / Psi_d
//   A_p^s[k][i] = phi_mu(r_i) f_{i mu},  mu = mu_p^s(k)
// so  d ln|psi| / d f_{i mu} = phi_mu(r_i) sum_p w_p sum_{k: mu_p(k) = mu} G_p[i][k].
// From there the reverse sweep runs through kappa, eta, the interaction
// layers (messages, h and the three g) and finally the filter networks.
//
// Kernels (the forward values come from the value pass, run just before):
//  k_bwd_net     groups of WB walkers; grid-stride over groups with a fixed
//                grid, each block summing its parameter gradients into its
//                own slot; writes the cotangents of the filter outputs.
//  k_bwd_filter  per (layer, channel) and a fixed set of blocks striding
//                over (walker, pair) rows; recomputes features and the
//                hidden layer, accumulates the filter gradients in registers.
//  k_bwd_reduce  sums the slots in a fixed order into the FP64 gradient.
// The fixed grids and slot order make the result independent of anything
// else running on the device.
#include "adj_util.h"
#include "gemm_lds.h"
#include "mfma_gemm.h"
#include "pn_internal.h"

namespace pn {
namespace {

constexpr int kSlotsNet = 512;     // blocks (and gradient slots) of k_bwd_net
constexpr int kSlotsFilter = 256;  // blocks per (layer, channel) of k_bwd_filter
constexpr int kFiltRows = 32;      // (walker, pair) rows per tile of k_bwd_filter

template <typename TN>
__global__ __launch_bounds__(kThreads) void k_bwd_net(Dims d, DevTables t, int64_t nw, int WB,
                                                      const TN* __restrict__ P, ParamLayout pl,
                                                      const TN* __restrict__ xval, const TN* __restrict__ hval,
                                                      const TN* __restrict__ filt, const double* __restrict__ phi,
                                                      const double* __restrict__ ginv, const double* __restrict__ wdet,
                                                      const double* __restrict__ ct_logabs, TN* __restrict__ ctw,
                                                      TN* __restrict__ gslot, int64_t n_params,
                                                      const double* __restrict__ ctfpart, int n_chunks,
                                                      const TN* __restrict__ cthv, const TN* __restrict__ ctkc,
                                                      const TN* __restrict__ ctec, TN* __restrict__ arena,
                                                      int64_t arena_elems) {
  extern __shared__ __align__(16) char smem[];
  const int N = d.N, DX = d.DX, DZ = d.DZ, M = d.M, L = d.L, NU = d.n_up;
  const int LDX = ld_pad<TN>(DX), LDZ = ld_pad<TN>(DZ), LDM = ld_pad<TN>((M + 15) & ~15);
  const int RW = WB * N;
  TN* slot = gslot + (size_t)blockIdx.x * n_params;
  int* pidx = reinterpret_cast<int*>(smem);
  TN* cw = reinterpret_cast<TN*>(pidx + ((N * N + 3) & ~3));  // [WB]
  TN* X = cw + ((WB + 3) & ~3);                                 // [RW][LDX]
  TN* CX = X + RW * LDX;                                        // [RW][LDX]
  // union region (heads, then layers): in LDS, or in this block's part of a
  // global arena when it does not fit beside X and CX
  TN* UN = arena ? arena + (size_t)blockIdx.x * arena_elems : CX + RW * LDX;
  // heads view
  TN* A = UN;                  // [RW][LDX]
  TN* B = A + RW * LDX;        // [RW][LDX]
  TN* Cb = B + RW * LDX;       // [RW][LDX]
  TN* CF = Cb + RW * LDX;      // [RW][LDM]
  // layers view
  TN* H = UN;                  // [RW][LDZ]
  TN* Z = H + RW * LDZ;
  TN* CZ = Z + RW * LDZ;
  TN* CH = CZ + RW * LDZ;
  const int64_t fl_stride = (int64_t)3 * d.n_pairs * DZ;
  const int64_t ng = (nw + WB - 1) / WB;
  for (int q = threadIdx.x; q < N * N; q += blockDim.x) pidx[q] = t.pair_index[q];
  bool first = true;
  for (int64_t grp = blockIdx.x; grp < ng; grp += gridDim.x, first = false) {
    const int64_t w0 = grp * WB;
    const int nwb = (int)min((int64_t)WB, nw - w0);
    const int R = nwb * N;
    __syncthreads();
    for (int q = threadIdx.x; q < nwb; q += blockDim.x) cw[q] = (TN)ct_logabs[w0 + q];
    const TN jas = (d.flags & PN_NET_NO_JASTROW) ? TN(0) : TN(1);  // a removed Jastrow factor gets no cotangent
    // ---- cotangent of the backflow, from the determinants ----
    for (int q = threadIdx.x; q < R * LDM; q += blockDim.x) CF[q] = 0;
    for (int q = threadIdx.x; q < R * DX; q += blockDim.x)
      X[(q / DX) * LDX + q % DX] = xval[((w0 + q / (N * DX)) * (L + 1) + L) * N * DX + q % (N * DX)];
    __syncthreads();
    const int gsz = d.n_up * d.n_up + d.n_dn * d.n_dn;
    for (int row = threadIdx.x; row < R; row += blockDim.x) {
      const int wl = row / N, i = row % N;
      const int64_t w = w0 + wl;
      const bool up = i < NU;
      const int n = up ? d.n_up : d.n_dn, ii = up ? i : i - NU;
      const int* dets = up ? t.det_up : t.det_dn;
      for (int p = 0; p < d.P; ++p) {
        const double wp = wdet[w * d.P + p];
        const double* G = ginv + (w * d.P + p) * gsz + (up ? 0 : d.n_up * d.n_up);
        for (int k = 0; k < n; ++k) CF[row * LDM + dets[p * n + k]] += (TN)(wp * G[ii * n + k]);
      }
      const double* ph = phi + (w * N + i) * M * 7;
      if (d.flags & PN_NET_NO_BACKFLOW) {
        for (int mu = 0; mu < M; ++mu) CF[row * LDM + mu] = 0;  // f = 1 does not depend on theta
      } else if (ctfpart) {
        // full adjoint: the determinant part supplies the cotangent of f
        // (its ln|psi| share included), summed over the coordinate chunks
        for (int mu = 0; mu < M; ++mu) {
          double v = 0.0;
          for (int c = 0; c < n_chunks; ++c) v += ctfpart[((w * n_chunks + c) * N + i) * M + mu];
          CF[row * LDM + mu] = (TN)v;
        }
      } else {
        for (int mu = 0; mu < M; ++mu) CF[row * LDM + mu] *= (TN)(ph[mu * 7]) * cw[wl];
      }
    }
    __syncthreads();
    // ---- Jastrow head (per walker): J = eta(sum_i x_i) ----
    {
      TN* Sv = CF + RW * LDM;  // [WB][LDX] s
      TN* U1 = Sv + WB * LDX;  // pre-activations
      TN* U2 = U1 + WB * LDX;
      TN* Y1 = U2 + WB * LDX;
      TN* C1 = Y1 + WB * LDX;  // cotangents
      TN* C2 = C1 + WB * LDX;
      for (int q = threadIdx.x; q < nwb * DX; q += blockDim.x) {
        const int wl = q / DX, x = q % DX;
        TN s = 0;
        for (int i = 0; i < N; ++i) s += X[(wl * N + i) * LDX + x];
        Sv[wl * LDX + x] = s;
      }
      __syncthreads();
      gemm_mfma<TN>(Sv, LDX, nwb, DX, P + pl.eW1, DX, U1, LDX, false, false);
      __syncthreads();
      for (int q = threadIdx.x; q < nwb * DX; q += blockDim.x) {
        const int r = q / DX, x = q % DX;
        U1[r * LDX + x] += P[pl.eb1 + x];
        Y1[r * LDX + x] = ssp(U1[r * LDX + x]);
      }
      __syncthreads();
      gemm_mfma<TN>(Y1, LDX, nwb, DX, P + pl.eW2, DX, U2, LDX, false, false);
      __syncthreads();
      for (int q = threadIdx.x; q < nwb * DX; q += blockDim.x) {
        const int r = q / DX, x = q % DX;
        U2[r * LDX + x] += P[pl.eb2 + x];
        // d/d u2 = cJ * W3[x] * ssp'(u2)
        const TN u2 = U2[r * LDX + x];
        TN c2 = jas * cw[r] * P[pl.eW3 + x] * sig(u2);
        if (ctec) {  // tangent-pass cotangents of ssp'(u2), ssp''(u2)
          const TN* ce = ctec + ((w0 + r) * 2 + 1) * 2 * DX;
          c2 += ce[x] * ssp2(u2) + ce[DX + x] * ssp3(u2);
        }
        C2[r * LDX + x] = c2;
      }
      __syncthreads();
      // dW3, db3
      for (int x = threadIdx.x; x < DX; x += blockDim.x) {
        TN s = 0;
        for (int r = 0; r < nwb; ++r) s += jas * ssp(U2[r * LDX + x]) * cw[r];
        slot[pl.eW3 + x] = first ? s : slot[pl.eW3 + x] + s;
      }
      if (threadIdx.x == 0) {
        TN s = 0;
        for (int r = 0; r < nwb; ++r) s += jas * cw[r];
        slot[pl.eb3] = first ? s : slot[pl.eb3] + s;
      }
      outer_mfma<TN, true>(U1, LDX, DX, C2, LDX, DX, nwb, slot + pl.eW2, first);
      colsum_acc<TN>(C2, LDX, DX, nwb, slot + pl.eb2, first);
      gemm_mfma_wt<TN>(C2, LDX, nwb, DX, P + pl.eW2, DX, C1, LDX, false);
      __syncthreads();
      for (int q = threadIdx.x; q < nwb * DX; q += blockDim.x) {
        const int r = q / DX, x = q % DX;
        const TN u1 = U1[r * LDX + x];
        TN c1 = C1[r * LDX + x] * sig(u1);
        if (ctec) {
          const TN* ce = ctec + ((w0 + r) * 2 + 0) * 2 * DX;
          c1 += ce[x] * ssp2(u1) + ce[DX + x] * ssp3(u1);
        }
        C1[r * LDX + x] = c1;
      }
      __syncthreads();
      outer_mfma<TN, false>(Sv, LDX, DX, C1, LDX, DX, nwb, slot + pl.eW1, first);
      colsum_acc<TN>(C1, LDX, DX, nwb, slot + pl.eb1, first);
      gemm_mfma_wt<TN>(C1, LDX, nwb, DX, P + pl.eW1, DX, C2, LDX, false);  // d/d s
      __syncthreads();
      for (int q = threadIdx.x; q < R * DX; q += blockDim.x) {
        const int row = q / DX, x = q % DX;
        CX[row * LDX + x] = C2[(row / N) * LDX + x];
      }
      __syncthreads();
    }
    // ---- backflow head: f = 1 + kappa(x_i) ----
    gemm_mfma<TN>(X, LDX, R, DX, P + pl.kW1, DX, A, LDX, false, false);
    __syncthreads();
    for (int q = threadIdx.x; q < R * DX; q += blockDim.x) {
      const int r = q / DX, x = q % DX;
      A[r * LDX + x] += P[pl.kb1 + x];
      B[r * LDX + x] = ssp(A[r * LDX + x]);
    }
    __syncthreads();
    gemm_mfma<TN>(B, LDX, R, DX, P + pl.kW2, DX, Cb, LDX, false, false);
    __syncthreads();
    for (int q = threadIdx.x; q < R * DX; q += blockDim.x) Cb[(q / DX) * LDX + q % DX] += P[pl.kb2 + q % DX];
    __syncthreads();
    outer_acc_ssp<TN>(Cb, LDX, DX, CF, LDM, M, R, slot + pl.kW3, first);
    colsum_acc<TN>(CF, LDM, M, R, slot + pl.kb3, first);
    // d/d y2 = CF W3^T  (W3 is [DX][M]; rows of the transposed product are M long)
    for (int q = threadIdx.x; q < R * DX; q += blockDim.x) {
      const int r = q / DX, x = q % DX;
      TN s = 0;
      for (int mu = 0; mu < M; ++mu) s += CF[r * LDM + mu] * P[pl.kW3 + x * M + mu];
      const TN u2 = Cb[r * LDX + x];
      TN c2 = s * sig(u2);  // d/d u2
      if (ctkc) {
        const int64_t wl = w0 + r / N;
        const TN* ck = ctkc + (wl * 2 + 1) * 2 * N * DX + (r % N) * DX + x;
        c2 += ck[0] * ssp2(u2) + ck[N * DX] * ssp3(u2);
      }
      B[r * LDX + x] = c2;
    }
    __syncthreads();
    outer_mfma<TN, true>(A, LDX, DX, B, LDX, DX, R, slot + pl.kW2, first);
    colsum_acc<TN>(B, LDX, DX, R, slot + pl.kb2, first);
    gemm_mfma_wt<TN>(B, LDX, R, DX, P + pl.kW2, DX, Cb, LDX, false);
    __syncthreads();
    for (int q = threadIdx.x; q < R * DX; q += blockDim.x) {
      const int r = q / DX, x = q % DX;
      const TN u1 = A[r * LDX + x];
      TN c1 = Cb[r * LDX + x] * sig(u1);  // d/d u1
      if (ctkc) {
        const int64_t wl = w0 + r / N;
        const TN* ck = ctkc + (wl * 2 + 0) * 2 * N * DX + (r % N) * DX + x;
        c1 += ck[0] * ssp2(u1) + ck[N * DX] * ssp3(u1);
      }
      Cb[r * LDX + x] = c1;
    }
    __syncthreads();
    outer_mfma<TN, false>(X, LDX, DX, Cb, LDX, DX, R, slot + pl.kW1, first);
    colsum_acc<TN>(Cb, LDX, DX, R, slot + pl.kb1, first);
    gemm_mfma_wt<TN>(Cb, LDX, R, DX, P + pl.kW1, DX, CX, LDX, true);
    __syncthreads();
    // ---- interaction layers, last to first ----
    for (int n = L - 1; n >= 0; --n) {
      const ParamLayout::Layer& Lp = pl.layer[n];
      for (int q = threadIdx.x; q < R * DX; q += blockDim.x)
        X[(q / DX) * LDX + q % DX] = xval[((w0 + q / (N * DX)) * (L + 1) + n) * N * DX + q % (N * DX)];
      for (int q = threadIdx.x; q < R * DZ; q += blockDim.x) {
        H[(q / DZ) * LDZ + q % DZ] = hval[((w0 + q / (N * DZ)) * L + n) * N * DZ + q % (N * DZ)];
        // the tangent pass's cotangent of the h values seeds the h adjoint
        CH[(q / DZ) * LDZ + q % DZ] = cthv ? cthv[((w0 + q / (N * DZ)) * L + n) * N * DZ + q % (N * DZ)] : TN(0);
      }
      __syncthreads();
      for (int ch = 0; ch < 3; ++ch) {
        // recompute the messages of this channel
        for (int q = threadIdx.x; q < R * DZ; q += blockDim.x) {
          const int row = q / DZ, z = q % DZ, wl = row / N, i = row % N;
          const TN* fv = filt + (w0 + wl) * fl_stride * L + n * fl_stride;
          TN acc = 0;
          if (ch < 2) {
            const bool want_up = (ch == 0) == (i < NU);
            for (int j = want_up ? 0 : NU; j < (want_up ? NU : N); ++j) {
              if (j == i) continue;
              acc += fv[(int64_t)pidx[i * N + j] * DZ + z] * H[(wl * N + j) * LDZ + z];
            }
          } else {
            for (int I = 0; I < d.NN; ++I) acc += fv[(int64_t)(d.n_ee + i * d.NN + I) * DZ + z] * P[pl.Y + I * DZ + z];
          }
          Z[row * LDZ + z] = acc;
        }
        __syncthreads();
        outer_mfma<TN, false>(Z, LDZ, DZ, CX, LDX, DX, R, slot + Lp.gW[ch], first);
        colsum_acc<TN>(CX, LDX, DX, R, slot + Lp.gb[ch], first);
        gemm_mfma_wt<TN>(CX, LDX, R, DX, P + Lp.gW[ch], DZ, CZ, LDZ, false);  // d/d z
        __syncthreads();
        if (ch < 2) {
          // d/d h_j += sum_i w_ij d/d z_i ; filter cotangent per pair
          for (int q = threadIdx.x; q < R * DZ; q += blockDim.x) {
            const int row = q / DZ, z = q % DZ, wl = row / N, j = row % N;
            const TN* fv = filt + (w0 + wl) * fl_stride * L + n * fl_stride;
            const bool want_up = (ch == 0) == (j < NU);
            TN acc = 0;
            for (int i = want_up ? 0 : NU; i < (want_up ? NU : N); ++i) {
              if (i == j) continue;
              acc += fv[(int64_t)pidx[i * N + j] * DZ + z] * CZ[(wl * N + i) * LDZ + z];
            }
            CH[row * LDZ + z] += acc;
          }
          const int p_lo = ch == 0 ? 0 : (d.n_up * (d.n_up - 1) + d.n_dn * (d.n_dn - 1)) / 2;
          const int p_hi = ch == 0 ? p_lo + (d.n_up * (d.n_up - 1) + d.n_dn * (d.n_dn - 1)) / 2 : d.n_ee;
          for (int q = threadIdx.x; q < nwb * (p_hi - p_lo) * DZ; q += blockDim.x) {
            const int wl = q / ((p_hi - p_lo) * DZ), rem = q % ((p_hi - p_lo) * DZ);
            const int p = p_lo + rem / DZ, z = rem % DZ;
            const int i = t.pair_ij[2 * p], j = t.pair_ij[2 * p + 1];
            const TN v = CZ[(wl * N + i) * LDZ + z] * H[(wl * N + j) * LDZ + z] +
                         CZ[(wl * N + j) * LDZ + z] * H[(wl * N + i) * LDZ + z];
            ctw[(((w0 + wl) * L + n) * d.n_pairs + p) * DZ + z] = v;
          }
        } else {
          for (int q = threadIdx.x; q < nwb * N * d.NN * DZ; q += blockDim.x) {
            const int wl = q / (N * d.NN * DZ), rem = q % (N * d.NN * DZ);
            const int i = rem / (d.NN * DZ), I = (rem / DZ) % d.NN, z = rem % DZ;
            const int p = d.n_ee + i * d.NN + I;
            ctw[(((w0 + wl) * L + n) * d.n_pairs + p) * DZ + z] = CZ[(wl * N + i) * LDZ + z] * P[pl.Y + I * DZ + z];
          }
          {
            // d/d Y_I = sum over layers and electrons of w_iI d/d z_i (this layer's share)
            for (int q = threadIdx.x; q < d.NN * DZ; q += blockDim.x) {
              const int I = q / DZ, z = q % DZ;
              TN s = 0;
              for (int row = 0; row < R; ++row) {
                const int wl = row / N, i = row % N;
                const TN* fv = filt + (w0 + wl) * fl_stride * L + n * fl_stride;
                s += fv[(int64_t)(d.n_ee + i * d.NN + I) * DZ + z] * CZ[row * LDZ + z];
              }
              const bool wr = first && n == L - 1;
              slot[pl.Y + q] = wr ? s : slot[pl.Y + q] + s;
            }
          }
        }
        __syncthreads();
      }
      // h = x W_h + b_h
      outer_mfma<TN, false>(X, LDX, DX, CH, LDZ, DZ, R, slot + Lp.hW, first);
      colsum_acc<TN>(CH, LDZ, DZ, R, slot + Lp.hb, first);
      gemm_mfma_wt<TN>(CH, LDZ, R, DZ, P + Lp.hW, DX, CX, LDX, true);
      __syncthreads();
    }
    // x^(0) = x0 for every electron
    colsum_acc<TN>(CX, LDX, DX, R, slot + pl.x0, first);
  }
}

// JETS: the cotangents also reach the radial derivatives (w'/d and w'') of
// the filter outputs (full adjoint).  With the jets of the hidden layer
//   u = e W1 + b1, ud = (e'/d) W1, u2 = e'' W1,
//   a0 = ssp(u), a1 = s ud, a2 = s u2 + s' (d ud)^2   (s = ssp'(u), s' = ssp''(u))
//   w = a0 W2 + b2, w'/d = a1 W2, w'' = a2 W2
// the reverse is
//   ct a_k = ct w_k W2^T,  dW2 += sum_k a_k^T ct w_k,  db2 += ct w
//   ct u  = ct a0 s + ct a1 s' ud + ct a2 (s' u2 + s'' (d ud)^2)
//   ct ud = ct a1 s + 2 ct a2 s' d (d ud),   ct u2 = ct a2 s
//   dW1 += e^T ct u + (e'/d)^T ct ud + e''^T ct u2,  db1 += ct u.
template <typename TN, bool JETS, int PT>
__global__ __launch_bounds__(kThreads) void k_bwd_filter(Dims d, DevTables t, int64_t nw, const double* __restrict__ r,
                                                         const TN* __restrict__ P, ParamLayout pl,
                                                         const TN* __restrict__ ctw, const TN* __restrict__ ctww,
                                                         const TN* __restrict__ ctwd, const TN* __restrict__ ctw2,
                                                         TN* __restrict__ fslot, int n_same) {
  extern __shared__ __align__(16) char smem[];
  constexpr int NJ = JETS ? 3 : 1;
  const int layer = blockIdx.y / 3, ch = blockIdx.y % 3;
  const int K = d.K, DZ = d.DZ, L = d.L;
  const int LDK = ld_pad<TN>(K), LDZ = ld_pad<TN>(DZ);
  constexpr int RPG = PT / 4;  // rows of a tile per lane group of the MFMA reduction
  const int p_lo = ch == 0 ? 0 : (ch == 1 ? n_same : d.n_ee);
  const int p_hi = ch == 0 ? n_same : (ch == 1 ? d.n_ee : d.n_pairs);
  const int np = p_hi - p_lo;
  const int64_t nrows = nw * np;
  double* dd = reinterpret_cast<double*>(smem);  // [PT]
  TN* E = reinterpret_cast<TN*>(dd + PT);        // [NJ][PT][LDK] feature jets
  TN* U = E + NJ * PT * LDK;                     // [NJ][PT][LDZ] hidden jets, then activations
  TN* CW = U + NJ * PT * LDZ;                    // [NJ][PT][LDZ] d/d (w, w'/d, w'')
  TN* CU = CW + NJ * PT * LDZ;                   // [NJ][PT][LDZ] d/d activations, then d/d hidden jets
  const ParamLayout::Layer& Lp = pl.layer[layer];
  const int fsz = K * DZ + DZ + DZ * DZ + DZ;
  // weight gradients dW1 = sum_k E_k^T CU_k and dW2 = sum_k U_k^T CW_k on
  // the matrix cores: every wavefront keeps its 16 x 16 output tiles in
  // registers across all row tiles; the reduction runs over the PT rows of
  // a tile (32, or 16 where 32 would exceed the LDS).
  typedef typename MfmaTile<TN>::acc_t acc_t;
  constexpr int kMaxT = 8;  // tiles per wavefront: (K/16 + DZ/16) * DZ/16 <= 32
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, c16 = lane & 15;
  const int nz = DZ / 16, nt1 = (K / 16) * nz, nt = nt1 + nz * nz;
  acc_t accs[kMaxT];
#pragma unroll
  for (int k = 0; k < kMaxT; ++k)
#pragma unroll
    for (int v = 0; v < 4; ++v) accs[k][v] = 0;
  TN bacc1 = 0, bacc2 = 0;  // thread z < DZ owns db1[z], db2[z]
  for (int64_t row0 = (int64_t)blockIdx.x * PT; row0 < nrows; row0 += (int64_t)gridDim.x * PT) {
    const int rows = (int)min((int64_t)PT, nrows - row0);
    __syncthreads();
    for (int q = threadIdx.x; q < PT; q += blockDim.x) {
      double v = 1.0;
      if (q < rows) {
        const int64_t gq = row0 + q, w = gq / np;
        const int p = p_lo + (int)(gq % np);
        const double* rw = r + w * d.N * 3;
        double x, y, z;
        if (p < d.n_ee) {
          const int i = t.pair_ij[2 * p], j = t.pair_ij[2 * p + 1];
          x = rw[3 * i] - rw[3 * j];
          y = rw[3 * i + 1] - rw[3 * j + 1];
          z = rw[3 * i + 2] - rw[3 * j + 2];
        } else {
          const int q2 = p - d.n_ee, i = q2 / d.NN, I = q2 % d.NN;
          x = rw[3 * i] - t.nuc_xyz[3 * I];
          y = rw[3 * i + 1] - t.nuc_xyz[3 * I + 1];
          z = rw[3 * i + 2] - t.nuc_xyz[3 * I + 2];
        }
        v = sqrt(x * x + y * y + z * z);
      }
      dd[q] = v;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < PT * K; q += blockDim.x) {
      const int row = q / K, k = q % K;
      TN e0 = 0, e1 = 0, e2 = 0;
      if (row < rows) {
        const double dv = dd[row], dm = dv - t.feat_mu[k], sg = t.feat_sig2inv[k];
        const double eg = exp(-dv - dm * dm * sg);
        e0 = (TN)(dv * dv * eg);
        if (JETS) {
          const double g1 = -1.0 - 2.0 * dm * sg, g2 = -2.0 * sg;
          e1 = (TN)((2.0 + dv * g1) * eg);                                  // e'/d
          e2 = (TN)((2.0 + 4.0 * dv * g1 + dv * dv * (g1 * g1 + g2)) * eg);  // e''
        }
      }
      E[row * LDK + k] = e0;
      if (JETS) {
        E[(PT + row) * LDK + k] = e1;
        E[(2 * PT + row) * LDK + k] = e2;
      }
    }
    for (int q = threadIdx.x; q < PT * DZ; q += blockDim.x) {
      const int row = q / DZ, z = q % DZ;
      TN v0 = 0, v1 = 0, v2 = 0;
      if (row < rows) {
        const int64_t gq = row0 + row, w = gq / np;
        const int p = p_lo + (int)(gq % np);
        const int64_t o = ((w * L + layer) * d.n_pairs + p) * DZ + z;
        v0 = ctw[o];
        if (JETS) {
          if (p < d.n_ee) v0 += ctww[((w * L + layer) * d.n_ee + p) * DZ + z];
          v1 = ctwd[o];
          v2 = ctw2[o];
        }
      }
      CW[row * LDZ + z] = v0;
      if (JETS) {
        CW[(PT + row) * LDZ + z] = v1;
        CW[(2 * PT + row) * LDZ + z] = v2;
      }
    }
    __syncthreads();
    for (int jet = 0; jet < NJ; ++jet) {
      gemm_mfma<TN>(E + jet * PT * LDK, LDK, PT, K, P + Lp.w1W[ch], DZ, U + jet * PT * LDZ, LDZ, false, false);
      gemm_mfma_wt<TN>(CW + jet * PT * LDZ, LDZ, PT, DZ, P + Lp.w2W[ch], DZ, CU + jet * PT * LDZ, LDZ, false);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < PT * DZ; q += blockDim.x) {
      const int row = q / DZ, z = q % DZ;
      const bool ok = row < rows;
      TN* u0 = U + row * LDZ + z;
      TN* c0 = CU + row * LDZ + z;
      const TN u = u0[0] + P[Lp.w1b[ch] + z];
      const TN s = sig(u);
      if (!JETS) {
        c0[0] = ok ? c0[0] * s : TN(0);
        u0[0] = ok ? ssp(u) : TN(0);  // hidden activation (zero on padding rows)
      } else {
        const TN s1 = ssp2(u), s2 = ssp3(u), dv = (TN)dd[row];
        const TN ud = u0[PT * LDZ], u2 = u0[2 * PT * LDZ], up = dv * ud;
        const TN ca0 = c0[0], ca1 = c0[PT * LDZ], ca2 = c0[2 * PT * LDZ];
        c0[0] = ok ? ca0 * s + ca1 * s1 * ud + ca2 * (s1 * u2 + s2 * up * up) : TN(0);
        c0[PT * LDZ] = ok ? ca1 * s + TN(2) * ca2 * s1 * dv * up : TN(0);
        c0[2 * PT * LDZ] = ok ? ca2 * s : TN(0);
        u0[0] = ok ? ssp(u) : TN(0);
        u0[PT * LDZ] = ok ? s * ud : TN(0);
        u0[2 * PT * LDZ] = ok ? s * u2 + s1 * up * up : TN(0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kMaxT; ++k) {
      const int tt = wv + k * (kThreads / 64);
      if (tt < nt) {
#pragma unroll
        for (int jet = 0; jet < NJ; ++jet) {
          const TN* X;
          const TN* Y;
          int ldx2, a0, b0;
          if (tt < nt1) {
            X = E + jet * PT * LDK;
            ldx2 = LDK;
            Y = CU + jet * PT * LDZ;
            a0 = (tt / nz) * 16;
            b0 = (tt % nz) * 16;
          } else {
            X = U + jet * PT * LDZ;
            ldx2 = LDZ;
            Y = CW + jet * PT * LDZ;
            a0 = ((tt - nt1) / nz) * 16;
            b0 = ((tt - nt1) % nz) * 16;
          }
          TN af[RPG], bf[RPG];
#pragma unroll
          for (int s2 = 0; s2 < RPG; ++s2) {
            af[s2] = X[(g * RPG + s2) * ldx2 + a0 + c16];
            bf[s2] = Y[(g * RPG + s2) * LDZ + b0 + c16];
          }
          accs[k] = MfmaChain<TN, RPG>::run(af, bf, accs[k], false);
        }
      }
    }
    if (threadIdx.x < DZ) {
      for (int row = 0; row < rows; ++row) {
        bacc1 += CU[row * LDZ + threadIdx.x];
        bacc2 += CW[row * LDZ + threadIdx.x];
      }
    }
  }
  TN* out = fslot + ((size_t)blockIdx.x * L * 3 + blockIdx.y) * fsz;
  // layout of a filter block: [w1W K x DZ][w1b DZ][w2W DZ x DZ][w2b DZ]
#pragma unroll
  for (int k = 0; k < kMaxT; ++k) {
    const int tt = wv + k * (kThreads / 64);
    if (tt < nt) {
      const bool first_mat = tt < nt1;
      const int a0 = first_mat ? (tt / nz) * 16 : ((tt - nt1) / nz) * 16;
      const int b0 = first_mat ? (tt % nz) * 16 : ((tt - nt1) % nz) * 16;
      const int base = first_mat ? 0 : K * DZ + DZ;
#pragma unroll
      for (int v = 0; v < 4; ++v) out[base + (a0 + MfmaTile<TN>::row_of(lane, v)) * DZ + b0 + c16] = accs[k][v];
    }
  }
  if (threadIdx.x < DZ) {
    out[K * DZ + threadIdx.x] = bacc1;
    out[K * DZ + DZ + DZ * DZ + threadIdx.x] = bacc2;
  }
}

template <typename TN>
__global__ __launch_bounds__(kThreads) void k_bwd_reduce(Dims d, ParamLayout pl, int64_t n_params, int n_net,
                                                         const TN* __restrict__ gslot, int n_filt,
                                                         const TN* __restrict__ fslot, int n_tan,
                                                         const TN* __restrict__ tslot, double* __restrict__ grad) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_params) return;
  const int fsz = d.K * d.DZ + d.DZ + d.DZ * d.DZ + d.DZ;
  // is q inside a filter block?
  for (int n = 0; n < d.L; ++n) {
    const int64_t f0 = pl.layer[n].w1W[0];
    if (q >= f0 && q < f0 + 3 * fsz) {
      const int seg = n * 3 + (int)((q - f0) / fsz), o = (int)((q - f0) % fsz);
      double s = 0.0;
      for (int b = 0; b < n_filt; ++b) s += (double)fslot[((size_t)b * d.L * 3 + seg) * fsz + o];
      grad[q] += s;
      return;
    }
  }
  double s = 0.0;
  for (int b = 0; b < n_net; ++b) s += (double)gslot[(size_t)b * n_params + q];
  for (int b = 0; b < n_tan; ++b) s += (double)tslot[(size_t)b * n_params + q];
  grad[q] += s;
}

}  // namespace

// elements of k_bwd_net's union region (head buffers, or layer buffers)
template <typename TN>
static size_t bwd_net_union(const Dims& d, int WB) {
  const int LDX = ld_pad<TN>(d.DX), LDZ = ld_pad<TN>(d.DZ), LDM = ld_pad<TN>((d.M + 15) & ~15);
  const size_t RW = (size_t)WB * d.N;
  const size_t heads = 3 * RW * LDX + RW * LDM + 6 * (size_t)WB * LDX;  // kappa buffers, then the eta ones
  const size_t layers = 4 * RW * LDZ;
  return std::max(heads, layers);
}

// LDS of k_bwd_net; with `arena` the union region lives in global memory
template <typename TN>
static size_t bwd_net_lds(const Dims& d, int WB, bool arena = false) {
  const int LDX = ld_pad<TN>(d.DX);
  const size_t RW = (size_t)WB * d.N;
  return (size_t)((d.N * d.N + 3) & ~3) * sizeof(int) +
         ((size_t)((WB + 3) & ~3) + 2 * RW * LDX + (arena ? 0 : bwd_net_union<TN>(d, WB))) * sizeof(TN);
}

template <typename TN>
static int bwd_wb(const Dims& d) {
  int wb = std::max(1, 64 / d.N);
  while (wb > 1 && bwd_net_lds<TN>(d, wb) > 80 * 1024) --wb;
  return wb;
}

// k_bwd_net keeps its union region in a global arena when the whole block
// does not fit in LDS (the 30-electron system in FP64)
template <typename TN>
static bool bwd_net_arena(const Dims& d) {
  return bwd_net_lds<TN>(d, bwd_wb<TN>(d)) > 160 * 1024;
}

// rows per tile of k_bwd_filter: 32, or 16 when 32 exceed the LDS
static int bwd_filter_rows(const Dims& d, bool fp32, bool full) {
  const int nj = full ? 3 : 1;
  const size_t tn = fp32 ? sizeof(float) : sizeof(double);
  const size_t ldk = fp32 ? ld_pad<float>(d.K) : ld_pad<double>(d.K);
  const size_t ldz = fp32 ? ld_pad<float>(d.DZ) : ld_pad<double>(d.DZ);
  for (int pt = kFiltRows; pt >= 16; pt /= 2)
    if (pt * sizeof(double) + (size_t)nj * pt * (ldk + 3 * ldz) * tn <= 160 * 1024) return pt;
  return 16;
}

static size_t filt_fsz(const Dims& d) { return (size_t)d.K * d.DZ + d.DZ + (size_t)d.DZ * d.DZ + d.DZ; }

size_t backward_scratch_bytes(const pn_ctx* c, int64_t tile, bool fp32) {
  const Dims& d = c->d;
  const size_t tn = fp32 ? sizeof(float) : sizeof(double);
  size_t b = 0;
  b += (size_t)kSlotsNet * c->pl.total * tn;                       // net slots
  b += (size_t)kSlotsFilter * d.L * 3 * filt_fsz(d) * tn;          // filter slots
  b += (size_t)tile * d.L * d.n_pairs * d.DZ * tn;                 // filter cotangents
  const bool arena = fp32 ? bwd_net_arena<float>(d) : bwd_net_arena<double>(d);
  if (arena)
    b += (size_t)kSlotsNet * (fp32 ? bwd_net_union<float>(d, bwd_wb<float>(d)) : bwd_net_union<double>(d, bwd_wb<double>(d))) *
         tn;
  return b + 1024;
}

bool backward_supported(const pn_ctx* c, bool fp32) {
  const Dims& d = c->d;
  if ((d.K / 16 + d.DZ / 16) * (d.DZ / 16) > 8 * (kThreads / 64)) return false;  // accumulator tiles per wave
  size_t lds = fp32 ? bwd_net_lds<float>(d, bwd_wb<float>(d), bwd_net_arena<float>(d))
                    : bwd_net_lds<double>(d, bwd_wb<double>(d), bwd_net_arena<double>(d));
  return lds <= 160 * 1024;
}

template <typename TN>
static void run_backward(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const TN* P, const double* ct,
                         char* ws, const WsLayout& L, double* grad, bool full) {
  const Dims& d = c->d;
  const int64_t np = c->pl.total;
  TN* gslot = reinterpret_cast<TN*>(ws + L.gpart);
  TN* fslot = gslot + (size_t)kSlotsNet * np;
  TN* ctw = fslot + (size_t)kSlotsFilter * d.L * 3 * filt_fsz(d);
  const int WB = bwd_wb<TN>(d);
  const bool use_arena = bwd_net_arena<TN>(d);
  TN* arena = use_arena ? ctw + (size_t)L.tile * d.L * d.n_pairs * d.DZ : nullptr;
  const int64_t arena_elems = use_arena ? (int64_t)bwd_net_union<TN>(d, WB) : 0;
  const size_t lds = bwd_net_lds<TN>(d, WB, use_arena);
  if (lds > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bwd_net<TN>), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  const int64_t ng = (nw + WB - 1) / WB;
  const int nb_net = (int)std::min<int64_t>(ng, kSlotsNet);
  hipLaunchKernelGGL(k_bwd_net<TN>, dim3(nb_net), dim3(kThreads), lds, s, d, c->t, nw, WB, P, c->pl,
                     reinterpret_cast<const TN*>(ws + L.xval), reinterpret_cast<const TN*>(ws + L.hval),
                     reinterpret_cast<const TN*>(ws + L.filt), reinterpret_cast<const double*>(ws + L.phi),
                     reinterpret_cast<const double*>(ws + L.ginv), reinterpret_cast<const double*>(ws + L.wdet), ct,
                     ctw, gslot, np, full ? reinterpret_cast<const double*>(ws + L.ctfpart) : nullptr, L.n_chunks,
                     full ? reinterpret_cast<const TN*>(ws + L.cthv) : nullptr,
                     full ? reinterpret_cast<const TN*>(ws + L.ctkc) : nullptr,
                     full ? reinterpret_cast<const TN*>(ws + L.ctec) : nullptr, arena, arena_elems);
  const int n_same = d.n_up * (d.n_up - 1) / 2 + d.n_dn * (d.n_dn - 1) / 2;
  const int64_t max_np = std::max<int64_t>(std::max(n_same, d.n_ee - n_same), (int64_t)d.N * d.NN);
  const int PT = bwd_filter_rows(d, sizeof(TN) == sizeof(float), full);
  const int nb_f = (int)std::min<int64_t>((nw * max_np + PT - 1) / PT, kSlotsFilter);
  const int nj = full ? 3 : 1;
  const size_t lds_f = PT * sizeof(double) + (size_t)nj * PT * (ld_pad<TN>(d.K) + 3 * ld_pad<TN>(d.DZ)) * sizeof(TN);
  auto filt_kernel = PT == 32 ? (full ? &k_bwd_filter<TN, true, 32> : &k_bwd_filter<TN, false, 32>)
                              : (full ? &k_bwd_filter<TN, true, 16> : &k_bwd_filter<TN, false, 16>);
  if (lds_f > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(filt_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_f);
  hipLaunchKernelGGL(filt_kernel, dim3(nb_f, d.L * 3), dim3(kThreads), lds_f, s, d, c->t, nw, r, P, c->pl, ctw,
                     full ? reinterpret_cast<const TN*>(ws + L.ctww) : nullptr,
                     full ? reinterpret_cast<const TN*>(ws + L.ctwd) : nullptr,
                     full ? reinterpret_cast<const TN*>(ws + L.ctw2) : nullptr, fslot, n_same);
  const int n_tan = full ? (int)std::min<int64_t>(nw, kSlotsTanAdj) : 0;
  hipLaunchKernelGGL(k_bwd_reduce<TN>, dim3((unsigned)((np + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, d,
                     c->pl, np, nb_net, gslot, nb_f, fslot, n_tan, full ? reinterpret_cast<const TN*>(ws + L.tslot) : nullptr,
                     grad);
}

void launch_backward(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const void* P, bool fp32, bool bf16,
                     const double* ct, char* ws, const WsLayout& L, double* grad_params, bool full) {
  (void)bf16;
  if (fp32)
    run_backward<float>(c, s, nw, r, static_cast<const float*>(P), ct, ws, L, grad_params, full);
  else
    run_backward<double>(c, s, nw, r, static_cast<const double*>(P), ct, ws, L, grad_params, full);
}

size_t backward_filter_lds_bytes(const Dims& d, bool fp32, bool full) {
  const int nj = full ? 3 : 1;
  const size_t tn = fp32 ? sizeof(float) : sizeof(double);
  const size_t ldk = fp32 ? ld_pad<float>(d.K) : ld_pad<double>(d.K);
  const size_t ldz = fp32 ? ld_pad<float>(d.DZ) : ld_pad<double>(d.DZ);
  const int pt = bwd_filter_rows(d, fp32, full);
  return pt * sizeof(double) + (size_t)nj * pt * (ldk + 3 * ldz) * tn;
}

}  // namespace pn
