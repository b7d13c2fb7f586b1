// SchNet-style interaction layers and the Jastrow / backflow heads
// (Methods, "PauliNet extension of SchNet"; Results, J = eta(sum_i x_i),
// f_i = kappa(x_i)), in two passes:
//
//  value pass   (k_net_value)   one block per group of walkers; computes the
//               activations and stores what the tangent pass needs: h^(n)
//               values and the ssp'(u), ssp''(u) of every head hidden unit.
//
//  tangent pass (k_net_tangent, in k_tangent.hip) one block per (walker,
//               coordinate chunk), using what the value pass stored.
#include "gemm_lds.h"
#include "mfma_gemm.h"
#include "pn_internal.h"

namespace pn {
namespace {

// ---------------------------------------------------------------- values --
template <typename TN>
__global__ __launch_bounds__(kThreads) void k_net_value(Dims d, DevTables t, int64_t nw, int WPB,
                                                        const TN* __restrict__ P, ParamLayout pl,
                                                        const TN* __restrict__ filt, TN* __restrict__ hval,
                                                        TN* __restrict__ kcoef, TN* __restrict__ ecoef,
                                                        double* __restrict__ fval, double* __restrict__ jval,
                                                        TN* __restrict__ xval, bool bf16) {
  extern __shared__ __align__(16) char smem[];
  const int N = d.N, DX = d.DX, DZ = d.DZ, M = d.M;
  const int64_t w0 = (int64_t)blockIdx.x * WPB;
  const int nwb = (int)min((int64_t)WPB, nw - w0);
  if (nwb <= 0) return;
  const int R = nwb * N;
  const int LDX = ld_pad<TN>(DX), LDW = ld_pad<TN>(max(DX, DZ));
  int* pidx = reinterpret_cast<int*>(smem);                      // [N][N]
  TN* X = reinterpret_cast<TN*>(pidx + ((N * N + 3) & ~3));      // [WPB*N][LDX]
  TN* H = X + WPB * N * LDX;                                     // [WPB*N][LDW]
  TN* Z = H + WPB * N * LDW;                                     // [WPB*N][LDW]
  TN* E = Z + WPB * N * LDW;                                     // [2][WPB][LDX] Jastrow scratch
  const int64_t fl_stride = (int64_t)3 * d.n_pairs * DZ;  // per layer
  const int64_t fw_stride = fl_stride * d.L;               // per walker

  for (int q = threadIdx.x; q < N * N; q += blockDim.x) pidx[q] = t.pair_index[q];
  for (int q = threadIdx.x; q < R * DX; q += blockDim.x) X[(q / DX) * LDX + q % DX] = P[pl.x0 + q % DX];
  __syncthreads();
  for (int n = 0; n < d.L; ++n) {
    const ParamLayout::Layer& Lp = pl.layer[n];
    if (xval)
      for (int q = threadIdx.x; q < R * DX; q += blockDim.x)
        xval[((w0 + q / (N * DX)) * (d.L + 1) + n) * N * DX + q % (N * DX)] = X[(q / DX) * LDX + q % DX];
    gemm_mfma<TN>(X, LDX, R, DX, P + Lp.hW, DZ, H, LDW, false, bf16);
    __syncthreads();
    for (int q = threadIdx.x; q < R * DZ; q += blockDim.x) {
      const int row = q / DZ, z = q % DZ;
      TN v = H[row * LDW + z] + P[Lp.hb + z];
      H[row * LDW + z] = v;
      hval[((w0 + row / N) * d.L + n) * N * DZ + (row % N) * DZ + z] = v;
    }
    __syncthreads();
    for (int ch = 0; ch < 3; ++ch) {
      for (int q = threadIdx.x; q < R * DZ; q += blockDim.x) {
        const int row = q / DZ, z = q % DZ, wl = row / N, i = row % N;
        const TN* fw = filt + (w0 + wl) * fw_stride + n * fl_stride;  // jet 0 = value
        TN acc = 0;
        if (ch < 2) {
          // electrons of this channel: same spin (ch 0) or opposite spin
          // (ch 1); j = i contributes w = 0.  Four partners per step, their
          // global and LDS reads issued before the products.
          const bool want_up = (ch == 0) == (i < d.n_up);
          const int j_lo = want_up ? 0 : d.n_up, j_hi = want_up ? d.n_up : N;
          const TN* hw = H + (size_t)wl * N * LDW + z;
          for (int j = j_lo; j < j_hi; j += 4) {
            TN wv[4], hv[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int jj = min(j + k, j_hi - 1);
              wv[k] = fw[(int64_t)max(pidx[i * N + jj], 0) * DZ + z];
              hv[k] = hw[(size_t)jj * LDW];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < 4; ++k) acc += (j + k < j_hi && j + k != i) ? wv[k] * hv[k] : TN(0);
          }
        } else {
          for (int I = 0; I < d.NN; I += 4) {
            TN wv[4], yv[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int II = min(I + k, d.NN - 1);
              wv[k] = fw[(int64_t)(d.n_ee + i * d.NN + II) * DZ + z];
              yv[k] = P[pl.Y + II * DZ + z];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < 4; ++k) acc += I + k < d.NN ? wv[k] * yv[k] : TN(0);
          }
        }
        Z[row * LDW + z] = acc;
      }
      __syncthreads();
      gemm_mfma<TN>(Z, LDW, R, DZ, P + Lp.gW[ch], DX, X, LDX, true, bf16);
      __syncthreads();
    }
    // the three channels' biases, added once
    for (int q = threadIdx.x; q < R * DX; q += blockDim.x) {
      const int x = q % DX;
      X[(q / DX) * LDX + x] += P[Lp.gb[0] + x] + P[Lp.gb[1] + x] + P[Lp.gb[2] + x];
    }
    __syncthreads();
  }
  if (xval)
    for (int q = threadIdx.x; q < R * DX; q += blockDim.x)
      xval[((w0 + q / (N * DX)) * (d.L + 1) + d.L) * N * DX + q % (N * DX)] = X[(q / DX) * LDX + q % DX];
  // ---- Jastrow head on s = sum_i x_i (rows = walkers) ----
  TN* S = E;                // [WPB][LDX]
  TN* U = E + WPB * LDX;    // [WPB][LDX]
  if (d.flags & PN_NET_NO_JASTROW) {
    for (int wl = threadIdx.x; wl < nwb; wl += blockDim.x) jval[w0 + wl] = 0.0;
  } else {
    for (int q = threadIdx.x; q < nwb * DX; q += blockDim.x) {
      int wl = q / DX, x = q % DX;
      TN s = 0;
      for (int i = 0; i < N; ++i) s += X[(wl * N + i) * LDX + x];
      S[wl * LDX + x] = s;
    }
    __syncthreads();
    for (int lay = 0; lay < 2; ++lay) {
      gemm_mfma<TN>(S, LDX, nwb, DX, P + (lay == 0 ? pl.eW1 : pl.eW2), DX, U, LDX, false, bf16);
      __syncthreads();
      for (int q = threadIdx.x; q < nwb * DX; q += blockDim.x) {
        int wl = q / DX, x = q % DX;
        TN u = U[wl * LDX + x] + P[(lay == 0 ? pl.eb1 : pl.eb2) + x];
        TN sg = sigmoid_d(u);
        ecoef[((w0 + wl) * 2 + lay) * 2 * DX + x] = sg;
        ecoef[((w0 + wl) * 2 + lay) * 2 * DX + DX + x] = sg * (TN(1) - sg);
        S[wl * LDX + x] = ssp(u);
      }
      __syncthreads();
    }
    for (int wl = threadIdx.x; wl < nwb; wl += blockDim.x) {
      TN acc = P[pl.eb3];
      for (int x = 0; x < DX; ++x) acc += maybe_bf16(S[wl * LDX + x], bf16) * maybe_bf16(P[pl.eW3 + x], bf16);
      jval[w0 + wl] = (double)acc;
    }
  }
  __syncthreads();
  if (d.flags & PN_NET_NO_BACKFLOW) {
    for (int q = threadIdx.x; q < R * M; q += blockDim.x) fval[(w0 + q / (N * M)) * N * M + q % (N * M)] = 1.0;
    return;
  }
  // ---- backflow head, per electron row ----
  gemm_mfma<TN>(X, LDX, R, DX, P + pl.kW1, DX, H, LDW, false, bf16);
  __syncthreads();
  for (int q = threadIdx.x; q < R * DX; q += blockDim.x) {
    int row = q / DX, x = q % DX;
    TN u = H[row * LDW + x] + P[pl.kb1 + x];
    TN sg = sigmoid_d(u);
    kcoef[(((w0 + row / N) * 2 + 0) * 2 + 0) * N * DX + (row % N) * DX + x] = sg;
    kcoef[(((w0 + row / N) * 2 + 0) * 2 + 1) * N * DX + (row % N) * DX + x] = sg * (TN(1) - sg);
    H[row * LDW + x] = ssp(u);
  }
  __syncthreads();
  gemm_mfma<TN>(H, LDW, R, DX, P + pl.kW2, DX, X, LDX, false, bf16);
  __syncthreads();
  for (int q = threadIdx.x; q < R * DX; q += blockDim.x) {
    int row = q / DX, x = q % DX;
    TN u = X[row * LDX + x] + P[pl.kb2 + x];
    TN sg = sigmoid_d(u);
    kcoef[(((w0 + row / N) * 2 + 1) * 2 + 0) * N * DX + (row % N) * DX + x] = sg;
    kcoef[(((w0 + row / N) * 2 + 1) * 2 + 1) * N * DX + (row % N) * DX + x] = sg * (TN(1) - sg);
    X[row * LDX + x] = ssp(u);
  }
  __syncthreads();
  gemm_mfma_cols<TN>(X, LDX, R, DX, P + pl.kW3, M, H, LDW, false, bf16);
  __syncthreads();
  for (int q = threadIdx.x; q < R * M; q += blockDim.x) {
    int row = q / M, mu = q % M;
    fval[(w0 + row / N) * N * M + (row % N) * M + mu] = 1.0 + (double)(H[row * LDW + mu] + P[pl.kb3 + mu]);
  }
}

}  // namespace

template <typename TN>
void launch_net_value(const pn_ctx* c, hipStream_t s, int64_t nw, const TN* P, char* ws, const WsLayout& L,
                      bool bf16) {
  const Dims& d = c->d;
  int64_t nb = (nw + L.wpb_value - 1) / L.wpb_value;
  if (L.lds_value > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_net_value<TN>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_value);
  hipLaunchKernelGGL(k_net_value<TN>, dim3((unsigned)nb), dim3(kThreads), L.lds_value, s, d, c->t, nw, L.wpb_value,
                     P, c->pl, reinterpret_cast<const TN*>(ws + L.filt), reinterpret_cast<TN*>(ws + L.hval),
                     reinterpret_cast<TN*>(ws + L.kcoef), reinterpret_cast<TN*>(ws + L.ecoef),
                     reinterpret_cast<double*>(ws + L.fval), reinterpret_cast<double*>(ws + L.jval),
                     L.xval ? reinterpret_cast<TN*>(ws + L.xval) : nullptr, bf16);
}

template <typename TN>
size_t value_lds_bytes(const Dims& d, int wpb) {
  const int LDX = ld_pad<TN>(d.DX), LDW = ld_pad<TN>(std::max(d.DX, d.DZ));
  return (size_t)((d.N * d.N + 3) & ~3) * sizeof(int) +
         ((size_t)wpb * d.N * (LDX + 2 * LDW) + 2 * (size_t)wpb * LDX) * sizeof(TN);
}

template void launch_net_value<double>(const pn_ctx*, hipStream_t, int64_t, const double*, char*, const WsLayout&,
                                       bool);
template void launch_net_value<float>(const pn_ctx*, hipStream_t, int64_t, const float*, char*, const WsLayout&,
                                      bool);
template size_t value_lds_bytes<double>(const Dims&, int);
template size_t value_lds_bytes<float>(const Dims&, int);

}  // namespace pn
