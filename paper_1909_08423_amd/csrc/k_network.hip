// SchNet-style interaction layers and the Jastrow / backflow heads
// (Methods, "PauliNet extension of SchNet"; Results, J = eta(sum_i x_i),
// f_i = kappa(x_i)), in two passes:
//
//  value pass   (k_net_value)   one block per group of walkers; computes the
//               activations and stores what the tangent pass needs: h^(n)
//               values and the ssp'(u), ssp''(u) of every head hidden unit.
//
//  tangent pass (k_net_tangent) one block per (walker, coordinate chunk).
//               A chunk is a range of T electron coordinates a; the block
//               carries, for every electron row i, the T first derivatives
//               d x_i / d r_a and one extra column holding the partial
//               Laplacian sum_{a in chunk} d^2 x_i / d r_a^2.  All maps are
//               applied per coordinate, so chunks are independent and the
//               partial Laplacians add up to the full one.
//
// Update rules per coordinate a (values come from the value pass):
//   Linear  y = x W + b           ->  y_a = x_a W,       y_L = x_L W
//   ssp     y = ssp(u)            ->  y_a = ssp'(u) u_a, y_L = ssp'(u) u_L
//                                                          + ssp''(u) sum_a u_a^2
//   message z_i = sum_j w_ij h_j  ->  z_a = sum_j (w_ij h_{j,a} + d_a w_ij h_j)
//           z_L = sum_j (w_ij h_{j,L} + sum_a (d2_a w_ij h_j + 2 d_a w_ij h_{j,a}))
// with d_a w_ij = (w'/d)(r_i - r_j)_a (delta_ik - delta_jk) for a = (k, alpha)
// and d2_a w_ij = w'' u_a^2 + (w'/d)(1 - u_a^2), u = (r_i - r_j) / d_ij, for
// k in {i, j}.
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
        int row = q / DZ, z = q % DZ, wl = row / N, i = row % N;
        const TN* fw = filt + (w0 + wl) * fw_stride + n * fl_stride;  // jet 0 = value
        TN acc = 0;
        if (ch < 2) {
          bool up_i = i < d.n_up;
          for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            bool same = (j < d.n_up) == up_i;
            if (same != (ch == 0)) continue;
            int p = pidx[i * N + j];
            acc += fw[(int64_t)p * DZ + z] * H[(wl * N + j) * LDW + z];
          }
        } else {
          for (int I = 0; I < d.NN; ++I) {
            int p = d.n_ee + i * d.NN + I;
            acc += fw[(int64_t)p * DZ + z] * P[pl.Y + I * DZ + z];
          }
        }
        Z[row * LDW + z] = acc;
      }
      __syncthreads();
      gemm_mfma<TN>(Z, LDW, R, DZ, P + Lp.gW[ch], DX, X, LDX, true, bf16);
      __syncthreads();
      for (int q = threadIdx.x; q < R * DX; q += blockDim.x) X[(q / DX) * LDX + q % DX] += P[Lp.gb[ch] + q % DX];
      __syncthreads();
    }
  }
  if (xval)
    for (int q = threadIdx.x; q < R * DX; q += blockDim.x)
      xval[((w0 + q / (N * DX)) * (d.L + 1) + d.L) * N * DX + q % (N * DX)] = X[(q / DX) * LDX + q % DX];
  // ---- Jastrow head on s = sum_i x_i (rows = walkers) ----
  TN* S = E;                // [WPB][LDX]
  TN* U = E + WPB * LDX;    // [WPB][LDX]
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
  __syncthreads();
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

// -------------------------------------------------------------- tangents --
constexpr int kCMax = 16;  // columns per chunk (T + 1) held in registers

template <typename TN>
__global__ __launch_bounds__(kThreads) void k_net_tangent(Dims d, DevTables t, int64_t nw, int T, int n_chunks,
                                                          const double* __restrict__ r, const TN* __restrict__ P,
                                                          ParamLayout pl, const TN* __restrict__ filt,
                                                          const TN* __restrict__ hval, const TN* __restrict__ kcoef,
                                                          const TN* __restrict__ ecoef, double* __restrict__ ftan,
                                                          double* __restrict__ jtan, bool bf16) {
  extern __shared__ __align__(16) char smem[];
  // XCD-aware order: blocks b, b+8, ... run on one XCD; keep a walker's chunks there.
  const int64_t nb = (int64_t)gridDim.x;
  const int64_t b = blockIdx.x;
  int64_t task;
  {
    const int64_t per = nb / 8, rem = nb % 8;
    const int64_t xcd = b % 8, slot = b / 8;
    task = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + slot;
  }
  const int64_t w = task / n_chunks;
  const int chunk = (int)(task % n_chunks);
  if (w >= nw) return;
  const int N = d.N, DX = d.DX, DZ = d.DZ, M = d.M;
  const int a0 = chunk * T;
  const int Tc = min(T, 3 * N - a0);
  const int C = Tc + 1;   // tangent columns + partial-Laplacian column
  const int LC = Tc;      // index of the Laplacian column
  const int R = N * C;    // rows: (electron i, column)
  const int e_lo = a0 / 3, e_hi = (a0 + Tc - 1) / 3;  // electrons with coordinates in the chunk
  const int LDX = ld_pad<TN>(DX), LDZ = ld_pad<TN>(DZ), LDHZ = max(2 * LDZ, LDX);
  double* rs = reinterpret_cast<double*>(smem);             // [N][3]
  int* pidx = reinterpret_cast<int*>(rs + 3 * kMaxElec);    // [N][N]
  TN* hvs = reinterpret_cast<TN*>(pidx + ((N * N + 3) & ~3));  // [N][DZ]
  TN* XT = hvs + N * DZ;                                    // [R][LDX]
  TN* HT = XT + R * LDX;                                    // [R][LDZ]  (layers)
  TN* ZT = HT + R * LDZ;                                    // [R][LDZ]  (layers)
  TN* KT = HT;                                              // [R][LDX]  (backflow head, over HT and ZT)
  TN* ES = HT + R * LDHZ;                                   // [2][C][LDX] Jastrow scratch
  const int NCE = e_hi - e_lo + 1;
  TN* cg = ES + 2 * C * LDX;                                // [NCE][N][4]  r_i - r_k, 1/|r_i - r_k|
  TN* cgn = cg + NCE * N * 4;                               // [NCE][NN][4] r_k - R_I, 1/|r_k - R_I|
  const double* rw = r + w * N * 3;
  for (int q = threadIdx.x; q < 3 * N; q += blockDim.x) rs[q] = rw[q];
  for (int q = threadIdx.x; q < N * N; q += blockDim.x) pidx[q] = t.pair_index[q];
  for (int q = threadIdx.x; q < R * LDX; q += blockDim.x) XT[q] = 0;
  __syncthreads();
  for (int q = threadIdx.x; q < NCE * N; q += blockDim.x) {
    const int k = e_lo + q / N, i = q % N;
    const double ux = rs[3 * i] - rs[3 * k], uy = rs[3 * i + 1] - rs[3 * k + 1], uz = rs[3 * i + 2] - rs[3 * k + 2];
    const double dd = sqrt(ux * ux + uy * uy + uz * uz);
    cg[4 * q + 0] = (TN)ux;
    cg[4 * q + 1] = (TN)uy;
    cg[4 * q + 2] = (TN)uz;
    cg[4 * q + 3] = i == k ? TN(0) : (TN)(1.0 / dd);
  }
  for (int q = threadIdx.x; q < NCE * d.NN; q += blockDim.x) {
    const int k = e_lo + q / d.NN, I = q % d.NN;
    const double ux = rs[3 * k] - t.nuc_xyz[3 * I], uy = rs[3 * k + 1] - t.nuc_xyz[3 * I + 1],
                 uz = rs[3 * k + 2] - t.nuc_xyz[3 * I + 2];
    cgn[4 * q + 0] = (TN)ux;
    cgn[4 * q + 1] = (TN)uy;
    cgn[4 * q + 2] = (TN)uz;
    cgn[4 * q + 3] = (TN)(1.0 / sqrt(ux * ux + uy * uy + uz * uz));
  }
  __syncthreads();
  const int64_t fl_stride = (int64_t)3 * d.n_pairs * DZ;
  for (int n = 0; n < d.L; ++n) {
    const ParamLayout::Layer& Lp = pl.layer[n];
    const TN* fw = filt + w * fl_stride * d.L + n * fl_stride;
    const TN* fv = fw;                                 // w
    const TN* fd = fw + (int64_t)d.n_pairs * DZ;       // w'/d
    const TN* f2 = fw + (int64_t)2 * d.n_pairs * DZ;   // w''
    const TN* hv = hval + (w * d.L + n) * N * DZ;
    for (int q = threadIdx.x; q < N * DZ; q += blockDim.x) hvs[q] = hv[q];
    if (n > 0) gemm_mfma<TN>(XT, LDX, R, DX, P + Lp.hW, DZ, HT, LDZ, false, bf16);
    __syncthreads();
    for (int ch = 0; ch < 2; ++ch) {
      for (int q = threadIdx.x; q < N * DZ; q += blockDim.x) {
        const int i = q / DZ, z = q % DZ;
        const bool up_i = i < d.n_up;
        TN acc[kCMax];
#pragma unroll
        for (int c = 0; c < kCMax; ++c) acc[c] = 0;
        if (n > 0) {
          for (int j = 0; j < N; ++j) {
            if (j == i || (((j < d.n_up) == up_i) != (ch == 0))) continue;
            const TN wv = fv[(int64_t)pidx[i * N + j] * DZ + z];
            const TN* hj = HT + (size_t)j * C * LDZ + z;
#pragma unroll
            for (int c = 0; c < kCMax; ++c)
              if (c < C) acc[c] += wv * hj[c * LDZ];
          }
        }
        TN* zi = ZT + (size_t)i * C * LDZ + z;
#pragma unroll
        for (int c = 0; c < kCMax; ++c)
          if (c < C) zi[c * LDZ] = acc[c];
        // derivatives of the filters with respect to the chunk's coordinates
        TN lap = 0;
        if (i >= e_lo && i <= e_hi) {
          const TN* gi = cg + (size_t)(i - e_lo) * N * 4;  // r_j - r_i
          for (int al = 0; al < 3; ++al) {
            const int c = 3 * i + al - a0;
            if (c < 0 || c >= Tc) continue;
            TN sv = 0;
            for (int j = 0; j < N; ++j) {
              if (j == i || (((j < d.n_up) == up_i) != (ch == 0))) continue;
              const int64_t p = pidx[i * N + j];
              const TN ua = -gi[4 * j + al];  // (r_i - r_j)_alpha
              const TN ur = ua * gi[4 * j + 3];
              const TN wd = fd[p * DZ + z], w2 = f2[p * DZ + z];
              const TN dw = wd * ua;
              const TN hj = hvs[j * DZ + z];
              sv += dw * hj;
              lap += (w2 * ur * ur + wd * (TN(1) - ur * ur)) * hj;
              if (n > 0) lap += TN(2) * dw * HT[((size_t)j * C + c) * LDZ + z];
            }
            zi[c * LDZ] += sv;
          }
        }
        for (int k = e_lo; k <= e_hi; ++k) {
          if (k == i || (((k < d.n_up) == up_i) != (ch == 0))) continue;
          const int64_t p = pidx[i * N + k];
          const TN* gk = cg + ((size_t)(k - e_lo) * N + i) * 4;  // r_i - r_k
          const TN wd = fd[p * DZ + z], w2 = f2[p * DZ + z];
          const TN hk = hvs[k * DZ + z];
          for (int al = 0; al < 3; ++al) {
            const int c = 3 * k + al - a0;
            if (c < 0 || c >= Tc) continue;
            const TN ua = gk[al];
            const TN ur = ua * gk[3];
            const TN dw = -wd * ua;  // d/dr_k of w(|r_i - r_k|)
            zi[c * LDZ] += dw * hk;
            lap += (w2 * ur * ur + wd * (TN(1) - ur * ur)) * hk;
            if (n > 0) lap += TN(2) * dw * HT[((size_t)k * C + c) * LDZ + z];
          }
        }
        zi[LC * LDZ] += lap;
      }
      __syncthreads();
      gemm_mfma<TN>(ZT, LDZ, R, DZ, P + Lp.gW[ch], DX, XT, LDX, true, bf16);
      __syncthreads();
    }
    // nuclear channel: only the chunk's own electrons have non-zero rows
    for (int q = threadIdx.x; q < (e_hi - e_lo + 1) * DZ; q += blockDim.x) {
      const int i = e_lo + q / DZ, z = q % DZ;
      TN* zi = ZT + (size_t)i * C * LDZ + z;
      for (int c = 0; c < C; ++c) zi[c * LDZ] = 0;
      TN lap = 0;
      for (int I = 0; I < d.NN; ++I) {
        const int64_t p = d.n_ee + i * d.NN + I;
        const TN* gn = cgn + ((size_t)(i - e_lo) * d.NN + I) * 4;
        const TN y = P[pl.Y + I * DZ + z];
        const TN wd = fd[p * DZ + z], w2 = f2[p * DZ + z];
        for (int al = 0; al < 3; ++al) {
          const int c = 3 * i + al - a0;
          if (c < 0 || c >= Tc) continue;
          const TN ua = gn[al];
          const TN ur = ua * gn[3];
          zi[c * LDZ] += wd * ua * y;
          lap += (w2 * ur * ur + wd * (TN(1) - ur * ur)) * y;
        }
      }
      zi[LC * LDZ] = lap;
    }
    __syncthreads();
    {
      const int row0 = e_lo * C, nrow = (e_hi - e_lo + 1) * C;
      gemm_mfma<TN>(ZT + (size_t)row0 * LDZ, LDZ, nrow, DZ, P + Lp.gW[2], DX, XT + (size_t)row0 * LDX, LDX, true,
                    bf16);
    }
    __syncthreads();
  }
  // ---- Jastrow head on sum_i x_i, rows = columns ----
  TN* S0 = ES;             // [C][LDX]
  TN* S1 = ES + C * LDX;   // [C][LDX]
  for (int q = threadIdx.x; q < C * DX; q += blockDim.x) {
    int col = q / DX, x = q % DX;
    TN s = 0;
    for (int i = 0; i < N; ++i) s += XT[((size_t)i * C + col) * LDX + x];
    S0[col * LDX + x] = s;
  }
  __syncthreads();
  for (int lay = 0; lay < 2; ++lay) {
    TN* Sin = lay == 0 ? S0 : S1;
    TN* Sout = lay == 0 ? S1 : S0;
    gemm_mfma<TN>(Sin, LDX, C, DX, P + (lay == 0 ? pl.eW1 : pl.eW2), DX, Sout, LDX, false, bf16);
    __syncthreads();
    const TN* ec = ecoef + (w * 2 + lay) * 2 * DX;
    for (int x = threadIdx.x; x < DX; x += blockDim.x) {
      TN s1 = ec[x], s2 = ec[DX + x];
      TN sq = 0;
      for (int col = 0; col < LC; ++col) {
        TN v = Sout[col * LDX + x];
        sq += v * v;
        Sout[col * LDX + x] = s1 * v;
      }
      Sout[LC * LDX + x] = s1 * Sout[LC * LDX + x] + s2 * sq;
    }
    __syncthreads();
  }
  double* jt = jtan + ((int64_t)w * n_chunks + chunk) * (T + 1);
  {
    // one wavefront per column: dot product with the output weights
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int col = wv; col < C; col += (int)(blockDim.x >> 6)) {
      TN acc = 0;
      for (int x = lane; x < DX; x += 64)
        acc += maybe_bf16(S0[col * LDX + x], bf16) * maybe_bf16(P[pl.eW3 + x], bf16);
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if (lane == 0) jt[col == LC ? T : col] = (double)acc;
    }
  }
  // ---- backflow head ----
  gemm_mfma<TN>(XT, LDX, R, DX, P + pl.kW1, DX, KT, LDX, false, bf16);
  __syncthreads();
  for (int lay = 0; lay < 2; ++lay) {
    TN* A = lay == 0 ? KT : XT;
    const int LDA = LDX;
    const TN* kc = kcoef + (w * 2 + lay) * 2 * N * DX;
    for (int q = threadIdx.x; q < N * DX; q += blockDim.x) {
      int i = q / DX, x = q % DX;
      TN s1 = kc[i * DX + x], s2 = kc[N * DX + i * DX + x];
      TN sq = 0;
      TN* ai = A + (size_t)i * C * LDA + x;
      for (int col = 0; col < LC; ++col) {
        TN v = ai[col * LDA];
        sq += v * v;
        ai[col * LDA] = s1 * v;
      }
      ai[LC * LDA] = s1 * ai[LC * LDA] + s2 * sq;
    }
    __syncthreads();
    if (lay == 0) {
      gemm_mfma<TN>(KT, LDX, R, DX, P + pl.kW2, DX, XT, LDX, false, bf16);
      __syncthreads();
    }
  }
  gemm_mfma_cols<TN>(XT, LDX, R, DX, P + pl.kW3, M, KT, LDX, false, bf16);
  __syncthreads();
  double* ft = ftan + ((int64_t)w * n_chunks + chunk) * N * (T + 1) * M;
  for (int q = threadIdx.x; q < R * M; q += blockDim.x) {
    int row = q / M, mu = q % M, i = row / C, col = row % C;
    ft[((int64_t)i * (T + 1) + (col == LC ? T : col)) * M + mu] = (double)KT[(size_t)row * LDX + mu];
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
void launch_net_tangent(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const TN* P, char* ws,
                        const WsLayout& L, bool bf16) {
  const Dims& d = c->d;
  int64_t nb = nw * L.n_chunks;
  if (L.lds_tangent > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_net_tangent<TN>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_tangent);
  hipLaunchKernelGGL(k_net_tangent<TN>, dim3((unsigned)nb), dim3(kThreads), L.lds_tangent, s, d, c->t, nw, L.T,
                     L.n_chunks, r, P, c->pl, reinterpret_cast<const TN*>(ws + L.filt),
                     reinterpret_cast<const TN*>(ws + L.hval), reinterpret_cast<const TN*>(ws + L.kcoef),
                     reinterpret_cast<const TN*>(ws + L.ecoef), reinterpret_cast<double*>(ws + L.ftan),
                     reinterpret_cast<double*>(ws + L.jtan), bf16);
}

template <typename TN>
size_t tangent_lds_bytes(const Dims& d, int T) {
  const int C = T + 1, R = d.N * C;
  const int LDX = ld_pad<TN>(d.DX), LDZ = ld_pad<TN>(d.DZ), LDHZ = std::max(2 * LDZ, LDX);
  const int NCE = std::min(d.N, T / 3 + 2);  // electrons a chunk of T coordinates can touch
  return 3 * kMaxElec * sizeof(double) + (size_t)((d.N * d.N + 3) & ~3) * sizeof(int) +
         ((size_t)d.N * d.DZ + (size_t)R * (LDX + LDHZ) + 2 * (size_t)C * LDX + (size_t)NCE * (d.N + d.NN) * 4) *
             sizeof(TN);
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
template void launch_net_tangent<double>(const pn_ctx*, hipStream_t, int64_t, const double*, const double*, char*,
                                         const WsLayout&, bool);
template void launch_net_tangent<float>(const pn_ctx*, hipStream_t, int64_t, const double*, const float*, char*,
                                        const WsLayout&, bool);
template size_t tangent_lds_bytes<double>(const Dims&, int);
template size_t tangent_lds_bytes<float>(const Dims&, int);
template size_t value_lds_bytes<double>(const Dims&, int);
template size_t value_lds_bytes<float>(const Dims&, int);

}  // namespace pn
