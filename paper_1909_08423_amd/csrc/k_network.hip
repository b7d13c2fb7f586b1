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
  const int DW = max(DX, DZ);
  TN* X = reinterpret_cast<TN*>(smem);  // [WPB*N][DX]
  TN* H = X + WPB * N * DX;              // [WPB*N][DW]
  TN* Z = H + WPB * N * DW;              // [WPB*N][DW]
  TN* E = Z + WPB * N * DW;              // [2][WPB][DX] Jastrow scratch
  const int64_t fl_stride = (int64_t)3 * d.n_pairs * DZ;  // per layer
  const int64_t fw_stride = fl_stride * d.L;               // per walker

  for (int q = threadIdx.x; q < R * DX; q += blockDim.x) X[q] = P[pl.x0 + q % DX];
  __syncthreads();
  for (int n = 0; n < d.L; ++n) {
    const ParamLayout::Layer& Lp = pl.layer[n];
    if (xval)
      for (int q = threadIdx.x; q < R * DX; q += blockDim.x)
        xval[((w0 + q / (N * DX)) * (d.L + 1) + n) * N * DX + q % (N * DX)] = X[q];
    gemm_xw<TN>(X, DX, R, DX, P + Lp.hW, DZ, H, DZ, false, bf16);
    __syncthreads();
    for (int q = threadIdx.x; q < R * DZ; q += blockDim.x) {
      TN v = H[q] + P[Lp.hb + q % DZ];
      H[q] = v;
      int row = q / DZ;
      hval[((w0 + row / N) * d.L + n) * N * DZ + (row % N) * DZ + q % DZ] = v;
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
            int p = t.pair_index[i * N + j];
            acc += fw[(int64_t)p * DZ + z] * H[(wl * N + j) * DZ + z];
          }
        } else {
          for (int I = 0; I < d.NN; ++I) {
            int p = d.n_ee + i * d.NN + I;
            acc += fw[(int64_t)p * DZ + z] * P[pl.Y + I * DZ + z];
          }
        }
        Z[q] = acc;
      }
      __syncthreads();
      gemm_xw<TN>(Z, DZ, R, DZ, P + Lp.gW[ch], DX, X, DX, true, bf16);
      __syncthreads();
      for (int q = threadIdx.x; q < R * DX; q += blockDim.x) X[q] += P[Lp.gb[ch] + q % DX];
      __syncthreads();
    }
  }
  if (xval)
    for (int q = threadIdx.x; q < R * DX; q += blockDim.x)
      xval[((w0 + q / (N * DX)) * (d.L + 1) + d.L) * N * DX + q % (N * DX)] = X[q];
  // ---- Jastrow head on s = sum_i x_i (rows = walkers) ----
  TN* S = E;               // [WPB][DX]
  TN* U = E + WPB * DX;    // [WPB][DX]
  for (int q = threadIdx.x; q < nwb * DX; q += blockDim.x) {
    int wl = q / DX, x = q % DX;
    TN s = 0;
    for (int i = 0; i < N; ++i) s += X[(wl * N + i) * DX + x];
    S[q] = s;
  }
  __syncthreads();
  for (int lay = 0; lay < 2; ++lay) {
    gemm_xw<TN>(S, DX, nwb, DX, P + (lay == 0 ? pl.eW1 : pl.eW2), DX, U, DX, false, bf16);
    __syncthreads();
    for (int q = threadIdx.x; q < nwb * DX; q += blockDim.x) {
      int wl = q / DX, x = q % DX;
      TN u = U[q] + P[(lay == 0 ? pl.eb1 : pl.eb2) + x];
      TN sg = sigmoid_d(u);
      ecoef[((w0 + wl) * 2 + lay) * 2 * DX + x] = sg;
      ecoef[((w0 + wl) * 2 + lay) * 2 * DX + DX + x] = sg * (TN(1) - sg);
      S[q] = ssp(u);
    }
    __syncthreads();
  }
  for (int wl = threadIdx.x; wl < nwb; wl += blockDim.x) {
    TN acc = P[pl.eb3];
    for (int x = 0; x < DX; ++x) acc += maybe_bf16(S[wl * DX + x], bf16) * maybe_bf16(P[pl.eW3 + x], bf16);
    jval[w0 + wl] = (double)acc;
  }
  __syncthreads();
  // ---- backflow head, per electron row ----
  TN* A1 = H;  // [R][DX]
  gemm_xw<TN>(X, DX, R, DX, P + pl.kW1, DX, A1, DX, false, bf16);
  __syncthreads();
  for (int q = threadIdx.x; q < R * DX; q += blockDim.x) {
    int row = q / DX, x = q % DX;
    TN u = A1[q] + P[pl.kb1 + x];
    TN sg = sigmoid_d(u);
    kcoef[(((w0 + row / N) * 2 + 0) * 2 + 0) * N * DX + (row % N) * DX + x] = sg;
    kcoef[(((w0 + row / N) * 2 + 0) * 2 + 1) * N * DX + (row % N) * DX + x] = sg * (TN(1) - sg);
    A1[q] = ssp(u);
  }
  __syncthreads();
  gemm_xw<TN>(A1, DX, R, DX, P + pl.kW2, DX, X, DX, false, bf16);
  __syncthreads();
  for (int q = threadIdx.x; q < R * DX; q += blockDim.x) {
    int row = q / DX, x = q % DX;
    TN u = X[q] + P[pl.kb2 + x];
    TN sg = sigmoid_d(u);
    kcoef[(((w0 + row / N) * 2 + 1) * 2 + 0) * N * DX + (row % N) * DX + x] = sg;
    kcoef[(((w0 + row / N) * 2 + 1) * 2 + 1) * N * DX + (row % N) * DX + x] = sg * (TN(1) - sg);
    X[q] = ssp(u);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < R * M; q += blockDim.x) {
    int row = q / M, mu = q % M;
    TN acc = P[pl.kb3 + mu];
    const TN* xr = X + row * DX;
    for (int x = 0; x < DX; ++x) acc += maybe_bf16(xr[x], bf16) * maybe_bf16(P[pl.kW3 + x * M + mu], bf16);
    fval[(w0 + row / N) * N * M + (row % N) * M + mu] = 1.0 + (double)acc;
  }
}

// -------------------------------------------------------------- tangents --
struct ChunkInfo {
  int a0, T, C;  // first coordinate, coordinates in the chunk, columns = T + 1
};

template <typename TN>
__device__ __forceinline__ void pair_geom(const double* rs, int i, int j, double& d, double* u) {
  double x = rs[3 * i] - rs[3 * j], y = rs[3 * i + 1] - rs[3 * j + 1], z = rs[3 * i + 2] - rs[3 * j + 2];
  d = sqrt(x * x + y * y + z * z);
  u[0] = x;
  u[1] = y;
  u[2] = z;
}

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
  const int DW = max(DX, DZ);
  double* rs = reinterpret_cast<double*>(smem);  // [N][3]
  TN* XT = reinterpret_cast<TN*>(rs + 3 * kMaxElec);  // [R][DX]
  TN* HT = XT + R * DX;                                 // [R][DW]
  TN* ZT = HT + R * DW;                                 // [R][DZ]
  TN* ES = ZT + R * DZ;                                 // [3][C][DX] Jastrow scratch
  const double* rw = r + w * N * 3;
  for (int q = threadIdx.x; q < 3 * N; q += blockDim.x) rs[q] = rw[q];
  for (int q = threadIdx.x; q < R * DX; q += blockDim.x) XT[q] = 0;
  __syncthreads();
  const int64_t fl_stride = (int64_t)3 * d.n_pairs * DZ;
  for (int n = 0; n < d.L; ++n) {
    const ParamLayout::Layer& Lp = pl.layer[n];
    const TN* fw = filt + w * fl_stride * d.L + n * fl_stride;
    const TN* fv = fw;                              // w
    const TN* fd = fw + (int64_t)d.n_pairs * DZ;    // w'/d
    const TN* f2 = fw + (int64_t)2 * d.n_pairs * DZ;  // w''
    const TN* hv = hval + (w * d.L + n) * N * DZ;
    if (n > 0) {
      gemm_xw<TN>(XT, DX, R, DX, P + Lp.hW, DZ, HT, DZ, false, bf16);
    } else {
      for (int q = threadIdx.x; q < R * DZ; q += blockDim.x) HT[q] = 0;
    }
    __syncthreads();
    for (int ch = 0; ch < 3; ++ch) {
      for (int q = threadIdx.x; q < R * DZ; q += blockDim.x) {
        const int row = q / DZ, z = q % DZ, i = row / C, col = row % C;
        TN acc = 0;
        if (ch < 2) {
          const bool up_i = i < d.n_up;
          for (int j = 0; j < N; ++j) {
            if (j == i || (((j < d.n_up) == up_i) != (ch == 0))) continue;
            const int p = t.pair_index[i * N + j];
            acc += fv[(int64_t)p * DZ + z] * HT[(j * C + col) * DZ + z];
          }
          if (col < LC) {
            const int a = a0 + col, k = a / 3, al = a % 3;
            if (k == i) {
              for (int j = 0; j < N; ++j) {
                if (j == i || (((j < d.n_up) == up_i) != (ch == 0))) continue;
                const int p = t.pair_index[i * N + j];
                TN dx = (TN)(rs[3 * i + al] - rs[3 * j + al]);
                acc += fd[(int64_t)p * DZ + z] * dx * hv[j * DZ + z];
              }
            } else if (k != i && (((k < d.n_up) == up_i) == (ch == 0))) {
              const int p = t.pair_index[i * N + k];
              TN dx = (TN)(rs[3 * k + al] - rs[3 * i + al]);
              acc += fd[(int64_t)p * DZ + z] * dx * hv[k * DZ + z];
            }
          } else {
            // second-derivative and cross terms of the chunk's coordinates
            for (int c2 = 0; c2 < LC; ++c2) {
              const int a = a0 + c2, k = a / 3, al = a % 3;
              if (k == i) {
                for (int j = 0; j < N; ++j) {
                  if (j == i || (((j < d.n_up) == up_i) != (ch == 0))) continue;
                  const int p = t.pair_index[i * N + j];
                  double dd, u[3];
                  pair_geom<TN>(rs, i, j, dd, u);
                  double ua = u[al] / dd;
                  TN wd = fd[(int64_t)p * DZ + z], w2 = f2[(int64_t)p * DZ + z];
                  TN d2w = w2 * (TN)(ua * ua) + wd * (TN)(1.0 - ua * ua);
                  TN dw = wd * (TN)u[al];
                  acc += d2w * hv[j * DZ + z] + TN(2) * dw * HT[(j * C + c2) * DZ + z];
                }
              } else if (((k < d.n_up) == up_i) == (ch == 0)) {
                const int p = t.pair_index[i * N + k];
                double dd, u[3];
                pair_geom<TN>(rs, i, k, dd, u);
                double ua = u[al] / dd;
                TN wd = fd[(int64_t)p * DZ + z], w2 = f2[(int64_t)p * DZ + z];
                TN d2w = w2 * (TN)(ua * ua) + wd * (TN)(1.0 - ua * ua);
                TN dw = -wd * (TN)u[al];  // d/dr_k of d_ik
                acc += d2w * hv[k * DZ + z] + TN(2) * dw * HT[(k * C + c2) * DZ + z];
              }
            }
          }
        } else {
          // nuclear channel: only coordinates of electron i itself contribute
          for (int I = 0; I < d.NN; ++I) {
            const int p = d.n_ee + i * d.NN + I;
            double u[3] = {rs[3 * i] - t.nuc_xyz[3 * I], rs[3 * i + 1] - t.nuc_xyz[3 * I + 1],
                           rs[3 * i + 2] - t.nuc_xyz[3 * I + 2]};
            double dd = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            TN y = P[pl.Y + I * DZ + z];
            TN wd = fd[(int64_t)p * DZ + z];
            if (col < LC) {
              const int a = a0 + col, k = a / 3, al = a % 3;
              if (k == i) acc += wd * (TN)u[al] * y;
            } else {
              TN w2 = f2[(int64_t)p * DZ + z];
              for (int c2 = 0; c2 < LC; ++c2) {
                const int a = a0 + c2, k = a / 3, al = a % 3;
                if (k != i) continue;
                double ua = u[al] / dd;
                acc += (w2 * (TN)(ua * ua) + wd * (TN)(1.0 - ua * ua)) * y;
              }
            }
          }
        }
        ZT[q] = acc;
      }
      __syncthreads();
      gemm_xw<TN>(ZT, DZ, R, DZ, P + Lp.gW[ch], DX, XT, DX, true, bf16);
      __syncthreads();
    }
  }
  // ---- Jastrow head on sum_i x_i, rows = columns ----
  TN* S = ES;              // [C][DX]
  TN* U = ES + C * DX;     // [C][DX]
  for (int q = threadIdx.x; q < C * DX; q += blockDim.x) {
    int col = q / DX, x = q % DX;
    TN s = 0;
    for (int i = 0; i < N; ++i) s += XT[(i * C + col) * DX + x];
    S[q] = s;
  }
  __syncthreads();
  for (int lay = 0; lay < 2; ++lay) {
    gemm_xw<TN>(S, DX, C, DX, P + (lay == 0 ? pl.eW1 : pl.eW2), DX, U, DX, false, bf16);
    __syncthreads();
    const TN* ec = ecoef + (w * 2 + lay) * 2 * DX;
    for (int x = threadIdx.x; x < DX; x += blockDim.x) {
      TN s1 = ec[x], s2 = ec[DX + x];
      TN sq = 0;
      for (int col = 0; col < LC; ++col) {
        TN v = U[col * DX + x];
        sq += v * v;
        S[col * DX + x] = s1 * v;
      }
      S[LC * DX + x] = s1 * U[LC * DX + x] + s2 * sq;
    }
    __syncthreads();
  }
  double* jt = jtan + ((int64_t)w * n_chunks + chunk) * (T + 1);
  for (int col = threadIdx.x; col < C; col += blockDim.x) {
    TN acc = 0;
    for (int x = 0; x < DX; ++x) acc += maybe_bf16(S[col * DX + x], bf16) * maybe_bf16(P[pl.eW3 + x], bf16);
    jt[col == LC ? T : col] = (double)acc;
  }
  __syncthreads();
  // ---- backflow head ----
  gemm_xw<TN>(XT, DX, R, DX, P + pl.kW1, DX, HT, DX, false, bf16);
  __syncthreads();
  for (int lay = 0; lay < 2; ++lay) {
    TN* A = lay == 0 ? HT : XT;
    const TN* kc = kcoef + (w * 2 + lay) * 2 * N * DX;
    for (int q = threadIdx.x; q < N * DX; q += blockDim.x) {
      int i = q / DX, x = q % DX;
      TN s1 = kc[i * DX + x], s2 = kc[N * DX + i * DX + x];
      TN sq = 0;
      for (int col = 0; col < LC; ++col) {
        TN v = A[(i * C + col) * DX + x];
        sq += v * v;
        A[(i * C + col) * DX + x] = s1 * v;
      }
      A[(i * C + LC) * DX + x] = s1 * A[(i * C + LC) * DX + x] + s2 * sq;
    }
    __syncthreads();
    if (lay == 0) {
      gemm_xw<TN>(HT, DX, R, DX, P + pl.kW2, DX, XT, DX, false, bf16);
      __syncthreads();
    }
  }
  double* ft = ftan + ((int64_t)w * n_chunks + chunk) * N * (T + 1) * M;
  for (int q = threadIdx.x; q < R * M; q += blockDim.x) {
    int row = q / M, mu = q % M, i = row / C, col = row % C;
    TN acc = 0;
    const TN* xr = XT + row * DX;
    for (int x = 0; x < DX; ++x) acc += maybe_bf16(xr[x], bf16) * maybe_bf16(P[pl.kW3 + x * M + mu], bf16);
    ft[((int64_t)i * (T + 1) + (col == LC ? T : col)) * M + mu] = (double)acc;
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
  int C = T + 1, R = d.N * C, DW = std::max(d.DX, d.DZ);
  return 3 * kMaxElec * sizeof(double) + (size_t)R * (d.DX + DW + d.DZ) * sizeof(TN) + 3 * C * d.DX * sizeof(TN);
}
template <typename TN>
size_t value_lds_bytes(const Dims& d, int wpb) {
  int DW = std::max(d.DX, d.DZ);
  return ((size_t)wpb * d.N * (d.DX + 2 * DW) + 2 * (size_t)wpb * d.DX) * sizeof(TN);
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
