// Adjoint of the network tangent pass: the parameter gradient of the
// coordinate derivatives of J and f (first derivatives and Laplacian), the
// second-order part of the full parameter adjoint (Methods, "PauliNet
// extension of SchNet"; J = eta(sum_i x_i), f_i = 1 + kappa(x_i)).
//
// The tangent pass maps, per coordinate chunk, the tangent columns and the
// partial-Laplacian column of the embeddings through
//   Linear  y_a = x_a W,                  y_L = x_L W
//   ssp     y_a = s1 u_a,                 y_L = s1 u_L + s2 sum_a u_a^2
//           (s1 = ssp'(u), s2 = ssp''(u) at the value-pass point u)
//   message z_a = sum_j (w_ij h_{j,a} + d_a w_ij h_j)
//           z_L = sum_j (w_ij h_{j,L} + sum_a (d2_a w_ij h_j + 2 d_a w_ij h_{j,a}))
// Its reverse, per (walker, chunk), with the cotangents of the backflow
// tangents and of J's tangents as input:
//   Linear  ct x = ct y W^T,              dW += x^T ct y   (rows = (electron, column))
//   ssp     ct u_a = s1 ct y_a + 2 s2 u_a ct y_L,  ct u_L = s1 ct y_L,
//           ct s1 = sum_a u_a ct y_a + u_L ct y_L,  ct s2 = ct y_L sum_a u_a^2
//   message ct h_{j,.} = sum_i w_ij ct z_{i,.} + 2 sum_a d_a w_ij ct z_{i,L}  (w_ij = w_ji)
//           ct w_ij   = sum_cols (h_{j,c} ct z_{i,c} + h_{i,c} ct z_{j,c})
//           and the source terms give cotangents of the value-pass h_j, of
//           w'/d and w'' per pair, and of the nuclear embeddings Y_I.
// The cotangents of the value-pass quantities (h values, ssp' and ssp'' of
// the heads, the filter values and radial derivatives) are summed over the
// walker's chunks and handed to the value-path adjoint.
//
// One 256-thread block per walker (grid-stride over walkers with a fixed
// grid); the block takes the walker's chunks one after the other and owns
// the walker's output rows, so every sum has a fixed order.  Parameter
// gradients go to the block's private slot.  The layer inputs x^(n) come from
// the forward tangent pass (saved per chunk); h = x W_h, the messages and the
// head pre-activations are recomputed.  The large row buffers sit in LDS, or
// (GA) in a per-block global arena when they do not fit.
#pragma once
#include "adj_util.h"
#include "gemm_lds.h"
#include "mfma_gemm.h"
#include "pn_internal.h"

namespace pn {

// Per-walker outputs of the tangent adjoint (sums over the walker's chunks).
template <typename TN>
struct TanAdjOut {
  TN* hv;  // [nw][L][N][DZ]        cotangent of the value-pass h
  TN* ww;  // [nw][L][n_ee][DZ]     cotangent of the ee filter values w
  TN* wd;  // [nw][L][n_pairs][DZ]  cotangent of w'/d
  TN* w2;  // [nw][L][n_pairs][DZ]  cotangent of w''
  TN* kc;  // [nw][2][2][N][DX]     cotangents of the backflow head's ssp', ssp''
  TN* ec;  // [nw][2][2][DX]        same for the Jastrow head
};

constexpr int tadj_nce_max(int T) { return (T + 4) / 3; }  // electrons a chunk of T coordinates touches

namespace {

// Forward activation of a head layer on the jets of one row group: columns
// 0..LC-1 are tangents, column LC the partial Laplacian.
template <typename TN, int C>
__device__ __forceinline__ void jet_act(const TN* E, TN* A, int ld, TN s1, TN s2, int x) {
  TN sq = 0;
#pragma unroll
  for (int col = 0; col < C - 1; ++col) {
    const TN v = E[col * ld + x];
    sq += v * v;
    A[col * ld + x] = s1 * v;
  }
  A[(C - 1) * ld + x] = s1 * E[(C - 1) * ld + x] + s2 * sq;
}
// Its reverse, in place on the cotangent CA (becomes the cotangent of E);
// returns the cotangents of s1 and s2.
template <typename TN, int C>
__device__ __forceinline__ void jet_act_adj(const TN* E, TN* CA, int ld, TN s1, TN s2, int x, TN& cs1, TN& cs2) {
  const TN cl = CA[(C - 1) * ld + x], el = E[(C - 1) * ld + x];
  TN a = el * cl, sq = 0;
#pragma unroll
  for (int col = 0; col < C - 1; ++col) {
    const TN v = E[col * ld + x], c = CA[col * ld + x];
    a += v * c;
    sq += v * v;
    CA[col * ld + x] = s1 * c + TN(2) * s2 * v * cl;
  }
  CA[(C - 1) * ld + x] = s1 * cl;
  cs1 = a;
  cs2 = cl * sq;
}

template <typename TN, int C, bool GA>
__global__ __launch_bounds__(kThreads) void k_net_tangent_adj(
    Dims d, DevTables t, int64_t nw, int n_chunks, const double* __restrict__ r, const TN* __restrict__ P,
    ParamLayout pl, const TN* __restrict__ filt, const TN* __restrict__ hval, const TN* __restrict__ kcoef,
    const TN* __restrict__ ecoef, const TN* __restrict__ xsave, const double* __restrict__ ctftan,
    const double* __restrict__ ctc, TanAdjOut<TN> out, TN* __restrict__ tslot, TN* __restrict__ garena,
    int64_t arena_elems, int64_t n_params) {
  constexpr int T = C - 1, LC = T;
  constexpr int NCEM = tadj_nce_max(T);
  extern __shared__ __align__(16) char smem[];
  const int N = d.N, DX = d.DX, DZ = d.DZ, M = d.M, NU = d.n_up, NN = d.NN, L = d.L, N3 = 3 * d.N;
  const int R = N * C, NP = N + NN;
  const int LDX = ld_pad<TN>(DX), LDZ = ld_pad<TN>(DZ), LDM = ld_pad<TN>((M + 15) & ~15);
  double* rs = reinterpret_cast<double*>(smem);                // [N][3]
  int* pidx = reinterpret_cast<int*>(rs + 3 * kMaxElec);       // [N][N]
  TN* cg = reinterpret_cast<TN*>(pidx + ((N * N + 3) & ~3));   // [NCEM][N][4]  r_i - r_k, 1/|r_i - r_k|
  TN* cgn = cg + NCEM * N * 4;                                 // [NCEM][NN][4] r_k - R_I, 1/|r_k - R_I|
  TN* hvs = cgn + NCEM * NN * 4;                               // [N][DZ] value-pass h of the layer
  TN* cthv = hvs + N * DZ;                                     // [N][DZ] its cotangent (this chunk)
  TN* tab = cthv + N * DZ;                                     // [2][NCEM][NP][DZ] ct of w'/d, w'' (chunk pairs)
  TN* arena = GA ? garena + (size_t)blockIdx.x * arena_elems : tab + 2 * NCEM * NP * DZ;
  TN* XS = arena;         // [R][LDX] layer input x^(n) (x^(L) for the heads)
  TN* CX = XS + R * LDX;  // [R][LDX] cotangent of the layer output
  TN* U = CX + R * LDX;   // union of the head and layer buffers
  TN* slot = tslot + (size_t)blockIdx.x * n_params;
  const int64_t fl_stride = (int64_t)3 * d.n_pairs * DZ;
  const int n_same = d.n_up * (d.n_up - 1) / 2 + d.n_dn * (d.n_dn - 1) / 2;
  const int64_t o_hv = (int64_t)L * N * DZ, o_ww = (int64_t)L * d.n_ee * DZ, o_wd = (int64_t)L * d.n_pairs * DZ;
  const int64_t o_kc = (int64_t)4 * N * DX, o_ec = (int64_t)4 * DX;
  for (int64_t q = threadIdx.x; q < n_params; q += blockDim.x) slot[q] = 0;
  for (int q = threadIdx.x; q < N * N; q += blockDim.x) pidx[q] = t.pair_index[q];
  for (int64_t w = blockIdx.x; w < nw; w += gridDim.x) {
    __syncthreads();
    for (int64_t q = threadIdx.x; q < o_hv; q += blockDim.x) out.hv[w * o_hv + q] = 0;
    for (int64_t q = threadIdx.x; q < o_ww; q += blockDim.x) out.ww[w * o_ww + q] = 0;
    for (int64_t q = threadIdx.x; q < o_wd; q += blockDim.x) {
      out.wd[w * o_wd + q] = 0;
      out.w2[w * o_wd + q] = 0;
    }
    for (int64_t q = threadIdx.x; q < o_kc; q += blockDim.x) out.kc[w * o_kc + q] = 0;
    for (int64_t q = threadIdx.x; q < o_ec; q += blockDim.x) out.ec[w * o_ec + q] = 0;
    for (int q = threadIdx.x; q < N3; q += blockDim.x) rs[q] = r[w * N3 + q];
    const double* cc = ctc + w * (N3 + 2);
    for (int chunk = 0; chunk < n_chunks; ++chunk) {
      __syncthreads();
      const int a0 = chunk * T, Tc = min(T, N3 - a0);
      const int e_lo = a0 / 3, e_hi = (a0 + Tc - 1) / 3, NCE = e_hi - e_lo + 1;
      const int64_t task = w * n_chunks + chunk;
      const TN* xs_base = xsave + (size_t)task * L * R * DX;
      for (int q = threadIdx.x; q < NCE * N; q += blockDim.x) {
        const int k = e_lo + q / N, i = q % N;
        const double ux = rs[3 * i] - rs[3 * k], uy = rs[3 * i + 1] - rs[3 * k + 1], uz = rs[3 * i + 2] - rs[3 * k + 2];
        cg[4 * q + 0] = (TN)ux;
        cg[4 * q + 1] = (TN)uy;
        cg[4 * q + 2] = (TN)uz;
        cg[4 * q + 3] = i == k ? TN(0) : (TN)(1.0 / sqrt(ux * ux + uy * uy + uz * uz));
      }
      for (int q = threadIdx.x; q < NCE * NN; q += blockDim.x) {
        const int k = e_lo + q / NN, I = q % NN;
        const double ux = rs[3 * k] - t.nuc_xyz[3 * I], uy = rs[3 * k + 1] - t.nuc_xyz[3 * I + 1],
                     uz = rs[3 * k + 2] - t.nuc_xyz[3 * I + 2];
        cgn[4 * q + 0] = (TN)ux;
        cgn[4 * q + 1] = (TN)uy;
        cgn[4 * q + 2] = (TN)uz;
        cgn[4 * q + 3] = (TN)(1.0 / sqrt(ux * ux + uy * uy + uz * uz));
      }
      for (int q = threadIdx.x; q < R * DX; q += blockDim.x)
        XS[(q / DX) * LDX + q % DX] = xs_base[(size_t)(L - 1) * R * DX + q];
      __syncthreads();
      // ================= Jastrow head, rows = columns =================
      if (d.flags & PN_NET_NO_JASTROW) {
        for (int q = threadIdx.x; q < R * DX; q += blockDim.x) CX[(q / DX) * LDX + q % DX] = 0;
        __syncthreads();
      } else {
        TN* S0 = U;
        TN* E1 = S0 + C * LDX;
        TN* A1 = E1 + C * LDX;
        TN* E2 = A1 + C * LDX;
        TN* A2 = E2 + C * LDX;
        TN* CT = A2 + C * LDX;
        TN* CT2 = CT + C * LDX;
        const TN* ec0 = ecoef + (w * 2 + 0) * 2 * DX;
        const TN* ec1 = ecoef + (w * 2 + 1) * 2 * DX;
        for (int q = threadIdx.x; q < C * DX; q += blockDim.x) {
          const int col = q / DX, x = q % DX;
          TN s = 0;
          for (int i = 0; i < N; ++i) s += XS[((size_t)i * C + col) * LDX + x];
          S0[col * LDX + x] = s;
        }
        __syncthreads();
        gemm_mfma<TN>(S0, LDX, C, DX, P + pl.eW1, DX, E1, LDX, false, false);
        __syncthreads();
        for (int x = threadIdx.x; x < DX; x += blockDim.x) jet_act<TN, C>(E1, A1, LDX, ec0[x], ec0[DX + x], x);
        __syncthreads();
        gemm_mfma<TN>(A1, LDX, C, DX, P + pl.eW2, DX, E2, LDX, false, false);
        __syncthreads();
        for (int x = threadIdx.x; x < DX; x += blockDim.x) {
          jet_act<TN, C>(E2, A2, LDX, ec1[x], ec1[DX + x], x);
          TN s = 0;
          const TN w3 = P[pl.eW3 + x];
#pragma unroll
          for (int col = 0; col < C; ++col) {
            const TN cj = col < LC ? (col < Tc ? (TN)cc[a0 + col] : TN(0)) : (TN)cc[N3];
            s += A2[col * LDX + x] * cj;
            CT[col * LDX + x] = cj * w3;
          }
          slot[pl.eW3 + x] += s;
          TN cs1, cs2;
          jet_act_adj<TN, C>(E2, CT, LDX, ec1[x], ec1[DX + x], x, cs1, cs2);
          out.ec[w * o_ec + 2 * DX + x] += cs1;
          out.ec[w * o_ec + 3 * DX + x] += cs2;
        }
        __syncthreads();
        outer_mfma<TN, false>(A1, LDX, DX, CT, LDX, DX, C, slot + pl.eW2, false);
        gemm_mfma_wt<TN>(CT, LDX, C, DX, P + pl.eW2, DX, CT2, LDX, false);
        __syncthreads();
        for (int x = threadIdx.x; x < DX; x += blockDim.x) {
          TN cs1, cs2;
          jet_act_adj<TN, C>(E1, CT2, LDX, ec0[x], ec0[DX + x], x, cs1, cs2);
          out.ec[w * o_ec + x] += cs1;
          out.ec[w * o_ec + DX + x] += cs2;
        }
        __syncthreads();
        outer_mfma<TN, false>(S0, LDX, DX, CT2, LDX, DX, C, slot + pl.eW1, false);
        gemm_mfma_wt<TN>(CT2, LDX, C, DX, P + pl.eW1, DX, CT, LDX, false);  // cotangent of sum_i x_i
        __syncthreads();
        for (int q = threadIdx.x; q < R * DX; q += blockDim.x) {
          const int row = q / DX, x = q % DX;
          CX[row * LDX + x] = CT[(row % C) * LDX + x];
        }
        __syncthreads();
      }
      // ================= backflow head, rows = (electron, column) =================
      if (!(d.flags & PN_NET_NO_BACKFLOW)) {
        TN* B1 = U;
        TN* B2 = B1 + R * LDX;
        TN* B3 = B2 + R * LDX;
        TN* CF = B3 + R * LDX;  // [R][LDM]
        const double* cf = ctftan + (size_t)task * R * M;
        for (int q = threadIdx.x; q < R * M; q += blockDim.x) CF[(q / M) * LDM + q % M] = (TN)cf[q];
        gemm_mfma<TN>(XS, LDX, R, DX, P + pl.kW1, DX, B1, LDX, false, false);  // K1
        __syncthreads();
        const TN* kc0 = kcoef + (w * 2 + 0) * 2 * N * DX;
        const TN* kc1 = kcoef + (w * 2 + 1) * 2 * N * DX;
        for (int q = threadIdx.x; q < N * DX; q += blockDim.x) {
          const int i = q / DX, x = q % DX;
          jet_act<TN, C>(B1 + (size_t)i * C * LDX, B2 + (size_t)i * C * LDX, LDX, kc0[q], kc0[N * DX + q], x);
        }
        __syncthreads();
        gemm_mfma<TN>(B2, LDX, R, DX, P + pl.kW2, DX, B1, LDX, false, false);  // K2 (over K1)
        __syncthreads();
        for (int q = threadIdx.x; q < N * DX; q += blockDim.x) {
          const int i = q / DX, x = q % DX;
          jet_act<TN, C>(B1 + (size_t)i * C * LDX, B3 + (size_t)i * C * LDX, LDX, kc1[q], kc1[N * DX + q], x);
        }
        __syncthreads();
        outer_acc<TN>(B3, LDX, DX, CF, LDM, M, R, slot + pl.kW3, false);  // kW3 is [DX][M]
        __syncthreads();
        for (int q = threadIdx.x; q < R * DX; q += blockDim.x) {
          const int row = q / DX, x = q % DX;
          TN s = 0;
          for (int mu = 0; mu < M; ++mu) s += CF[row * LDM + mu] * P[pl.kW3 + x * M + mu];
          B3[row * LDX + x] = s;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < N * DX; q += blockDim.x) {
          const int i = q / DX, x = q % DX;
          TN cs1, cs2;
          jet_act_adj<TN, C>(B1 + (size_t)i * C * LDX, B3 + (size_t)i * C * LDX, LDX, kc1[q], kc1[N * DX + q], x, cs1,
                             cs2);
          out.kc[w * o_kc + 2 * N * DX + q] += cs1;
          out.kc[w * o_kc + 3 * N * DX + q] += cs2;
        }
        __syncthreads();
        outer_mfma<TN, false>(B2, LDX, DX, B3, LDX, DX, R, slot + pl.kW2, false);
        gemm_mfma_wt<TN>(B3, LDX, R, DX, P + pl.kW2, DX, B1, LDX, false);  // ct of the first activation
        __syncthreads();
        gemm_mfma<TN>(XS, LDX, R, DX, P + pl.kW1, DX, B2, LDX, false, false);  // K1 again
        __syncthreads();
        for (int q = threadIdx.x; q < N * DX; q += blockDim.x) {
          const int i = q / DX, x = q % DX;
          TN cs1, cs2;
          jet_act_adj<TN, C>(B2 + (size_t)i * C * LDX, B1 + (size_t)i * C * LDX, LDX, kc0[q], kc0[N * DX + q], x, cs1,
                             cs2);
          out.kc[w * o_kc + q] += cs1;
          out.kc[w * o_kc + N * DX + q] += cs2;
        }
        __syncthreads();
        outer_mfma<TN, false>(XS, LDX, DX, B1, LDX, DX, R, slot + pl.kW1, false);
        gemm_mfma_wt<TN>(B1, LDX, R, DX, P + pl.kW1, DX, CX, LDX, true);
        __syncthreads();
      }
      // ================= interaction layers, last to first =================
      TN* HB = U;             // [R][LDZ] h tangents, recomputed
      TN* ZB = HB + R * LDZ;  // [R][LDZ] messages, then their cotangent
      TN* CH = ZB + R * LDZ;  // [R][LDZ] cotangent of the h tangents
      TN* twd = tab;                     // [NCEM][NP][DZ]
      TN* tw2 = tab + NCEM * NP * DZ;    // [NCEM][NP][DZ]
      for (int n = L - 1; n >= 0; --n) {
        const ParamLayout::Layer& Lp = pl.layer[n];
        const bool hn = n > 0;  // x^(0) is the same for every walker: no h tangents in layer 0
        const TN* fv = filt + (w * L + n) * fl_stride;
        const TN* fd = fv + (int64_t)d.n_pairs * DZ;
        const TN* f2 = fv + (int64_t)2 * d.n_pairs * DZ;
        const TN* hv = hval + (w * L + n) * N * DZ;
        for (int q = threadIdx.x; q < N * DZ; q += blockDim.x) {
          hvs[q] = hv[q];
          cthv[q] = 0;
        }
        for (int q = threadIdx.x; q < 2 * NCEM * NP * DZ; q += blockDim.x) tab[q] = 0;
        for (int q = threadIdx.x; q < R * DZ; q += blockDim.x) CH[(q / DZ) * LDZ + q % DZ] = 0;
        if (hn)
          for (int q = threadIdx.x; q < R * DX; q += blockDim.x)
            XS[(q / DX) * LDX + q % DX] = xs_base[(size_t)(n - 1) * R * DX + q];
        __syncthreads();
        if (hn) gemm_mfma<TN>(XS, LDX, R, DX, P + Lp.hW, DZ, HB, LDZ, false, false);
        __syncthreads();
        for (int ch = 0; ch < 3; ++ch) {
          // ---- recompute this channel's tangent messages into ZB ----
          if (ch < 2) {
            for (int q = threadIdx.x; q < N * DZ; q += blockDim.x) {
              const int i = q / DZ, z = q % DZ;
              const bool want_up = (ch == 0) == (i < NU);
              const int j_lo = want_up ? 0 : NU, j_hi = want_up ? NU : N;
              TN acc[C];
#pragma unroll
              for (int c = 0; c < C; ++c) acc[c] = 0;
              if (hn) {
                for (int j = j_lo; j < j_hi; ++j) {
                  if (j == i) continue;
                  const TN wv = fv[(int64_t)pidx[i * N + j] * DZ + z];
                  const TN* hj = HB + (size_t)j * C * LDZ + z;
#pragma unroll
                  for (int c = 0; c < C; ++c) acc[c] += wv * hj[c * LDZ];
                }
              }
              TN* zi = ZB + (size_t)i * C * LDZ + z;
              TN lap = acc[LC];
              if (i >= e_lo && i <= e_hi) {
                const TN* gi = cg + (size_t)(i - e_lo) * N * 4;
                const int c0 = 3 * i - a0;
                TN sv0 = 0, sv1 = 0, sv2 = 0;
                for (int j = j_lo; j < j_hi; ++j) {
                  if (j == i) continue;
                  const int64_t p = pidx[i * N + j];
                  const TN wd = fd[p * DZ + z], w2 = f2[p * DZ + z];
                  const TN hj = hvs[j * DZ + z], inv = gi[4 * j + 3];
                  const TN* hjc = HB + (size_t)j * C * LDZ + z;
#pragma unroll
                  for (int al = 0; al < 3; ++al) {
                    const int c = c0 + al;
                    if (c < 0 || c >= Tc) continue;
                    const TN ua = -gi[4 * j + al], ur = ua * inv, dw = wd * ua;
                    if (al == 0) sv0 += dw * hj;
                    if (al == 1) sv1 += dw * hj;
                    if (al == 2) sv2 += dw * hj;
                    lap += (w2 * ur * ur + wd * (TN(1) - ur * ur)) * hj;
                    if (hn) lap += TN(2) * dw * hjc[c * LDZ];
                  }
                }
#pragma unroll
                for (int c = 0; c < C; ++c) {
                  const int al = c - c0;
                  if (al == 0) acc[c] += sv0;
                  if (al == 1) acc[c] += sv1;
                  if (al == 2) acc[c] += sv2;
                }
              }
#pragma unroll
              for (int c = 0; c < LC; ++c) zi[c * LDZ] = acc[c];
              for (int k = max(e_lo, j_lo); k <= min(e_hi, j_hi - 1); ++k) {
                if (k == i) continue;
                const TN* gk = cg + ((size_t)(k - e_lo) * N + i) * 4;
                const int64_t p = pidx[i * N + k];
                const TN wd = fd[p * DZ + z], w2 = f2[p * DZ + z];
                const TN hk = hvs[k * DZ + z];
                const TN* hkc = HB + (size_t)k * C * LDZ + z;
#pragma unroll
                for (int al = 0; al < 3; ++al) {
                  const int c = 3 * k + al - a0;
                  if (c < 0 || c >= Tc) continue;
                  const TN ua = gk[al], ur = ua * gk[3], dw = -wd * ua;
                  zi[c * LDZ] += dw * hk;
                  lap += (w2 * ur * ur + wd * (TN(1) - ur * ur)) * hk;
                  if (hn) lap += TN(2) * dw * hkc[c * LDZ];
                }
              }
              zi[LC * LDZ] = lap;
            }
          } else {
            for (int q = threadIdx.x; q < NCE * DZ; q += blockDim.x) {
              const int i = e_lo + q / DZ, z = q % DZ;
              TN acc[C];
#pragma unroll
              for (int c = 0; c < C; ++c) acc[c] = 0;
              const int c0 = 3 * i - a0;
              for (int I = 0; I < NN; ++I) {
                const TN* gn = cgn + ((size_t)(i - e_lo) * NN + I) * 4;
                const TN y = P[pl.Y + I * DZ + z];
                const int64_t p = d.n_ee + i * NN + I;
                const TN wd = fd[p * DZ + z], w2 = f2[p * DZ + z];
#pragma unroll
                for (int c = 0; c < T; ++c) {
                  const int al = c - c0;
                  if (al < 0 || al > 2 || c >= Tc) continue;
                  const TN ua = gn[al], ur = ua * gn[3];
                  acc[c] += wd * ua * y;
                  acc[LC] += (w2 * ur * ur + wd * (TN(1) - ur * ur)) * y;
                }
              }
              TN* zi = ZB + (size_t)i * C * LDZ + z;
#pragma unroll
              for (int c = 0; c < C; ++c) zi[c * LDZ] = acc[c];
            }
          }
          __syncthreads();
          // ---- g_c: x += z G_c ----
          const int r0 = ch < 2 ? 0 : e_lo * C, nr = ch < 2 ? R : NCE * C;
          outer_mfma<TN, false>(ZB + (size_t)r0 * LDZ, LDZ, DZ, CX + (size_t)r0 * LDX, LDX, DX, nr, slot + Lp.gW[ch],
                                false);
          __syncthreads();
          gemm_mfma_wt<TN>(CX + (size_t)r0 * LDX, LDX, nr, DX, P + Lp.gW[ch], DZ, ZB + (size_t)r0 * LDZ, LDZ, false);
          __syncthreads();
          if (ch < 2) {
            // ---- pass A: rows j; cotangents through w_ij (row i) and the
            //      sources of the chunk electrons e != j on row e ----
            for (int q = threadIdx.x; q < N * DZ; q += blockDim.x) {
              const int j = q / DZ, z = q % DZ;
              const bool want_up = (ch == 0) == (j < NU);
              const int i_lo = want_up ? 0 : NU, i_hi = want_up ? NU : N;
              TN acc[C];
#pragma unroll
              for (int c = 0; c < C; ++c) acc[c] = 0;
              if (hn) {
                for (int i = i_lo; i < i_hi; ++i) {
                  if (i == j) continue;
                  const TN wv = fv[(int64_t)pidx[i * N + j] * DZ + z];
                  const TN* ci = ZB + (size_t)i * C * LDZ + z;
#pragma unroll
                  for (int c = 0; c < C; ++c) acc[c] += wv * ci[c * LDZ];
                }
              }
              TN chv = 0;
              const TN hvj = hvs[j * DZ + z];
              for (int e = max(e_lo, i_lo); e <= min(e_hi, i_hi - 1); ++e) {
                if (e == j) continue;
                const TN* gq = cg + ((size_t)(e - e_lo) * N + j) * 4;  // r_j - r_e
                const int64_t p = pidx[e * N + j];
                const TN wd = fd[p * DZ + z], w2 = f2[p * DZ + z];
                const TN ctzL = ZB[((size_t)e * C + LC) * LDZ + z];
                const int c0 = 3 * e - a0;
                TN cwd = 0, cw2 = 0, s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
                for (int al = 0; al < 3; ++al) {
                  const int c = c0 + al;
                  if (c < 0 || c >= Tc) continue;
                  const TN ua = -gq[al], ur = ua * gq[3], ur2 = ur * ur;
                  const TN ctzc = ZB[((size_t)e * C + c) * LDZ + z];
                  const TN d2 = w2 * ur2 + wd * (TN(1) - ur2);
                  chv += wd * ua * ctzc + d2 * ctzL;
                  cwd += ua * hvj * ctzc + (TN(1) - ur2) * hvj * ctzL;
                  cw2 += ur2 * hvj * ctzL;
                  if (hn) {
                    const TN v = TN(2) * wd * ua * ctzL;
                    if (al == 0) s0 += v;
                    if (al == 1) s1 += v;
                    if (al == 2) s2 += v;
                    cwd += TN(2) * ua * HB[((size_t)j * C + c) * LDZ + z] * ctzL;
                  }
                }
#pragma unroll
                for (int c = 0; c < C; ++c) {
                  const int al = c - c0;
                  if (al == 0) acc[c] += s0;
                  if (al == 1) acc[c] += s1;
                  if (al == 2) acc[c] += s2;
                }
                twd[((size_t)(e - e_lo) * NP + j) * DZ + z] += cwd;
                tw2[((size_t)(e - e_lo) * NP + j) * DZ + z] += cw2;
              }
              if (hn) {
                TN* chj = CH + (size_t)j * C * LDZ + z;
#pragma unroll
                for (int c = 0; c < C; ++c) chj[c * LDZ] += acc[c];
              }
              cthv[j * DZ + z] += chv;
            }
            // cotangent of the filter values of this channel's pairs
            {
              const int p_lo = ch == 0 ? 0 : n_same, p_hi = ch == 0 ? n_same : d.n_ee;
              TN* ow = out.ww + w * o_ww + (int64_t)n * d.n_ee * DZ;
              if (hn)
                for (int q = threadIdx.x; q < (p_hi - p_lo) * DZ; q += blockDim.x) {
                  const int p = p_lo + q / DZ, z = q % DZ;
                  const int i = t.pair_ij[2 * p], j = t.pair_ij[2 * p + 1];
                  const TN* hi = HB + (size_t)i * C * LDZ + z;
                  const TN* hj = HB + (size_t)j * C * LDZ + z;
                  const TN* zi = ZB + (size_t)i * C * LDZ + z;
                  const TN* zj = ZB + (size_t)j * C * LDZ + z;
                  TN s = 0;
#pragma unroll
                  for (int c = 0; c < C; ++c) s += hj[c * LDZ] * zi[c * LDZ] + hi[c * LDZ] * zj[c * LDZ];
                  ow[(int64_t)p * DZ + z] += s;
                }
            }
            __syncthreads();
            // ---- pass B: chunk electrons e; the sources of e's coordinates on rows j ----
            for (int q = threadIdx.x; q < NCE * DZ; q += blockDim.x) {
              const int e = e_lo + q / DZ, z = q % DZ;
              const bool want_up = (ch == 0) == (e < NU);
              const int j_lo = want_up ? 0 : NU, j_hi = want_up ? NU : N;
              const TN* gi = cg + (size_t)(e - e_lo) * N * 4;  // r_j - r_e
              const TN hve = hvs[e * DZ + z];
              const int c0 = 3 * e - a0;
              TN chv = 0, s0 = 0, s1 = 0, s2 = 0;
              for (int j = j_lo; j < j_hi; ++j) {
                if (j == e) continue;
                const int64_t p = pidx[e * N + j];
                const TN wd = fd[p * DZ + z], w2 = f2[p * DZ + z];
                const TN inv = gi[4 * j + 3];
                const TN ctzL = ZB[((size_t)j * C + LC) * LDZ + z];
                TN cwd = 0, cw2 = 0;
#pragma unroll
                for (int al = 0; al < 3; ++al) {
                  const int c = c0 + al;
                  if (c < 0 || c >= Tc) continue;
                  const TN ua = -gi[4 * j + al], ur = ua * inv, ur2 = ur * ur;
                  const TN ctzc = ZB[((size_t)j * C + c) * LDZ + z];
                  const TN d2 = w2 * ur2 + wd * (TN(1) - ur2);
                  chv += wd * ua * ctzc + d2 * ctzL;
                  cwd += ua * hve * ctzc + (TN(1) - ur2) * hve * ctzL;
                  cw2 += ur2 * hve * ctzL;
                  if (hn) {
                    const TN v = TN(2) * wd * ua * ctzL;
                    if (al == 0) s0 += v;
                    if (al == 1) s1 += v;
                    if (al == 2) s2 += v;
                    cwd += TN(2) * ua * HB[((size_t)e * C + c) * LDZ + z] * ctzL;
                  }
                }
                twd[((size_t)(e - e_lo) * NP + j) * DZ + z] += cwd;
                tw2[((size_t)(e - e_lo) * NP + j) * DZ + z] += cw2;
              }
              if (hn) {
#pragma unroll
                for (int al = 0; al < 3; ++al) {
                  const int c = c0 + al;
                  if (c < 0 || c >= Tc) continue;
                  CH[((size_t)e * C + c) * LDZ + z] += al == 0 ? s0 : (al == 1 ? s1 : s2);
                }
              }
              cthv[e * DZ + z] += chv;
            }
          } else {
            // ---- nuclear channel: w'/d, w'' of the chunk electrons' e-n pairs ----
            for (int q = threadIdx.x; q < NCE * DZ; q += blockDim.x) {
              const int e = e_lo + q / DZ, z = q % DZ;
              const int c0 = 3 * e - a0;
              const TN ctzL = ZB[((size_t)e * C + LC) * LDZ + z];
              for (int I = 0; I < NN; ++I) {
                const TN* gn = cgn + ((size_t)(e - e_lo) * NN + I) * 4;
                const TN y = P[pl.Y + I * DZ + z];
                TN cwd = 0, cw2 = 0;
#pragma unroll
                for (int al = 0; al < 3; ++al) {
                  const int c = c0 + al;
                  if (c < 0 || c >= Tc) continue;
                  const TN ua = gn[al], ur = ua * gn[3], ur2 = ur * ur;
                  const TN ctzc = ZB[((size_t)e * C + c) * LDZ + z];
                  cwd += ua * y * ctzc + (TN(1) - ur2) * y * ctzL;
                  cw2 += ur2 * y * ctzL;
                }
                twd[((size_t)(e - e_lo) * NP + N + I) * DZ + z] += cwd;
                tw2[((size_t)(e - e_lo) * NP + N + I) * DZ + z] += cw2;
              }
            }
            // d/dY_I (its share from the tangents)
            for (int q = threadIdx.x; q < NN * DZ; q += blockDim.x) {
              const int I = q / DZ, z = q % DZ;
              TN s = 0;
              for (int e = e_lo; e <= e_hi; ++e) {
                const TN* gn = cgn + ((size_t)(e - e_lo) * NN + I) * 4;
                const int64_t p = d.n_ee + e * NN + I;
                const TN wd = fd[p * DZ + z], w2 = f2[p * DZ + z];
                const TN ctzL = ZB[((size_t)e * C + LC) * LDZ + z];
                const int c0 = 3 * e - a0;
#pragma unroll
                for (int al = 0; al < 3; ++al) {
                  const int c = c0 + al;
                  if (c < 0 || c >= Tc) continue;
                  const TN ua = gn[al], ur = ua * gn[3], ur2 = ur * ur;
                  const TN ctzc = ZB[((size_t)e * C + c) * LDZ + z];
                  s += wd * ua * ctzc + (w2 * ur2 + wd * (TN(1) - ur2)) * ctzL;
                }
              }
              slot[pl.Y + q] += s;
            }
          }
          __syncthreads();
        }
        // ---- h = x W_h: weight gradient and the cotangent of x^(n) ----
        if (hn) {
          outer_mfma<TN, false>(XS, LDX, DX, CH, LDZ, DZ, R, slot + Lp.hW, false);
          gemm_mfma_wt<TN>(CH, LDZ, R, DZ, P + Lp.hW, DX, CX, LDX, true);
        }
        // ---- this chunk's share of the value-pass cotangents ----
        for (int q = threadIdx.x; q < N * DZ; q += blockDim.x) out.hv[w * o_hv + (int64_t)n * N * DZ + q] += cthv[q];
        {
          TN* owd = out.wd + w * o_wd + (int64_t)n * d.n_pairs * DZ;
          TN* ow2 = out.w2 + w * o_wd + (int64_t)n * d.n_pairs * DZ;
          for (int q = threadIdx.x; q < NCE * NP * DZ; q += blockDim.x) {
            const int el = q / (NP * DZ), part = (q / DZ) % NP, z = q % DZ;
            const int e = e_lo + el;
            int64_t p;
            TN vd = twd[q], v2 = tw2[q];
            if (part < N) {
              if (part == e) continue;
              if (part >= e_lo && part <= e_hi) {
                if (part < e) continue;  // the pair is summed by its lower chunk electron
                const size_t q2 = ((size_t)(part - e_lo) * NP + e) * DZ + z;
                vd += twd[q2];
                v2 += tw2[q2];
              }
              p = pidx[e * N + part];
            } else {
              p = d.n_ee + (int64_t)e * NN + (part - N);
            }
            owd[p * DZ + z] += vd;
            ow2[p * DZ + z] += v2;
          }
        }
        __syncthreads();
      }
    }
  }
}

template <typename TN, int C>
void launch_ta_c(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const TN* P, char* ws,
                 const WsLayout& L) {
  const Dims& d = c->d;
  const int nb = (int)std::min<int64_t>(nw, kSlotsTanAdj);
  TanAdjOut<TN> o{reinterpret_cast<TN*>(ws + L.cthv), reinterpret_cast<TN*>(ws + L.ctww),
                  reinterpret_cast<TN*>(ws + L.ctwd), reinterpret_cast<TN*>(ws + L.ctw2),
                  reinterpret_cast<TN*>(ws + L.ctkc), reinterpret_cast<TN*>(ws + L.ctec)};
  TN* tslot = reinterpret_cast<TN*>(ws + L.tslot);
  TN* garena = tslot + (size_t)kSlotsTanAdj * c->pl.total;
  auto go = [&](auto kern) {
    if (L.lds_tadj > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)L.lds_tadj);
    hipLaunchKernelGGL(kern, dim3(nb), dim3(kThreads), L.lds_tadj, s, d, c->t, nw, L.n_chunks, r, P, c->pl,
                       reinterpret_cast<const TN*>(ws + L.filt), reinterpret_cast<const TN*>(ws + L.hval),
                       reinterpret_cast<const TN*>(ws + L.kcoef), reinterpret_cast<const TN*>(ws + L.ecoef),
                       reinterpret_cast<const TN*>(ws + L.xsave), reinterpret_cast<const double*>(ws + L.ctftan),
                       reinterpret_cast<const double*>(ws + L.ctc), o, tslot, garena, (int64_t)L.tadj_arena,
                       (int64_t)c->pl.total);
  };
  if (L.tadj_global)
    go(&k_net_tangent_adj<TN, C, true>);
  else
    go(&k_net_tangent_adj<TN, C, false>);
}

}  // namespace

// LDS bytes of the tangent adjoint block (small tables, plus the row
// buffers when they are kept in LDS) and the row-buffer elements.
template <typename TN>
size_t tangent_adj_arena_elems(const Dims& d, int T) {
  const int C = T + 1, R = d.N * C;
  const size_t LDX = ld_pad<TN>(d.DX), LDZ = ld_pad<TN>(d.DZ), LDM = ld_pad<TN>((d.M + 15) & ~15);
  const size_t u = std::max(std::max(3 * R * LDZ, 3 * R * LDX + R * LDM), 7 * (size_t)C * LDX);
  return 2 * R * LDX + u;
}
template <typename TN>
size_t tangent_adj_lds_bytes(const Dims& d, int T, bool global_arena) {
  const int NCEM = tadj_nce_max(T), NP = d.N + d.NN;
  size_t tn = (size_t)NCEM * (d.N + d.NN) * 4 + 2 * (size_t)d.N * d.DZ + 2 * (size_t)NCEM * NP * d.DZ;
  if (!global_arena) tn += tangent_adj_arena_elems<TN>(d, T);
  return 3 * kMaxElec * sizeof(double) + (size_t)((d.N * d.N + 3) & ~3) * sizeof(int) + tn * sizeof(TN);
}

template <typename TN>
void launch_net_tangent_adj(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const TN* P, char* ws,
                            const WsLayout& L) {
  switch (L.T + 1) {
    case 2: launch_ta_c<TN, 2>(c, s, nw, r, P, ws, L); break;
    case 3: launch_ta_c<TN, 3>(c, s, nw, r, P, ws, L); break;
    case 4: launch_ta_c<TN, 4>(c, s, nw, r, P, ws, L); break;
    case 5: launch_ta_c<TN, 5>(c, s, nw, r, P, ws, L); break;
    case 6: launch_ta_c<TN, 6>(c, s, nw, r, P, ws, L); break;
    case 7: launch_ta_c<TN, 7>(c, s, nw, r, P, ws, L); break;
    default: break;  // the planner only picks T in 1..6 for the full adjoint
  }
}

}  // namespace pn
