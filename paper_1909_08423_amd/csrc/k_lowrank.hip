// Multideterminant expansion through one LU per spin (all FP64).
//
// The expansion sum_p c_p det A_p^up det A_p^down (Results, eq. "ansatz")
// has members that differ from the first determinant in a few orbitals.
// Write A_0 for the first determinant's matrix of one spin, G_0 = A_0^{-1}
// and Theta = Phi~ G_0 (rows: the orbitals occupied in some determinant but
// not in the first, "virtual rows"; columns: the first determinant's slots).
// If determinant p replaces the orbitals of slots h_1..h_k by v_1..v_k, the
// matrix determinant lemma gives
//
//   det A_p = s_p det A_0 det D_p,   D_p[j][l] = Theta[v_j][h_l]   (k x k),
//
// with s_p the sign of the row order.  For a coordinate a, with
// T_a = d_a Phi~ (the table derivative), B_a = T_a G_0 and N_a = the first
// determinant's rows of B_a (= d_a A_0 G_0):
//
//   d_a ln det A_0 = tr N_a,        Xi_a = d_a Theta = B_a - Theta N_a,
//   d_a ln det D_p = tr(D_p^{-1} Xi_a[v][h]),
//
// and with L the Laplacian of the table, Lambda = L G_0 and S = sum_a Xi_a N_a:
//
//   lap ln det A_0 = tr Lambda[occ] - sum_a tr(N_a^2),
//   sum_a d2_a Theta = Lambda - Theta Lambda[occ] - 2 S,
//   lap ln det D_p = tr(D_p^{-1} (sum_a d2_a Theta)[v][h])
//                    - sum_a tr((D_p^{-1} Xi_a[v][h])^2).
//
// The per-coordinate work is one product T_a G_0 per spin instead of one
// per determinant.  The formulas divide by det A_0 through G_0: a walker
// whose first determinant is singular, or small against another member
// (|det D_p| > kRatioMax), is handed to the direct per-determinant kernels
// through a device-side list.
//
//  k_lr_value    one wavefront per (walker, spin): Theta, each D_p, its
//                determinant and inverse (Gauss-Jordan in registers), the
//                members' (ln|det|, sign) in the direct path's layout, and
//                the hand-back flag.
//  k_lr_list     one block per tile: the flagged walkers, ascending, and
//                their count.
//  k_lr_tangent  one block per walker, over the coordinate chunks of the
//                network tangent pass: the table derivatives, B_a and Xi_a,
//                the members' gradients, the determinant sum per coordinate
//                (as in the direct path), then the Laplacian terms; writes
//                the gradient and the walker's Laplacian / |grad|^2 partials.
#include <math.h>

#include <type_traits>

#include <algorithm>

#include "pn_internal.h"

namespace pn {
namespace {

constexpr int kWaves = kThreads / 64;
constexpr double kRatioMax = 1e4;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// In-place inverse of the leading k x k block of a (identity beyond it) by
// Gauss-Jordan elimination with partial pivoting (largest |a[r][c]|, ties to
// the lowest row); returns the determinant, 0 for a singular block (a is then
// undefined).
__device__ __forceinline__ double gj_inverse(double (&a)[kMaxExc][kMaxExc], int k) {
  int piv[kMaxExc];
  double det = 1.0;
#pragma unroll
  for (int c = 0; c < kMaxExc; ++c) {
    int bi = c;
    double best = fabs(a[c][c]);
#pragma unroll
    for (int r = c + 1; r < kMaxExc; ++r) {
      const double v = fabs(a[r][c]);
      if (r < k && v > best) {
        best = v;
        bi = r;
      }
    }
    piv[c] = bi;
    if (bi != c) det = -det;
#pragma unroll
    for (int r = c + 1; r < kMaxExc; ++r) {
      if (r == bi) {
#pragma unroll
        for (int col = 0; col < kMaxExc; ++col) {
          const double tmp = a[c][col];
          a[c][col] = a[r][col];
          a[r][col] = tmp;
        }
      }
    }
    const double pv = a[c][c];
    if (pv == 0.0) return 0.0;
    det *= pv;
    const double inv = 1.0 / pv;
    a[c][c] = 1.0;
#pragma unroll
    for (int col = 0; col < kMaxExc; ++col) a[c][col] *= inv;
#pragma unroll
    for (int r = 0; r < kMaxExc; ++r) {
      if (r == c) continue;
      const double f = a[r][c];
      a[r][c] = 0.0;
#pragma unroll
      for (int col = 0; col < kMaxExc; ++col) a[r][col] -= f * a[c][col];
    }
  }
#pragma unroll
  for (int c = kMaxExc - 1; c >= 0; --c) {
#pragma unroll
    for (int col = c + 1; col < kMaxExc; ++col) {
      if (piv[c] == col) {
#pragma unroll
        for (int r = 0; r < kMaxExc; ++r) {
          const double tmp = a[r][c];
          a[r][c] = a[r][col];
          a[r][col] = tmp;
        }
      }
    }
  }
  return det;
}

__device__ __forceinline__ int theta_size(const Dims& d) { return d.nv[0] * d.n_up + d.nv[1] * d.n_dn; }

__global__ __launch_bounds__(kThreads) void k_lr_value(Dims d, DevTables t, int64_t nw,
                                                       const double* __restrict__ phi,
                                                       const double* __restrict__ fval,
                                                       const double* __restrict__ g0,
                                                       const double* __restrict__ ld0,
                                                       double* __restrict__ theta, double* __restrict__ dinv,
                                                       double* __restrict__ ldet, int* __restrict__ flag) {
  extern __shared__ __align__(16) double lsm[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t task = (int64_t)blockIdx.x * kWaves + wv;
  if (task >= nw * 2) return;
  const int64_t w = task >> 1;
  const int s = (int)(task & 1);
  const int n = s ? d.n_dn : d.n_up, e0 = s ? d.n_up : 0, nv = s ? d.nv[1] : d.nv[0];
  const int N = d.N, M = d.M, P = d.P;
  const int gsz = d.n_up * d.n_up + d.n_dn * d.n_dn;
  const int nvmax = max(d.nv[0], d.nv[1]), nmax = max(d.n_up, d.n_dn);
  double* ts = lsm + (size_t)wv * nvmax * nmax;
  if (n == 0) {
    for (int p = lane; p < P; p += 64) {
      ldet[((w * P + p) * 2 + s) * 2] = 0.0;
      ldet[((w * P + p) * 2 + s) * 2 + 1] = 1.0;
    }
    if (lane == 0) flag[w * 2 + s] = 0;
    return;
  }
  const double* G = g0 + w * gsz + (s ? d.n_up * d.n_up : 0);
  const double l0 = ld0[(w * 2 + s) * 2], s0 = ld0[(w * 2 + s) * 2 + 1];
  const bool ref_ok = l0 > -INFINITY;
  double* Th = theta + w * theta_size(d) + (s ? d.nv[0] * d.n_up : 0);
  if (ref_ok) {
    const double* ph = phi + w * N * M * 7;
    const double* fv = fval + w * N * M;
    for (int q = lane; q < nv * n; q += 64) {
      const int v = q / n, k = q % n, orb = t.lr_vorb[s * M + v];
      double acc = 0.0;
      for (int i = 0; i < n; ++i) {
        const size_t e = (size_t)(e0 + i) * M + orb;
        acc += ph[e * 7] * fv[e] * G[i * n + k];
      }
      Th[q] = acc;
      ts[q] = acc;
    }
  }
  wave_sync();
  bool bad = !ref_ok;
  for (int p = lane; p < P; p += 64) {
    const int k = t.lr_k[p * 2 + s];
    double* di = dinv + ((w * P + p) * 2 + s) * (kMaxExc * kMaxExc);
    double lnd = 0.0, sd = 1.0;
    if (!ref_ok) {
      lnd = -INFINITY;
      sd = 0.0;
    } else if (k > 0) {
      const int* hl = t.lr_hole + (p * 2 + s) * kMaxExc;
      const int* pt = t.lr_part + (p * 2 + s) * kMaxExc;
      double a[kMaxExc][kMaxExc];
#pragma unroll
      for (int j = 0; j < kMaxExc; ++j)
#pragma unroll
        for (int l = 0; l < kMaxExc; ++l)
          a[j][l] = (j < k && l < k) ? ts[pt[j] * n + hl[l]] : (j == l ? 1.0 : 0.0);
      const double det = gj_inverse(a, k);
      if (det == 0.0) {
        lnd = -INFINITY;
        sd = 0.0;
#pragma unroll
        for (int q = 0; q < kMaxExc * kMaxExc; ++q) di[q] = 0.0;
      } else {
        lnd = log(fabs(det));
        sd = det > 0 ? 1.0 : -1.0;
        if (fabs(det) > kRatioMax) bad = true;
#pragma unroll
        for (int j = 0; j < kMaxExc; ++j)
#pragma unroll
          for (int l = 0; l < kMaxExc; ++l) di[j * kMaxExc + l] = a[j][l];
      }
    }
    ldet[((w * P + p) * 2 + s) * 2] = l0 + lnd;
    ldet[((w * P + p) * 2 + s) * 2 + 1] = s0 * sd * t.lr_sign[p * 2 + s];
  }
  const unsigned long long any_bad = __ballot(bad);
  if (lane == 0) flag[w * 2 + s] = any_bad ? 1 : 0;
}

// The walkers of the tile with either spin flagged, ascending, in list[0..],
// and their count in list[nw] (one block of 1024 threads).
__global__ __launch_bounds__(1024) void k_lr_list(int64_t nw, const int* __restrict__ flag, int* __restrict__ list) {
  __shared__ int scan[1024];
  __shared__ int base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int64_t w0 = 0; w0 < nw; w0 += 1024) {
    const int64_t w = w0 + threadIdx.x;
    const int f = (w < nw) ? ((flag[2 * w] | flag[2 * w + 1]) ? 1 : 0) : 0;
    scan[threadIdx.x] = f;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int v = threadIdx.x >= (unsigned)o ? scan[threadIdx.x - o] : 0;
      __syncthreads();
      scan[threadIdx.x] += v;
      __syncthreads();
    }
    if (f) list[base + scan[threadIdx.x] - 1] = (int)w;
    __syncthreads();
    if (threadIdx.x == 1023) base += scan[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) list[nw] = base;
}

// Element offsets of the tangent kernel's LDS regions (doubles, then ints).
struct LrLds {
  int gsz, thsz, bsz, R0, R1;
  size_t G0, TH, TB, LT, BM, SS, YY, TRN, TRN2, GPA, QACC, DELTA, DINV, WD, LAPC, SQC, SCAL, PF, n_dbl;
  size_t ROWORB, n_int;
};

__host__ __device__ inline LrLds lr_lds(const Dims& d, int T) {
  LrLds o{};
  o.gsz = d.n_up * d.n_up + d.n_dn * d.n_dn;
  o.thsz = d.nv[0] * d.n_up + d.nv[1] * d.n_dn;
  o.R0 = d.n_up + d.nv[0];
  o.R1 = d.n_dn + d.nv[1];
  o.bsz = o.R0 * d.n_up + o.R1 * d.n_dn;
  size_t off = 0;
  auto take = [&](size_t n) {
    size_t r = off;
    off += (n + 1) & ~size_t(1);  // keep 16-byte alignment
    return r;
  };
  o.G0 = take(o.gsz);
  o.TH = take(o.thsz);
  o.TB = take((size_t)T * d.M * d.N);
  o.LT = take((size_t)d.M * d.N);
  o.BM = take((size_t)T * o.bsz);
  o.SS = take(o.thsz);
  o.YY = take(o.thsz);
  o.TRN = take((size_t)T * 2);
  o.TRN2 = take((size_t)T * 2);
  o.GPA = take((size_t)d.P * T * 2);
  o.QACC = take((size_t)d.P * 2);
  o.DELTA = take(d.P);
  o.DINV = take((size_t)d.P * 2 * kMaxExc * kMaxExc);
  o.WD = take(d.P);
  o.LAPC = take(T);
  o.SQC = take(T);
  o.SCAL = take(8);
  o.PF = take((size_t)2 * d.N * d.M);
  o.n_dbl = off;
  o.ROWORB = 0;
  o.n_int = o.R0 + o.R1;
  return o;
}

// WIDE: spins of 8 or more electrons, blocks of over 40 KB of LDS (at most
// two per CU, so a wave may hold up to 256 registers): slot blocking in
// steps 2 and 3 and the next chunk's tangents of the first 8 step-1 items
// requested ahead.  Otherwise one slot per item, no prefetch, and at most
// 128 registers (four blocks per CU).
template <bool WIDE>
__global__ __launch_bounds__(kThreads, WIDE ? 2 : 4) void k_lr_tangent(Dims d, DevTables t, int64_t nw, int T, int n_chunks,
                                                         const double* __restrict__ geo,
                                                         const double* __restrict__ phi,
                                                         const double* __restrict__ fval,
                                                         const double* __restrict__ ftan,
                                                         const double* __restrict__ jtan,
                                                         const double* __restrict__ g0,
                                                         const double* __restrict__ theta,
                                                         const double* __restrict__ dinv,
                                                         const double* __restrict__ wdet,
                                                         const int* __restrict__ flag, double* __restrict__ grad,
                                                         double* __restrict__ partial) {
  extern __shared__ __align__(16) double sm[];
  const int64_t w = blockIdx.x;
  if (w >= nw || (flag[2 * w] | flag[2 * w + 1])) return;  // the direct path takes this walker
  const LrLds o = lr_lds(d, T);
  const int N = d.N, M = d.M, P = d.P, nu = d.n_up, nd = d.n_dn;
  const int tid = threadIdx.x, nth = blockDim.x;
  double* G0s = sm + o.G0;
  double* THs = sm + o.TH;
  double* TB = sm + o.TB;      // [T][N][M] table derivatives of the chunk (orbital fastest)
  double* LT = sm + o.LT;      // [M][N] Laplacian of the table, summed over chunks
  double* BM = sm + o.BM;      // [T][bsz] B_a rows (first determinant's, then virtual) per spin
  double* SS = sm + o.SS;      // [thsz] S = sum_a Xi_a N_a
  double* YY = sm + o.YY;      // [thsz] sum_a d2_a Theta on the virtual rows
  double* TRN = sm + o.TRN;    // [T][2] tr N_a
  double* TRN2 = sm + o.TRN2;  // [T][2] tr N_a^2
  double* GPA = sm + o.GPA;    // [P][T][2] d_a ln|D_p|, each spin's minor
  double* QACC = sm + o.QACC;  // [P][2] sum_a tr((D^-1 Xi_a)^2), each spin
  double* DELTA = sm + o.DELTA;
  double* DI = sm + o.DINV;    // [P][2][kMaxExc^2]
  double* WD = sm + o.WD;      // [P]
  double* LAPC = sm + o.LAPC;
  double* SQC = sm + o.SQC;
  double* SCAL = sm + o.SCAL;  // lap, |grad|^2, sum tr N^2 (up, down), tr Lambda[occ] (up, down)
  double* PF = sm + o.PF;      // [2][N][M] phi_mu(r_i) and f_{i mu} of the walker
  int* ROWORB = reinterpret_cast<int*>(sm + o.n_dbl);

  const int gsz = o.gsz, thsz = o.thsz, bsz = o.bsz;
  const int sB1 = o.R0 * nu, sT1 = d.nv[0] * nu;  // offsets of the down-spin rows
  auto soffB = [&](int s) { return s ? sB1 : 0; };
  auto soffT = [&](int s) { return s ? sT1 : 0; };
  auto ns = [&](int s) { return s ? nd : nu; };
  auto e0s = [&](int s) { return s ? nu : 0; };

  for (int q = tid; q < gsz; q += nth) G0s[q] = g0[w * gsz + q];
  for (int q = tid; q < thsz; q += nth) {
    THs[q] = theta[w * thsz + q];
    SS[q] = 0.0;
  }
  for (int q = tid; q < M * N; q += nth) LT[q] = 0.0;
  for (int q = tid; q < P * 2 * kMaxExc * kMaxExc; q += nth) DI[q] = dinv[w * P * 2 * kMaxExc * kMaxExc + q];
  for (int q = tid; q < P; q += nth) {
    WD[q] = wdet[w * P + q];
    QACC[2 * q] = QACC[2 * q + 1] = 0.0;
  }
  for (int q = tid; q < o.R0 + o.R1; q += nth) {
    const int s = q >= o.R0, r = s ? q - o.R0 : q, n = ns(s);
    ROWORB[q] = r < n ? (s ? t.det_dn[r] : t.det_up[r]) : t.lr_vorb[s * M + (r - n)];
  }
  if (tid < 8) SCAL[tid] = 0.0;
  for (int q = tid; q < N * M; q += nth) {
    PF[q] = phi[((size_t)w * N * M + q) * 7];
    PF[N * M + q] = fval[(size_t)w * N * M + q];
  }
  __syncthreads();

  const double* ph = phi + w * N * M * 7;
  const double* fv = fval + w * N * M;
  const double* g = geo + w * kGeoStride(N);
  const int Tp = T + 1, NTM = N * Tp * M;
  // the first chunk's tangents of the step-1 items held in registers, and
  // the items' (i, column, mu) decoded once (the same in every chunk; M <= 128
  // and columns <= 17 fit their 8-bit fields)
  constexpr int kItems = WIDE ? 8 : 1;  // step-1 items per thread kept in registers
  double ftv[kItems];
  int pk[kItems];
#pragma unroll
  for (int u = 0; u < kItems; ++u) {
    const int q = tid + u * nth;
    if (q >= NTM) break;
    ftv[u] = ftan[(size_t)w * n_chunks * NTM + q];
    pk[u] = ((q / (Tp * M)) << 16) | (((q / M) % Tp) << 8) | (q % M);
  }
  for (int chunk = 0; chunk < n_chunks; ++chunk) {
    const int a0 = chunk * T, Tc = min(T, 3 * N - a0);
    const double* ft = ftan + ((size_t)w * n_chunks + chunk) * NTM;
    const double* jt = jtan + ((size_t)w * n_chunks + chunk) * Tp;
    // 1. table derivatives T_a[mu][i] and the chunk's part of the table
    //    Laplacian, read in the memory order of the network tangents.  A
    //    thread's items (i, column, mu) are the same in every chunk: phi
    //    and f come from LDS (copied once per walker), and the tangents of
    //    the first kItems items for the next chunk are requested into
    //    registers at the end of this step, so the HBM latency overlaps
    //    steps 2 to 5.
    {
#pragma unroll
      for (int u = 0; u < kItems; ++u) {
        const int q = tid + u * nth;
        if (q >= NTM) break;
        const int i = pk[u] >> 16, col = (pk[u] >> 8) & 255, mu = pk[u] & 255;
        const double* pj = ph + ((size_t)i * M + mu) * 7;
        const double f = PF[N * M + i * M + mu];
        if (col < Tc) {
          const int a = a0 + col, k = a / 3, al = a % 3;
          double v = PF[i * M + mu] * ftv[u];
          if (k == i) v += pj[1 + al] * f;
          TB[((size_t)col * N + i) * M + mu] = v;
        } else if (col == T) {
          double v = PF[i * M + mu] * ftv[u];
          for (int c2 = 0; c2 < Tc; ++c2) {
            const int a = a0 + c2, k = a / 3, al = a % 3;
            if (k != i) continue;
            v += pj[4 + al] * f + 2.0 * pj[1 + al] * ft[((size_t)i * Tp + c2) * M + mu];
          }
          LT[mu * N + i] += v;
        }
      }
      for (int q = tid + kItems * nth; q < NTM; q += nth) {  // items past the register-resident ones
        const int i = q / (Tp * M), col = (q / M) % Tp, mu = q % M;
        const double* pj = ph + ((size_t)i * M + mu) * 7;
        const double f = fv[i * M + mu];
        if (col < Tc) {
          const int a = a0 + col, k = a / 3, al = a % 3;
          double v = pj[0] * ft[q];
          if (k == i) v += pj[1 + al] * f;
          TB[((size_t)col * N + i) * M + mu] = v;
        } else if (col == T) {
          double v = pj[0] * ft[q];
          for (int c2 = 0; c2 < Tc; ++c2) {
            const int a = a0 + c2, k = a / 3, al = a % 3;
            if (k != i) continue;
            v += pj[4 + al] * f + 2.0 * pj[1 + al] * ft[((size_t)i * Tp + c2) * M + mu];
          }
          LT[mu * N + i] += v;
        }
      }
      if (chunk + 1 < n_chunks) {
        const double* ftn = ft + (size_t)NTM;  // the next chunk's tangents follow this chunk's
#pragma unroll
        for (int u = 0; u < kItems; ++u) {
          const int q = tid + u * nth;
          if (q >= NTM) break;
          ftv[u] = ftn[q];
        }
      }
    }
    __syncthreads();
    // 2. B_a = T_a G_0 on the first determinant's rows and the virtual rows;
    //    an item is SL consecutive slots k of one row (independent sums
    //    sharing the row's reads; SL = 4 from 8 electrons of a spin on)
    auto step2 = [&](auto sl_tag) {
      constexpr int SL = decltype(sl_tag)::value;
      const int nq0 = o.R0 * ((nu + SL - 1) / SL), nq1 = o.R1 * ((nd + SL - 1) / SL), nq = nq0 + nq1;
      for (int q = tid; q < Tc * nq; q += nth) {
        const int col = q / nq, rem = q % nq;
        const int s = rem >= nq0, rq = rem - (s ? nq0 : 0), n = ns(s), nks = (n + SL - 1) / SL;
        const int r = rq / nks, k0 = (rq % nks) * SL;
        const double* tb = TB + ((size_t)col * N + e0s(s)) * M + ROWORB[s * o.R0 + r];
        const double* Gs = G0s + (s ? nu * nu : 0);
        double acc[SL];
#pragma unroll
        for (int u = 0; u < SL; ++u) acc[u] = 0.0;
        for (int i = 0; i < n; ++i) {
          const double x = tb[i * M];
#pragma unroll
          for (int u = 0; u < SL; ++u) acc[u] += x * Gs[i * n + min(k0 + u, n - 1)];
        }
        double* B = BM + (size_t)col * bsz + soffB(s) + r * n;
#pragma unroll
        for (int u = 0; u < SL; ++u)
          if (k0 + u < n) B[k0 + u] = acc[u];
      }
    };
    if constexpr (WIDE)
      step2(std::integral_constant<int, 4>());
    else
      step2(std::integral_constant<int, 1>());
    __syncthreads();
    // 3. Xi_a = B_a - Theta N_a on the virtual rows (in place; an item is
    //    SL consecutive slots of one row, as in step 2), and tr N_a, tr N_a^2 per
    //    (coordinate, spin) by one wavefront (lane k: row k), summed across
    //    the lanes in a fixed order
    {
      auto xi = [&](auto sl_tag) {
        constexpr int SL = decltype(sl_tag)::value;
        const int nq0 = d.nv[0] * ((nu + SL - 1) / SL), nq1 = d.nv[1] * ((nd + SL - 1) / SL), nq = nq0 + nq1;
        for (int q = tid; q < Tc * nq; q += nth) {
          const int col = q / nq, rem = q % nq;
          const int s = rem >= nq0, rq = rem - (s ? nq0 : 0), n = ns(s), nks = (n + SL - 1) / SL;
          const int v = rq / nks, k0 = (rq % nks) * SL;
          double* B = BM + (size_t)col * bsz + soffB(s);
          const double* th = THs + soffT(s) + v * n;
          double acc[SL];
#pragma unroll
          for (int u = 0; u < SL; ++u) acc[u] = B[(n + v) * n + min(k0 + u, n - 1)];
          for (int l = 0; l < n; ++l) {
            const double x = th[l];
#pragma unroll
            for (int u = 0; u < SL; ++u) acc[u] -= x * B[l * n + min(k0 + u, n - 1)];
          }
#pragma unroll
          for (int u = 0; u < SL; ++u)
            if (k0 + u < n) B[(n + v) * n + k0 + u] = acc[u];
        }
      };
      if constexpr (WIDE)
        xi(std::integral_constant<int, 4>());
      else
        xi(std::integral_constant<int, 1>());
      const int lane = tid & 63, wv = tid >> 6, nwv = nth >> 6;
      for (int cs = wv; cs < Tc * 2; cs += nwv) {
        const int col = cs / 2, s = cs % 2, n = ns(s);
        const double* B = BM + (size_t)col * bsz + soffB(s);
        double tr = 0.0, tr2 = 0.0;
        if (lane < n) {
          tr = B[lane * n + lane];
          for (int l = 0; l < n; ++l) tr2 += B[lane * n + l] * B[l * n + lane];
        }
        for (int off = 32; off > 0; off >>= 1) {
          tr += __shfl_xor(tr, off, 64);
          tr2 += __shfl_xor(tr2, off, 64);
        }
        if (lane == 0) {
          TRN[col * 2 + s] = tr;
          TRN2[col * 2 + s] = tr2;
        }
      }
    }
    __syncthreads();
    // 4. S += sum_a Xi_a N_a (virtual rows x all slots), and per member
    //    d_a ln|D_p| and tr((D_p^-1 Xi_a)^2)
    for (int q = tid; q < thsz + 2 * P; q += nth) {
      if (q < thsz) {
        const int s = q >= sT1, rr = q - soffT(s), n = ns(s);
        const int v = rr / n, h = rr % n;
        double acc = SS[q];
        for (int col = 0; col < Tc; ++col) {
          const double* B = BM + (size_t)col * bsz + soffB(s);
          for (int k = 0; k < n; ++k) acc += B[(n + v) * n + k] * B[k * n + h];
        }
        SS[q] = acc;
      } else {
        // member p, spin s: d_a ln|det D_p| = tr(D^-1 Xi_a[v][h]) and
        // tr((D^-1 Xi_a[v][h])^2) for the chunk's coordinates
        const int p = (q - thsz) >> 1, s = (q - thsz) & 1;
        const int k = t.lr_k[p * 2 + s];
        double qsum = QACC[p * 2 + s];
        const int n = ns(s);
        const int* hl = t.lr_hole + (p * 2 + s) * kMaxExc;
        const int* pt = t.lr_part + (p * 2 + s) * kMaxExc;
        const double* Di = DI + (p * 2 + s) * kMaxExc * kMaxExc;
        for (int col = 0; col < Tc; ++col) {
          double gp = 0.0;
          if (k > 0) {
            const double* B = BM + (size_t)col * bsz + soffB(s);
            double X[kMaxExc][kMaxExc], Mx[kMaxExc][kMaxExc];
#pragma unroll
            for (int j = 0; j < kMaxExc; ++j)
#pragma unroll
              for (int l = 0; l < kMaxExc; ++l) X[j][l] = (j < k && l < k) ? B[(n + pt[j]) * n + hl[l]] : 0.0;
#pragma unroll
            for (int l = 0; l < kMaxExc; ++l)
#pragma unroll
              for (int l2 = 0; l2 < kMaxExc; ++l2) {
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < kMaxExc; ++j) acc += Di[l * kMaxExc + j] * X[j][l2];
                Mx[l][l2] = acc;
              }
#pragma unroll
            for (int l = 0; l < kMaxExc; ++l) {
              gp += Mx[l][l];
#pragma unroll
              for (int l2 = 0; l2 < kMaxExc; ++l2) qsum += Mx[l][l2] * Mx[l2][l];
            }
          }
          GPA[(p * T + col) * 2 + s] = gp;
        }
        QACC[p * 2 + s] = qsum;
      }
    }
    __syncthreads();
    // 5. determinant sum per coordinate (one wavefront per coordinate, lanes
    //    over members, summed across the lanes in a fixed order), gamma and J
    {
      const int lane = tid & 63, wv = tid >> 6, nwv = nth >> 6;
      for (int col = wv; col < Tc; col += nwv) {
        const int a = a0 + col, k = a / 3, al = a % 3;
        const double trn = TRN[col * 2] + TRN[col * 2 + 1];
        double dpsi = 0.0, wsq = 0.0;
        for (int p = lane; p < P; p += 64) {
          const double gp = trn + GPA[(p * T + col) * 2] + GPA[(p * T + col) * 2 + 1];
          dpsi += WD[p] * gp;
          wsq += WD[p] * gp * gp;
        }
        for (int off = 32; off > 0; off >>= 1) {
          dpsi += __shfl_xor(dpsi, off, 64);
          wsq += __shfl_xor(wsq, off, 64);
        }
        if (lane == 0) {
          const double gtot = g[4 + 6 * k + al] + jt[col] + dpsi;
          grad[w * N * 3 + a] = gtot;
          LAPC[col] = wsq - dpsi * dpsi + g[4 + 6 * k + 3 + al];
          SQC[col] = gtot * gtot;
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      double lap = SCAL[0], sq = SCAL[1], t2u = SCAL[2], t2d = SCAL[3];
      for (int col = 0; col < Tc; ++col) {
        lap += LAPC[col];
        sq += SQC[col];
        t2u += TRN2[col * 2];
        t2d += TRN2[col * 2 + 1];
      }
      SCAL[0] = lap + jt[T];
      SCAL[1] = sq;
      SCAL[2] = t2u;
      SCAL[3] = t2d;
    }
    // the next chunk's first writes (TB, LT) are not read by thread 0 here,
    // and its TRN2 writes follow two more barriers
  }
  __syncthreads();
  // 6. Lambda = L G_0 on all rows (into the B buffer)
  for (int q = tid; q < bsz; q += nth) {
    const int s = q >= sB1, rr = q - soffB(s), n = ns(s);
    const int r = rr / n, k = rr % n;
    const double* lt = LT + (size_t)ROWORB[s * o.R0 + r] * N + e0s(s);
    const double* Gs = G0s + (s ? nu * nu : 0);
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += lt[i] * Gs[i * n + k];
    BM[q] = acc;
  }
  __syncthreads();
  // 7. Y = Lambda[virtual] - Theta Lambda[occ] - 2 S; tr Lambda[occ]
  for (int q = tid; q < thsz + 2; q += nth) {
    if (q < thsz) {
      const int s = q >= sT1, rr = q - soffT(s), n = ns(s);
      const int v = rr / n, h = rr % n;
      const double* Lm = BM + soffB(s);
      const double* th = THs + soffT(s) + v * n;
      double acc = Lm[(n + v) * n + h] - 2.0 * SS[q];
      for (int l = 0; l < n; ++l) acc -= th[l] * Lm[l * n + h];
      YY[q] = acc;
    } else {
      const int s = q - thsz, n = ns(s);
      const double* Lm = BM + soffB(s);
      double tr = 0.0;
      for (int k = 0; k < n; ++k) tr += Lm[k * n + k];
      SCAL[4 + s] = tr;
    }
  }
  __syncthreads();
  // 8. each member's Laplacian of ln|det|, both spins
  for (int p = tid; p < P; p += nth) {
    double dl = SCAL[4] + SCAL[5] - SCAL[2] - SCAL[3] - QACC[2 * p] - QACC[2 * p + 1];
    for (int s = 0; s < 2; ++s) {
      const int k = t.lr_k[p * 2 + s];
      if (k == 0) continue;
      const int n = ns(s);
      const int* hl = t.lr_hole + (p * 2 + s) * kMaxExc;
      const int* pt = t.lr_part + (p * 2 + s) * kMaxExc;
      const double* Di = DI + (p * 2 + s) * kMaxExc * kMaxExc;
      const double* Y = YY + soffT(s);
      for (int l = 0; l < k; ++l)
        for (int j = 0; j < k; ++j) dl += Di[l * kMaxExc + j] * Y[pt[j] * n + hl[l]];
    }
    DELTA[p] = dl;
  }
  __syncthreads();
  double* pw = partial + (size_t)w * n_chunks * 2;
  for (int q = tid; q < n_chunks * 2; q += nth) {
    if (q >= 2) pw[q] = 0.0;
  }
  if (tid == 0) {
    double dl = 0.0;
    for (int p = 0; p < P; ++p) dl += WD[p] * DELTA[p];
    pw[0] = SCAL[0] + dl;
    pw[1] = SCAL[1];
  }
}

}  // namespace

size_t lowrank_tangent_lds_bytes(const Dims& d, int T) {
  const LrLds o = lr_lds(d, T);
  return o.n_dbl * sizeof(double) + o.n_int * sizeof(int);
}

void launch_lowrank_value(const pn_ctx* c, hipStream_t s, int64_t nw, char* ws, const WsLayout& L, double* logabs,
                          double* sign) {
  const Dims& d = c->d;
  double* g0 = reinterpret_cast<double*>(ws + L.g0);
  double* ld0 = reinterpret_cast<double*>(ws + L.ld0);
  int* flag = reinterpret_cast<int*>(ws + L.lrflag);
  int* list = reinterpret_cast<int*>(ws + L.lrlist);
  // 1. the first determinant's LU per spin
  Dims d1 = d;
  d1.P = 1;
  launch_slater_lu(c, d1, s, nw, ws, L, g0, ld0, nullptr, nullptr, (nw * 2 + kThreads - 1) / kThreads,
                   (nw * 2 + kWaves - 1) / kWaves);
  // 2. excitation table, members' minors, hand-back flags
  const size_t lds = (size_t)kWaves * std::max(d.nv[0], d.nv[1]) * std::max(d.n_up, d.n_dn) * sizeof(double);
  hipLaunchKernelGGL(k_lr_value, dim3((unsigned)((nw * 2 + kWaves - 1) / kWaves)), dim3(kThreads), lds, s, d, c->t,
                     nw, reinterpret_cast<const double*>(ws + L.phi), reinterpret_cast<const double*>(ws + L.fval), g0,
                     ld0, reinterpret_cast<double*>(ws + L.theta), reinterpret_cast<double*>(ws + L.dinv),
                     reinterpret_cast<double*>(ws + L.ldet), flag);
  // 3. the handed-back walkers go through the direct LU of every member
  hipLaunchKernelGGL(k_lr_list, dim3(1), dim3(1024), 0, s, nw, flag, list);
  const int64_t nmat = nw * d.P * 2;
  launch_slater_lu(c, d, s, nw, ws, L, reinterpret_cast<double*>(ws + L.ginv), reinterpret_cast<double*>(ws + L.ldet),
                   list, list + nw, std::min<int64_t>((nmat + kThreads - 1) / kThreads, kListGrid),
                   std::min<int64_t>((nmat + kWaves - 1) / kWaves, kListGrid));
  launch_combine_value(c, s, nw, ws, L, logabs, sign);
}

void launch_lowrank_tangent(const pn_ctx* c, hipStream_t s, int64_t nw, char* ws, const WsLayout& L, double* grad) {
  const Dims& d = c->d;
  const int* flag = reinterpret_cast<const int*>(ws + L.lrflag);
  const int* list = reinterpret_cast<const int*>(ws + L.lrlist);
  auto go = [&](auto kern) {
    if (L.lds_lr > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)L.lds_lr);
    hipLaunchKernelGGL(kern, dim3((unsigned)nw), dim3(kThreads), L.lds_lr, s, d, c->t, nw, L.T, L.n_chunks,
                       reinterpret_cast<const double*>(ws + L.geo), reinterpret_cast<const double*>(ws + L.phi),
                       reinterpret_cast<const double*>(ws + L.fval), reinterpret_cast<const double*>(ws + L.ftan),
                       reinterpret_cast<const double*>(ws + L.jtan), reinterpret_cast<const double*>(ws + L.g0),
                       reinterpret_cast<const double*>(ws + L.theta), reinterpret_cast<const double*>(ws + L.dinv),
                       reinterpret_cast<const double*>(ws + L.wdet), flag, grad,
                       reinterpret_cast<double*>(ws + L.partial));
  };
  if (std::max(d.n_up, d.n_dn) >= 8 && L.lds_lr > 40 * 1024)
    go(&k_lr_tangent<true>);
  else
    go(&k_lr_tangent<false>);
  // the handed-back walkers: direct determinant tangents
  launch_slater_tangent(c, s, nw, nullptr, ws, L, grad, nullptr, list, list + nw);
}

}  // namespace pn
