// Full adjoint, determinant part (FP64): cotangents on d ln|psi| / d r, on
// the Laplacian of ln|psi| and on E_loc are carried back through the
// multideterminant sum and the Slater determinants to the backflow f and
// its coordinate derivatives (the table entries).
//
// Per walker, with cotangents cg_a on d_a ln|psi| (a over the 3N
// coordinates), cl on the Laplacian, ce on E_loc = -1/2 (lap + |grad|^2) + V
// (Methods, eq. "monte-carlo"; V does not depend on the parameters) and c0
// on ln|psi|:
//   cg'_a = cg_a - ce grad_a,   cl' = cl - ce / 2.
// The determinant sum (w_p = c_p D_p / Psi_d, g_pa = d_a ln|D_p|,
// Delta_p = lap ln|D_p|, both spins added):
//   d_a ln|Psi_d| = sum_p w_p g_pa
//   lap ln|Psi_d| = sum_p w_p (Delta_p + |g_p|^2) - |d ln|Psi_d||^2
// gives
//   ct g_pa    = w_p (cg'_a + 2 cl' (g_pa - d_a ln|Psi_d|))
//   ct Delta_p = cl' w_p
//   ct l_p     = w_p (c~_p - sum_q w_q c~_q) + c0 w_p
//   c~_p       = sum_a cg'_a g_pa + cl' (Delta_p + |g_p|^2 - 2 g_p . d ln|Psi_d|)
// with l_p = ln|c_p D_p|.  Per determinant and spin, with G = A^{-1},
// M_a = G T_a (T_a = d A / d r_a) and L the Laplacian of A:
//   g_a = tr M_a,  Delta = tr(G L) - sum_a tr(M_a^2),  l = ln|det A|
//   ct A   = (Q G)^T,  Q = ct_l I - sum_a ct_g_a M_a - ct_Delta G L + 2 ct_Delta sum_a M_a^2
//   ct T_a = ((ct_g_a I - 2 ct_Delta M_a) G)^T
//   ct L   = ct_Delta G^T
// The table entries A = phi f, T_a = d_a phi f + phi d_a f and (per chunk of
// coordinates) L = sum_{a in chunk} (d_a^2 phi f + 2 d_a phi d_a f) + phi lap_chunk f
// pass these on to f, its tangents and its partial Laplacians.
//
//  k_adj_combine  one wavefront per walker: the per-walker and
//                 per-determinant cotangents above.
//  k_adj_slater   one block per (walker, coordinate chunk); the block takes
//                 the (determinant, spin) pairs one after the other, so every
//                 accumulation into the backflow cotangents happens in a
//                 fixed order.
#include <math.h>

#include "pn_internal.h"

namespace pn {
namespace {

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// detres: [nw][n_chunks][P][2][T+1] (d_a ln det per chunk coordinate, chunk
// Laplacian part at T); ctc out: [nw][3N+2] (cg', cl', c0);
// ctdet out: [nw][P][3N+2] (ct g_pa, ct Delta_p, ct l_p).
__global__ __launch_bounds__(kThreads) void k_adj_combine(Dims d, int64_t nw, int T, int n_chunks,
                                                          const double* __restrict__ detres,
                                                          const double* __restrict__ wdet,
                                                          const double* __restrict__ gradf,
                                                          const double* __restrict__ ct_logabs,
                                                          const double* __restrict__ ct_grad,
                                                          const double* __restrict__ ct_lap,
                                                          const double* __restrict__ ct_eloc,
                                                          double* __restrict__ ctc, double* __restrict__ ctdet) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (w >= nw) return;
  const int N3 = 3 * d.N, P = d.P, Tp = T + 1;
  const double ce = ct_eloc ? ct_eloc[w] : 0.0;
  const double cl = (ct_lap ? ct_lap[w] : 0.0) - 0.5 * ce;
  const double c0 = ct_logabs ? ct_logabs[w] : 0.0;
  double* cc = ctc + w * (N3 + 2);
  for (int a = lane; a < N3; a += 64)
    cc[a] = (ct_grad ? ct_grad[w * N3 + a] : 0.0) - ce * gradf[w * N3 + a];
  if (lane == 0) {
    cc[N3] = cl;
    cc[N3 + 1] = c0;
  }
  const double* wd = wdet + w * P;
  const double* dr = detres + (size_t)w * n_chunks * P * 2 * Tp;
  auto gpa = [&](int p, int a) {
    const double* x = dr + ((size_t)(a / T) * P * 2 + 2 * p) * Tp + a % T;
    return x[0] + x[Tp];
  };
  // d_a ln|Psi_d| for the lane's coordinates (at most 3 kMaxElec / 64 = 3 per lane)
  double dps[3], cgp[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int a = lane + 64 * s;
    double v = 0.0;
    if (a < N3)
      for (int p = 0; p < P; ++p) v += wd[p] * gpa(p, a);
    dps[s] = v;
    cgp[s] = a < N3 ? (ct_grad ? ct_grad[w * N3 + a] : 0.0) - ce * gradf[w * N3 + a] : 0.0;
  }
  // c~_p, then ct l_p = w_p (c~_p - sum_q w_q c~_q) + c0 w_p; c~_p is kept in ctdet[p][N3 + 1] meanwhile
  double wct = 0.0;
  for (int p = 0; p < P; ++p) {
    double* cd = ctdet + (w * P + p) * (N3 + 2);
    double sg = 0.0, g2 = 0.0, gd = 0.0;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int a = lane + 64 * s;
      if (a < N3) {
        const double g = gpa(p, a);
        sg += cgp[s] * g;
        g2 += g * g;
        gd += g * dps[s];
        cd[a] = wd[p] * (cgp[s] + 2.0 * cl * (g - dps[s]));
      }
    }
    sg = wave_sum_d(sg);
    g2 = wave_sum_d(g2);
    gd = wave_sum_d(gd);
    double Dp = 0.0;
    for (int ch = 0; ch < n_chunks; ++ch) {
      const double* x = dr + ((size_t)ch * P * 2 + 2 * p) * Tp + T;
      Dp += x[0] + x[Tp];
    }
    const double ct = sg + cl * (Dp + g2 - 2.0 * gd);
    wct += wd[p] * ct;
    if (lane == 0) {
      cd[N3] = cl * wd[p];
      cd[N3 + 1] = ct;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int p = lane; p < P; p += 64) {
    double* cd = ctdet + (w * P + p) * (N3 + 2);
    cd[N3 + 1] = wd[p] * (cd[N3 + 1] - wct) + c0 * wd[p];
  }
}

// ctftan out: [nw][n_chunks][N][T+1][M] (cotangents of f's tangents and, at
// column T, of the chunk's partial Laplacian of f); ctfpart out:
// [nw][n_chunks][N][M] (the chunk's share of the cotangent of f itself).
__global__ __launch_bounds__(kThreads) void k_adj_slater(Dims d, DevTables t, int64_t nw, int T, int n_chunks,
                                                         const double* __restrict__ phi,
                                                         const double* __restrict__ fval,
                                                         const double* __restrict__ ftan,
                                                         const double* __restrict__ ginv,
                                                         const double* __restrict__ ctdet,
                                                         double* __restrict__ ctftan, double* __restrict__ ctfpart) {
  extern __shared__ __align__(16) char smem[];
  const int64_t task = blockIdx.x;
  const int64_t w = task / n_chunks;
  const int chunk = (int)(task % n_chunks);
  if (w >= nw) return;
  const int N = d.N, M = d.M, P = d.P, N3 = 3 * N;
  const int a0 = chunk * T, Tc = min(T, N3 - a0), C = Tc + 1, LC = Tc, Tp = T + 1;
  const int NM = max(max(d.n_up, d.n_dn), 1);
  double* TB = reinterpret_cast<double*>(smem);  // [C][M][N] table derivatives
  double* ctT = TB + (size_t)C * M * N;          // [C][N][M] cotangents of f tangents (col LC: Laplacian)
  double* ctv = ctT + (size_t)C * N * M;         // [N][M]    cotangent of f
  double* G = ctv + (size_t)N * M;               // [n][n]
  double* Ms = G + (size_t)NM * NM;              // [C][n][n] M_a = G T_a (col LC: G L)
  double* MG = Ms + (size_t)C * NM * NM;         // [C][n][n] M_a G
  double* Q = MG + (size_t)C * NM * NM;          // [n][n]

  const double* ph = phi + w * N * M * 7;
  const double* fv = fval + w * N * M;
  const double* ft = ftan + (w * n_chunks + chunk) * N * Tp * M;
  for (int q = threadIdx.x; q < C * M * N; q += blockDim.x) {
    const int col = q / (M * N), mu = (q / N) % M, i = q % N;
    const double* pj = ph + ((size_t)i * M + mu) * 7;
    const double f = fv[i * M + mu];
    double v;
    if (col < LC) {
      const int a = a0 + col, k = a / 3, al = a % 3;
      v = pj[0] * ft[((size_t)i * Tp + col) * M + mu];
      if (k == i) v += pj[1 + al] * f;
    } else {
      v = pj[0] * ft[((size_t)i * Tp + T) * M + mu];
      for (int c2 = 0; c2 < LC; ++c2) {
        const int a = a0 + c2, k = a / 3, al = a % 3;
        if (k != i) continue;
        v += pj[4 + al] * f + 2.0 * pj[1 + al] * ft[((size_t)i * Tp + c2) * M + mu];
      }
    }
    TB[q] = v;
  }
  for (int q = threadIdx.x; q < C * N * M + N * M; q += blockDim.x) ctT[q] = 0.0;
  __syncthreads();
  const int gsz = d.n_up * d.n_up + d.n_dn * d.n_dn;
  for (int ps = 0; ps < 2 * P; ++ps) {
    const int p = ps / 2, spin = ps % 2;
    const int n = spin == 0 ? d.n_up : d.n_dn;
    if (n == 0) continue;  // an empty spin block has det = 1 and no derivatives
    const int e0 = spin == 0 ? 0 : d.n_up;
    const int* occ = spin == 0 ? t.det_up + p * d.n_up : t.det_dn + p * d.n_dn;
    const double* cd = ctdet + (w * P + p) * (N3 + 2);
    const double cD = cd[N3], cl0 = chunk == 0 ? cd[N3 + 1] : 0.0;
    const double* Gg = ginv + (w * P + p) * gsz + (spin == 0 ? 0 : d.n_up * d.n_up);
    const int nn = n * n;
    for (int q = threadIdx.x; q < nn; q += blockDim.x) G[q] = Gg[q];
    __syncthreads();
    for (int q = threadIdx.x; q < C * nn; q += blockDim.x) {
      const int col = q / nn, x = (q / n) % n, y = q % n;
      const double* tb = TB + (size_t)col * M * N + e0 + y;
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += G[x * n + k] * tb[(size_t)occ[k] * N];
      Ms[q] = s;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < Tc * nn; q += blockDim.x) {
      const int col = q / nn, x = (q / n) % n, y = q % n;
      const double* mr = Ms + ((size_t)col * n + x) * n;
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += mr[k] * G[k * n + y];
      MG[q] = s;
    }
    for (int q = threadIdx.x; q < nn; q += blockDim.x) {
      const int x = q / n, y = q % n;
      double v = (x == y ? cl0 : 0.0) - cD * Ms[((size_t)LC * n + x) * n + y];
      for (int col = 0; col < Tc; ++col) {
        const double* mc = Ms + (size_t)col * nn;
        double sq = 0.0;
        for (int k = 0; k < n; ++k) sq += mc[x * n + k] * mc[k * n + y];
        v += -cd[a0 + col] * mc[x * n + y] + 2.0 * cD * sq;
      }
      Q[q] = v;
    }
    __syncthreads();
    // (x, k): electron e0 + x, orbital occ[k]; distinct within a determinant
    for (int q = threadIdx.x; q < nn; q += blockDim.x) {
      const int x = q / n, k = q % n, mu = occ[k], i = e0 + x;
      const double* pj = ph + ((size_t)i * M + mu) * 7;
      double cA = 0.0;
      for (int m = 0; m < n; ++m) cA += Q[x * n + m] * G[m * n + k];
      const double gxk = G[x * n + k], cL = cD * gxk;
      double vs = cA * pj[0];
      for (int col = 0; col < Tc; ++col) {
        const int a = a0 + col;
        const double cT = cd[a] * gxk - 2.0 * cD * MG[((size_t)col * n + x) * n + k];
        double v = cT * pj[0];
        if (a / 3 == i) {
          const int al = a % 3;
          v += 2.0 * cL * pj[1 + al];
          vs += cT * pj[1 + al] + cL * pj[4 + al];
        }
        ctT[((size_t)col * N + i) * M + mu] += v;
      }
      ctT[((size_t)LC * N + i) * M + mu] += cL * pj[0];
      ctv[i * M + mu] += vs;
    }
    __syncthreads();
  }
  double* co = ctftan + (size_t)task * N * Tp * M;
  for (int q = threadIdx.x; q < N * Tp * M; q += blockDim.x) {
    const int i = q / (Tp * M), col = (q / M) % Tp, mu = q % M;
    co[q] = col < Tc ? ctT[((size_t)col * N + i) * M + mu] : (col == T ? ctT[((size_t)LC * N + i) * M + mu] : 0.0);
  }
  double* cv = ctfpart + (size_t)task * N * M;
  for (int q = threadIdx.x; q < N * M; q += blockDim.x) cv[q] = ctv[q];
}

}  // namespace

size_t adj_slater_lds_bytes(const Dims& d, int T) {
  const int C = T + 1, NM = std::max(std::max(d.n_up, d.n_dn), 1);
  return ((size_t)2 * C * d.M * d.N + (size_t)d.N * d.M + (size_t)(2 + 2 * C) * NM * NM) * sizeof(double);
}

void launch_adj_det(const pn_ctx* c, hipStream_t s, int64_t nw, const WsLayout& L, char* ws, const double* ct_logabs,
                    const double* ct_grad, const double* ct_lap, const double* ct_eloc) {
  const Dims& d = c->d;
  const int wpb = kThreads / 64;
  hipLaunchKernelGGL(k_adj_combine, dim3((unsigned)((nw + wpb - 1) / wpb)), dim3(kThreads), 0, s, d, nw, L.T,
                     L.n_chunks, reinterpret_cast<const double*>(ws + L.detres),
                     reinterpret_cast<const double*>(ws + L.wdet), reinterpret_cast<const double*>(ws + L.gradf),
                     ct_logabs, ct_grad, ct_lap, ct_eloc, reinterpret_cast<double*>(ws + L.ctc),
                     reinterpret_cast<double*>(ws + L.ctdet));
  const size_t lds = adj_slater_lds_bytes(d, L.T);
  if (lds > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_adj_slater), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  hipLaunchKernelGGL(k_adj_slater, dim3((unsigned)(nw * L.n_chunks)), dim3(kThreads), lds, s, d, c->t, nw, L.T,
                     L.n_chunks, reinterpret_cast<const double*>(ws + L.phi),
                     reinterpret_cast<const double*>(ws + L.fval), reinterpret_cast<const double*>(ws + L.ftan),
                     reinterpret_cast<const double*>(ws + L.ginv), reinterpret_cast<const double*>(ws + L.ctdet),
                     reinterpret_cast<double*>(ws + L.ctftan), reinterpret_cast<double*>(ws + L.ctfpart));
}

}  // namespace pn
