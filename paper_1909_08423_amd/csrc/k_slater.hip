// Slater determinants of the backflowed orbitals, the multideterminant sum,
// their coordinate derivatives and the local energy (all FP64).
//
// A_p^s[k][i] = phi_{mu_p^s(k)}(r_i) f_{i mu_p^s(k)}   over electrons i of
// spin s (Results, eq. "ansatz"; antisymmetry by the determinant).
//
//  k_slater_value    one wavefront per (walker, determinant, spin): LU with
//                    partial pivoting (ties to the lowest row), ln|det|,
//                    sign, and G = A^{-1}; for spin blocks of at most 8
//                    electrons k_slater_value_lane takes one matrix per lane
//                    (Gauss-Jordan in registers, same pivoting rule).
//  k_combine_value   signed log-sum-exp of c_p det_up det_down; weights
//                    w_p = c_p D_p / Psi_d; ln|psi| = gamma + J + ln|Psi_d|.
//  k_slater_tangent  one block per (walker, coordinate chunk).  For every
//                    coordinate a of the chunk: T_a = d A / d r_a,
//                    d_a ln det = tr(G T_a), and the chunk's part of the
//                    Laplacian tr(G L) - sum_a tr((G T_a)^2).  Then the
//                    determinant sum per coordinate:
//                      d_a ln Psi_d  = sum_p w_p g_pa
//                      d2_a ln Psi_d = sum_p w_p (D2_pa + g_pa^2) - (d_a ln Psi_d)^2
//                    and gamma and J are added.
//  k_finalize        lap = sum of chunk partials;
//                    E_loc = -1/2 (lap + |grad|^2) + V  (Methods, eq.
//                    "monte-carlo").
#include <math.h>

#include "pn_internal.h"

namespace pn {
namespace {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

constexpr int kWaves = kThreads / 64;

// With wlist set, the (determinant, spin) matrices of the listed walkers
// only (*wcount of them), taken by a grid-stride loop.
__global__ __launch_bounds__(kThreads) void k_slater_value(Dims d, DevTables t, int64_t nw,
                                                           const double* __restrict__ phi,
                                                           const double* __restrict__ fval,
                                                           double* __restrict__ ginv, double* __restrict__ ldet,
                                                           const int* __restrict__ wlist,
                                                           const int* __restrict__ wcount) {
  extern __shared__ __align__(16) char smem[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int NM = max(d.n_up, d.n_dn), LD = NM + 1;
  double* A = reinterpret_cast<double*>(smem) + (size_t)wv * 2 * NM * LD;
  double* X = A + NM * LD;
  int* perm = reinterpret_cast<int*>(reinterpret_cast<double*>(smem) + (size_t)kWaves * 2 * NM * LD) + wv * kMaxSpin;
  const int64_t nmat = (wlist ? (int64_t)*wcount : nw) * d.P * 2;
  for (int64_t mat = (int64_t)blockIdx.x * kWaves + wv; mat < nmat; mat += (int64_t)gridDim.x * kWaves) {
  const int spin = (int)(mat % 2);
  const int p = (int)((mat / 2) % d.P);
  const int64_t w = wlist ? (int64_t)wlist[mat / (2 * d.P)] : mat / (2 * d.P);
  const int n = spin == 0 ? d.n_up : d.n_dn;
  const int e0 = spin == 0 ? 0 : d.n_up;
  const int* occ = spin == 0 ? t.det_up + p * d.n_up : t.det_dn + p * d.n_dn;
  const int N = d.N, M = d.M;
  const int gsz = d.n_up * d.n_up + d.n_dn * d.n_dn;
  double* G = ginv + (w * d.P + p) * gsz + (spin == 0 ? 0 : d.n_up * d.n_up);
  double* ld = ldet + ((w * d.P + p) * 2 + spin) * 2;
  if (n == 0) {
    if (lane == 0) {
      ld[0] = 0.0;
      ld[1] = 1.0;
    }
    continue;
  }
  const double* ph = phi + w * N * M * 7;
  const double* fv = fval + w * N * M;
  for (int q = lane; q < n * n; q += 64) {
    int k = q / n, i = q % n;
    int mu = occ[k], e = e0 + i;
    A[k * LD + i] = ph[((size_t)e * M + mu) * 7] * fv[(size_t)e * M + mu];
  }
  if (lane < n) perm[lane] = lane;
  wave_sync();
  double logabs = 0.0, sgn = 1.0;
  bool singular = false;
  for (int c = 0; c < n; ++c) {
    // pivot: largest |A[r][c]|, r >= c, ties to the lowest row
    double best = -1.0;
    int bi = n;
    if (lane >= c && lane < n) {
      best = fabs(A[lane * LD + c]);
      bi = lane;
    }
    for (int o = 32; o > 0; o >>= 1) {
      double ob = __shfl_xor(best, o, 64);
      int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (bi != c) {
      for (int col = lane; col < n; col += 64) {
        double tmp = A[c * LD + col];
        A[c * LD + col] = A[bi * LD + col];
        A[bi * LD + col] = tmp;
      }
      if (lane == 0) {
        int tp = perm[c];
        perm[c] = perm[bi];
        perm[bi] = tp;
      }
      sgn = -sgn;
    }
    wave_sync();
    const double pv = A[c * LD + c];
    if (pv == 0.0) {
      singular = true;
      break;
    }
    logabs += log(fabs(pv));
    if (pv < 0) sgn = -sgn;
    for (int r = c + 1 + lane; r < n; r += 64) A[r * LD + c] /= pv;
    wave_sync();
    const int m = n - c - 1;
    for (int q = lane; q < m * m; q += 64) {
      int r = c + 1 + q / m, col = c + 1 + q % m;
      A[r * LD + col] -= A[r * LD + c] * A[c * LD + col];
    }
    wave_sync();
  }
  if (singular) {
    if (lane == 0) {
      ld[0] = -INFINITY;
      ld[1] = 0.0;
    }
    for (int q = lane; q < n * n; q += 64) G[q] = 0.0;
    wave_sync();
    continue;
  }
  if (lane == 0) {
    ld[0] = logabs;
    ld[1] = sgn;
  }
  // column j of A^{-1} = U^{-1} L^{-1} P e_j ; lane j, work column X[.][j]
  if (lane < n) {
    const int j = lane;
    for (int r = 0; r < n; ++r) {
      double v = (perm[r] == j) ? 1.0 : 0.0;
      for (int s2 = 0; s2 < r; ++s2) v -= A[r * LD + s2] * X[s2 * LD + j];
      X[r * LD + j] = v;
    }
    for (int r = n - 1; r >= 0; --r) {
      double v = X[r * LD + j];
      for (int s2 = r + 1; s2 < n; ++s2) v -= A[r * LD + s2] * X[s2 * LD + j];
      X[r * LD + j] = v / A[r * LD + r];
    }
  }
  wave_sync();
  for (int q = lane; q < n * n; q += 64) G[q] = X[(q / n) * LD + q % n];
  wave_sync();
  }
}

// Small determinants (n <= NMAX): one lane per (walker, determinant, spin).
// Gauss-Jordan inversion in registers with partial pivoting (largest
// |a[r][c]|, ties to the lowest row): ln|det| and sign from the pivots, then
// the column swaps undone in reverse order give G = A^{-1}.  Every loop is
// unrolled over NMAX, so the matrix stays in registers.
template <int NMAX>
__global__ __launch_bounds__(kThreads) void k_slater_value_lane(Dims d, DevTables t, int64_t nw,
                                                                const double* __restrict__ phi,
                                                                const double* __restrict__ fval,
                                                                double* __restrict__ ginv, double* __restrict__ ldet,
                                                                const int* __restrict__ wlist,
                                                                const int* __restrict__ wcount) {
  const int64_t nmat = (wlist ? (int64_t)*wcount : nw) * d.P * 2;
  for (int64_t mat = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; mat < nmat;
       mat += (int64_t)gridDim.x * blockDim.x) {
  const int spin = (int)(mat % 2);
  const int p = (int)((mat / 2) % d.P);
  const int64_t w = wlist ? (int64_t)wlist[mat / (2 * d.P)] : mat / (2 * d.P);
  const int n = spin == 0 ? d.n_up : d.n_dn;
  const int e0 = spin == 0 ? 0 : d.n_up;
  const int* occ = spin == 0 ? t.det_up + p * d.n_up : t.det_dn + p * d.n_dn;
  const int N = d.N, M = d.M;
  const int gsz = d.n_up * d.n_up + d.n_dn * d.n_dn;
  double* G = ginv + (w * d.P + p) * gsz + (spin == 0 ? 0 : d.n_up * d.n_up);
  double* ld = ldet + ((w * d.P + p) * 2 + spin) * 2;
  if (n == 0) {
    ld[0] = 0.0;
    ld[1] = 1.0;
    continue;
  }
  const double* ph = phi + w * N * M * 7;
  const double* fv = fval + w * N * M;
  double a[NMAX][NMAX];
  int oc[NMAX];
#pragma unroll
  for (int k = 0; k < NMAX; ++k) oc[k] = k < n ? occ[k] : 0;
#pragma unroll
  for (int k = 0; k < NMAX; ++k)
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
      const size_t q = (size_t)(e0 + i) * M + oc[k];
      a[k][i] = (k < n && i < n) ? ph[q * 7] * fv[q] : (k == i ? 1.0 : 0.0);  // identity padding
    }
  int piv[NMAX];
  double logabs = 0.0, sgn = 1.0;
  bool singular = false;
#pragma unroll
  for (int c = 0; c < NMAX; ++c) {
    int bi = c;
    double best = fabs(a[c][c]);
#pragma unroll
    for (int r = c + 1; r < NMAX; ++r) {
      const double v = fabs(a[r][c]);
      if (r < n && v > best) {
        best = v;
        bi = r;
      }
    }
    piv[c] = bi;
    if (bi != c) sgn = -sgn;
#pragma unroll
    for (int r = c + 1; r < NMAX; ++r) {
      if (r == bi) {
#pragma unroll
        for (int col = 0; col < NMAX; ++col) {
          const double tmp = a[c][col];
          a[c][col] = a[r][col];
          a[r][col] = tmp;
        }
      }
    }
    double pv = a[c][c];
    if (c < n) {
      if (pv == 0.0) {
        singular = true;
        pv = 1.0;
      }
      logabs += log(fabs(pv));
      if (pv < 0) sgn = -sgn;
    }
    const double inv = 1.0 / pv;
    a[c][c] = 1.0;
#pragma unroll
    for (int col = 0; col < NMAX; ++col) a[c][col] *= inv;
#pragma unroll
    for (int r = 0; r < NMAX; ++r) {
      if (r == c) continue;
      const double f = a[r][c];
      a[r][c] = 0.0;
#pragma unroll
      for (int col = 0; col < NMAX; ++col) a[r][col] -= f * a[c][col];
    }
  }
  // undo the row interchanges as column interchanges, last first
#pragma unroll
  for (int c = NMAX - 1; c >= 0; --c) {
#pragma unroll
    for (int col = c + 1; col < NMAX; ++col) {
      if (piv[c] == col) {
#pragma unroll
        for (int r = 0; r < NMAX; ++r) {
          const double tmp = a[r][c];
          a[r][c] = a[r][col];
          a[r][col] = tmp;
        }
      }
    }
  }
  if (singular) {
    ld[0] = -INFINITY;
    ld[1] = 0.0;
  } else {
    ld[0] = logabs;
    ld[1] = sgn;
  }
  // a now holds A^{-1}[electron][orbital slot]
#pragma unroll
  for (int i = 0; i < NMAX; ++i)
#pragma unroll
    for (int k = 0; k < NMAX; ++k)
      if (i < n && k < n) G[i * n + k] = singular ? 0.0 : a[i][k];
  }
}

__global__ __launch_bounds__(kThreads) void k_combine_value(Dims d, DevTables t, int64_t nw,
                                                            const double* __restrict__ geo,
                                                            const double* __restrict__ jval,
                                                            const double* __restrict__ ldet,
                                                            double* __restrict__ wdet, double* __restrict__ ldpsi,
                                                            double* __restrict__ logabs, double* __restrict__ sign) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  const int P = d.P;
  const double* ld = ldet + w * P * 4;
  double m = -INFINITY;
  for (int p = 0; p < P; ++p) {
    double l = t.ci_log[p] + ld[4 * p] + ld[4 * p + 2];
    if (l > m) m = l;
  }
  double S = 0.0;
  if (m > -INFINITY) {
    for (int p = 0; p < P; ++p) {
      double l = t.ci_log[p] + ld[4 * p] + ld[4 * p + 2];
      double s = t.ci_sign[p] * ld[4 * p + 1] * ld[4 * p + 3];
      S += s * exp(l - m);
    }
  }
  double* wd = wdet + w * P;
  const double* g = geo + w * kGeoStride(d.N);
  if (S == 0.0) {
    for (int p = 0; p < P; ++p) wd[p] = 0.0;
    ldpsi[w] = -INFINITY;
    logabs[w] = -INFINITY;
    sign[w] = 0.0;
    return;
  }
  for (int p = 0; p < P; ++p) {
    double l = t.ci_log[p] + ld[4 * p] + ld[4 * p + 2];
    double s = t.ci_sign[p] * ld[4 * p + 1] * ld[4 * p + 3];
    wd[p] = (l > -INFINITY) ? s * exp(l - m) / S : 0.0;
  }
  double lp = m + log(fabs(S));
  ldpsi[w] = lp;
  logabs[w] = g[1] + jval[w] + lp;
  sign[w] = S > 0 ? 1.0 : -1.0;
}

template <int NMAX>
__global__ __launch_bounds__(kThreads) void k_slater_tangent(Dims d, DevTables t, int64_t nw, int T, int n_chunks,
                                                             const double* __restrict__ geo,
                                                             const double* __restrict__ phi,
                                                             const double* __restrict__ fval,
                                                             const double* __restrict__ ftan,
                                                             const double* __restrict__ jtan,
                                                             const double* __restrict__ ginv,
                                                             const double* __restrict__ wdet,
                                                             double* __restrict__ grad, double* __restrict__ partial,
                                                             double* __restrict__ detres,
                                                             const int* __restrict__ wlist,
                                                             const int* __restrict__ wcount) {
  extern __shared__ __align__(16) char smem[];
  // one (walker, chunk) task per iteration; with wlist set only the listed
  // walkers' tasks (*wcount walkers), taken by a grid-stride loop
  const int64_t ntask = (wlist ? (int64_t)*wcount : nw) * n_chunks;
  for (int64_t it = blockIdx.x; it < ntask; it += gridDim.x) {
  const int64_t w = wlist ? (int64_t)wlist[it / n_chunks] : it / n_chunks;
  const int chunk = (int)(it % n_chunks);
  const int64_t task = w * n_chunks + chunk;
  const int N = d.N, M = d.M, P = d.P;
  const int a0 = chunk * T, Tc = min(T, 3 * N - a0), C = Tc + 1, LC = Tc;
  const int NM = max(max(d.n_up, d.n_dn), 1);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double* TB = reinterpret_cast<double*>(smem);       // [C][M][N] table derivatives
  double* gres = TB + (size_t)C * M * N;              // [P][2][T]
  double* dres = gres + (size_t)P * 2 * T;            // [P][2]
  double* scr = dres + (size_t)P * 2;                 // per wave scratch, SW doubles
  const int SW = C * NM * NM + 2 * C * NM;

  const double* ph = phi + w * N * M * 7;
  const double* fv = fval + w * N * M;
  const double* ft = ftan + (w * n_chunks + chunk) * N * (T + 1) * M;
  // table derivatives: column col = d/dr_a (a = a0 + col), column LC = chunk Laplacian
  for (int q = threadIdx.x; q < C * M * N; q += blockDim.x) {
    int col = q / (M * N), mu = (q / N) % M, i = q % N;
    const double* pj = ph + ((size_t)i * M + mu) * 7;
    double f = fv[i * M + mu];
    if (col < LC) {
      int a = a0 + col, k = a / 3, al = a % 3;
      double v = pj[0] * ft[((size_t)i * (T + 1) + col) * M + mu];
      if (k == i) v += pj[1 + al] * f;
      TB[q] = v;
    } else {
      double v = pj[0] * ft[((size_t)i * (T + 1) + T) * M + mu];
      for (int c2 = 0; c2 < LC; ++c2) {
        int a = a0 + c2, k = a / 3, al = a % 3;
        if (k != i) continue;
        v += pj[4 + al] * f + 2.0 * pj[1 + al] * ft[((size_t)i * (T + 1) + c2) * M + mu];
      }
      TB[q] = v;
    }
  }
  __syncthreads();
  // per (determinant, spin), one wavefront each; its lanes take (column,
  // row x) pairs and form row x of M_a = G T_a for all columns at once
  const int gsz = d.n_up * d.n_up + d.n_dn * d.n_dn;
  for (int ps = wv; ps < P * 2; ps += kWaves) {
    const int p = ps / 2, spin = ps % 2;
    const int n = spin == 0 ? d.n_up : d.n_dn;
    const int e0 = spin == 0 ? 0 : d.n_up;
    const int* occ = spin == 0 ? t.det_up + p * d.n_up : t.det_dn + p * d.n_dn;
    double* gr = gres + (size_t)ps * T;
    if (n == 0) {
      for (int col = lane; col < Tc; col += 64) gr[col] = 0.0;
      if (lane == 0) dres[ps] = 0.0;
      continue;
    }
    const double* Gg = ginv + (w * P + p) * gsz + (spin == 0 ? 0 : d.n_up * d.n_up);
    double* Ms = scr + (size_t)wv * SW;     // [C][n][n] rows of M_a
    double* gpart = Ms + (size_t)C * NM * NM;  // [C][n] diagonal of M_a, or tr(G L) parts
    double* qpart = gpart + (size_t)C * NM;    // [C][n] sum_y M[x][y] M[y][x]
    for (int it = lane; it < C * n; it += 64) {
      const int col = it / n, x = it % n;
      const double* tb = TB + (size_t)col * M * N + e0;
      double row[NMAX];
#pragma unroll
      for (int y = 0; y < NMAX; ++y) row[y] = 0.0;
      for (int k = 0; k < n; ++k) {
        const double gxk = Gg[x * n + k];
        const double* tk = tb + (size_t)occ[k] * N;
#pragma unroll
        for (int y = 0; y < NMAX; ++y)
          if (y < n) row[y] += gxk * tk[y];
      }
      double* mr = Ms + ((size_t)col * n + x) * n;
#pragma unroll
      for (int y = 0; y < NMAX; ++y)
        if (y < n) mr[y] = row[y];
    }
    wave_sync();
    for (int it = lane; it < C * n; it += 64) {
      const int col = it / n, x = it % n;
      const double* mc = Ms + (size_t)col * n * n;
      gpart[col * n + x] = mc[x * n + x];  // the Laplacian column gives tr(G L)
      double q = 0.0;
      if (col != LC)
        for (int y = 0; y < n; ++y) q += mc[x * n + y] * mc[y * n + x];
      qpart[col * n + x] = q;
    }
    wave_sync();
    double sq = 0.0;
    for (int col = lane; col < C; col += 64) {
      double tr = 0.0, q = 0.0;
      for (int x = 0; x < n; ++x) {
        tr += gpart[col * n + x];
        q += qpart[col * n + x];
      }
      if (col < LC) {
        gr[col] = tr;
        sq += q;
      } else {
        dres[ps] = tr;  // tr(G L)
      }
    }
    sq = wave_sum(sq);
    wave_sync();
    if (lane == 0) dres[ps] -= sq;
    wave_sync();
  }
  __syncthreads();
  // per-determinant results for the adjoint pass: [P][2][T+1] per (walker,
  // chunk): d_a ln det for the chunk's coordinates, then the chunk's part of
  // the Laplacian of ln det at index T
  if (detres) {
    double* dr = detres + (size_t)task * P * 2 * (T + 1);
    for (int q = threadIdx.x; q < P * 2 * (T + 1); q += blockDim.x) {
      const int ps = q / (T + 1), col = q % (T + 1);
      dr[q] = col < Tc ? gres[(size_t)ps * T + col] : (col == T ? dres[ps] : 0.0);
    }
  }
  // determinant sum per coordinate, then gamma and J
  const double* g = geo + w * kGeoStride(N);
  const double* jt = jtan + (w * n_chunks + chunk) * (T + 1);
  const double* wd = wdet + w * P;
  if (threadIdx.x < 64) {
    double lap_part = 0.0, sq_part = 0.0;
    for (int col = lane; col < Tc; col += 64) {
      const int a = a0 + col, k = a / 3, al = a % 3;
      double dpsi = 0.0, wsq = 0.0;
      for (int p = 0; p < P; ++p) {
        double gp = gres[(2 * p) * T + col] + gres[(2 * p + 1) * T + col];
        dpsi += wd[p] * gp;
        wsq += wd[p] * gp * gp;
      }
      lap_part += wsq - dpsi * dpsi + g[4 + 6 * k + 3 + al];
      double gtot = g[4 + 6 * k + al] + jt[col] + dpsi;
      grad[w * N * 3 + a] = gtot;
      sq_part += gtot * gtot;
    }
    lap_part = wave_sum(lap_part);
    sq_part = wave_sum(sq_part);
    if (lane == 0) {
      double dl = 0.0;
      for (int p = 0; p < P; ++p) dl += wd[p] * (dres[2 * p] + dres[2 * p + 1]);
      partial[(w * n_chunks + chunk) * 2] = lap_part + dl + jt[T];
      partial[(w * n_chunks + chunk) * 2 + 1] = sq_part;
    }
  }
  __syncthreads();  // the next task overwrites the tables
  }
}

__global__ __launch_bounds__(kThreads) void k_finalize(Dims d, int64_t nw, int n_chunks, const double* __restrict__ geo,
                                                       const double* __restrict__ partial, double* __restrict__ lap,
                                                       double* __restrict__ eloc) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  double l = 0.0, s = 0.0;
  for (int c = 0; c < n_chunks; ++c) {
    l += partial[(w * n_chunks + c) * 2];
    s += partial[(w * n_chunks + c) * 2 + 1];
  }
  if (lap) lap[w] = l;
  if (eloc) eloc[w] = -0.5 * (l + s) + geo[w * kGeoStride(d.N)];
}

}  // namespace

// LU of every (walker, determinant, spin) matrix of the dims `d` (which may
// restrict the expansion to its first determinant), written to G / ld; with
// a walker list, the listed walkers only, on a fixed grid.
void launch_slater_lu(const pn_ctx* c, const Dims& d, hipStream_t s, int64_t nw, char* ws, const WsLayout& L,
                      double* G, double* ld, const int* wlist, const int* wcount, int64_t nb_lane, int64_t nb_wave) {
  const int NM = std::max(d.n_up, d.n_dn);
  if (NM <= 8) {
    auto kern = NM <= 4 ? &k_slater_value_lane<4> : (NM <= 6 ? &k_slater_value_lane<6> : &k_slater_value_lane<8>);
    hipLaunchKernelGGL(kern, dim3((unsigned)std::max<int64_t>(nb_lane, 1)), dim3(kThreads), 0, s, d, c->t, nw,
                       reinterpret_cast<const double*>(ws + L.phi), reinterpret_cast<const double*>(ws + L.fval), G, ld,
                       wlist, wcount);
  } else {
    size_t lds = (size_t)kWaves * 2 * NM * (NM + 1) * sizeof(double) + kWaves * kMaxSpin * sizeof(int);
    hipLaunchKernelGGL(k_slater_value, dim3((unsigned)std::max<int64_t>(nb_wave, 1)), dim3(kThreads), lds, s, d, c->t,
                       nw, reinterpret_cast<const double*>(ws + L.phi), reinterpret_cast<const double*>(ws + L.fval), G,
                       ld, wlist, wcount);
  }
}

void launch_slater_value(const pn_ctx* c, hipStream_t s, int64_t nw, char* ws, const WsLayout& L, double* logabs,
                         double* sign) {
  const Dims& d = c->d;
  int64_t nmat = nw * d.P * 2;
  launch_slater_lu(c, d, s, nw, ws, L, reinterpret_cast<double*>(ws + L.ginv), reinterpret_cast<double*>(ws + L.ldet),
                   nullptr, nullptr, (nmat + kThreads - 1) / kThreads, (nmat + kWaves - 1) / kWaves);
  launch_combine_value(c, s, nw, ws, L, logabs, sign);
}

void launch_combine_value(const pn_ctx* c, hipStream_t s, int64_t nw, char* ws, const WsLayout& L, double* logabs,
                          double* sign) {
  const Dims& d = c->d;
  int64_t nb2 = (nw + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_combine_value, dim3((unsigned)nb2), dim3(kThreads), 0, s, d, c->t, nw,
                     reinterpret_cast<const double*>(ws + L.geo), reinterpret_cast<const double*>(ws + L.jval),
                     reinterpret_cast<const double*>(ws + L.ldet), reinterpret_cast<double*>(ws + L.wdet),
                     reinterpret_cast<double*>(ws + L.ldpsi), logabs, sign);
}

size_t slater_tangent_lds_bytes(const Dims& d, int T) {
  const int C = T + 1, NM = std::max(std::max(d.n_up, d.n_dn), 1);
  return ((size_t)C * d.M * d.N + (size_t)d.P * 2 * T + d.P * 2 + (size_t)kWaves * (C * NM * NM + 2 * C * NM)) *
         sizeof(double);
}

void launch_slater_tangent(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, char* ws, const WsLayout& L,
                           double* grad, double* detres, const int* wlist, const int* wcount) {
  const Dims& d = c->d;
  (void)r;
  size_t lds = slater_tangent_lds_bytes(d, L.T);
  const int NM = std::max(d.n_up, d.n_dn);
  // a listed subset (walkers the low-rank path hands back) runs on a fixed grid
  const int64_t nb = wlist ? std::min<int64_t>(nw * L.n_chunks, kListGrid) : nw * L.n_chunks;
  auto go = [&](auto kern) {
    if (lds > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
    hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(kThreads), lds, s, d, c->t, nw, L.T,
                       L.n_chunks, reinterpret_cast<const double*>(ws + L.geo),
                       reinterpret_cast<const double*>(ws + L.phi), reinterpret_cast<const double*>(ws + L.fval),
                       reinterpret_cast<const double*>(ws + L.ftan), reinterpret_cast<const double*>(ws + L.jtan),
                       reinterpret_cast<const double*>(ws + L.ginv), reinterpret_cast<const double*>(ws + L.wdet),
                       grad, reinterpret_cast<double*>(ws + L.partial), detres, wlist, wcount);
  };
  if (NM <= 8)
    go(&k_slater_tangent<8>);
  else if (NM <= 16)
    go(&k_slater_tangent<16>);
  else
    go(&k_slater_tangent<32>);
}

void launch_finalize(const pn_ctx* c, hipStream_t s, int64_t nw, char* ws, const WsLayout& L, double* grad,
                     double* lap, double* eloc) {
  (void)grad;
  int64_t nb = (nw + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)nb), dim3(kThreads), 0, s, c->d, nw, L.n_chunks,
                     reinterpret_cast<const double*>(ws + L.geo), reinterpret_cast<const double*>(ws + L.partial),
                     lap, eloc);
}

}  // namespace pn
