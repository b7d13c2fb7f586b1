// Gradient of sum_w ct_w ln|psi_w| in the orbital values at the nuclei of
// the cusp correction (Methods, "Cusp conditions": the paper optimizes
// them), FP64.
//
// Inside r_cusp of nucleus I the on-centre s part of MO mu is replaced by
// s~(rho) = sgn(s0) exp(a0 + a1 rho + ... + a4 rho^4), whose coefficients
// depend on the nucleus value s0 (a0 = ln|s0|, a1 = -Z (eta0 + s0) / s0,
// a2..a4 by the matching conditions at r_cusp), so
//   d s~(rho) / d s0 = s~(rho) sum_k (d a_k / d s0) rho^k
// (the derivatives d a_k / d s0 come from the host set-up).  With
// A_p^s[k][i] = phi_mu(r_i) f_{i mu},  d ln|Psi_d| / d phi_mu(r_i) =
// f_{i mu} sum_p w_p sum_{k: mu_p(k) = mu} G_p[i][k], and
//   d ln|psi| / d s0[I][mu] = sum_{i: |r_i - R_I| < r_cusp} that * d s~(rho_i) / d s0.
//
// k_cusp_grad: a fixed grid of blocks strides over walkers; thread (i, mu)
// accumulates into its own LDS entries [i][I][mu] in walker order; each block
// then sums its electrons into its slot.  k_cusp_reduce adds the slots in
// block order, so the result is reproducible bit for bit.
#include <math.h>

#include "pn_internal.h"

namespace pn {
namespace {

constexpr int kSlotsCusp = 256;

__global__ __launch_bounds__(kThreads) void k_cusp_grad(Dims d, DevTables t, int64_t nw, const double* __restrict__ r,
                                                        const double* __restrict__ ginv,
                                                        const double* __restrict__ wdet,
                                                        const double* __restrict__ fval,
                                                        const double* __restrict__ ct, double* __restrict__ slot) {
  extern __shared__ __align__(16) char smem[];
  double* acc = reinterpret_cast<double*>(smem);  // [N][NN][M]
  const int N = d.N, NN = d.NN, M = d.M, P = d.P, NU = d.n_up;
  const int gsz = d.n_up * d.n_up + d.n_dn * d.n_dn;
  for (int q = threadIdx.x; q < N * NN * M; q += blockDim.x) acc[q] = 0.0;
  __syncthreads();
  for (int64_t w = blockIdx.x; w < nw; w += gridDim.x) {
    const double cw = ct[w];
    for (int q = threadIdx.x; q < N * M; q += blockDim.x) {
      const int i = q / M, mu = q % M;
      const double* ri = r + (w * N + i) * 3;
      for (int I = 0; I < NN; ++I) {
        if (!t.cusp_on[I * M + mu]) continue;
        const double x = ri[0] - t.nuc_xyz[3 * I], y = ri[1] - t.nuc_xyz[3 * I + 1], z = ri[2] - t.nuc_xyz[3 * I + 2];
        const double rho = sqrt(x * x + y * y + z * z);
        if (!(rho < d.cusp_rc)) continue;
        // f_{i mu} sum_p w_p sum_{k: mu_p(k) = mu} G_p[i][k]
        const bool up = i < NU;
        const int n = up ? d.n_up : d.n_dn, ii = up ? i : i - NU;
        const int* dets = up ? t.det_up : t.det_dn;
        double D = 0.0;
        for (int p = 0; p < P; ++p) {
          const double* G = ginv + (w * P + p) * gsz + (up ? 0 : d.n_up * d.n_up);
          double s = 0.0;
          for (int k = 0; k < n; ++k)
            if (dets[p * n + k] == mu) s += G[ii * n + k];
          D += wdet[w * P + p] * s;
        }
        const double* al = t.cusp_alpha + ((size_t)I * M + mu) * 5;
        const double* da = t.cusp_dalpha + ((size_t)I * M + mu) * 5;
        const double pr = al[0] + rho * (al[1] + rho * (al[2] + rho * (al[3] + rho * al[4])));
        const double dp = da[0] + rho * (da[1] + rho * (da[2] + rho * (da[3] + rho * da[4])));
        const double sv = t.cusp_sign[I * M + mu] * exp(pr);
        acc[((size_t)i * NN + I) * M + mu] += cw * D * fval[(w * N + i) * M + mu] * sv * dp;
      }
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < NN * M; q += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < N; ++i) s += acc[(size_t)i * NN * M + q];
    slot[(size_t)blockIdx.x * NN * M + q] = s;
  }
}

__global__ __launch_bounds__(kThreads) void k_cusp_reduce(int n, int nslots, const double* __restrict__ slot,
                                                          double* __restrict__ grad) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  double s = 0.0;
  for (int b = 0; b < nslots; ++b) s += slot[(size_t)b * n + q];
  grad[q] += s;
}

}  // namespace

size_t cusp_grad_lds_bytes(const Dims& d) { return (size_t)d.N * d.NN * d.M * sizeof(double); }

void launch_cusp_grad(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, char* ws, const WsLayout& L,
                      const double* ct, double* slot, double* grad) {
  const Dims& d = c->d;
  const int nb = (int)std::min<int64_t>(nw, kSlotsCusp);
  const size_t lds = cusp_grad_lds_bytes(d);
  if (lds > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cusp_grad), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  hipLaunchKernelGGL(k_cusp_grad, dim3(nb), dim3(kThreads), lds, s, d, c->t, nw, r,
                     reinterpret_cast<const double*>(ws + L.ginv), reinterpret_cast<const double*>(ws + L.wdet),
                     reinterpret_cast<const double*>(ws + L.fval), ct, slot);
  const int n = d.NN * d.M;
  hipLaunchKernelGGL(k_cusp_reduce, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, n, nb, slot, grad);
}

}  // namespace pn
