// Pair geometry, Coulomb potential, electronic cusp factor and the
// cusp-corrected Gaussian orbitals with their coordinate derivatives.
//
// One workgroup per walker.  Output per walker (FP64):
//   geo: V, gamma, then per electron  d gamma/d r_i (3)  and the diagonal
//        second derivatives d^2 gamma / d r_{i,a}^2 (3)
//   phi: [N][M][7]  phi_mu(r_i), its gradient and diagonal second
//        derivatives with respect to r_i.
//
// V = sum_{i<j} 1/r_ij - sum_{i,I} Z_I / r_iI + V_nn  (the electronic
// Hamiltonian in E_loc, Methods eq. "monte-carlo").
// gamma = sum_{i<j} -c_ij / (1 + r_ij), c_ij = 1/2 for opposite spins and
// 1/4 for same spins (Methods, "Cusp conditions").
// Orbitals: phi_mu = sum_b C_{b mu} chi_b with primitive normalised s/p
// Gaussians; inside r_cusp of nucleus I the on-centre s part is replaced
// by sign * exp(a0 + a1 rho + a2 rho^2 + a3 rho^3 + a4 rho^4) (the Ma et al.
// scheme the paper cites; coefficients are set up on the host).
#include "pn_internal.h"

namespace pn {
namespace {

__device__ __forceinline__ double block_sum(double v, double* red) {
  // wave64 shuffle reduction, then across waves through LDS
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0) {
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
    red[0] = s;
  }
  __syncthreads();
  s = red[0];
  __syncthreads();
  return s;
}

constexpr int kEG = 8;  // electrons per basis-staging group

__global__ __launch_bounds__(kThreads) void k_geometry_orbitals(Dims d, DevTables t, const double* __restrict__ r,
                                                                double* __restrict__ geo, double* __restrict__ phi) {
  extern __shared__ __align__(16) char smem[];
  const int w = blockIdx.x;
  const int N = d.N, NN = d.NN, NB = d.NB, M = d.M;
  double* rs = reinterpret_cast<double*>(smem);   // [N][3]
  double* red = rs + 3 * kMaxElec;                  // [8]
  double* chi = red + 8;                            // [kEG][NB][7]
  const double* rw = r + (size_t)w * N * 3;
  for (int k = threadIdx.x; k < 3 * N; k += blockDim.x) rs[k] = rw[k];
  __syncthreads();

  // --- potential and gamma value (one term per pair) ---
  double v = 0, gam = 0;
  const int n_ee = d.n_ee;
  for (int p = threadIdx.x; p < n_ee + N * NN; p += blockDim.x) {
    if (p < n_ee) {
      int i = t.pair_ij[2 * p], j = t.pair_ij[2 * p + 1];
      double dx = rs[3 * i] - rs[3 * j], dy = rs[3 * i + 1] - rs[3 * j + 1], dz = rs[3 * i + 2] - rs[3 * j + 2];
      double rij = sqrt(dx * dx + dy * dy + dz * dz);
      v += 1.0 / rij;
      double c = ((i < d.n_up) == (j < d.n_up)) ? 0.25 : 0.5;
      gam += -c / (1.0 + rij);
    } else {
      int q = p - n_ee, i = q / NN, I = q % NN;
      double dx = rs[3 * i] - t.nuc_xyz[3 * I], dy = rs[3 * i + 1] - t.nuc_xyz[3 * I + 1],
             dz = rs[3 * i + 2] - t.nuc_xyz[3 * I + 2];
      v -= t.charge[I] / sqrt(dx * dx + dy * dy + dz * dz);
    }
  }
  v = block_sum(v, red);
  gam = block_sum(gam, red);
  const int GS = kGeoStride(N);
  double* gw = geo + (size_t)w * GS;
  if (threadIdx.x == 0) {
    gw[0] = v + d.v_nn;
    gw[1] = gam;
    gw[2] = 0;
    gw[3] = 0;
  }
  // --- gamma derivatives per electron coordinate ---
  for (int q = threadIdx.x; q < 3 * N; q += blockDim.x) {
    int i = q / 3, a = q % 3;
    double g1 = 0, g2 = 0;
    for (int j = 0; j < N; ++j) {
      if (j == i) continue;
      double dx = rs[3 * i] - rs[3 * j], dy = rs[3 * i + 1] - rs[3 * j + 1], dz = rs[3 * i + 2] - rs[3 * j + 2];
      double rij = sqrt(dx * dx + dy * dy + dz * dz);
      double c = ((i < d.n_up) == (j < d.n_up)) ? 0.25 : 0.5;
      double op = 1.0 + rij;
      double f1 = c / (op * op);          // dF/dr for F = -c/(1+r)
      double f2 = -2.0 * c / (op * op * op);
      double ua = (a == 0 ? dx : (a == 1 ? dy : dz)) / rij;
      g1 += f1 * ua;
      g2 += f2 * ua * ua + f1 / rij * (1.0 - ua * ua);
    }
    gw[4 + 6 * i + a] = g1;
    gw[4 + 6 * i + 3 + a] = g2;
  }

  // --- orbitals, electrons in groups of kEG ---
  double* phw = phi + (size_t)w * N * M * 7;
  for (int e0 = 0; e0 < N; e0 += kEG) {
    const int ne = min(kEG, N - e0);
    __syncthreads();
    // basis jets: (electron, shell)
    for (int q = threadIdx.x; q < ne * d.n_shell; q += blockDim.x) {
      int ie = q / d.n_shell, sh = q % d.n_shell, i = e0 + ie;
      int C = t.shell_center[sh];
      double a = t.shell_exp[sh], nrm = t.shell_norm[sh];
      double x[3] = {rs[3 * i] - t.nuc_xyz[3 * C], rs[3 * i + 1] - t.nuc_xyz[3 * C + 1],
                     rs[3 * i + 2] - t.nuc_xyz[3 * C + 2]};
      double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
      double g = nrm * exp(-a * r2);
      double* out = chi + ((size_t)ie * NB + t.shell_first[sh]) * 7;
      if (t.shell_l[sh] == 0) {
        out[0] = g;
        for (int b = 0; b < 3; ++b) {
          out[1 + b] = -2.0 * a * x[b] * g;
          out[4 + b] = (4.0 * a * a * x[b] * x[b] - 2.0 * a) * g;
        }
      } else {
        for (int c = 0; c < 3; ++c) {
          double* o = out + 7 * c;
          o[0] = x[c] * g;
          for (int b = 0; b < 3; ++b) {
            double dcb = (b == c) ? 1.0 : 0.0;
            o[1 + b] = (dcb - 2.0 * a * x[c] * x[b]) * g;
            o[4 + b] = (-4.0 * a * dcb * x[b] - 2.0 * a * x[c] + 4.0 * a * a * x[c] * x[b] * x[b]) * g;
          }
        }
      }
    }
    __syncthreads();
    // MO contraction and cusp correction: (electron, MO)
    for (int q = threadIdx.x; q < ne * M; q += blockDim.x) {
      int ie = q / M, mu = q % M, i = e0 + ie;
      double acc[7] = {0, 0, 0, 0, 0, 0, 0};
      const double* ch = chi + (size_t)ie * NB * 7;
      for (int b = 0; b < NB; ++b) {
        double cb = t.mo[(size_t)b * M + mu];
#pragma unroll
        for (int k = 0; k < 7; ++k) acc[k] += cb * ch[7 * b + k];
      }
      if (d.cusp_rc > 0) {
        for (int I = 0; I < NN; ++I) {
          if (!t.cusp_on[I * M + mu]) continue;
          double x[3] = {rs[3 * i] - t.nuc_xyz[3 * I], rs[3 * i + 1] - t.nuc_xyz[3 * I + 1],
                         rs[3 * i + 2] - t.nuc_xyz[3 * I + 2]};
          double rho = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
          if (!(rho < d.cusp_rc)) continue;
          // remove the on-centre s part
          for (int k = t.s_first[I]; k < t.s_first[I + 1]; ++k) {
            double cb = t.mo[(size_t)t.s_basis[k] * M + mu];
            const double* cs = ch + 7 * t.s_basis[k];
#pragma unroll
            for (int m = 0; m < 7; ++m) acc[m] -= cb * cs[m];
          }
          // add sign * exp(p(rho)) as a radial function
          const double* al = t.cusp_alpha + ((size_t)I * M + mu) * 5;
          double p = al[0] + rho * (al[1] + rho * (al[2] + rho * (al[3] + rho * al[4])));
          double p1 = al[1] + rho * (2 * al[2] + rho * (3 * al[3] + rho * 4 * al[4]));
          double p1_over_r = al[1] / rho + 2 * al[2] + rho * (3 * al[3] + rho * 4 * al[4]);
          double p2 = 2 * al[2] + rho * (6 * al[3] + rho * 12 * al[4]);
          double gv = t.cusp_sign[I * M + mu] * exp(p);
          double g1r = gv * p1_over_r;       // g'/rho
          double g2 = gv * (p2 + p1 * p1);   // g''
          acc[0] += gv;
          for (int b = 0; b < 3; ++b) {
            double ub = x[b] / rho;
            acc[1 + b] += g1r * x[b];
            acc[4 + b] += g2 * ub * ub + g1r * (1.0 - ub * ub);
          }
        }
      }
      double* o = phw + ((size_t)i * M + mu) * 7;
#pragma unroll
      for (int k = 0; k < 7; ++k) o[k] = acc[k];
    }
  }
}

}  // namespace

void launch_geometry_orbitals(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, char* ws,
                              const WsLayout& L) {
  const Dims& d = c->d;
  size_t lds = (3 * kMaxElec + 8 + (size_t)kEG * d.NB * 7) * sizeof(double);
  hipLaunchKernelGGL(k_geometry_orbitals, dim3((unsigned)nw), dim3(kThreads), lds, s, d, c->t, r,
                     reinterpret_cast<double*>(ws + L.geo), reinterpret_cast<double*>(ws + L.phi));
}

}  // namespace pn
