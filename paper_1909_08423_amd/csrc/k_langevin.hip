// Langevin Monte Carlo sampling of |psi|^2 (Methods, "Ansatz optimization";
// Table 2): the drift-diffusion moves of Umrigar, Nightingale and Runge
// (J. Chem. Phys. 99, 2865 (1993)) as simplified in the paper, where the
// step is clipped below the distance to the nearest nucleus instead of their
// radial step proposal.
//
// One step for every walker (all electrons at once):
//   d_i(r)  = tau grad_i ln|psi|(r), rescaled to length <= min_I |r_i - R_I|
//   r'      = m(r) + sqrt(tau) xi,        m(r) = r + d(r)
//   ln A    = 2 (ln|psi(r')| - ln|psi(r)|) - (|r - m(r')|^2 - |r' - m(r)|^2) / (2 tau)
//   accept  u < A (Metropolis-Hastings with the forward and backward
//           Gaussian proposal densities)
//   tau    <- tau exp(k (a - a*)) after the step (a: batch acceptance)
// ln|psi| and its gradient at r' come from pn_eval; the kept walkers carry
// theirs from step to step, so each step evaluates the wavefunction once.
// Random numbers: Philox4x32-10 with counter (walker, step, call, 0), the
// normals of call j by Box-Muller for coordinates 2j and 2j + 1, the
// acceptance uniform from call 0xFFFFFFFF (the Metropolis step's scheme).
#include <math.h>

#include "philox.h"
#include "pn_internal.h"

namespace pn {
namespace {

// tau g_i rescaled to at most the distance of r_i to the nearest nucleus
__device__ __forceinline__ void clipped_drift(const double* ri, const double* gi, const double* nuc, int NN, double tau,
                                              double d[3]) {
  d[0] = tau * gi[0];
  d[1] = tau * gi[1];
  d[2] = tau * gi[2];
  if (NN == 0) return;
  double dist2 = INFINITY;
  for (int I = 0; I < NN; ++I) {
    const double x = ri[0] - nuc[3 * I], y = ri[1] - nuc[3 * I + 1], z = ri[2] - nuc[3 * I + 2];
    dist2 = fmin(dist2, x * x + y * y + z * z);
  }
  const double dist = sqrt(dist2), nrm = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  if (nrm > dist) {
    const double sc = dist / nrm;
    d[0] *= sc;
    d[1] *= sc;
    d[2] *= sc;
  }
}

__global__ __launch_bounds__(kThreads) void k_lang_propose(int64_t nw, int N, const double* __restrict__ r,
                                                           const double* __restrict__ g, const double* __restrict__ nuc,
                                                           int NN, const double* __restrict__ tau_p, uint64_t seed,
                                                           int64_t step, double* __restrict__ rp,
                                                           double* __restrict__ qf) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  const double tau = *tau_p, st = sqrt(tau);
  const int ncoord = 3 * N;
  const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  const double* rw = r + w * ncoord;
  const double* gw = g + w * ncoord;
  double* pw = rp + w * ncoord;
  // diffusion part first
  for (int j = 0; 2 * j < ncoord; ++j) {
    uint32_t c[4] = {(uint32_t)w, (uint32_t)step, (uint32_t)j, 0u};
    philox4x32_10(c, k0, k1);
    const double u1 = u53(c[0], c[1]), u2 = u53(c[2], c[3]);
    const double rad = sqrt(-2.0 * log(u1)), ang = 2.0 * M_PI * u2;
    pw[2 * j] = st * (rad * cos(ang));
    if (2 * j + 1 < ncoord) pw[2 * j + 1] = st * (rad * sin(ang));
  }
  double q = 0.0;
  for (int i = 0; i < N; ++i) {
    double d[3];
    clipped_drift(rw + 3 * i, gw + 3 * i, nuc, NN, tau, d);
    for (int a = 0; a < 3; ++a) {
      const double m = rw[3 * i + a] + d[a], v = m + pw[3 * i + a];
      const double e = v - m;
      q += e * e;
      pw[3 * i + a] = v;
    }
  }
  qf[w] = q;
}

__global__ __launch_bounds__(kThreads) void k_lang_accept(int64_t nw, int N, double* __restrict__ r,
                                                          double* __restrict__ la, double* __restrict__ g,
                                                          const double* __restrict__ rp,
                                                          const double* __restrict__ lap,
                                                          const double* __restrict__ gp,
                                                          const double* __restrict__ nuc, int NN,
                                                          const double* __restrict__ tau_p, uint64_t seed, int64_t step,
                                                          const double* __restrict__ qf, int* __restrict__ acc) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  const double tau = *tau_p;
  const int ncoord = 3 * N;
  double* rw = r + w * ncoord;
  const double* pw = rp + w * ncoord;
  const double* gpw = gp + w * ncoord;
  double qb = 0.0;
  for (int i = 0; i < N; ++i) {
    double d[3];
    clipped_drift(pw + 3 * i, gpw + 3 * i, nuc, NN, tau, d);
    for (int a = 0; a < 3; ++a) {
      const double e = rw[3 * i + a] - (pw[3 * i + a] + d[a]);
      qb += e * e;
    }
  }
  uint32_t c[4] = {(uint32_t)w, (uint32_t)step, kAcceptCall, 0u};
  philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  const double u = u53(c[0], c[1]);
  const double log_a = 2.0 * (lap[w] - la[w]) - (qb - qf[w]) / (2.0 * tau);
  const bool ok = u < exp(log_a);
  acc[w] = ok ? 1 : 0;
  if (ok) {
    for (int a = 0; a < ncoord; ++a) {
      rw[a] = pw[a];
      g[w * ncoord + a] = gpw[a];
    }
    la[w] = lap[w];
  }
}

// one block: batch acceptance, the step's statistics and the next tau
__global__ __launch_bounds__(kThreads) void k_lang_adapt(int64_t nw, const int* __restrict__ acc,
                                                         double* __restrict__ tau_p, double target, double rate,
                                                         double* __restrict__ stats) {
  __shared__ double red[kThreads / 64];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < nw; k += blockDim.x) s += acc[k];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < kThreads / 64; ++k) t += red[k];
    const double a = t / (double)nw, tau = *tau_p;
    stats[0] = a;
    stats[1] = tau;
    *tau_p = tau * exp(rate * (a - target));
  }
}

struct LangWs {
  size_t eval, rp, la, lap, sg, sgp, g, gp, qf, acc, total;
};

LangWs lang_layout(const pn_ctx* c, int64_t nw, pn_precision prec) {
  LangWs L{};
  size_t eb = 0;
  pn_workspace_bytes(c, nw, prec, PN_OUT_LOGABS | PN_OUT_GRAD, &eb);
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t nc = (size_t)nw * c->d.N * 3 * 8, n1 = (size_t)nw * 8;
  size_t off = 0;
  L.eval = off;
  off = al(off + eb);
  L.rp = off;
  off = al(off + nc);
  L.g = off;
  off = al(off + nc);
  L.gp = off;
  off = al(off + nc);
  L.la = off;
  off = al(off + n1);
  L.lap = off;
  off = al(off + n1);
  L.sg = off;
  off = al(off + n1);
  L.sgp = off;
  off = al(off + n1);
  L.qf = off;
  off = al(off + n1);
  L.acc = off;
  off = al(off + (size_t)nw * 4);
  L.total = off;
  return L;
}

}  // namespace
}  // namespace pn

using namespace pn;

extern "C" {

pn_status pn_langevin_workspace_bytes(const pn_ctx* c, int64_t nw, pn_precision prec, size_t* bytes) {
  if (!c || !bytes || nw < 1 || prec < PN_PREC_FP64 || prec > PN_PREC_NET_BF16) return PN_ERR_INVALID_ARG;
  *bytes = lang_layout(c, nw, prec).total;
  return PN_OK;
}

pn_status pn_langevin_run(const pn_ctx* c, hipStream_t s, int64_t nw, double* r, const double* params,
                          pn_precision prec, const pn_langevin_hparams* hp, double* tau, int32_t n_steps,
                          uint64_t seed, int64_t step0, double* stats, void* ws, size_t ws_bytes) {
  if (!c || !hp || prec < PN_PREC_FP64 || prec > PN_PREC_NET_BF16) return PN_ERR_INVALID_ARG;
  if (nw < 1 || n_steps < 0 || step0 < 0) return PN_ERR_INVALID_ARG;
  if (!r || !params || !tau || !ws || (n_steps > 0 && !stats)) return PN_ERR_INVALID_ARG;
  if (!(hp->target_accept > 0 && hp->target_accept < 1) || !(hp->adapt_rate >= 0)) return PN_ERR_INVALID_ARG;
  const LangWs L = lang_layout(c, nw, prec);
  if (ws_bytes < L.total) return PN_ERR_WORKSPACE_TOO_SMALL;
  if (n_steps == 0) return PN_OK;
  char* base = static_cast<char*>(ws);
  void* wse = base + L.eval;
  const size_t wse_bytes = L.rp - L.eval;
  double* rp = reinterpret_cast<double*>(base + L.rp);
  double* g = reinterpret_cast<double*>(base + L.g);
  double* gp = reinterpret_cast<double*>(base + L.gp);
  double* la = reinterpret_cast<double*>(base + L.la);
  double* lap = reinterpret_cast<double*>(base + L.lap);
  double* sg = reinterpret_cast<double*>(base + L.sg);
  double* sgp = reinterpret_cast<double*>(base + L.sgp);
  double* qf = reinterpret_cast<double*>(base + L.qf);
  int* acc = reinterpret_cast<int*>(base + L.acc);
  const unsigned nb = (unsigned)((nw + kThreads - 1) / kThreads);
  pn_status st = pn_eval(c, s, nw, r, params, prec, la, sg, g, nullptr, nullptr, wse, wse_bytes);
  if (st != PN_OK) return st;
  for (int32_t k = 0; k < n_steps; ++k) {
    const int64_t step = step0 + k;
    hipLaunchKernelGGL(k_lang_propose, dim3(nb), dim3(kThreads), 0, s, nw, c->d.N, r, g, c->t.nuc_xyz, c->d.NN, tau,
                       seed, step, rp, qf);
    st = pn_eval(c, s, nw, rp, params, prec, lap, sgp, gp, nullptr, nullptr, wse, wse_bytes);
    if (st != PN_OK) return st;
    hipLaunchKernelGGL(k_lang_accept, dim3(nb), dim3(kThreads), 0, s, nw, c->d.N, r, la, g, rp, lap, gp,
                       c->t.nuc_xyz, c->d.NN, tau, seed, step, qf, acc);
    hipLaunchKernelGGL(k_lang_adapt, dim3(1), dim3(kThreads), 0, s, nw, acc, tau, hp->target_accept, hp->adapt_rate,
                       stats + 2 * k);
  }
  if (hipGetLastError() != hipSuccess) return PN_ERR_DEVICE;
  return PN_OK;
}

}  // extern "C"
