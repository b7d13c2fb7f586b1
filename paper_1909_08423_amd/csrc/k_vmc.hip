// One VMC step of a job (Methods, "Ansatz optimization"; Table 2):
// Metropolis move on |psi|^2, local energy, smooth clipping, the Hermitian
// gradient estimator (eq. "trainig") and AdamW.  The wavefunction work goes
// through pn_eval / pn_eval_backward; this file holds the sampling,
// statistics and optimizer kernels and the step sequence.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key =
// seed (low, high 32 bits), counter = (walker, step, call, 0).  Each call
// gives two uniforms in (0, 1) built from 53 bits,
//   u = ((x0 >> 5) 2^26 + (x1 >> 6) + 1/2) 2^-53,
// turned into two normals by Box-Muller.  Call 0xFFFFFFFF gives the
// acceptance uniform.
#include <math.h>

#include <algorithm>

#include "philox.h"
#include "pn_internal.h"

namespace pn {
namespace {

// Proposal r' = r + sigma xi for walker w (all its coordinates).
__device__ __forceinline__ void propose_walker(int64_t w, int ncoord, const double* __restrict__ r,
                                               double* __restrict__ rp, double sigma, uint64_t seed, int64_t step) {
  const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  for (int j = 0; 2 * j < ncoord; ++j) {
    uint32_t c[4] = {(uint32_t)w, (uint32_t)step, (uint32_t)j, 0u};
    philox4x32_10(c, k0, k1);
    const double u1 = u53(c[0], c[1]), u2 = u53(c[2], c[3]);
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = 2.0 * M_PI * u2;
    const int a = 2 * j;
    rp[w * ncoord + a] = r[w * ncoord + a] + sigma * rad * cos(ang);
    if (a + 1 < ncoord) rp[w * ncoord + a + 1] = r[w * ncoord + a + 1] + sigma * rad * sin(ang);
  }
}

// Metropolis acceptance of walker w: u < |psi(r')|^2 / |psi(r)|^2.
__device__ __forceinline__ void accept_walker(int64_t w, int ncoord, double* __restrict__ r,
                                              const double* __restrict__ rp, const double* __restrict__ la,
                                              const double* __restrict__ lap, uint64_t seed, int64_t step,
                                              int* __restrict__ acc) {
  uint32_t c[4] = {(uint32_t)w, (uint32_t)step, kAcceptCall, 0u};
  philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  const double u = u53(c[0], c[1]);
  const bool ok = u < exp(2.0 * (lap[w] - la[w]));
  acc[w] = ok ? 1 : 0;
  if (ok)
    for (int a = 0; a < ncoord; ++a) r[w * ncoord + a] = rp[w * ncoord + a];
}

__global__ __launch_bounds__(kThreads) void k_propose(int64_t nw, int ncoord, const double* __restrict__ r,
                                                      double* __restrict__ rp, double sigma, uint64_t seed,
                                                      int64_t step) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w < nw) propose_walker(w, ncoord, r, rp, sigma, seed, step);
}

__global__ __launch_bounds__(kThreads) void k_accept(int64_t nw, int ncoord, double* __restrict__ r,
                                                     const double* __restrict__ rp, const double* __restrict__ la,
                                                     const double* __restrict__ lap, uint64_t seed, int64_t step,
                                                     int* __restrict__ acc) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w < nw) accept_walker(w, ncoord, r, rp, la, lap, seed, step, acc);
}

constexpr int kClipThreads = 1024;

__device__ double block_sum_d(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = 0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];  // same order in every thread
  __syncthreads();
  return s;
}

// One block: median, mean absolute deviation, clipped energies, the
// per-walker weights 2/B (E~ - L) and the step statistics.
__device__ void clip_job(int64_t nw, int npow2, const double* __restrict__ eloc, const int* __restrict__ acc,
                         double q, double* __restrict__ ct, double* __restrict__ stats, char* smem) {
  double* red = reinterpret_cast<double*>(smem);  // [16]
  double* srt = red + 16;                          // [npow2]
  const int B = (int)nw;
  double nonfin = 0, sum = 0, acc_sum = 0;
  for (int k = threadIdx.x; k < npow2; k += blockDim.x) {
    double e = k < B ? eloc[k] : INFINITY;
    if (k < B) {
      if (!isfinite(e)) {
        nonfin += 1;
        e = INFINITY;
      } else {
        sum += e;
      }
      acc_sum += acc[k];
    }
    srt[k] = e;
  }
  nonfin = block_sum_d(nonfin, red);
  sum = block_sum_d(sum, red);
  acc_sum = block_sum_d(acc_sum, red);
  // bitonic sort, ascending
  for (int size = 2; size <= npow2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int k = threadIdx.x; k < npow2; k += blockDim.x) {
        const int pk = k ^ stride;
        if (pk > k) {
          const bool up = (k & size) == 0;
          const double a = srt[k], b = srt[pk];
          if ((a > b) == up) {
            srt[k] = b;
            srt[pk] = a;
          }
        }
      }
    }
  }
  __syncthreads();
  const double med = (B & 1) ? srt[B / 2] : 0.5 * (srt[B / 2 - 1] + srt[B / 2]);
  const double mean = sum / B;
  double dev = 0, var = 0;
  for (int k = threadIdx.x; k < B; k += blockDim.x) {
    dev += fabs(eloc[k] - med);
    var += (eloc[k] - mean) * (eloc[k] - mean);
  }
  dev = block_sum_d(dev, red) / B;
  var = block_sum_d(var, red) / B;
  const double wdw = q * dev;
  const bool ok = nonfin == 0;
  double csum = 0;
  for (int k = threadIdx.x; k < B; k += blockDim.x) {
    const double e = eloc[k], dv = fabs(e - med);
    const double ec = (wdw == 0.0 || dv <= wdw) ? e : med + copysign(1.0, e - med) * wdw * (1.0 + log(dv / wdw));
    ct[k] = ec;  // clipped energy for now
    csum += ec;
  }
  csum = block_sum_d(csum, red);
  const double Lm = csum / B;
  for (int k = threadIdx.x; k < B; k += blockDim.x) ct[k] = ok ? 2.0 / B * (ct[k] - Lm) : 0.0;
  if (threadIdx.x == 0) {
    stats[0] = ok ? mean : NAN;
    stats[1] = ok ? sqrt(var) : NAN;
    stats[2] = acc_sum / B;
    stats[3] = ok ? Lm : NAN;
    stats[4] = nonfin;
    stats[5] = ok ? 1.0 : 0.0;
    stats[6] = ok ? med : NAN;
    stats[7] = ok ? wdw : NAN;
  }
}

__global__ __launch_bounds__(kClipThreads) void k_clip(int64_t nw, int npow2, const double* __restrict__ eloc,
                                                       const int* __restrict__ acc, double q,
                                                       double* __restrict__ ct, double* __restrict__ stats) {
  extern __shared__ __align__(16) char smem[];
  clip_job(nw, npow2, eloc, acc, q, ct, stats, smem);
}

__global__ __launch_bounds__(kThreads) void k_fill0(int64_t n, double* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.0;
}

// AdamW update of parameter i at step t (decoupled weight decay,
// learning rate lr0 / (1 + t / t0), bias-corrected moments).
__device__ __forceinline__ void adamw_elem(int64_t i, double* __restrict__ th, const double* __restrict__ g,
                                           double* __restrict__ m, double* __restrict__ v, int64_t t,
                                           const pn_vmc_hparams& hp) {
  const double lr = hp.lr0 / (1.0 + (double)t / hp.t0);
  const double bc1 = 1.0 - pow(hp.beta1, (double)(t + 1)), bc2 = 1.0 - pow(hp.beta2, (double)(t + 1));
  const double gi = g[i];
  const double mi = hp.beta1 * m[i] + (1.0 - hp.beta1) * gi;
  const double vi = hp.beta2 * v[i] + (1.0 - hp.beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] = th[i] * (1.0 - lr * hp.weight_decay) - lr * (mi / bc1) / (sqrt(vi / bc2) + hp.eps);
}

__global__ __launch_bounds__(kThreads) void k_adamw(int64_t n, double* __restrict__ th, const double* __restrict__ g,
                                                    double* __restrict__ m, double* __restrict__ v, int64_t t,
                                                    pn_vmc_hparams hp, const double* __restrict__ stats) {
  if (stats[5] == 0.0) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    adamw_elem(i, th, g, m, v, t, hp);
}

// ---- grouped launches over the job slots of a serving step ----
// Every slot's pointers and sizes travel in the kernel arguments, so a
// grouped step copies and allocates nothing.  wblk / pblk are prefix sums
// of each slot's blocks over walkers / over parameters; a block finds its
// slot by a search over at most kGroupMax entries.
constexpr int kGroupMax = 16;

struct GroupSlot {
  int64_t nw, np;
  int ncoord, npow2;
  double* r;
  double* rp;
  const double* la;
  const double* lap;
  int* acc;
  const double* eloc;
  double* ct;
  double* stats;
  double* th;
  double* gp;
  double* m;
  double* v;
  uint64_t seed;
  int64_t step;
};

struct Group {
  int n;
  int64_t wblk[kGroupMax + 1];
  int64_t pblk[kGroupMax + 1];
  GroupSlot s[kGroupMax];
};

__device__ __forceinline__ int slot_of(const int64_t* blk, int n, int64_t b) {
  int k = 0;
  while (k + 1 < n && b >= blk[k + 1]) ++k;
  return k;
}

__global__ __launch_bounds__(kThreads) void kg_propose(Group G, double sigma) {
  const int k = slot_of(G.wblk, G.n, blockIdx.x);
  const GroupSlot& S = G.s[k];
  const int64_t w = (blockIdx.x - G.wblk[k]) * blockDim.x + threadIdx.x;
  if (w < S.nw) propose_walker(w, S.ncoord, S.r, S.rp, sigma, S.seed, S.step);
}

__global__ __launch_bounds__(kThreads) void kg_accept(Group G) {
  const int k = slot_of(G.wblk, G.n, blockIdx.x);
  const GroupSlot& S = G.s[k];
  const int64_t w = (blockIdx.x - G.wblk[k]) * blockDim.x + threadIdx.x;
  if (w < S.nw) accept_walker(w, S.ncoord, S.r, S.rp, S.la, S.lap, S.seed, S.step, S.acc);
}

__global__ __launch_bounds__(kClipThreads) void kg_clip(Group G, double q) {
  extern __shared__ __align__(16) char smem[];
  const GroupSlot& S = G.s[blockIdx.x];
  clip_job(S.nw, S.npow2, S.eloc, S.acc, q, S.ct, S.stats, smem);
}

__global__ __launch_bounds__(kThreads) void kg_fill0(Group G) {
  const int k = slot_of(G.pblk, G.n, blockIdx.x);
  const GroupSlot& S = G.s[k];
  const int64_t i = (blockIdx.x - G.pblk[k]) * blockDim.x + threadIdx.x;
  if (i < S.np) S.gp[i] = 0.0;
}

__global__ __launch_bounds__(kThreads) void kg_adamw(Group G, pn_vmc_hparams hp) {
  const int k = slot_of(G.pblk, G.n, blockIdx.x);
  const GroupSlot& S = G.s[k];
  if (S.stats[5] == 0.0) return;
  const int64_t i = (blockIdx.x - G.pblk[k]) * blockDim.x + threadIdx.x;
  if (i < S.np) adamw_elem(i, S.th, S.gp, S.m, S.v, S.step, hp);
}

struct VmcWs {
  size_t eval, rp, la, lap, sg, sgp, ct, gp, acc, total;
};

VmcWs vmc_layout(const pn_ctx* c, int64_t nw, pn_precision prec) {
  VmcWs L{};
  size_t eb = 0;
  pn_workspace_bytes(c, nw, prec, PN_OUT_ALL, &eb);
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  size_t off = 0;
  L.eval = off;
  off = al(off + eb);
  L.rp = off;
  off = al(off + (size_t)nw * c->d.N * 3 * 8);
  L.la = off;
  off = al(off + (size_t)nw * 8);
  L.lap = off;
  off = al(off + (size_t)nw * 8);
  L.sg = off;
  off = al(off + (size_t)nw * 8);
  L.sgp = off;
  off = al(off + (size_t)nw * 8);
  L.ct = off;
  off = al(off + (size_t)nw * 8);
  L.gp = off;
  off = al(off + (size_t)c->pl.total * 8);
  L.acc = off;
  off = al(off + (size_t)nw * 4);
  L.total = off;
  return L;
}

}  // namespace
}  // namespace pn

using namespace pn;

extern "C" {

pn_status pn_vmc_workspace_bytes(const pn_ctx* c, int64_t nw, pn_precision prec, size_t* bytes) {
  if (!c || !bytes || nw < 1 || nw > 16384 || prec < PN_PREC_FP64 || prec > PN_PREC_NET_BF16)
    return PN_ERR_INVALID_ARG;
  *bytes = vmc_layout(c, nw, prec).total;
  return PN_OK;
}

}  // extern "C"

namespace pn {
namespace {
pn_status check_job(const pn_ctx* c, const pn_vmc_job* job, pn_precision prec, const pn_vmc_hparams* hp, void* ws,
                    size_t ws_bytes) {
  if (!c || !job || !hp || !ws || prec < PN_PREC_FP64 || prec > PN_PREC_NET_BF16) return PN_ERR_INVALID_ARG;
  const int64_t B = job->n_walkers;
  if (B < 1 || B > 16384) return PN_ERR_UNSUPPORTED_SHAPE;
  if (!job->r || !job->params || !job->adam_m || !job->adam_v || !job->eloc || !job->stats || job->step < 0)
    return PN_ERR_INVALID_ARG;
  if (!(hp->sigma > 0) || !(hp->t0 > 0) || !(hp->clip_q > 0)) return PN_ERR_INVALID_ARG;
  if (ws_bytes < vmc_layout(c, B, prec).total) return PN_ERR_WORKSPACE_TOO_SMALL;
  return PN_OK;
}
}  // namespace
}  // namespace pn

extern "C" {

pn_status pn_job_bytes(const pn_ctx* c, int64_t nw, pn_precision prec, size_t* resident, size_t* scratch) {
  if (!c || !resident || !scratch || nw < 1 || nw > 16384 || prec < PN_PREC_FP64 || prec > PN_PREC_NET_BF16)
    return PN_ERR_INVALID_ARG;
  *resident = 8 * ((size_t)nw * c->d.N * 3 + 3 * (size_t)c->pl.total + (size_t)nw + 8);
  *scratch = vmc_layout(c, nw, prec).total;
  return PN_OK;
}

pn_status pn_vmc_step(const pn_ctx* c, hipStream_t s, const pn_vmc_job* job, pn_precision prec,
                      const pn_vmc_hparams* hp, void* ws, size_t ws_bytes) {
  const pn_status chk = check_job(c, job, prec, hp, ws, ws_bytes);
  if (chk != PN_OK) return chk;
  const int64_t B = job->n_walkers;
  const VmcWs L = vmc_layout(c, B, prec);
  char* base = static_cast<char*>(ws);
  void* wse = base + L.eval;
  const size_t wse_bytes = L.rp - L.eval;
  double* rp = reinterpret_cast<double*>(base + L.rp);
  double* la = reinterpret_cast<double*>(base + L.la);
  double* lap = reinterpret_cast<double*>(base + L.lap);
  double* sg = reinterpret_cast<double*>(base + L.sg);
  double* sgp = reinterpret_cast<double*>(base + L.sgp);
  double* ct = reinterpret_cast<double*>(base + L.ct);
  double* gp = reinterpret_cast<double*>(base + L.gp);
  int* acc = reinterpret_cast<int*>(base + L.acc);
  const int ncoord = 3 * c->d.N;
  const unsigned nb = (unsigned)((B + kThreads - 1) / kThreads);
  pn_status st;
  // 1-3: Metropolis
  st = pn_eval(c, s, B, job->r, job->params, prec, la, sg, nullptr, nullptr, nullptr, wse, wse_bytes);
  if (st != PN_OK) return st;
  hipLaunchKernelGGL(k_propose, dim3(nb), dim3(kThreads), 0, s, B, ncoord, job->r, rp, hp->sigma, job->seed,
                     job->step);
  st = pn_eval(c, s, B, rp, job->params, prec, lap, sgp, nullptr, nullptr, nullptr, wse, wse_bytes);
  if (st != PN_OK) return st;
  hipLaunchKernelGGL(k_accept, dim3(nb), dim3(kThreads), 0, s, B, ncoord, job->r, rp, la, lap, job->seed, job->step,
                     acc);
  // 4: local energy at the new positions
  st = pn_eval(c, s, B, job->r, job->params, prec, la, sg, nullptr, nullptr, job->eloc, wse, wse_bytes);
  if (st != PN_OK) return st;
  // 5: clipping and estimator weights
  int npow2 = 1;
  while (npow2 < B) npow2 <<= 1;
  const size_t lds = (16 + (size_t)npow2) * sizeof(double);
  if (lds > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_clip), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  hipLaunchKernelGGL(k_clip, dim3(1), dim3(kClipThreads), lds, s, B, npow2, job->eloc, acc, hp->clip_q, ct,
                     job->stats);
  // 6: gradient
  const int64_t np = c->pl.total;
  const unsigned nbp = (unsigned)std::min<int64_t>((np + kThreads - 1) / kThreads, 2048);
  hipLaunchKernelGGL(k_fill0, dim3(nbp), dim3(kThreads), 0, s, np, gp);
  st = pn_eval_backward(c, s, B, job->r, job->params, prec, ct, nullptr, nullptr, nullptr, gp, wse, wse_bytes);
  if (st != PN_OK) return st;
  // 7: AdamW
  hipLaunchKernelGGL(k_adamw, dim3(nbp), dim3(kThreads), 0, s, np, job->params, gp, job->adam_m, job->adam_v,
                     job->step, *hp, job->stats);
  if (hipGetLastError() != hipSuccess) return PN_ERR_DEVICE;
  return PN_OK;
}

pn_status pn_serve_step(hipStream_t s, const pn_job_slot* slots, int32_t n_slots, pn_precision prec,
                        const pn_vmc_hparams* hp) {
  if (n_slots < 0 || (n_slots > 0 && !slots) || !hp) return PN_ERR_INVALID_ARG;
  for (int32_t k = 0; k < n_slots; ++k) {
    const pn_status chk = check_job(slots[k].ctx, &slots[k].job, prec, hp, slots[k].ws, slots[k].ws_bytes);
    if (chk != PN_OK) return chk;
  }
  // the slots, kGroupMax at a time: each phase of the step is one launch per
  // job for the wavefunction work and one grouped launch over the slots for
  // the rest, so every job's step computes what pn_vmc_step computes
  for (int32_t k0 = 0; k0 < n_slots; k0 += kGroupMax) {
    const int nk = std::min<int32_t>(kGroupMax, n_slots - k0);
    const pn_job_slot* sl = slots + k0;
    Group G{};
    G.n = nk;
    int npow2_max = 1;
    for (int k = 0; k < nk; ++k) {
      const pn_ctx* c = sl[k].ctx;
      const int64_t B = sl[k].job.n_walkers;
      const VmcWs L = vmc_layout(c, B, prec);
      char* base = static_cast<char*>(sl[k].ws);
      GroupSlot& S = G.s[k];
      S.nw = B;
      S.np = c->pl.total;
      S.ncoord = 3 * c->d.N;
      int npow2 = 1;
      while (npow2 < B) npow2 <<= 1;
      S.npow2 = npow2;
      npow2_max = std::max(npow2_max, npow2);
      S.r = sl[k].job.r;
      S.rp = reinterpret_cast<double*>(base + L.rp);
      S.la = reinterpret_cast<const double*>(base + L.la);
      S.lap = reinterpret_cast<const double*>(base + L.lap);
      S.acc = reinterpret_cast<int*>(base + L.acc);
      S.eloc = sl[k].job.eloc;
      S.ct = reinterpret_cast<double*>(base + L.ct);
      S.stats = sl[k].job.stats;
      S.th = sl[k].job.params;
      S.gp = reinterpret_cast<double*>(base + L.gp);
      S.m = sl[k].job.adam_m;
      S.v = sl[k].job.adam_v;
      S.seed = sl[k].job.seed;
      S.step = sl[k].job.step;
      G.wblk[k + 1] = G.wblk[k] + (B + kThreads - 1) / kThreads;
      G.pblk[k + 1] = G.pblk[k] + (S.np + kThreads - 1) / kThreads;
    }
    auto eval_all = [&](bool at_proposal, bool with_eloc) -> pn_status {
      for (int k = 0; k < nk; ++k) {
        const pn_ctx* c = sl[k].ctx;
        const int64_t B = sl[k].job.n_walkers;
        const VmcWs L = vmc_layout(c, B, prec);
        char* base = static_cast<char*>(sl[k].ws);
        const double* rr = at_proposal ? reinterpret_cast<const double*>(base + L.rp) : sl[k].job.r;
        double* la = reinterpret_cast<double*>(base + (at_proposal ? L.lap : L.la));
        double* sg = reinterpret_cast<double*>(base + (at_proposal ? L.sgp : L.sg));
        const pn_status st = pn_eval(c, s, B, rr, sl[k].job.params, prec, la, sg, nullptr, nullptr,
                                     with_eloc ? sl[k].job.eloc : nullptr, base + L.eval, L.rp - L.eval);
        if (st != PN_OK) return st;
      }
      return PN_OK;
    };
    pn_status st;
    // 1-3: Metropolis
    if ((st = eval_all(false, false)) != PN_OK) return st;
    hipLaunchKernelGGL(kg_propose, dim3((unsigned)G.wblk[nk]), dim3(kThreads), 0, s, G, hp->sigma);
    if ((st = eval_all(true, false)) != PN_OK) return st;
    hipLaunchKernelGGL(kg_accept, dim3((unsigned)G.wblk[nk]), dim3(kThreads), 0, s, G);
    // 4: local energy at the new positions
    if ((st = eval_all(false, true)) != PN_OK) return st;
    // 5: clipping and estimator weights, one block per job
    const size_t lds = (16 + (size_t)npow2_max) * sizeof(double);
    if (lds > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&kg_clip), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
    hipLaunchKernelGGL(kg_clip, dim3(nk), dim3(kClipThreads), lds, s, G, hp->clip_q);
    // 6: gradient
    hipLaunchKernelGGL(kg_fill0, dim3((unsigned)G.pblk[nk]), dim3(kThreads), 0, s, G);
    for (int k = 0; k < nk; ++k) {
      const pn_ctx* c = sl[k].ctx;
      const int64_t B = sl[k].job.n_walkers;
      const VmcWs L = vmc_layout(c, B, prec);
      char* base = static_cast<char*>(sl[k].ws);
      st = pn_eval_backward(c, s, B, sl[k].job.r, sl[k].job.params, prec, reinterpret_cast<double*>(base + L.ct),
                            nullptr, nullptr, nullptr, reinterpret_cast<double*>(base + L.gp), base + L.eval,
                            L.rp - L.eval);
      if (st != PN_OK) return st;
    }
    // 7: AdamW
    hipLaunchKernelGGL(kg_adamw, dim3((unsigned)G.pblk[nk]), dim3(kThreads), 0, s, G, *hp);
  }
  if (hipGetLastError() != hipSuccess) return PN_ERR_DEVICE;
  return PN_OK;
}

}  // extern "C"
