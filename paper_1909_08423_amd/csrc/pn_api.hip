// Host side of the C ABI: context creation (validation, pair and
// determinant tables, nuclear-cusp polynomials), workspace planning and the
// launch sequence of the walker-evaluation path.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "pn_internal.h"

namespace pn {

template <typename TN>
size_t tangent_lds_bytes(const Dims& d, int T, int stage);
template <typename TN>
size_t value_lds_bytes(const Dims& d, int wpb);
size_t slater_tangent_lds_bytes(const Dims& d, int T);
template <typename TN>
size_t filter_lds_bytes(const Dims& d, int PT);
bool tangent_chunk_supported(int T);
void launch_backward(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const void* P, bool fp32,
                     bool bf16, const double* ct, char* ws, const WsLayout& L, double* grad_params, bool full);
size_t backward_filter_lds_bytes(const Dims& d, bool fp32, bool full);
size_t adj_slater_lds_bytes(const Dims& d, int T);
template <typename TN>
size_t tangent_adj_arena_elems(const Dims& d, int T);
template <typename TN>
size_t tangent_adj_lds_bytes(const Dims& d, int T, bool global_arena);
size_t backward_scratch_bytes(const pn_ctx* c, int64_t tile, bool fp32);
bool backward_supported(const pn_ctx* c, bool fp32);

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kWsBudget = size_t(6) << 30;  // walker tiles keep the workspace below ~6 GiB
constexpr size_t kLdsMax = 160 * 1024;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

ParamLayout make_layout(const Dims& d) {
  ParamLayout pl{};
  int64_t off = 0;
  auto take = [&](int64_t n) {
    int64_t o = off;
    off += n;
    return o;
  };
  const int64_t K = d.K, X = d.DX, Z = d.DZ;
  pl.x0 = take(X);
  pl.Y = take((int64_t)d.NN * Z);
  for (int n = 0; n < d.L; ++n) {
    ParamLayout::Layer& Lp = pl.layer[n];
    for (int c = 0; c < 3; ++c) {
      Lp.w1W[c] = take(K * Z);
      Lp.w1b[c] = take(Z);
      Lp.w2W[c] = take(Z * Z);
      Lp.w2b[c] = take(Z);
    }
    Lp.hW = take(X * Z);
    Lp.hb = take(Z);
    for (int c = 0; c < 3; ++c) {
      Lp.gW[c] = take(Z * X);
      Lp.gb[c] = take(X);
    }
  }
  pl.eW1 = take(X * X);
  pl.eb1 = take(X);
  pl.eW2 = take(X * X);
  pl.eb2 = take(X);
  pl.eW3 = take(X);
  pl.eb3 = take(1);
  pl.kW1 = take(X * X);
  pl.kb1 = take(X);
  pl.kW2 = take(X * X);
  pl.kb2 = take(X);
  pl.kW3 = take(X * d.M);
  pl.kb3 = take(d.M);
  pl.total = off;
  return pl;
}

template <typename T>
T* dev_copy(const std::vector<T>& v, hipError_t* err) {
  T* p = nullptr;
  size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(T);
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    *err = e;
    return nullptr;
  }
  if (!v.empty()) e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) *err = e;
  return p;
}

// Solve the 3x3 system M a = b by Gaussian elimination with partial pivoting.
bool solve3(double M[3][3], double b[3], double x[3]) {
  int idx[3] = {0, 1, 2};
  for (int c = 0; c < 3; ++c) {
    int piv = c;
    for (int r = c + 1; r < 3; ++r)
      if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
    if (M[piv][c] == 0.0) return false;
    if (piv != c) {
      for (int k = 0; k < 3; ++k) std::swap(M[c][k], M[piv][k]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < 3; ++r) {
      double l = M[r][c] / M[c][c];
      for (int k = c; k < 3; ++k) M[r][k] -= l * M[c][k];
      b[r] -= l * b[c];
    }
  }
  (void)idx;
  for (int r = 2; r >= 0; --r) {
    double v = b[r];
    for (int k = r + 1; k < 3; ++k) v -= M[r][k] * x[k];
    x[r] = v / M[r][r];
  }
  return true;
}

}  // namespace

// Workspace plan for `nw` walkers; net_bytes = sizeof of the network type.
// mode 0: forward with derivatives; 1: value-path adjoint; 2: full adjoint
// (cotangents on the gradient, Laplacian and E_loc); 3: value pass only.
// The tangent pass's buffers exist in modes 0 and 2 only.
enum { kPlanForward = 0, kPlanValueAdjoint = 1, kPlanFullAdjoint = 2, kPlanValueOnly = 3 };

// chunk size of the full adjoint: the largest T in 1..6 whose tangent-adjoint
// block keeps its row buffers in LDS; when none fits, the row buffers go to a
// per-block global arena and T is the largest whose small tables fit.  The
// forward tangent pass runs with the same chunks, so its block must fit too.
void plan_full_adjoint(const Dims& d, bool fp64, WsLayout& L) {
  auto lds = [&](int T, bool ga) {
    const size_t fwd = fp64 ? tangent_lds_bytes<double>(d, T, 0) : tangent_lds_bytes<float>(d, T, 0);
    if (fwd > kLdsMax) return fwd;
    return fp64 ? tangent_adj_lds_bytes<double>(d, T, ga) : tangent_adj_lds_bytes<float>(d, T, ga);
  };
  const int ncoord = 3 * d.N;
  L.T = 0;
  for (int pass = 0; pass < 2 && L.T == 0; ++pass) {
    const bool ga = pass == 1;
    for (int T = std::min(6, ncoord); T >= 1; --T) {
      if (!tangent_chunk_supported(T)) continue;
      if (lds(T, ga) <= kLdsMax && adj_slater_lds_bytes(d, T) <= kLdsMax) {
        L.T = T;
        L.tadj_global = ga;
        break;
      }
    }
  }
  if (L.T == 0) L.T = 1;  // reported unsupported by the caller (LDS over the limit)
  L.lds_tadj = lds(L.T, L.tadj_global);
  L.lds_adjdet = adj_slater_lds_bytes(d, L.T);
  L.tadj_arena = fp64 ? tangent_adj_arena_elems<double>(d, L.T) : tangent_adj_arena_elems<float>(d, L.T);
}

// `budget`: workspace bytes the walker tile is sized for; min_tile: the
// smallest tile (the library's own budget keeps tiles of >= 256 walkers).
WsLayout plan(const pn_ctx* c, int64_t nw, pn_precision prec, int mode, size_t budget_bytes = kWsBudget,
              int64_t min_tile = 256) {
  const Dims& d = c->d;
  const bool fp64 = prec == PN_PREC_FP64;
  const bool backward = mode == kPlanValueAdjoint || mode == kPlanFullAdjoint, full = mode == kPlanFullAdjoint;
  const size_t tn = fp64 ? sizeof(double) : sizeof(float);
  WsLayout L{};
  L.full = full;
  // chunking of the 3N coordinates for the tangent pass: the largest chunk
  // whose block fits the LDS budget; at equal chunk the form that stages the
  // filter tables in LDS (measured: a larger chunk without staging beats a
  // smaller staged one, e.g. Ne-like FP32 T 10 vs 8, 2.25 vs 2.59 ms, and
  // FP64 T 5 vs 3, 4.28 vs 5.39 ms).  Two 256-thread blocks per CU (80 KB each) unless
  // that leaves chunks of fewer than 3 coordinates (large systems, where the
  // per-chunk work of the heads would be repeated 3N times): then one block
  // per CU with all 160 KB, if that at least doubles the chunk.
  const int ncoord = 3 * d.N;
  auto lds_of = [&](int T, int stage) {
    return fp64 ? tangent_lds_bytes<double>(d, T, stage) : tangent_lds_bytes<float>(d, T, stage);
  };
  auto pick = [&](size_t budget, int& T_out, bool& stage_out) {
    T_out = 0;
    for (int nc = 1; nc <= ncoord && T_out == 0; ++nc) {
      const int T = (ncoord + nc - 1) / nc;
      if (!tangent_chunk_supported(T)) continue;
      for (int pass = 0; pass < 2; ++pass) {
        const bool stage = pass == 0;
        if (lds_of(T, stage ? 2 : 0) <= budget || (!stage && T == 1)) {
          T_out = T;
          stage_out = stage;
          break;
        }
      }
    }
  };
  size_t budget = 80 * 1024;
  pick(budget, L.T, L.stage_filters);
  if (L.T < 3) {
    int T2;
    bool st2;
    pick(kLdsMax, T2, st2);
    if (T2 >= 2 * L.T) {
      budget = kLdsMax;
      L.T = T2;
      L.stage_filters = st2;
    }
  }
  if (full) {
    // the forward tangent pass runs with the adjoint's chunking
    plan_full_adjoint(d, fp64, L);
    L.stage_filters = lds_of(L.T, 2) <= budget;
  }
  L.n_chunks = (ncoord + L.T - 1) / L.T;
  L.lds_tangent = lds_of(L.T, L.stage_filters ? 2 : 0);
  // a block that takes more than half the CU's LDS runs alone on it: 512
  // threads keep two waves per SIMD (chunks of at most 6 coordinates)
  L.tan_threads = (L.lds_tangent > kLdsMax / 2 && L.T <= 6) ? 512 : 256;
  L.wpb_value = std::max(1, 64 / d.N);
  while (L.wpb_value > 1 &&
         (fp64 ? value_lds_bytes<double>(d, L.wpb_value) : value_lds_bytes<float>(d, L.wpb_value)) > 64 * 1024)
    L.wpb_value /= 2;
  L.lds_value = fp64 ? value_lds_bytes<double>(d, L.wpb_value) : value_lds_bytes<float>(d, L.wpb_value);
  // 32 pair rows per filter block (measured: 64 rows, two blocks per CU, are
  // 20 % slower in FP32), halved while the tile exceeds 64 KB of LDS
  L.filt_rows = 32;
  while (L.filt_rows > 16 &&
         (fp64 ? filter_lds_bytes<double>(d, L.filt_rows) : filter_lds_bytes<float>(d, L.filt_rows)) > 64 * 1024)
    L.filt_rows /= 2;
  L.lds_filter = fp64 ? filter_lds_bytes<double>(d, L.filt_rows) : filter_lds_bytes<float>(d, L.filt_rows);
  // determinants of the forward pass through one LU per spin when the
  // expansion allows it (and the caller did not ask for the direct path)
  L.lowrank = (mode == kPlanForward || mode == kPlanValueOnly) && d.lr && !(d.flags & PN_DET_DIRECT);
  L.lds_lr = L.lowrank ? lowrank_tangent_lds_bytes(d, L.T) : 0;
  if (L.lds_lr > kLdsMax) L.lowrank = false;

  const int N = d.N, M = d.M, P = d.P, Tp = L.T + 1;
  const bool tangents = mode == kPlanForward || mode == kPlanFullAdjoint;
  const size_t gsz = (size_t)d.n_up * d.n_up + (size_t)d.n_dn * d.n_dn;
  // bytes per walker of every tile-sized region
  auto per_walker = [&](bool with_bwd) {
    size_t b = 0;
    b += align_up(kGeoStride(N) * 8);
    b += (size_t)N * M * 7 * 8;
    b += (size_t)d.L * 3 * d.n_pairs * d.DZ * tn;
    b += (size_t)d.L * N * d.DZ * tn;
    b += (size_t)4 * N * d.DX * tn + 4 * d.DX * tn;
    b += (size_t)N * M * 8 + 8;
    b += (size_t)P * gsz * 8 + (size_t)P * 4 * 8 + (size_t)P * 8 + 8;
    if (tangents) b += (size_t)L.n_chunks * N * Tp * M * 8 + (size_t)L.n_chunks * Tp * 8 + (size_t)L.n_chunks * 2 * 8;
    b += (size_t)N * 3 * 8;
    if (with_bwd) b += (size_t)(d.L + 1) * N * d.DX * tn;
    if (L.lowrank)
      b += (gsz + 4 + (size_t)d.nv[0] * d.n_up + (size_t)d.nv[1] * d.n_dn + (size_t)P * 2 * kMaxExc * kMaxExc) * 8 +
           3 * 4;
    if (full) {
      const size_t nc = L.n_chunks, N3 = 3 * N;
      b += nc * d.L * N * Tp * d.DX * tn;                     // xsave
      b += nc * P * 2 * Tp * 8 + N3 * 8 + (N3 + 2) * 8 + (size_t)P * (N3 + 2) * 8 + 8;
      b += nc * N * Tp * M * 8 + nc * N * M * 8;              // ctftan, ctfpart
      b += ((size_t)d.L * N * d.DZ + (size_t)d.L * d.n_ee * d.DZ + 2 * (size_t)d.L * d.n_pairs * d.DZ +
            4 * (size_t)N * d.DX + 4 * (size_t)d.DX) * tn;
    }
    return b;
  };
  size_t pw = per_walker(backward);
  // bytes that do not scale with the tile: the converted parameters and the
  // alignment of every region
  const size_t fixed = (fp64 ? 0 : align_up((size_t)c->pl.total * sizeof(float))) + 64 * kAlign;
  const size_t avail = budget_bytes > fixed ? budget_bytes - fixed : 0;
  int64_t tile = std::max<int64_t>(min_tile, (int64_t)(avail / std::max<size_t>(pw, 1)));
  tile = std::min<int64_t>(tile, std::max<int64_t>(nw, 1));
  L.tile = tile;
  size_t off = 0;
  auto region = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.params_net = region(fp64 ? 0 : (size_t)c->pl.total * sizeof(float));
  L.geo = region((size_t)tile * kGeoStride(N) * 8);
  L.phi = region((size_t)tile * N * M * 7 * 8);
  L.filt = region((size_t)tile * d.L * 3 * d.n_pairs * d.DZ * tn);
  L.hval = region((size_t)tile * d.L * N * d.DZ * tn);
  L.kcoef = region((size_t)tile * 4 * N * d.DX * tn);
  L.ecoef = region((size_t)tile * 4 * d.DX * tn);
  L.fval = region((size_t)tile * N * M * 8);
  L.jval = region((size_t)tile * 8);
  L.ginv = region((size_t)tile * P * gsz * 8);
  L.ldet = region((size_t)tile * P * 4 * 8);
  L.wdet = region((size_t)tile * P * 8);
  L.ldpsi = region((size_t)tile * 8);
  L.ftan = region(tangents ? (size_t)tile * L.n_chunks * N * Tp * M * 8 : 0);
  L.jtan = region(tangents ? (size_t)tile * L.n_chunks * Tp * 8 : 0);
  L.partial = region(tangents ? (size_t)tile * L.n_chunks * 2 * 8 : 0);
  // grad scratch for calls that want lap/eloc without grad
  L.adj = region((size_t)tile * std::max(N * 3, 2) * 8);
  L.xval = 0;
  L.gpart = 0;
  if (backward) {
    L.xval = region((size_t)tile * (d.L + 1) * N * d.DX * tn);
    L.gpart = region(backward_scratch_bytes(c, tile, !fp64));
  }
  if (L.lowrank) {
    L.g0 = region((size_t)tile * gsz * 8);
    L.ld0 = region((size_t)tile * 4 * 8);
    L.theta = region((size_t)tile * ((size_t)d.nv[0] * d.n_up + (size_t)d.nv[1] * d.n_dn) * 8);
    L.dinv = region((size_t)tile * P * 2 * kMaxExc * kMaxExc * 8);
    L.lrflag = region((size_t)tile * 2 * 4);
    L.lrlist = region((size_t)(tile + 1) * 4);
  }
  if (full) {
    const size_t nc = L.n_chunks, N3 = 3 * N;
    L.xsave = region((size_t)tile * nc * d.L * N * Tp * d.DX * tn);
    L.detres = region((size_t)tile * nc * P * 2 * Tp * 8);
    L.gradf = region((size_t)tile * N3 * 8);
    L.ctc = region((size_t)tile * (N3 + 2) * 8);
    L.ctdet = region((size_t)tile * P * (N3 + 2) * 8);
    L.ctftan = region((size_t)tile * nc * N * Tp * M * 8);
    L.ctfpart = region((size_t)tile * nc * N * M * 8);
    L.cthv = region((size_t)tile * d.L * N * d.DZ * tn);
    L.ctww = region((size_t)tile * d.L * d.n_ee * d.DZ * tn);
    L.ctwd = region((size_t)tile * d.L * d.n_pairs * d.DZ * tn);
    L.ctw2 = region((size_t)tile * d.L * d.n_pairs * d.DZ * tn);
    L.ctkc = region((size_t)tile * 4 * N * d.DX * tn);
    L.ctec = region((size_t)tile * 4 * d.DX * tn);
    L.ct0 = region((size_t)tile * 8);
    L.tslot = region(((size_t)kSlotsTanAdj * c->pl.total + (L.tadj_global ? (size_t)kSlotsTanAdj * L.tadj_arena : 0)) *
                     tn);
  }
  L.total = off;
  return L;
}

// ---- optional stage timing ----
namespace {
void harvest_set(pn_ctx::Timing* T, int set) {
  for (int k = 0; k < pn_ctx::Timing::kStages; ++k) {
    if (!T->rec[set][k]) continue;
    float ms = 0.f;
    if (hipEventSynchronize(T->ev[set][k][1]) == hipSuccess &&
        hipEventElapsedTime(&ms, T->ev[set][k][0], T->ev[set][k][1]) == hipSuccess) {
      T->ms[k] += ms;
      T->cnt[k] += 1;
    }
    T->rec[set][k] = false;
  }
}
struct StageClock {
  pn_ctx::Timing* T;
  hipStream_t s;
  StageClock(const pn_ctx* c, hipStream_t st) : T(c->timing && c->timing->on ? c->timing : nullptr), s(st) {
    if (T) harvest_set(T, T->cur);
  }
  void begin(int k) {
    if (T) (void)hipEventRecord(T->ev[T->cur][k][0], s);
  }
  void end(int k) {
    if (!T) return;
    (void)hipEventRecord(T->ev[T->cur][k][1], s);
    T->rec[T->cur][k] = true;
  }
  void next_set() {
    if (!T) return;
    T->cur = (T->cur + 1) % pn_ctx::Timing::kSets;
    harvest_set(T, T->cur);
  }
};
}  // namespace

// ---- allocation-free evaluation (pn_eval_noalloc) ----
// A file-scope device array serves as the workspace of pn_eval_noalloc.
// Host code never passes the array's name to a kernel: each device's copy
// has its own address, taken once per device by hipGetSymbolAddress at
// context creation (with that device current) and kept in scratch_ptr.
namespace {
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) char scratch[kScratchBytes];
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

void scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (scratch_ptr[dev]) return;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) scratch_ptr[dev] = p;
  else (void)hipGetLastError();
}

void* scratch_of(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(scratch_mu);
  return scratch_ptr[dev];
}
}  // namespace

}  // namespace pn

using namespace pn;

namespace {
pn_status eval_impl(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const double* params,
                    pn_precision prec, double* logabs, double* sign, double* grad, double* lap, double* eloc, char* base,
                    const WsLayout& L);
}

extern "C" {

const char* pn_status_string(pn_status s) {
  switch (s) {
    case PN_OK: return "ok";
    case PN_ERR_INVALID_ARG: return "invalid argument";
    case PN_ERR_UNSUPPORTED_SHAPE: return "unsupported shape";
    case PN_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case PN_ERR_DEVICE: return "device error";
    case PN_ERR_BUDGET: return "over budget";
  }
  return "unknown status";
}

pn_status pn_ctx_create(const pn_system_desc* sys, const pn_net_desc* net, pn_ctx** out) {
  if (!out) return PN_ERR_INVALID_ARG;
  *out = nullptr;
  if (!sys || !net) return PN_ERR_INVALID_ARG;
  if (sys->n_nuc < 1 || !sys->nuc_xyz || !sys->charge || sys->n_shell < 1 || !sys->shell_center ||
      !sys->shell_l || !sys->shell_exp || sys->n_mo < 1 || !sys->mo_coeff || sys->n_det < 1 || !sys->ci ||
      sys->n_up < 0 || sys->n_down < 0 || sys->n_up + sys->n_down < 1 || (sys->n_up > 0 && !sys->det_up) ||
      (sys->n_down > 0 && !sys->det_down) || !(sys->cusp_radius >= 0))
    return PN_ERR_INVALID_ARG;
  if (net->flags & ~(PN_NET_NO_JASTROW | PN_NET_NO_BACKFLOW | PN_DET_DIRECT)) return PN_ERR_INVALID_ARG;
  if (net->n_feat < 1 || net->dim_x < 1 || net->dim_z < 1 || net->n_layers < 1 || !(net->feat_cutoff > 0))
    return PN_ERR_INVALID_ARG;
  const int N = sys->n_up + sys->n_down;
  auto mfma_dim = [](int v) { return v == 16 || v == 32 || v == 64 || v == 128; };
  if (!mfma_dim(net->n_feat) || !mfma_dim(net->dim_x) || !mfma_dim(net->dim_z)) return PN_ERR_UNSUPPORTED_SHAPE;
  if (sys->n_up > kMaxSpin || sys->n_down > kMaxSpin || N > kMaxElec || sys->n_det > kMaxDet ||
      net->dim_x > 128 || net->dim_z > 128 || net->n_feat > 64 || net->n_layers > kMaxLayers ||
      sys->n_nuc > kMaxNuc || sys->n_mo > net->dim_x)
    return PN_ERR_UNSUPPORTED_SHAPE;
  int NB = 0;
  for (int s = 0; s < sys->n_shell; ++s) {
    if (sys->shell_l[s] < 0 || sys->shell_l[s] > 1) return PN_ERR_UNSUPPORTED_SHAPE;
    if (sys->shell_center[s] < 0 || sys->shell_center[s] >= sys->n_nuc || !(sys->shell_exp[s] > 0))
      return PN_ERR_INVALID_ARG;
    NB += 2 * sys->shell_l[s] + 1;
  }
  const int M = sys->n_mo, P = sys->n_det, NN = sys->n_nuc;
  for (int p = 0; p < P; ++p) {
    for (int k = 0; k < sys->n_up; ++k)
      if (sys->det_up[p * sys->n_up + k] < 0 || sys->det_up[p * sys->n_up + k] >= M) return PN_ERR_INVALID_ARG;
    for (int k = 0; k < sys->n_down; ++k)
      if (sys->det_down[p * sys->n_down + k] < 0 || sys->det_down[p * sys->n_down + k] >= M)
        return PN_ERR_INVALID_ARG;
  }

  pn_ctx* c = new pn_ctx();
  Dims& d = c->d;
  d.N = N;
  d.n_up = sys->n_up;
  d.n_dn = sys->n_down;
  d.NN = NN;
  d.NB = NB;
  d.M = M;
  d.P = P;
  d.K = net->n_feat;
  d.DX = net->dim_x;
  d.DZ = net->dim_z;
  d.L = net->n_layers;
  d.flags = net->flags;
  d.n_ee = N * (N - 1) / 2;
  d.n_pairs = d.n_ee + N * NN;
  d.n_shell = sys->n_shell;
  d.feat_rc = net->feat_cutoff;
  d.cusp_rc = sys->cusp_radius;
  double vnn = 0.0;
  for (int I = 0; I < NN; ++I)
    for (int J = I + 1; J < NN; ++J) {
      double dx = sys->nuc_xyz[3 * I] - sys->nuc_xyz[3 * J], dy = sys->nuc_xyz[3 * I + 1] - sys->nuc_xyz[3 * J + 1],
             dz = sys->nuc_xyz[3 * I + 2] - sys->nuc_xyz[3 * J + 2];
      vnn += sys->charge[I] * sys->charge[J] / sqrt(dx * dx + dy * dy + dz * dz);
    }
  d.v_nn = vnn;
  c->pl = make_layout(d);
  if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
  scratch_setup(c->device);

  // ---- host tables ----
  std::vector<double> nuc(sys->nuc_xyz, sys->nuc_xyz + 3 * NN), chg(sys->charge, sys->charge + NN);
  std::vector<int> sc(sys->shell_center, sys->shell_center + d.n_shell), sl(sys->shell_l, sys->shell_l + d.n_shell);
  std::vector<double> se(sys->shell_exp, sys->shell_exp + d.n_shell), sn(d.n_shell);
  std::vector<int> sfirst(d.n_shell);
  int b = 0;
  for (int s = 0; s < d.n_shell; ++s) {
    double a = se[s];
    sn[s] = sl[s] == 0 ? pow(2.0 * a / M_PI, 0.75) : pow(128.0 * pow(a, 5) / pow(M_PI, 3), 0.25);
    sfirst[s] = b;
    b += 2 * sl[s] + 1;
  }
  std::vector<double> mo(sys->mo_coeff, sys->mo_coeff + (size_t)NB * M);
  std::vector<int> du(sys->det_up, sys->det_up + (size_t)P * d.n_up), dd(sys->det_down, sys->det_down + (size_t)P * d.n_dn);
  std::vector<double> clog(P), csign(P);
  for (int p = 0; p < P; ++p) {
    clog[p] = log(fabs(sys->ci[p]));
    csign[p] = sys->ci[p] > 0 ? 1.0 : (sys->ci[p] < 0 ? -1.0 : 0.0);
  }
  // s functions grouped by nucleus
  std::vector<int> s_first(NN + 1, 0), s_basis;
  std::vector<double> s_exp, s_norm;
  for (int I = 0; I < NN; ++I) {
    s_first[I] = (int)s_basis.size();
    for (int s = 0; s < d.n_shell; ++s)
      if (sc[s] == I && sl[s] == 0) {
        s_basis.push_back(sfirst[s]);
        s_exp.push_back(se[s]);
        s_norm.push_back(sn[s]);
      }
  }
  s_first[NN] = (int)s_basis.size();
  // nuclear cusp polynomials (Ma et al. scheme, nucleus value as input)
  std::vector<int> cusp_on((size_t)NN * M, 0);
  std::vector<double> cusp_sign((size_t)NN * M, 0.0), cusp_alpha((size_t)NN * M * 5, 0.0),
      cusp_dalpha((size_t)NN * M * 5, 0.0);
  int n_on = 0;
  if (d.cusp_rc > 0) {
    const double rc = d.cusp_rc;
    for (int I = 0; I < NN; ++I) {
      if (s_first[I] == s_first[I + 1]) continue;
      for (int mu = 0; mu < M; ++mu) {
        // uncorrected orbital at the nucleus
        double phi0 = 0.0;
        for (int s = 0; s < d.n_shell; ++s) {
          double dx = nuc[3 * I] - nuc[3 * sc[s]], dy = nuc[3 * I + 1] - nuc[3 * sc[s] + 1],
                 dz = nuc[3 * I + 2] - nuc[3 * sc[s] + 2];
          double g = sn[s] * exp(-se[s] * (dx * dx + dy * dy + dz * dz));
          if (sl[s] == 0) {
            phi0 += mo[(size_t)sfirst[s] * M + mu] * g;
          } else {
            double x[3] = {dx, dy, dz};
            for (int k = 0; k < 3; ++k) phi0 += mo[(size_t)(sfirst[s] + k) * M + mu] * x[k] * g;
          }
        }
        double s0u = 0.0, sv = 0.0, s1 = 0.0, s2 = 0.0;
        for (int k = s_first[I]; k < s_first[I + 1]; ++k) {
          double cn = mo[(size_t)s_basis[k] * M + mu] * s_norm[k], a = s_exp[k];
          double e = exp(-a * rc * rc);
          s0u += cn;
          sv += cn * e;
          s1 += cn * (-2.0 * a * rc) * e;
          s2 += cn * (4.0 * a * a * rc * rc - 2.0 * a) * e;
        }
        double s0 = sys->cusp_nuc_value ? sys->cusp_nuc_value[(size_t)I * M + mu] : s0u;
        if (s0 == 0.0 || !(sv * s0 > 0.0)) continue;
        double eta0 = phi0 - s0u;
        double a0 = log(fabs(s0));
        double a1 = -sys->charge[I] * (eta0 + s0) / s0;
        double X1 = log(fabs(sv)), X2 = s1 / sv, X3 = s2 / sv - X2 * X2;
        double Mm[3][3] = {{rc * rc, rc * rc * rc, rc * rc * rc * rc},
                           {2 * rc, 3 * rc * rc, 4 * rc * rc * rc},
                           {2.0, 6 * rc, 12 * rc * rc}};
        double Md[3][3];  // solve3 eliminates in place: keep a copy for the derivative system
        for (int a = 0; a < 3; ++a)
          for (int b2 = 0; b2 < 3; ++b2) Md[a][b2] = Mm[a][b2];
        double rhs[3] = {X1 - a0 - a1 * rc, X2 - a1, X3}, sol[3];
        if (!solve3(Mm, rhs, sol)) continue;
        size_t q = (size_t)I * M + mu;
        cusp_on[q] = 1;
        cusp_sign[q] = s0 > 0 ? 1.0 : -1.0;
        cusp_alpha[5 * q + 0] = a0;
        cusp_alpha[5 * q + 1] = a1;
        cusp_alpha[5 * q + 2] = sol[0];
        cusp_alpha[5 * q + 3] = sol[1];
        cusp_alpha[5 * q + 4] = sol[2];
        // d alpha / d s0: a0 = ln|s0|, a1 = -Z (eta0 + s0) / s0, a2..a4 from the
        // linear system whose right-hand side depends on a0 and a1
        const double da0 = 1.0 / s0, da1 = sys->charge[I] * eta0 / (s0 * s0);
        double rhs_d[3] = {-da0 - da1 * rc, -da1, 0.0}, sol_d[3];
        if (solve3(Md, rhs_d, sol_d)) {
          cusp_dalpha[5 * q + 0] = da0;
          cusp_dalpha[5 * q + 1] = da1;
          for (int k = 0; k < 3; ++k) cusp_dalpha[5 * q + 2 + k] = sol_d[k];
        }
        ++n_on;
      }
    }
  }
  c->n_cusp_on = n_on;
  // features
  std::vector<double> fmu(d.K), fs(d.K);
  for (int k = 0; k < d.K; ++k) {
    double q = d.K > 1 ? double(k) / double(d.K - 1) : 0.0;
    fmu[k] = d.feat_rc * q * q;
    double sg = (1.0 + d.feat_rc * q) / 7.0;
    fs[k] = 1.0 / (sg * sg);
  }
  // pairs: same-spin ee (i<j), then opposite-spin ee, then e-n
  std::vector<int> pij, pidx((size_t)N * N, -1);
  for (int pass = 0; pass < 2; ++pass)
    for (int i = 0; i < N; ++i)
      for (int j = i + 1; j < N; ++j) {
        bool same = (i < d.n_up) == (j < d.n_up);
        if (same != (pass == 0)) continue;
        int p = (int)pij.size() / 2;
        pij.push_back(i);
        pij.push_back(j);
        pidx[(size_t)i * N + j] = p;
        pidx[(size_t)j * N + i] = p;
      }

  // the expansion as excitations of its first determinant (low-rank path):
  // per (determinant, spin) the hole slots of the first determinant's rows,
  // the particle orbitals replacing them (as rows of the spin's virtual
  // list), and the sign of the row order
  std::vector<int> lrk((size_t)P * 2, 0), lrh((size_t)P * 2 * kMaxExc, 0), lrp((size_t)P * 2 * kMaxExc, 0),
      lrv((size_t)2 * M, 0);
  std::vector<double> lrs((size_t)P * 2, 1.0);
  int lr_ok = P >= 2 ? 1 : 0;
  d.nv[0] = d.nv[1] = 0;
  for (int sp = 0; sp < 2 && lr_ok; ++sp) {
    const int n = sp == 0 ? d.n_up : d.n_dn;
    const int* occ = sp == 0 ? du.data() : dd.data();
    std::vector<int> slot(M, -1), vrow(M, -1);
    for (int k = 0; k < n && lr_ok; ++k) {
      if (slot[occ[k]] >= 0) lr_ok = 0;  // repeated orbital: the first determinant vanishes
      slot[occ[k]] = k;
    }
    for (int p = 0; p < P && lr_ok; ++p) {
      const int* op = occ + (size_t)p * n;
      std::vector<char> in_p(M, 0);
      for (int k = 0; k < n; ++k) {
        if (in_p[op[k]]) lr_ok = 0;
        in_p[op[k]] = 1;
      }
      std::vector<int> holes, parts;
      for (int k = 0; k < n; ++k)
        if (!in_p[occ[k]]) holes.push_back(k);
      for (int k = 0; k < n; ++k)
        if (slot[op[k]] < 0) parts.push_back(op[k]);
      std::sort(parts.begin(), parts.end());
      if (!lr_ok || (int)holes.size() > kMaxExc || holes.size() != parts.size()) {
        lr_ok = 0;
        break;
      }
      std::vector<int> seq(occ, occ + n);
      for (size_t j = 0; j < holes.size(); ++j) seq[holes[j]] = parts[j];
      int inversions = 0;
      std::vector<int> pos(n);
      for (int k = 0; k < n; ++k) pos[k] = (int)(std::find(seq.begin(), seq.end(), op[k]) - seq.begin());
      for (int a = 0; a < n; ++a)
        for (int b2 = a + 1; b2 < n; ++b2) inversions += pos[a] > pos[b2];
      const size_t q = (size_t)p * 2 + sp;
      lrs[q] = (inversions & 1) ? -1.0 : 1.0;
      lrk[q] = (int)holes.size();
      for (size_t j = 0; j < holes.size(); ++j) {
        if (vrow[parts[j]] < 0) {
          vrow[parts[j]] = d.nv[sp];
          lrv[(size_t)sp * M + d.nv[sp]] = parts[j];
          ++d.nv[sp];
        }
        lrh[q * kMaxExc + j] = holes[j];
        lrp[q * kMaxExc + j] = vrow[parts[j]];
      }
    }
  }
  d.lr = lr_ok;
  if (!lr_ok) d.nv[0] = d.nv[1] = 0;

  hipError_t err = hipSuccess;
  DevTables& t = c->t;
  t.nuc_xyz = dev_copy(nuc, &err);
  t.charge = dev_copy(chg, &err);
  t.shell_center = dev_copy(sc, &err);
  t.shell_l = dev_copy(sl, &err);
  t.shell_exp = dev_copy(se, &err);
  t.shell_norm = dev_copy(sn, &err);
  t.shell_first = dev_copy(sfirst, &err);
  t.mo = dev_copy(mo, &err);
  t.det_up = dev_copy(du, &err);
  t.det_dn = dev_copy(dd, &err);
  t.ci_log = dev_copy(clog, &err);
  t.ci_sign = dev_copy(csign, &err);
  t.cusp_on = dev_copy(cusp_on, &err);
  t.cusp_sign = dev_copy(cusp_sign, &err);
  t.cusp_alpha = dev_copy(cusp_alpha, &err);
  t.cusp_dalpha = dev_copy(cusp_dalpha, &err);
  t.s_first = dev_copy(s_first, &err);
  t.s_basis = dev_copy(s_basis, &err);
  t.s_exp = dev_copy(s_exp, &err);
  t.s_norm = dev_copy(s_norm, &err);
  t.feat_mu = dev_copy(fmu, &err);
  t.feat_sig2inv = dev_copy(fs, &err);
  t.pair_ij = dev_copy(pij, &err);
  t.pair_index = dev_copy(pidx, &err);
  t.lr_k = dev_copy(lrk, &err);
  t.lr_hole = dev_copy(lrh, &err);
  t.lr_part = dev_copy(lrp, &err);
  t.lr_sign = dev_copy(lrs, &err);
  t.lr_vorb = dev_copy(lrv, &err);
  if (err != hipSuccess) {
    pn_ctx_destroy(c);
    return PN_ERR_DEVICE;
  }
  *out = c;
  return PN_OK;
}

void pn_ctx_destroy(pn_ctx* c) {
  if (!c) return;
  if (c->timing) {
    for (int a = 0; a < pn_ctx::Timing::kSets; ++a)
      for (int k = 0; k < pn_ctx::Timing::kStages; ++k)
        for (int e = 0; e < 2; ++e)
          if (c->timing->ev[a][k][e]) (void)hipEventDestroy(c->timing->ev[a][k][e]);
    delete c->timing;
  }
  void* ptrs[] = {c->t.nuc_xyz, c->t.charge, c->t.shell_center, c->t.shell_l, c->t.shell_exp, c->t.shell_norm,
                  c->t.shell_first, c->t.mo, c->t.det_up, c->t.det_dn, c->t.ci_log, c->t.ci_sign, c->t.cusp_on,
                  c->t.cusp_sign, c->t.cusp_alpha, c->t.cusp_dalpha, c->t.s_first, c->t.s_basis, c->t.s_exp, c->t.s_norm,
                  c->t.feat_mu, c->t.feat_sig2inv, c->t.pair_ij, c->t.pair_index, c->t.lr_k, c->t.lr_hole,
                  c->t.lr_part, c->t.lr_sign, c->t.lr_vorb};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete c;
}

int64_t pn_param_count(const pn_ctx* c) { return c ? c->pl.total : -1; }

pn_status pn_param_layout(const pn_ctx* c, pn_param_entry* e, int32_t cap, int32_t* n) {
  if (!c || !n || cap < 0 || (cap > 0 && !e)) return PN_ERR_INVALID_ARG;
  const Dims& d = c->d;
  const ParamLayout& pl = c->pl;
  int32_t k = 0;
  auto put = [&](const char* name, int64_t off, int32_t r0, int32_t r1) {
    if (k < cap) {
      pn_param_entry& x = e[k];
      memset(&x, 0, sizeof(x));
      snprintf(x.name, sizeof(x.name), "%s", name);
      x.offset = off;
      x.ndim = r1 > 0 ? 2 : 1;
      x.shape[0] = r0;
      x.shape[1] = r1;
    }
    ++k;
  };
  static const char* chn[3] = {"same", "opp", "nuc"};
  char buf[32];
  put("x0", pl.x0, d.DX, 0);
  put("Y", pl.Y, d.NN, d.DZ);
  for (int l = 0; l < d.L; ++l) {
    const ParamLayout::Layer& Lp = pl.layer[l];
    for (int ch = 0; ch < 3; ++ch) {
      snprintf(buf, sizeof(buf), "l%d.w_%s.W1", l, chn[ch]);
      put(buf, Lp.w1W[ch], d.K, d.DZ);
      snprintf(buf, sizeof(buf), "l%d.w_%s.b1", l, chn[ch]);
      put(buf, Lp.w1b[ch], d.DZ, 0);
      snprintf(buf, sizeof(buf), "l%d.w_%s.W2", l, chn[ch]);
      put(buf, Lp.w2W[ch], d.DZ, d.DZ);
      snprintf(buf, sizeof(buf), "l%d.w_%s.b2", l, chn[ch]);
      put(buf, Lp.w2b[ch], d.DZ, 0);
    }
    snprintf(buf, sizeof(buf), "l%d.h.W", l);
    put(buf, Lp.hW, d.DX, d.DZ);
    snprintf(buf, sizeof(buf), "l%d.h.b", l);
    put(buf, Lp.hb, d.DZ, 0);
    for (int ch = 0; ch < 3; ++ch) {
      snprintf(buf, sizeof(buf), "l%d.g_%s.W", l, chn[ch]);
      put(buf, Lp.gW[ch], d.DZ, d.DX);
      snprintf(buf, sizeof(buf), "l%d.g_%s.b", l, chn[ch]);
      put(buf, Lp.gb[ch], d.DX, 0);
    }
  }
  put("eta.W1", pl.eW1, d.DX, d.DX);
  put("eta.b1", pl.eb1, d.DX, 0);
  put("eta.W2", pl.eW2, d.DX, d.DX);
  put("eta.b2", pl.eb2, d.DX, 0);
  put("eta.W3", pl.eW3, d.DX, 1);
  put("eta.b3", pl.eb3, 1, 0);
  put("kappa.W1", pl.kW1, d.DX, d.DX);
  put("kappa.b1", pl.kb1, d.DX, 0);
  put("kappa.W2", pl.kW2, d.DX, d.DX);
  put("kappa.b2", pl.kb2, d.DX, 0);
  put("kappa.W3", pl.kW3, d.DX, d.M);
  put("kappa.b3", pl.kb3, d.M, 0);
  *n = k;
  return k <= cap ? PN_OK : PN_ERR_INVALID_ARG;
}

pn_status pn_workspace_bytes(const pn_ctx* c, int64_t nw, pn_precision prec, uint32_t out_mask, size_t* bytes) {
  if (!c || !bytes || nw < 0 || prec < PN_PREC_FP64 || prec > PN_PREC_NET_BF16 || (out_mask & ~PN_OUT_ALL))
    return PN_ERR_INVALID_ARG;
  // a value-only call plans its own (larger) walker tile, so a workspace for
  // calls with derivatives covers it as well
  size_t b = plan(c, nw, prec, kPlanValueOnly).total;
  if (out_mask & (PN_OUT_GRAD | PN_OUT_LAP | PN_OUT_ELOC)) b = std::max(b, plan(c, nw, prec, kPlanForward).total);
  if (out_mask & PN_OUT_ADJOINT) b = std::max(b, plan(c, nw, prec, kPlanValueAdjoint).total);
  *bytes = b;
  return PN_OK;
}

pn_status pn_workspace_bytes_full(const pn_ctx* c, int64_t nw, pn_precision prec, size_t* bytes) {
  if (!c || !bytes || nw < 0 || prec < PN_PREC_FP64 || prec > PN_PREC_NET_BF16) return PN_ERR_INVALID_ARG;
  *bytes = std::max(std::max(plan(c, nw, prec, kPlanForward).total, plan(c, nw, prec, kPlanValueAdjoint).total),
                    std::max(plan(c, nw, prec, kPlanFullAdjoint).total, plan(c, nw, prec, kPlanValueOnly).total));
  return PN_OK;
}

pn_status pn_eval_plan(const pn_ctx* c, int64_t nw, pn_precision prec, int32_t kind, pn_plan_info* out) {
  if (!c || !out || nw < 0 || prec < PN_PREC_FP64 || prec > PN_PREC_NET_BF16 || kind < 0 || kind > 3)
    return PN_ERR_INVALID_ARG;
  const WsLayout L = plan(c, nw, prec, kind);
  memset(out, 0, sizeof(*out));
  out->tile_walkers = L.tile;
  out->chunk_coords = L.T;
  out->n_chunks = L.n_chunks;
  out->lowrank = L.lowrank ? 1 : 0;
  out->workspace_bytes = L.total;
  return PN_OK;
}

pn_status pn_eval(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const double* params,
                  pn_precision prec, double* logabs, double* sign, double* grad, double* lap, double* eloc, void* ws,
                  size_t ws_bytes) {
  if (!c || nw < 0 || prec < PN_PREC_FP64 || prec > PN_PREC_NET_BF16) return PN_ERR_INVALID_ARG;
  if (nw == 0) return PN_OK;
  if (!r || !params || !logabs || !sign || !ws) return PN_ERR_INVALID_ARG;
  WsLayout L = plan(c, nw, prec, (grad || lap || eloc) ? kPlanForward : kPlanValueOnly);
  if (ws_bytes < L.total) return PN_ERR_WORKSPACE_TOO_SMALL;
  if (L.lds_tangent > kLdsMax) return PN_ERR_UNSUPPORTED_SHAPE;
  return eval_impl(c, s, nw, r, params, prec, logabs, sign, grad, lap, eloc, static_cast<char*>(ws), L);
}

pn_status pn_eval_noalloc(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const double* params,
                          pn_precision prec, double* logabs, double* sign, double* grad, double* lap, double* eloc) {
  if (!c || nw < 0 || prec < PN_PREC_FP64 || prec > PN_PREC_NET_BF16) return PN_ERR_INVALID_ARG;
  if (nw == 0) return PN_OK;
  if (!r || !params || !logabs || !sign) return PN_ERR_INVALID_ARG;
  char* base = static_cast<char*>(scratch_of(c->device));
  if (!base) return PN_ERR_DEVICE;
  // walker tiles sized for the static scratch (down to one walker)
  WsLayout L = plan(c, nw, prec, (grad || lap || eloc) ? kPlanForward : kPlanValueOnly, kScratchBytes, 1);
  if (L.total > kScratchBytes) return PN_ERR_WORKSPACE_TOO_SMALL;
  if (L.lds_tangent > kLdsMax) return PN_ERR_UNSUPPORTED_SHAPE;
  return eval_impl(c, s, nw, r, params, prec, logabs, sign, grad, lap, eloc, base, L);
}

}  // extern "C"

namespace {
pn_status eval_impl(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const double* params,
                    pn_precision prec, double* logabs, double* sign, double* grad, double* lap, double* eloc, char* base,
                    const WsLayout& L) {
  // PN_PREC_NET_BF16: BF16 operands in the tangent (derivative) products
  // only; the value pass stays FP32 (BF16 values of f, J and of the stored
  // filter values and slopes move E_loc by far more than FP32 does)
  const bool fp64 = prec == PN_PREC_FP64, bf16 = prec == PN_PREC_NET_BF16;
  const bool derivs = grad || lap || eloc;
  const Dims& d = c->d;
  const bool no_net = (d.flags & (PN_NET_NO_JASTROW | PN_NET_NO_BACKFLOW)) == (PN_NET_NO_JASTROW | PN_NET_NO_BACKFLOW);
  const void* P = params;
  StageClock clk(c, s);
  if (!fp64) {
    clk.begin(0);
    launch_convert_params(s, c->pl.total, params, reinterpret_cast<float*>(base + L.params_net));
    clk.end(0);
    P = base + L.params_net;
  }
  for (int64_t w0 = 0; w0 < nw; w0 += L.tile) {
    const int64_t n = std::min<int64_t>(L.tile, nw - w0);
    const double* rt = r + w0 * d.N * 3;
    clk.begin(1);
    launch_geometry_orbitals(c, s, n, rt, base, L);
    clk.end(1);
    if (no_net) {
      // neither Jastrow factor nor backflow: f = 1, J = 0 and no network work
      launch_fill(s, n * d.N * d.M, reinterpret_cast<double*>(base + L.fval), 1.0);
      launch_fill(s, n, reinterpret_cast<double*>(base + L.jval), 0.0);
    } else if (fp64) {
      clk.begin(2);
      launch_filters<double>(c, s, n, rt, static_cast<const double*>(P), base, L, false);
      clk.end(2);
      clk.begin(3);
      launch_net_value<double>(c, s, n, static_cast<const double*>(P), base, L, false);
      clk.end(3);
    } else {
      clk.begin(2);
      launch_filters<float>(c, s, n, rt, static_cast<const float*>(P), base, L, false);
      clk.end(2);
      clk.begin(3);
      launch_net_value<float>(c, s, n, static_cast<const float*>(P), base, L, false);
      clk.end(3);
    }
    clk.begin(4);
    if (L.lowrank)
      launch_lowrank_value(c, s, n, base, L, logabs + w0, sign + w0);
    else
      launch_slater_value(c, s, n, base, L, logabs + w0, sign + w0);
    clk.end(4);
    if (derivs) {
      clk.begin(5);
      if (no_net) {
        launch_fill(s, n * L.n_chunks * d.N * (L.T + 1) * d.M, reinterpret_cast<double*>(base + L.ftan), 0.0);
        launch_fill(s, n * L.n_chunks * (L.T + 1), reinterpret_cast<double*>(base + L.jtan), 0.0);
      } else if (fp64) {
        launch_net_tangent<double>(c, s, n, rt, static_cast<const double*>(P), base, L, false);
      } else {
        launch_net_tangent<float>(c, s, n, rt, static_cast<const float*>(P), base, L, bf16);
      }
      clk.end(5);
      double* g = grad ? grad + w0 * d.N * 3 : reinterpret_cast<double*>(base + L.adj);
      clk.begin(6);
      if (L.lowrank)
        launch_lowrank_tangent(c, s, n, base, L, g);
      else
        launch_slater_tangent(c, s, n, rt, base, L, g);
      clk.end(6);
      clk.begin(7);
      launch_finalize(c, s, n, base, L, g, lap ? lap + w0 : nullptr, eloc ? eloc + w0 : nullptr);
      clk.end(7);
    }
    clk.next_set();
  }
  if (hipGetLastError() != hipSuccess) return PN_ERR_DEVICE;
  return PN_OK;
}
}  // namespace

extern "C" {

pn_status pn_eval_backward(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const double* params,
                           pn_precision prec, const double* ct_logabs, const double* ct_grad, const double* ct_lap,
                           const double* ct_eloc, double* grad_params, void* ws, size_t ws_bytes) {
  if (!c || nw < 0 || prec < PN_PREC_FP64 || prec > PN_PREC_NET_BF16) return PN_ERR_INVALID_ARG;
  if (nw == 0) return PN_OK;
  if (!r || !params || !grad_params || !ws) return PN_ERR_INVALID_ARG;
  const bool full = ct_grad || ct_lap || ct_eloc;
  if (!full && !ct_logabs) return PN_OK;  // every cotangent is zero
  if ((c->d.flags & (PN_NET_NO_JASTROW | PN_NET_NO_BACKFLOW)) == (PN_NET_NO_JASTROW | PN_NET_NO_BACKFLOW))
    return PN_OK;  // without both heads psi does not depend on the parameters
  const bool fp64 = prec == PN_PREC_FP64, bf16 = prec == PN_PREC_NET_BF16;
  if (!backward_supported(c, !fp64)) return PN_ERR_UNSUPPORTED_SHAPE;
  WsLayout L = plan(c, nw, prec, full ? kPlanFullAdjoint : kPlanValueAdjoint);
  if (ws_bytes < L.total) return PN_ERR_WORKSPACE_TOO_SMALL;
  const Dims& d = c->d;
  if (full && (L.lds_tadj > kLdsMax || L.lds_adjdet > kLdsMax || L.lds_tangent > kLdsMax ||
               backward_filter_lds_bytes(d, !fp64, true) > kLdsMax))
    return PN_ERR_UNSUPPORTED_SHAPE;
  char* base = static_cast<char*>(ws);
  const void* P = params;
  if (!fp64) {
    launch_convert_params(s, c->pl.total, params, reinterpret_cast<float*>(base + L.params_net));
    P = base + L.params_net;
  }
  // the forward pass is recomputed here (nothing is kept between calls); its
  // ln|psi| and sign go to scratch
  double* la = reinterpret_cast<double*>(base + L.adj);
  double* sg = la + L.tile;
  for (int64_t w0 = 0; w0 < nw; w0 += L.tile) {
    const int64_t n = std::min<int64_t>(L.tile, nw - w0);
    const double* rt = r + w0 * d.N * 3;
    launch_geometry_orbitals(c, s, n, rt, base, L);
    if (fp64) {
      launch_filters<double>(c, s, n, rt, static_cast<const double*>(P), base, L, false);
      launch_net_value<double>(c, s, n, static_cast<const double*>(P), base, L, false);
    } else {
      launch_filters<float>(c, s, n, rt, static_cast<const float*>(P), base, L, false);
      launch_net_value<float>(c, s, n, static_cast<const float*>(P), base, L, false);
    }
    launch_slater_value(c, s, n, base, L, la, sg);
    const double* ctl = ct_logabs ? ct_logabs + w0 : nullptr;
    if (full) {
      // coordinate derivatives with the layer inputs and per-determinant
      // results kept, then the determinant and network-tangent adjoints
      if (fp64)
        launch_net_tangent<double>(c, s, n, rt, static_cast<const double*>(P), base, L, false,
                                   reinterpret_cast<double*>(base + L.xsave));
      else
        launch_net_tangent<float>(c, s, n, rt, static_cast<const float*>(P), base, L, bf16,
                                  reinterpret_cast<float*>(base + L.xsave));
      launch_slater_tangent(c, s, n, rt, base, L, reinterpret_cast<double*>(base + L.gradf),
                            reinterpret_cast<double*>(base + L.detres));
      launch_adj_det(c, s, n, L, base, ctl, ct_grad ? ct_grad + w0 * d.N * 3 : nullptr, ct_lap ? ct_lap + w0 : nullptr,
                     ct_eloc ? ct_eloc + w0 : nullptr);
      if (fp64)
        launch_net_tangent_adj<double>(c, s, n, rt, static_cast<const double*>(P), base, L);
      else
        launch_net_tangent_adj<float>(c, s, n, rt, static_cast<const float*>(P), base, L);
      if (!ctl) {
        launch_fill0(s, n, reinterpret_cast<double*>(base + L.ct0));
        ctl = reinterpret_cast<const double*>(base + L.ct0);
      }
    }
    launch_backward(c, s, n, rt, P, !fp64, bf16, ctl, base, L, grad_params, full);
  }
  if (hipGetLastError() != hipSuccess) return PN_ERR_DEVICE;
  return PN_OK;
}

pn_status pn_eval_backward_cusp(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const double* params,
                                pn_precision prec, const double* ct_logabs, double* grad_cusp, void* ws,
                                size_t ws_bytes) {
  if (!c || nw < 0 || prec < PN_PREC_FP64 || prec > PN_PREC_NET_BF16) return PN_ERR_INVALID_ARG;
  if (nw == 0) return PN_OK;
  if (!r || !params || !ct_logabs || !grad_cusp || !ws) return PN_ERR_INVALID_ARG;
  if (c->n_cusp_on == 0) return PN_OK;  // no corrected orbital: the gradient is zero
  const Dims& d = c->d;
  if (cusp_grad_lds_bytes(d) > kLdsMax) return PN_ERR_UNSUPPORTED_SHAPE;
  const bool fp64 = prec == PN_PREC_FP64;
  WsLayout L = plan(c, nw, prec, kPlanValueAdjoint);
  if (ws_bytes < L.total) return PN_ERR_WORKSPACE_TOO_SMALL;
  char* base = static_cast<char*>(ws);
  const void* P = params;
  if (!fp64) {
    launch_convert_params(s, c->pl.total, params, reinterpret_cast<float*>(base + L.params_net));
    P = base + L.params_net;
  }
  const bool no_net = (d.flags & (PN_NET_NO_JASTROW | PN_NET_NO_BACKFLOW)) == (PN_NET_NO_JASTROW | PN_NET_NO_BACKFLOW);
  double* la = reinterpret_cast<double*>(base + L.adj);
  double* sg = la + L.tile;
  double* slot = reinterpret_cast<double*>(base + L.gpart);  // per-block partial sums
  for (int64_t w0 = 0; w0 < nw; w0 += L.tile) {
    const int64_t n = std::min<int64_t>(L.tile, nw - w0);
    const double* rt = r + w0 * d.N * 3;
    launch_geometry_orbitals(c, s, n, rt, base, L);
    if (no_net) {
      launch_fill(s, n * d.N * d.M, reinterpret_cast<double*>(base + L.fval), 1.0);
      launch_fill(s, n, reinterpret_cast<double*>(base + L.jval), 0.0);
    } else if (fp64) {
      launch_filters<double>(c, s, n, rt, static_cast<const double*>(P), base, L, false);
      launch_net_value<double>(c, s, n, static_cast<const double*>(P), base, L, false);
    } else {
      launch_filters<float>(c, s, n, rt, static_cast<const float*>(P), base, L, false);
      launch_net_value<float>(c, s, n, static_cast<const float*>(P), base, L, false);
    }
    launch_slater_value(c, s, n, base, L, la, sg);
    launch_cusp_grad(c, s, n, rt, base, L, ct_logabs + w0, slot, grad_cusp);
  }
  if (hipGetLastError() != hipSuccess) return PN_ERR_DEVICE;
  return PN_OK;
}

pn_status pn_stage_timing(pn_ctx* c, int enable) {
  if (!c) return PN_ERR_INVALID_ARG;
  if (enable) {
    if (!c->timing) {
      c->timing = new pn_ctx::Timing();
      for (int a = 0; a < pn_ctx::Timing::kSets; ++a)
        for (int k = 0; k < pn_ctx::Timing::kStages; ++k)
          for (int e = 0; e < 2; ++e)
            if (hipEventCreate(&c->timing->ev[a][k][e]) != hipSuccess) return PN_ERR_DEVICE;
    }
    for (int k = 0; k < pn_ctx::Timing::kStages; ++k) {
      c->timing->ms[k] = 0;
      c->timing->cnt[k] = 0;
    }
    c->timing->on = true;
  } else if (c->timing) {
    c->timing->on = false;
  }
  return PN_OK;
}

pn_status pn_stage_times(pn_ctx* c, double* ms, int64_t* cnt, int n) {
  if (!c || !ms || !cnt || n < PN_N_STAGES) return PN_ERR_INVALID_ARG;
  for (int k = 0; k < n; ++k) {
    ms[k] = 0;
    cnt[k] = 0;
  }
  if (!c->timing) return PN_OK;
  for (int a = 0; a < pn_ctx::Timing::kSets; ++a) harvest_set(c->timing, a);
  for (int k = 0; k < PN_N_STAGES; ++k) {
    ms[k] = c->timing->ms[k];
    cnt[k] = c->timing->cnt[k];
  }
  return PN_OK;
}

}  // extern "C"
