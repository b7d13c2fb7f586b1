// Internal definitions shared by the host API and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/paulinet.h"

namespace pn {

constexpr int kMaxLayers = 8;
constexpr int kMaxNuc = 64;
constexpr int kMaxElec = 64;
constexpr int kMaxSpin = 32;
constexpr int kMaxDet = 64;
constexpr int kThreads = 256;
constexpr int kMaxExc = 4;      // largest excitation rank of the low-rank determinant path
constexpr int kListGrid = 1024;  // blocks of a grid-stride launch over a device-side walker list

// Offsets (in elements) of every tensor inside the flat parameter blob.
struct ParamLayout {
  int64_t x0, Y;
  struct Layer {
    int64_t w1W[3], w1b[3], w2W[3], w2b[3];
    int64_t hW, hb;
    int64_t gW[3], gb[3];
  } layer[kMaxLayers];
  int64_t eW1, eb1, eW2, eb2, eW3, eb3;
  int64_t kW1, kb1, kW2, kb2, kW3, kb3;
  int64_t total;
};

// Problem sizes, passed by value to every kernel.
struct Dims {
  int N, n_up, n_dn, NN, NB, M, P;
  int K, DX, DZ, L;
  int n_ee;      // N (N - 1) / 2 electron pairs i < j
  int n_pairs;   // n_ee + N * NN
  int n_shell;
  double feat_rc;
  double cusp_rc;
  double v_nn;   // nuclear repulsion, a constant of the geometry
  int flags;     // PN_NET_NO_JASTROW | PN_NET_NO_BACKFLOW | PN_DET_DIRECT
  // low-rank determinant path: every determinant differs from the first in
  // at most kMaxExc orbitals per spin (lr = 1); nv[s] virtual orbitals
  // (occupied somewhere, not in the first determinant) per spin
  int lr;
  int nv[2];
};

// Device-resident copies of the system tables (owned by the context).
struct DevTables {
  double* nuc_xyz;     // [NN][3]
  double* charge;      // [NN]
  int* shell_center;   // [n_shell]
  int* shell_l;        // [n_shell]
  double* shell_exp;   // [n_shell]
  double* shell_norm;  // [n_shell]
  int* shell_first;    // [n_shell] first basis index
  double* mo;          // [NB][M]
  int* det_up;         // [P][n_up]
  int* det_dn;         // [P][n_dn]
  double* ci_log;      // [P] ln|c_p|
  double* ci_sign;     // [P] sign c_p
  // nuclear cusp correction, per (nucleus, MO)
  int* cusp_on;        // [NN][M]
  double* cusp_sign;   // [NN][M]
  double* cusp_alpha;  // [NN][M][5]
  double* cusp_dalpha; // [NN][M][5] derivatives of the coefficients in the nucleus value
  int* s_first;        // [NN+1] CSR offsets into s_basis
  int* s_basis;        // basis index of each s function, grouped by nucleus
  double* s_exp;       // exponent of each s function (same order)
  double* s_norm;      // normalisation of each s function
  // distance features
  double* feat_mu;     // [K]
  double* feat_sig2inv;// [K] 1 / sigma_k^2
  // pairs
  int* pair_ij;        // [n_ee][2] (i < j)
  int* pair_index;     // [N][N] unified pair index of the ee pair, -1 on the diagonal
  // low-rank determinant path, per (determinant p, spin s) relative to the
  // first determinant: rank k, hole slots of the first determinant's rows,
  // particle rows (indices into the spin's virtual list), sign of the row
  // permutation from "first determinant with holes replaced" to the listed order
  int* lr_k;           // [P][2]
  int* lr_hole;        // [P][2][kMaxExc]
  int* lr_part;        // [P][2][kMaxExc]
  double* lr_sign;     // [P][2]
  int* lr_vorb;        // [2][M] orbital of each virtual row of spin s
};

// Workspace regions for one walker tile (byte offsets from ws base).
struct WsLayout {
  int64_t tile;        // walkers per tile
  int T;               // coordinates per tangent chunk
  int n_chunks;
  int wpb_value;       // walkers per block in the value network kernel
  size_t lds_tangent;  // dynamic LDS of the tangent kernel
  int tan_threads;     // threads per tangent block: 256 (two blocks per CU) or 512 (one block, all LDS)
  size_t lds_value;
  size_t lds_filter;
  int filt_rows;       // pairs per block in the filter kernel
  bool stage_filters;  // tangent pass copies the layer's filter tables to LDS
  // offsets
  size_t params_net;   // converted params (float) when the network is FP32/BF16
  size_t geo;          // [tile][GEO] V, gamma, then per electron grad(3) + hess diag(3)
  size_t phi;          // [tile][N][M][7] value, grad(3), d2 diag(3)
  size_t filt;         // [tile][L][3][n_pairs][DZ]  (w, w'/d, w'')  net type
  size_t hval;         // [tile][L][N][DZ]                           net type
  size_t kcoef;        // [tile][2][2][N][DX] (ssp', ssp'') per kappa hidden layer
  size_t ecoef;        // [tile][2][2][DX]
  size_t fval;         // [tile][N][M]  double
  size_t jval;         // [tile]        double
  size_t ginv;         // [tile][P][n_up*n_up + n_dn*n_dn] inverse matrices
  size_t ldet;         // [tile][P][2][2] (ln|det|, sign) per spin
  size_t wdet;         // [tile][P] signed determinant weights
  size_t ldpsi;        // [tile] ln|psi_d|
  size_t ftan;         // [tile][n_chunks][N][T+1][M] double
  size_t jtan;         // [tile][n_chunks][T+1] double
  size_t partial;      // [tile][n_chunks][2]
  size_t xval;         // [tile][L+1][N][DX] activations (backward only)
  size_t adj;          // backward scratch
  size_t gpart;        // [n_blocks][n_params] per-block parameter gradients
  // full adjoint (cotangents on grad / lap / E_loc)
  bool full;
  bool tadj_global;    // tangent-adjoint row buffers in a global arena (else LDS)
  size_t lds_tadj;     // dynamic LDS of the tangent adjoint
  size_t lds_adjdet;   // dynamic LDS of the determinant adjoint
  size_t tadj_arena;   // elements of one block's row buffers
  size_t xsave;        // [tile][n_chunks][L][N(T+1)][DX] net type: layer inputs of the tangent pass
  size_t detres;       // [tile][n_chunks][P][2][T+1] per-determinant derivatives
  size_t gradf;        // [tile][3N] gradient of ln|psi|
  size_t ctc;          // [tile][3N+2] (ct grad', ct lap', ct ln|psi|)
  size_t ctdet;        // [tile][P][3N+2] (ct g_pa, ct Delta_p, ct l_p)
  size_t ctftan;       // [tile][n_chunks][N][T+1][M] ct of f tangents / partial Laplacians
  size_t ctfpart;      // [tile][n_chunks][N][M] ct of f, per chunk
  size_t cthv;         // [tile][L][N][DZ]       net type
  size_t ctww;         // [tile][L][n_ee][DZ]    net type
  size_t ctwd;         // [tile][L][n_pairs][DZ] net type
  size_t ctw2;         // [tile][L][n_pairs][DZ] net type
  size_t ctkc;         // [tile][2][2][N][DX]    net type
  size_t ctec;         // [tile][2][2][DX]       net type
  size_t ct0;          // [tile] zeros (absent ln|psi| cotangent)
  size_t tslot;        // [kSlotsTanAdj][n_params] + global arena, net type
  // low-rank determinant path (forward only)
  bool lowrank;
  size_t lds_lr;       // dynamic LDS of the low-rank tangent kernel
  size_t g0;           // [tile][n_up^2 + n_dn^2] inverse of the first determinant per spin
  size_t ld0;          // [tile][2][2] its (ln|det|, sign) per spin
  size_t theta;        // [tile][nv_up n_up + nv_dn n_dn] excitation table
  size_t dinv;         // [tile][P][2][kMaxExc^2] inverse of each determinant's minor
  size_t lrflag;       // [tile][2] int: walker handed to the direct path
  size_t lrlist;       // [tile + 1] int: those walkers (ascending), then their count
  size_t total;
};

constexpr int kSlotsTanAdj = 512;  // blocks (and gradient slots) of the tangent adjoint

constexpr int kGeoStride(int N) { return 4 + 6 * N; }  // V, gamma, lap_gamma, pad, N*(grad3, hess3)

// Electrons whose coordinates a chunk of T coordinates starting at a
// multiple of T can hold: exactly T / 3 when 3 divides T (chunks then start
// on an electron boundary), else at most T / 3 + 2.
__host__ __device__ constexpr int chunk_elecs_max(int N, int T) {
  return (T % 3 == 0 ? T / 3 : T / 3 + 2) < N ? (T % 3 == 0 ? T / 3 : T / 3 + 2) : N;
}

}  // namespace pn

struct pn_ctx {
  pn::Dims d;
  pn::ParamLayout pl;
  pn::DevTables t;
  int device;
  int n_cusp_on;
  // optional per-stage timing (profiling only; not part of the immutable state)
  struct Timing {
    static constexpr int kSets = 64, kStages = PN_N_STAGES;
    bool on = false;
    hipEvent_t ev[kSets][kStages][2] = {};
    bool rec[kSets][kStages] = {};
    int cur = 0;
    double ms[kStages] = {};
    int64_t cnt[kStages] = {};
  };
  mutable Timing* timing = nullptr;
};

namespace pn {

// ---------------------------------------------------------------- helpers --
__device__ __forceinline__ double sigmoid_d(double x) { return 1.0 / (1.0 + exp(-x)); }
__device__ __forceinline__ float sigmoid_d(float x) { return 1.0f / (1.0f + __expf(-x)); }

// Shifted softplus ssp(x) = ln(1 + e^x) - ln 2, evaluated stably.
__device__ __forceinline__ double ssp(double x) {
  return (x > 0 ? x + log1p(exp(-x)) : log1p(exp(x))) - 0.69314718055994530942;
}
__device__ __forceinline__ float ssp(float x) {
  return (x > 0.f ? x + log1pf(__expf(-x)) : log1pf(__expf(x))) - 0.69314718f;
}

// LDS row stride with 16 bytes of padding (keeps 16-byte alignment, spreads
// rows over the banks).
template <typename T>
__host__ __device__ constexpr int ld_pad(int D) {
  return D + 16 / (int)sizeof(T);
}

}  // namespace pn

// Launchers implemented in the kernel translation units.
namespace pn {
void launch_geometry_orbitals(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, char* ws,
                              const WsLayout& L);
template <typename TN>
void launch_filters(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const TN* P, char* ws,
                    const WsLayout& L, bool bf16);
template <typename TN>
void launch_net_value(const pn_ctx* c, hipStream_t s, int64_t nw, const TN* P, char* ws, const WsLayout& L,
                      bool bf16);
template <typename TN>
void launch_net_tangent(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const TN* P, char* ws,
                        const WsLayout& L, bool bf16, TN* xsave = nullptr);
void launch_slater_value(const pn_ctx* c, hipStream_t s, int64_t nw, char* ws, const WsLayout& L,
                         double* logabs, double* sign);
void launch_slater_lu(const pn_ctx* c, const Dims& d, hipStream_t s, int64_t nw, char* ws, const WsLayout& L,
                      double* G, double* ld, const int* wlist, const int* wcount, int64_t nb_lane, int64_t nb_wave);
void launch_combine_value(const pn_ctx* c, hipStream_t s, int64_t nw, char* ws, const WsLayout& L, double* logabs,
                          double* sign);
void launch_slater_tangent(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, char* ws,
                           const WsLayout& L, double* grad, double* detres = nullptr, const int* wlist = nullptr,
                           const int* wcount = nullptr);
size_t lowrank_tangent_lds_bytes(const Dims& d, int T);
void launch_lowrank_value(const pn_ctx* c, hipStream_t s, int64_t nw, char* ws, const WsLayout& L, double* logabs,
                          double* sign);
void launch_lowrank_tangent(const pn_ctx* c, hipStream_t s, int64_t nw, char* ws, const WsLayout& L, double* grad);
void launch_finalize(const pn_ctx* c, hipStream_t s, int64_t nw, char* ws, const WsLayout& L, double* grad,
                     double* lap, double* eloc);
void launch_convert_params(hipStream_t s, int64_t n, const double* src, float* dst);
void launch_fill0(hipStream_t s, int64_t n, double* dst);
void launch_fill(hipStream_t s, int64_t n, double* dst, double v);
size_t cusp_grad_lds_bytes(const Dims& d);
void launch_cusp_grad(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, char* ws, const WsLayout& L,
                      const double* ct, double* slot, double* grad);
void launch_adj_det(const pn_ctx* c, hipStream_t s, int64_t nw, const WsLayout& L, char* ws, const double* ct_logabs,
                    const double* ct_grad, const double* ct_lap, const double* ct_eloc);
template <typename TN>
void launch_net_tangent_adj(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const TN* P, char* ws,
                            const WsLayout& L);
}  // namespace pn
