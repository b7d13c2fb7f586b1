/*
 * paulinet.h -- C ABI of the MI355X (gfx950) PauliNet walker-evaluation
 * library.
 *
 * The library evaluates, for a batch of Monte Carlo walkers r (all electron
 * positions), the PauliNet wavefunction of Hermann, Schaetzle and Noe
 * (arXiv:1909.08423, Results eq. "ansatz"):
 *
 *   psi(r) = exp(gamma(r) + J(r)) sum_p c_p det[phi~_up] det[phi~_down],
 *   phi~_{mu i}(r) = phi_mu(r_i) f_{mu i}(r),
 *
 * with a Gaussian-orbital baseline phi_mu corrected at the nuclei (Methods,
 * "Cusp conditions"), the electronic cusp factor gamma (same section), and a
 * SchNet-style network giving the Jastrow factor J and the backflow f
 * (Methods, "PauliNet extension of SchNet").  Per walker it returns
 * ln|psi|, sign psi, the gradient and Laplacian of ln|psi| in the electron
 * coordinates and the local energy
 *
 *   E_loc = -1/2 (lap ln|psi| + |grad ln|psi||^2) + V        (Methods,
 *                                                    eq. "monte-carlo")
 *
 * and, for the VMC update, the parameter gradient of sum_w ct_w ln|psi_w|
 * (the adjoint needed by the Hermitian estimator, Methods eq. "trainig").
 *
 * Conventions
 *  - Every pointer argument is a DEVICE pointer unless marked [host].
 *  - Calls enqueue work on the given HIP stream and return; they never
 *    synchronise.  Errors detectable on the host (null pointers, shapes,
 *    workspace size) are returned before anything is enqueued; a non-OK
 *    status means nothing was enqueued.
 *  - The caller owns every device buffer, including the workspace.  The
 *    library allocates device memory only in pn_ctx_create (small copies of
 *    the system tables) and frees it in pn_ctx_destroy.
 *  - Per-walker numerical outcomes are data, not errors: an exactly
 *    cancelling determinant sum gives logabs = -inf and sign = 0.
 *  - Electrons 0..n_up-1 are spin up, the rest spin down.  Coordinates are
 *    in bohr, energies in hartree.
 *  - Limits: n_up, n_down <= 32; n_elec <= 64; n_det <= 64; n_nuc <= 64;
 *    n_feat, dim_x and dim_z each one of 16, 32, 64, 128; n_mo <= dim_x;
 *    n_layers <= 8; shells are s (l = 0) or p (l = 1).  Anything else
 *    returns PN_ERR_UNSUPPORTED_SHAPE.
 */
#ifndef PAULINET_H
#define PAULINET_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PN_OK = 0,
  PN_ERR_INVALID_ARG = 1,
  PN_ERR_UNSUPPORTED_SHAPE = 2,
  PN_ERR_WORKSPACE_TOO_SMALL = 4,
  PN_ERR_DEVICE = 5,
  PN_ERR_BUDGET = 6
} pn_status;

/* Arithmetic of the network (distance features, filters, interaction
 * layers, Jastrow and backflow heads).  Geometry, orbitals, determinants,
 * their derivatives and E_loc are always FP64.  In the BF16 form only the
 * dense products of the derivative (tangent) pass take BF16 operands; the
 * value pass (filters, layers and heads on the values) stays FP32, because
 * BF16 values of the backflow, the Jastrow factor and the stored filter
 * values move E_loc by orders of magnitude more than FP32 rounding does,
 * while BF16 tangent products leave the batch-mean E_loc at the FP32 level. */
typedef enum {
  PN_PREC_FP64 = 0,     /* network in FP64                                  */
  PN_PREC_NET_FP32 = 1, /* network in FP32                                  */
  PN_PREC_NET_BF16 = 2  /* FP32 value pass; tangent products BF16 operands,
                           FP32 accumulation                                */
} pn_precision;

typedef struct pn_ctx pn_ctx; /* opaque; immutable after create */

/* The system (Results, "Hartree-Fock baseline"; Methods, "Computational
 * details"): nuclei, one primitive Gaussian per shell, MO coefficients and
 * the determinant expansion.  All arrays are [host] and copied at create. */
typedef struct {
  int32_t n_nuc;
  const double* nuc_xyz;      /* [n_nuc][3]                                */
  const double* charge;       /* [n_nuc]                                   */
  int32_t n_up, n_down;
  int32_t n_shell;
  const int32_t* shell_center; /* [n_shell] nucleus index                  */
  const int32_t* shell_l;      /* [n_shell] 0 = s, 1 = p                   */
  const double* shell_exp;     /* [n_shell] Gaussian exponent              */
  int32_t n_mo;
  const double* mo_coeff;      /* [n_basis][n_mo]; n_basis = sum(2l+1),
                                  basis order = shell order, then x, y, z  */
  int32_t n_det;
  const int32_t* det_up;       /* [n_det][n_up] orbital indices            */
  const int32_t* det_down;     /* [n_det][n_down]                          */
  const double* ci;            /* [n_det] determinant coefficients c_p     */
  double cusp_radius;          /* nuclear cusp correction radius; 0 = off  */
  const double* cusp_nuc_value; /* [n_nuc][n_mo] corrected on-centre s-part
                                   value at each nucleus (the variational
                                   nucleus value); NULL = uncorrected s(0) */
} pn_system_desc;

/* Network shape (Methods, SchNet extension and featurisation; Table 2). */
typedef struct {
  int32_t n_feat;     /* K, number of distance features e_k             */
  double feat_cutoff; /* r_c in mu_k = r_c q_k^2, sigma_k = (1+r_c q_k)/7 */
  int32_t dim_x;      /* D_x, electron embedding width                  */
  int32_t dim_z;      /* D_z, message width                             */
  int32_t n_layers;   /* L, interaction layers                          */
  int32_t flags;      /* ansatz variant: PN_NET_NO_JASTROW, PN_NET_NO_BACKFLOW (or 0) */
} pn_net_desc;

/* Ansatz variants (Results: the paper compares single- and multi-determinant
 * baselines with a Jastrow factor only or with Jastrow and backflow; single
 * vs multiple determinants is just n_det).  A removed head is identically
 * J = 0 or f = 1: its parameters stay in the blob but receive exactly zero
 * gradient, and with both heads removed the network is not evaluated. */
#define PN_NET_NO_JASTROW 1
#define PN_NET_NO_BACKFLOW 2

/* Determinant path of the forward evaluation.  When every determinant of
 * the expansion differs from the first one in at most 4 orbitals per spin
 * (single, double, ... excitations; Results, eq. "ansatz": the
 * multideterminant sum), pn_eval evaluates the expansion through one LU of
 * the first determinant per spin: det A_p = det A_0 det(Theta[v][h]) with
 * the excitation table Theta = Phi~ A_0^{-1}, and the coordinate derivatives
 * through T_a A_0^{-1} (one product per spin and coordinate instead of one
 * per determinant).  This is exact up to rounding; walkers whose first
 * determinant is singular or small against another member (ratio above
 * 1e4) are evaluated member by member instead.  PN_DET_DIRECT in
 * pn_net_desc.flags forces the member-by-member path for every walker.
 * The adjoints always take the member-by-member path. */
#define PN_DET_DIRECT 4

/* Create a context: validates shapes, builds the pair and determinant
 * tables and the nuclear-cusp polynomials on the host, copies them to the
 * current device.  *out is NULL on error. */
pn_status pn_ctx_create(const pn_system_desc* sys, const pn_net_desc* net, pn_ctx** out);
void pn_ctx_destroy(pn_ctx* ctx);

/* Number of entries of the flat FP64 parameter blob.  Layout (Linear is
 * y = x W + b, W stored [in][out] row-major):
 *   x0[D_x], Y[n_nuc][D_z];
 *   per layer: for c in (+,-,n): w1W[K][D_z] w1b[D_z] w2W[D_z][D_z] w2b[D_z];
 *              hW[D_x][D_z] hb[D_z];
 *              for c in (+,-,n): gW[D_z][D_x] gb[D_x];
 *   eta:   W1[D_x][D_x] b1[D_x] W2[D_x][D_x] b2[D_x] W3[D_x][1] b3[1];
 *   kappa: W1[D_x][D_x] b1[D_x] W2[D_x][D_x] b2[D_x] W3[D_x][n_mo] b3[n_mo]. */
int64_t pn_param_count(const pn_ctx* ctx);

/* One named tensor of the parameter blob: element offset, rank (1 or 2)
 * and shape (rows, columns; columns 0 for a vector).  Names: "x0", "Y",
 * "l<n>.w_<c>.W1|b1|W2|b2", "l<n>.h.W|b", "l<n>.g_<c>.W|b" with c in
 * {same, opp, nuc}, "eta.W1".."eta.b3", "kappa.W1".."kappa.b3". */
typedef struct {
  char name[32];
  int64_t offset;
  int32_t ndim;
  int32_t shape[2];
} pn_param_entry;

/* Fills entries[0 .. cap-1] ([host]) in blob order and sets *n to the total
 * number of tensors; returns PN_ERR_INVALID_ARG (with *n set) when cap is
 * too small, so a call with cap = 0 queries the count. */
pn_status pn_param_layout(const pn_ctx* ctx, pn_param_entry* entries, int32_t cap, int32_t* n);

/* Outputs a pn_eval call produces (out_mask of pn_workspace_bytes): a call
 * whose grad, lap and eloc are all NULL runs the value pass only and needs
 * no tangent buffers. */
#define PN_OUT_LOGABS 1u  /* logabs and sign (always produced) */
#define PN_OUT_GRAD 2u
#define PN_OUT_LAP 4u
#define PN_OUT_ELOC 8u
#define PN_OUT_ADJOINT 16u /* also pn_eval_backward with only ct_logabs */
#define PN_OUT_ALL 31u

/* Workspace bytes for the calls out_mask names, with n_walkers walkers at
 * the given precision: pn_eval calls whose non-NULL outputs are among its
 * PN_OUT_LOGABS / GRAD / LAP / ELOC bits (LOGABS alone: value-only calls,
 * which need no tangent buffers; any of GRAD, LAP, ELOC: the full forward
 * pass), and with PN_OUT_ADJOINT pn_eval_backward with only ct_logabs (the
 * value-path adjoint, whose per-block gradient slots can dominate small
 * batches).  Batches larger than the internal walker tile are processed tile
 * by tile, so the size stops growing at the tile.  PN_ERR_INVALID_ARG for
 * bits outside PN_OUT_ALL; a call that needs more than the workspace it is
 * given returns PN_ERR_WORKSPACE_TOO_SMALL. */
pn_status pn_workspace_bytes(const pn_ctx* ctx, int64_t n_walkers, pn_precision prec, uint32_t out_mask,
                             size_t* bytes);

/* Workspace bytes that also cover pn_eval_backward with cotangents on the
 * gradient, Laplacian or local energy (the full adjoint keeps the layer
 * inputs of the tangent pass and per-chunk cotangent tables per walker
 * tile); never less than pn_workspace_bytes. */
pn_status pn_workspace_bytes_full(const pn_ctx* ctx, int64_t n_walkers, pn_precision prec, size_t* bytes);

/* How a call with n_walkers walkers is carried out: walkers per internal
 * tile, coordinates per chunk of the tangent (derivative) pass, number of
 * chunks, whether the determinants take the low-rank path (PN_DET_DIRECT),
 * and the workspace bytes of that call.  kind: 0 = pn_eval with derivative
 * outputs, 1 = pn_eval_backward with only ct_logabs (value-path adjoint),
 * 2 = pn_eval_backward with coordinate cotangents (full adjoint), 3 =
 * pn_eval without derivative outputs (value pass only).  [host] out. */
typedef struct {
  int64_t tile_walkers;
  int32_t chunk_coords;
  int32_t n_chunks;
  int32_t lowrank;
  int32_t reserved;
  size_t workspace_bytes;
} pn_plan_info;

pn_status pn_eval_plan(const pn_ctx* ctx, int64_t n_walkers, pn_precision prec, int32_t kind, pn_plan_info* out);

/* Forward evaluation (the hot path).
 *   r       [B][n_elec][3] FP64 walker positions
 *   params  [pn_param_count] FP64 parameter blob (converted internally to
 *           the network precision)
 *   logabs  [B] ln|psi|          sign [B] in {-1, 0, +1}
 *   grad    [B][n_elec][3] d ln|psi| / d r, or NULL
 *   lap     [B] Laplacian of ln|psi|, or NULL
 *   eloc    [B] local energy, or NULL
 * If grad, lap and eloc are all NULL only the value pass runs. */
pn_status pn_eval(const pn_ctx* ctx, hipStream_t stream, int64_t n_walkers, const double* r,
                  const double* params, pn_precision prec, double* logabs, double* sign,
                  double* grad, double* lap, double* eloc, void* ws, size_t ws_bytes);

/* pn_eval without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The workspace is a
 * static device array of 128 MiB inside the library (one per GPU, held until
 * the process ends; its address is taken when a context is created on that
 * GPU).  Batches of any size are processed in walker tiles that fit it, so a
 * large batch runs in more, smaller tiles than pn_eval uses; the results are
 * those of pn_eval.  A shape whose single walker needs more than 128 MiB of
 * workspace returns PN_ERR_WORKSPACE_TOO_SMALL; PN_ERR_DEVICE if the array's
 * address could not be taken.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (different streams, or other host
 * threads) race and must be serialised by the caller.  Nothing in the array
 * needs to start at zero. */
pn_status pn_eval_noalloc(const pn_ctx* ctx, hipStream_t stream, int64_t n_walkers, const double* r,
                          const double* params, pn_precision prec, double* logabs, double* sign, double* grad,
                          double* lap, double* eloc);

/* Parameter adjoint of the evaluation:
 *   grad_params[t] += sum_w ( ct_logabs[w] d ln|psi_w| / d theta_t
 *                           + sum_a ct_grad[w][a] d (d_a ln|psi_w|) / d theta_t
 *                           + ct_lap[w] d (lap ln|psi_w|) / d theta_t
 *                           + ct_eloc[w] d E_loc,w / d theta_t )
 * Each cotangent pointer may be NULL (= zero); ct_grad is [B][n_elec][3],
 * the others [B].  With only ct_logabs this is the value-path adjoint that
 * the Hermitian gradient estimator needs (Methods eq. "trainig": weights
 * 2 (E_loc - L) / B); with ct_grad, ct_lap or ct_eloc it is the full
 * adjoint through the coordinate derivatives, the Laplacian's second-order
 * terms included (d E_loc / d theta = -1/2 d(lap + |grad|^2) / d theta,
 * since V does not depend on theta), and needs pn_workspace_bytes_full
 * bytes of workspace.  grad_params is [pn_param_count] FP64 and is
 * ACCUMULATED into.  The forward values are recomputed inside the call
 * (nothing is stored between calls).  Per-walker contributions are reduced
 * in a fixed order, so the result does not depend on what else runs on the
 * device.  In the BF16 mode the recomputed value pass is FP32 and the
 * recomputed tangent pass (full adjoint) takes BF16 operands; the adjoint
 * products are FP32.  Shapes whose adjoint blocks exceed the LDS limit
 * return PN_ERR_UNSUPPORTED_SHAPE. */
pn_status pn_eval_backward(const pn_ctx* ctx, hipStream_t stream, int64_t n_walkers,
                           const double* r, const double* params, pn_precision prec,
                           const double* ct_logabs, const double* ct_grad, const double* ct_lap,
                           const double* ct_eloc, double* grad_params, void* ws, size_t ws_bytes);

/* Gradient in the orbital values at the nuclei (Methods, "Cusp conditions":
 * the corrected on-centre s part of each MO takes the value s0 at the
 * nucleus, which the paper optimizes; s0 is the cusp_nuc_value of the system
 * description, or its default):
 *   grad_cusp[I][mu] += sum_w ct_logabs[w] d ln|psi_w| / d s0[I][mu]
 * grad_cusp is [n_nuc][n_mo] FP64, accumulated into; entries of pairs
 * without correction stay unchanged.  Only electrons inside the cusp radius
 * of a nucleus contribute.  The forward values are recomputed (workspace of
 * pn_workspace_bytes); the sum has a fixed order.  To train s0, create the
 * context again with the new values (the context is immutable). */
pn_status pn_eval_backward_cusp(const pn_ctx* ctx, hipStream_t stream, int64_t n_walkers,
                                const double* r, const double* params, pn_precision prec,
                                const double* ct_logabs, double* grad_cusp, void* ws, size_t ws_bytes);

/* ---- Langevin Monte Carlo sampling ----------------------------------------
 * Methods, "Ansatz optimization" (Table 2: target acceptance 57 %, 50
 * discarded steps, 1 decorrelation step, resampling every 100 iterations):
 * drift-diffusion moves of Umrigar et al. (1993) with the step clipped below
 * the nearest-nucleus distance.  Per walker and step, all electrons at once:
 *   d_i = tau d_i ln|psi|, rescaled to length <= min_I |r_i - R_I|;
 *   r' = r + d(r) + sqrt(tau) xi;
 *   accept if u < A, ln A = 2 (ln|psi(r')| - ln|psi(r)|)
 *                         - (|r - r' - d(r')|^2 - |r' - r - d(r)|^2) / (2 tau);
 *   after the step tau <- tau exp(adapt_rate (acceptance - target_accept)).
 * xi and u come from Philox4x32-10 keyed by `seed`, counter (walker, step,
 * call, 0) as in pn_vmc_step (step = step0 + k for the k-th step). */
typedef struct {
  double target_accept; /* in (0, 1); 0.57 in the paper */
  double adapt_rate;    /* >= 0; 0 keeps tau fixed */
} pn_langevin_hparams;

pn_status pn_langevin_workspace_bytes(const pn_ctx* ctx, int64_t n_walkers, pn_precision prec, size_t* bytes);

/* n_steps steps on the walkers r ([B][n_elec][3] FP64, updated in place).
 * tau: [1] FP64 device scalar, read at every step and updated by the
 * adaptation (so consecutive calls continue the schedule).  stats:
 * [n_steps][2] FP64 device output (acceptance of the step, tau used).  One
 * wavefunction evaluation (value and gradient) per step plus one at the
 * start; the discarded and decorrelation steps of a schedule are simply
 * more steps. */
pn_status pn_langevin_run(const pn_ctx* ctx, hipStream_t stream, int64_t n_walkers, double* r,
                          const double* params, pn_precision prec, const pn_langevin_hparams* hp,
                          double* tau, int32_t n_steps, uint64_t seed, int64_t step0, double* stats,
                          void* ws, size_t ws_bytes);

/* ---- one VMC step of a job (serving) -------------------------------------
 * Methods, "Ansatz optimization": the walkers sample |psi|^2 by Metropolis
 * moves, the loss is the mean clipped local energy, its gradient comes from
 * the Hermitian estimator (eq. "trainig") and the parameters follow AdamW
 * with the decaying learning rate lr0 / (1 + t / t0) (Table 2).
 *
 * pn_vmc_step enqueues, on `stream`, for one job:
 *   1. ln|psi| at r (current parameters);
 *   2. all-electron Gaussian proposal r' = r + sigma xi, xi from the
 *      counter-based Philox4x32-10 generator keyed by `seed` with counter
 *      (walker, step, call, 0) (two Box-Muller normals per call, call =
 *      0, 1, ...; the acceptance uniform uses call 0xFFFFFFFF);
 *   3. ln|psi| at r' and acceptance when u < exp(2 (ln|psi'| - ln|psi|));
 *   4. E_loc at the new r;
 *   5. clipping: median m and mean absolute deviation delta of E_loc,
 *      window w = clip_q * delta, E~ = E inside the window, else
 *      m + sgn(E - m) w (1 + ln(|E - m| / w)); L = mean E~;
 *   6. g = (2 / B) sum_w (E~_w - L) d ln|psi_w| / d theta;
 *   7. AdamW on the FP64 parameters with step t = `step`.
 * A step whose E_loc has a non-finite value skips 6 and 7 (stats[5] = 0).
 * All buffers are the caller's; the call does not synchronise.  Results are
 * deterministic and independent of other work on the device.
 * Limits: n_walkers <= 16384 (the clipping statistics run in one block). */
typedef struct {
  double sigma;        /* Metropolis step, bohr (0.3)                      */
  double lr0, t0;      /* learning rate lr0 / (1 + t / t0) (0.01, 200)    */
  double clip_q;       /* clipping window in mean deviations (5)          */
  double beta1, beta2, eps, weight_decay; /* AdamW (0.9, 0.999, 1e-8, 0.01) */
} pn_vmc_hparams;

typedef struct {
  int64_t n_walkers;
  double* r;           /* [B][n_elec][3] walker positions, updated        */
  double* params;      /* [n_params] FP64 parameters, updated             */
  double* adam_m;      /* [n_params] first moment, updated (start at 0)   */
  double* adam_v;      /* [n_params] second moment, updated (start at 0)  */
  double* eloc;        /* [B] out: E_loc at the new positions             */
  double* stats;       /* [8] out: mean E_loc, std E_loc, acceptance,
                          clipped mean L, non-finite count, step applied
                          (1/0), median, clipping window                  */
  uint64_t seed;
  int64_t step;        /* t: RNG counter and AdamW step (0 for the first) */
} pn_vmc_job;

/* Workspace bytes for pn_vmc_step with n_walkers walkers. */
pn_status pn_vmc_workspace_bytes(const pn_ctx* ctx, int64_t n_walkers, pn_precision prec, size_t* bytes);
pn_status pn_vmc_step(const pn_ctx* ctx, hipStream_t stream, const pn_vmc_job* job, pn_precision prec,
                      const pn_vmc_hparams* hp, void* ws, size_t ws_bytes);

/* ---- continuous batching: one step of every active job ------------------
 * Device bytes of a job, for admission by memory: `resident` covers what
 * the job keeps between steps (walkers, parameters, both AdamW moments,
 * E_loc and the 8 statistics, all FP64), `scratch` the per-step workspace
 * (pn_vmc_workspace_bytes).  [host] outputs. */
pn_status pn_job_bytes(const pn_ctx* ctx, int64_t n_walkers, pn_precision prec, size_t* resident,
                       size_t* scratch);

/* One active job of a serving step: its context (system and network shape),
 * its state (pn_vmc_job: walkers, parameters, moments, E_loc, statistics,
 * seed and step counter t) and its workspace of pn_vmc_workspace_bytes. */
typedef struct {
  const pn_ctx* ctx;
  pn_vmc_job job;
  void* ws;
  size_t ws_bytes;
} pn_job_slot;

/* One VMC step (the seven parts listed under pn_vmc_step) of every job in
 * slots[0 .. n_slots-1] ([host] array; jobs of different systems, electron
 * counts and walker counts), as one launch sequence on `stream`: for each
 * part, the wavefunction evaluations run job by job and the proposal,
 * acceptance, clipping, gradient clearing and AdamW run as one launch over
 * all slots (16 slots per launch), with every slot's pointers passed in the
 * kernel arguments (nothing is allocated or copied).  Each job's results
 * equal those of pn_vmc_step on the same state bit for bit, whatever the
 * other slots hold; the caller advances each job's `step` afterwards.  Every
 * slot is validated before anything is enqueued.  Slots must not share
 * state or workspace buffers. */
pn_status pn_serve_step(hipStream_t stream, const pn_job_slot* slots, int32_t n_slots, pn_precision prec,
                        const pn_vmc_hparams* hp);

/* Per-stage kernel timing, for profiling.  When enabled, pn_eval records
 * a HIP event before and after each of its stages on the call's stream.
 * pn_stage_times waits for the recorded events and returns, per stage, the
 * summed duration in milliseconds and the number of timed launches since
 * timing was enabled; it synchronises with those events (not for use on a
 * latency-critical path).  Stages, in order: 0 parameter conversion,
 * 1 geometry + orbitals, 2 filters, 3 network values, 4 determinants,
 * 5 network tangents, 6 determinant tangents, 7 finalize.  n_stages of the
 * output arrays must be >= 8. */
#define PN_N_STAGES 8
pn_status pn_stage_timing(pn_ctx* ctx, int enable);
pn_status pn_stage_times(pn_ctx* ctx, double* ms_sum /*[host]*/, int64_t* count /*[host]*/, int n_stages);

const char* pn_status_string(pn_status s);

#ifdef __cplusplus
}
#endif

#endif /* PAULINET_H */
