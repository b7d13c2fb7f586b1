// Tangent pass of the network: first derivatives and partial Laplacian of
// every electron embedding, the Jastrow factor and the backflow, with
// respect to one chunk of electron coordinates (Methods, "PauliNet
// extension of SchNet"; Results, J = eta(sum_i x_i), f_i = kappa(x_i)).
//
// One 256-thread block per (walker, chunk); two blocks share a CU, so one
// block's barriers and load latencies overlap the other's work.  The chunk holds T = C - 1 coordinates
// a = a0 .. a0 + T - 1 (the last chunk may be ragged; its missing
// coordinates are zero columns).  For every electron row i the block keeps,
// in LDS, the T derivative columns d x_i / d r_a and one column with
// sum_{a in chunk} d^2 x_i / d r_a^2.  Each map is applied per coordinate,
// so the chunks are independent and their partial Laplacians add up:
//
//   Linear  y = x W + b     ->  y_a = x_a W,        y_L = x_L W
//   ssp     y = ssp(u)      ->  y_a = ssp'(u) u_a,  y_L = ssp'(u) u_L + ssp''(u) sum_a u_a^2
//   message z_i = sum_j w_ij h_j  with w_ij = w(|r_i - r_j|):
//           z_a = sum_j (w_ij h_{j,a} + d_a w_ij h_j)
//           z_L = sum_j (w_ij h_{j,L} + sum_a (d2_a w_ij h_j + 2 d_a w_ij h_{j,a}))
//     where, for a = (k, alpha) and u = r_i - r_j,
//           d_a w_ij  = (w'/d) u_alpha (delta_ik - delta_jk)
//           d2_a w_ij = w'' (u_alpha/d)^2 + (w'/d) (1 - (u_alpha/d)^2)   (k in {i, j})
//
// The values (h, w, w'/d, w'', ssp', ssp'') come from the value pass.  The
// dense products run on the matrix cores (mfma_gemm.h); the message sums are
// register-blocked over the C columns, which are a template parameter.
// Per layer the block passes five barriers: after the staging and the h
// product, and after each channel's message sums and product.  The nuclear
// channel's
// messages (non-zero only in rows of the chunk's own electrons, as the
// nuclei do not move) are extra items of channel 0's sums, and their product
// follows channel 0's in the same phase, on the same tile-to-wave map.
// With STAGE the layer's filter values and the chunk electrons' filter
// derivatives are copied to LDS first (coalesced), so the message sums read
// only LDS; without it (systems whose pair tables do not fit) they read the
// value pass's output in global memory.
//
// This file is included by k_tangent_f32.hip and k_tangent_f64.hip, which
// instantiate it for one network type each.
#pragma once
#include "gemm_lds.h"
#include "mfma_gemm.h"
#include "pn_internal.h"

namespace pn {

constexpr int kThreadsT = 256;

namespace {

// Block-wide global-to-LDS copy of n 16-byte units without registers: wave
// wv moves runs of 64 units, lane l the l-th unit of a run (the LDS address
// of a run is wave-uniform, as the load-to-LDS instruction requires).  The
// data land asynchronously; a barrier (which waits for outstanding loads)
// makes them visible.
__device__ __forceinline__ void dma16(uint4* __restrict__ dst, const uint4* __restrict__ src, int n, int lane,
                                      int wv, int nwv) {
  for (int b = wv * 64; b < n; b += nwv * 64)
    if (b + lane < n) __builtin_amdgcn_global_load_lds(src + b + lane, dst + b, 16, 0, 0);
}

// Head activation as the epilogue of the product that feeds it (chunks of
// three coordinates in the FP32 tile layout, where a lane's four results are
// the four columns of one row group: electron i = 4 rt + lane / 16 for the
// backflow head, the summed embedding for the Jastrow head):
//   y_a = s1 v_a (a < 3),   y_L = s1 v_L + s2 sum_a v_a^2
// with the value pass's slopes s1 = ssp'(u), s2 = ssp''(u) of the feature.
// h tangents of a 3-coordinate chunk in the FP32 tile layout, where a lane
// holds the four jet columns of one electron at one feature: stored as one
// 16-byte unit per (electron, feature), h[j * stride + 4 z + c], so that the
// message sums read a partner's four columns with one LDS read.
struct HStore4 {
  float* h;
  int n_elec, stride;
  static constexpr bool kOwnStore = true;
  template <typename A>
  __device__ void operator()(int, int, A&) const {}
  template <typename A>
  __device__ void store(int rt, int col, const A& c) const {
    const int j = 4 * rt + (((int)threadIdx.x & 63) >> 4);
    if (j < n_elec) *reinterpret_cast<float4*>(h + j * stride + 4 * col) = make_float4(c[0], c[1], c[2], c[3]);
  }
};

template <typename TN>
struct HeadAct {
  const TN* s;  // [2][rows][DX] slopes (s1 block, then s2 block)
  int n_rows, DX;
  bool per_row;  // backflow: slopes per electron; Jastrow: one row
  template <typename A>
  __device__ void operator()(int rt, int col, A& c) const {
    const int i = per_row ? min(4 * rt + (((int)threadIdx.x & 63) >> 4), n_rows - 1) : 0;
    const TN s1 = s[i * DX + col], s2 = s[(n_rows + i) * DX + col];
    TN sq = 0;
    sq += c[0] * c[0];
    sq += c[1] * c[1];
    sq += c[2] * c[2];
    c[0] = s1 * c[0];
    c[1] = s1 * c[1];
    c[2] = s1 * c[2];
    c[3] = s1 * c[3] + s2 * sq;
  }
};

// BF16 is a template parameter so that the FP32 and FP64 instantiations
// carry no BF16 operand code (smaller kernels, fewer instruction-cache
// misses).  NT threads per block: 256 with two blocks per CU (80 KB of LDS
// each), or 512 with one block per CU when a block takes all 160 KB (two
// waves per SIMD either way, so the register budget is the same).
template <typename TN, int C, bool STAGE, bool BF16, int NT>
__global__ __launch_bounds__(NT, 512 / NT) void k_net_tangent(Dims d, DevTables t, int64_t nw, int n_chunks,
                                                           const double* __restrict__ r, const TN* __restrict__ P,
                                                           ParamLayout pl, const TN* __restrict__ filt,
                                                           const TN* __restrict__ hval, const TN* __restrict__ kcoef,
                                                           const TN* __restrict__ ecoef, double* __restrict__ ftan,
                                                           double* __restrict__ jtan, TN* __restrict__ xsave,
                                                           bool) {
  constexpr bool bf16 = BF16;
  constexpr int T = C - 1, LC = T;
  // message sums: rows per item (RB), partners per step (JB, operands of a
  // step within 256 bytes per lane), chunk electrons per row (KK) and
  // own-row partners whose filter slopes are requested together (KO)
  constexpr int RB = C <= 4 ? 4 : (C <= 5 ? 3 : (C <= 8 ? 2 : 1));
  constexpr int JB0 = 256 / (int)(sizeof(TN) * (RB + C));
  constexpr int JBM = sizeof(TN) == 4 ? 3 : 1;
  constexpr int JB = JB0 < 1 ? 1 : (JB0 > JBM ? JBM : JB0);
  constexpr int KK = T % 3 == 0 ? T / 3 : T / 3 + 2;  // chunks start at multiples of T
  constexpr int KO = sizeof(TN) == 4 ? 8 : 4;
  // row blocks (and the pair-coefficient table) pay off without staged
  // tables and with narrow chunks (measured: 30-electron chunks of three
  // coordinates gain, chunks of ten coordinates of ten electrons lose)
  constexpr bool kRowBlocks = !STAGE && C <= 4;
  // chunks of three coordinates in the FP32 tile layout keep the h tangents
  // interleaved by column ([N][4 DZ + 4]; see HStore4)
  constexpr bool kH4 = kRowBlocks && C == 4 && sizeof(TN) == 4;
  // row blocks over chunks that touch one electron (T = 1 or 3) split the
  // chunk electron's own-row terms over partner groups of threads (partial
  // sums added in a fixed order) instead of leaving them to the one wave
  // that holds the row: up to 8 groups in FP32, 2 in FP64 (LDS)
  constexpr bool kSplitOwn = kRowBlocks && (T == 1 || T == 3);
  constexpr int kSplitG = sizeof(TN) == 4 ? 8 : 2;
  // the same chunks also move the chunk electron's terms in the other rows
  // (pairs (i, k), which only the row blocks of k's channel have) to a pass
  // over all threads after the same barrier
  constexpr bool kSplitK = kSplitOwn;
  extern __shared__ __align__(16) char smem[];
  // XCD-aware order: blocks b, b+8, ... run on one XCD; keep a walker's chunks there.
  const int64_t nb = (int64_t)gridDim.x;
  const int64_t b = blockIdx.x;
  int64_t task;
  {
    const int64_t per = nb / 8, rem = nb % 8;
    const int64_t xcd = b % 8, slot = b / 8;
    task = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + slot;
  }
  const int64_t w = task / n_chunks;
  const int chunk = (int)(task % n_chunks);
  if (w >= nw) return;
  const int N = d.N, DX = d.DX, DZ = d.DZ, M = d.M, NU = d.n_up;
  const int a0 = chunk * T;
  const int Tc = min(T, 3 * N - a0);   // coordinates present in this chunk
  const int R = N * C;                  // rows: (electron i, column)
  const int e_lo = a0 / 3, e_hi = (a0 + Tc - 1) / 3;
  const int NCE = e_hi - e_lo + 1;
  const int LDX = ld_pad<TN>(DX), LDZ = ld_pad<TN>(DZ), LDHZ = max(2 * LDZ, LDX);
  // interleaved h tangents: electron stride (16 bytes of padding spread the
  // four electrons of a tile over the banks) and column step
  const int SH4 = 4 * DZ + 4, HCS = kH4 ? 1 : LDZ;
  double* rs = reinterpret_cast<double*>(smem);                 // [N][3]
  int* pidx = reinterpret_cast<int*>(rs + 3 * kMaxElec);        // [N][N]
  TN* hvs = reinterpret_cast<TN*>(pidx + ((N * N + 3) & ~3));   // [N][DZ]
  TN* XT = hvs + N * DZ;                                        // [R][LDX]
  TN* HT = XT + R * LDX;                                        // [R][LDZ]  (layers)
  TN* ZT = HT + R * LDZ;                                        // [R][LDZ]  (layers)
  TN* KT = HT;                                                  // [R][LDX]  (backflow head)
  const int nce_max = chunk_elecs_max(N, T);                    // chunk electrons, at most
  TN* ES = HT + R * LDHZ;  // [2][C][LDX] Jastrow head; in the layers [NCE][C][LDZ] nuclear messages
  TN* ZN = ES;
  // [NCE][N][4] geometry, or [NCE][N][8] pair coefficients (row blocks, below)
  TN* cg = ES + max(2 * C * LDX, nce_max * C * LDZ);
  TN* cgn = cg + NCE * N * (kRowBlocks ? 8 : 4);                // [NCE][NN][4] r_k - R_I, 1/|r_k - R_I|
  const int NP = N + d.NN;                                      // partners of a chunk electron
  TN* wvs = cgn + NCE * d.NN * 4;                               // [n_ee][DZ]      (STAGE) w, all ee pairs
  TN* wds = wvs + (STAGE ? d.n_ee * DZ : 0);                    // [NCE][NP][DZ]   (STAGE) w'/d
  TN* w2s = wds + (STAGE ? NCE * NP * DZ : 0);                   // [NCE][NP][DZ]   (STAGE) w''
  int* prow = reinterpret_cast<int*>(wvs);  // (row blocks, never staged) [blocks][N][4] pair indices
  // (kSplitOwn) [groups][4][DZ] partial own-row sums of the partner groups
  TN* ownp = reinterpret_cast<TN*>(prow + ((NU + 3) / 4 + (N - NU + 3) / 4) * N * 4);
  const double* rw = r + w * N * 3;
  for (int q = threadIdx.x; q < 3 * N; q += blockDim.x) rs[q] = rw[q];
  for (int q = threadIdx.x; q < N * N; q += blockDim.x) pidx[q] = t.pair_index[q];
  {
    const uint4 z4 = {0u, 0u, 0u, 0u};
    uint4* x4 = reinterpret_cast<uint4*>(XT);
    for (int q = threadIdx.x; q < R * LDX * (int)sizeof(TN) / 16; q += blockDim.x) x4[q] = z4;
  }
  constexpr int V = 16 / sizeof(TN);  // elements per 16-byte unit
  __syncthreads();
  if constexpr (!kRowBlocks) {
    // [NCE][N][4]: r_i - r_k and 1/|r_i - r_k| for chunk electron k
    for (int q = threadIdx.x; q < NCE * N; q += blockDim.x) {
      const int k = e_lo + q / N, i = q % N;
      const double ux = rs[3 * i] - rs[3 * k], uy = rs[3 * i + 1] - rs[3 * k + 1], uz = rs[3 * i + 2] - rs[3 * k + 2];
      cg[4 * q + 0] = (TN)ux;
      cg[4 * q + 1] = (TN)uy;
      cg[4 * q + 2] = (TN)uz;
      cg[4 * q + 3] = i == k ? TN(0) : (TN)(1.0 / sqrt(ux * ux + uy * uy + uz * uz));
    }
  } else {
    // Pair coefficients of chunk electron k and electron j != k, with
    // u = r_k - r_j, rho = u / |u| and m_alpha = 1 for the chunk's columns of k
    // (a = 3k + alpha present in the chunk), else 0:
    //   g_alpha = m_alpha u_alpha,  A = sum m_alpha rho_alpha^2,  B = sum m_alpha (1 - rho_alpha^2)
    // so that d_a w_kj = (w'/d) g_alpha and sum_a d2_a w_kj = w'' A + (w'/d) B;
    // zero for j = k.
    for (int q = threadIdx.x; q < NCE * N; q += blockDim.x) {
      const int k = e_lo + q / N, j = q % N;
      const double u[3] = {rs[3 * k] - rs[3 * j], rs[3 * k + 1] - rs[3 * j + 1], rs[3 * k + 2] - rs[3 * j + 2]};
      const double inv = j == k ? 0.0 : 1.0 / sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      double A = 0, B = 0;
      for (int al = 0; al < 3; ++al) {
        const int col = 3 * k + al - a0;
        const bool m = j != k && col >= 0 && col < Tc;
        const double rho = u[al] * inv;
        cg[8 * q + al] = m ? (TN)u[al] : TN(0);
        if (m) {
          A += rho * rho;
          B += 1.0 - rho * rho;
        }
      }
      cg[8 * q + 3] = (TN)A;
      cg[8 * q + 4] = (TN)B;
      cg[8 * q + 5] = cg[8 * q + 6] = cg[8 * q + 7] = TN(0);
    }
    // Pair indices of each row block's RB = 4 rows with every electron j, one
    // 16-byte unit per (block, j): prow[(blk * N + j) * 4 + r].  Rows past
    // the block repeat its last row, and (row, row) reads pair 0; the sums
    // mask both.
    static_assert(RB == 4, "row blocks of four rows");
    const int nbu = (NU + RB - 1) / RB, nbd = (N - NU + RB - 1) / RB;
    for (int q = threadIdx.x; q < (nbu + nbd) * N * RB; q += blockDim.x) {
      const int r = q % RB, j = (q / RB) % N, blk = q / (RB * N);
      const bool upb = blk < nbu;
      const int i0 = upb ? blk * RB : NU + (blk - nbu) * RB;
      const int nr = min(RB, (upb ? NU : N) - i0);
      prow[q] = max(pidx[(i0 + min(r, nr - 1)) * N + j], 0);
    }
  }
  for (int q = threadIdx.x; q < NCE * d.NN; q += blockDim.x) {
    const int k = e_lo + q / d.NN, I = q % d.NN;
    const double ux = rs[3 * k] - t.nuc_xyz[3 * I], uy = rs[3 * k + 1] - t.nuc_xyz[3 * I + 1],
                 uz = rs[3 * k + 2] - t.nuc_xyz[3 * I + 2];
    cgn[4 * q + 0] = (TN)ux;
    cgn[4 * q + 1] = (TN)uy;
    cgn[4 * q + 2] = (TN)uz;
    cgn[4 * q + 3] = (TN)(1.0 / sqrt(ux * ux + uy * uy + uz * uz));
  }
  const int64_t fl_stride = (int64_t)3 * d.n_pairs * DZ;
  for (int n = 0; n < d.L; ++n) {
    const ParamLayout::Layer& Lp = pl.layer[n];
    const TN* fw = filt + w * fl_stride * d.L + n * fl_stride;
    const TN* fv = fw;                                 // w
    const TN* fd = fw + (int64_t)d.n_pairs * DZ;       // w'/d
    const TN* f2 = fw + (int64_t)2 * d.n_pairs * DZ;   // w''
    const TN* hv = hval + (w * d.L + n) * N * DZ;
    // the adjoint pass re-reads the layer inputs x^(n), n >= 1 (x^(0) has no tangents)
    if (xsave && n > 0) {
      TN* xs = xsave + (((size_t)w * n_chunks + chunk) * d.L + (n - 1)) * R * DX;
      for (int q = threadIdx.x; q < R * DX; q += blockDim.x) xs[q] = XT[(q / DX) * LDX + q % DX];
    }
    // Staging of the layer's tables: h values, then (STAGE) the filter values
    // of all electron pairs and the rows (chunk electron k, partner) of w'/d
    // and w''.  Global-to-LDS loads (16 bytes per lane, no registers): all of
    // them are in flight together, and the h product below proceeds while
    // they land; the barrier after it waits for them.
    {
      const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6, nwv = (int)blockDim.x >> 6;
      dma16(reinterpret_cast<uint4*>(hvs), reinterpret_cast<const uint4*>(hv), N * DZ / V, lane, wv, nwv);
      if constexpr (STAGE) {
        dma16(reinterpret_cast<uint4*>(wvs), reinterpret_cast<const uint4*>(fv), d.n_ee * DZ / V, lane, wv, nwv);
        const int U16 = DZ / V, nD = NCE * NP * U16;
        const uint4 z4 = {0u, 0u, 0u, 0u};
        for (int b = wv * 64; b < nD; b += nwv * 64) {
          const int q = b + lane;
          int64_t p = -1;
          if (q < nD) {
            const int row = q / U16, k = e_lo + row / NP, part = row % NP;
            p = part < N ? (part == k ? -1 : pidx[k * N + part]) : d.n_ee + k * d.NN + (part - N);
          }
          if (p >= 0) {
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const uint4*>(fd + p * DZ) + q % U16,
                                             reinterpret_cast<uint4*>(wds) + b, 16, 0, 0);
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const uint4*>(f2 + p * DZ) + q % U16,
                                             reinterpret_cast<uint4*>(w2s) + b, 16, 0, 0);
          } else if (q < nD) {  // a chunk electron paired with itself: zeros
            reinterpret_cast<uint4*>(wds)[q] = z4;
            reinterpret_cast<uint4*>(w2s)[q] = z4;
          }
        }
      }
      if (n > 0) {
        if constexpr (kH4)
          gemm_mfma<TN, true, HStore4>(XT, LDX, R, DX, P + Lp.hW, DZ, HT, LDZ, false, bf16,
                                       HStore4{reinterpret_cast<float*>(HT), N, SH4});
        else
          gemm_mfma<TN, true>(XT, LDX, R, DX, P + Lp.hW, DZ, HT, LDZ, false, bf16);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);  // this wave's loads to LDS have landed
    __syncthreads();
    for (int ch = 0; ch < 2; ++ch) {
      if constexpr (!kRowBlocks) {
        // One item per (row, feature z), two partners per step.
        // channel 0 also takes the nuclear messages, which only rows of the
        // chunk's own electrons have (extra items; their product joins
        // channel 0's)
        const int n_items = N * DZ + (ch == 0 ? NCE * DZ : 0);
        for (int q = threadIdx.x; q < n_items; q += blockDim.x) {
          if (q >= N * DZ) {
            const int i = e_lo + (q - N * DZ) / DZ, z = q % DZ;
            TN* zn = ZN + (size_t)(i - e_lo) * C * LDZ + z;
            TN acc[C];
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c] = 0;
            const int c0 = 3 * i - a0;
            for (int I = 0; I < d.NN; ++I) {
              const TN* gn = cgn + ((size_t)(i - e_lo) * d.NN + I) * 4;
              const TN y = P[pl.Y + I * DZ + z];
              TN wd, w2;
              if constexpr (STAGE) {
                wd = wds[((i - e_lo) * NP + N + I) * DZ + z];
                w2 = w2s[((i - e_lo) * NP + N + I) * DZ + z];
              } else {
                const int64_t p = d.n_ee + i * d.NN + I;
                wd = fd[p * DZ + z];
                w2 = f2[p * DZ + z];
              }
#pragma unroll
              for (int c = 0; c < T; ++c) {
                const int al = c - c0;
                if (al < 0 || al > 2 || c >= Tc) continue;
                const TN ua = gn[al];
                const TN ur = ua * gn[3];
                acc[c] += wd * ua * y;
                acc[LC] += (w2 * ur * ur + wd * (TN(1) - ur * ur)) * y;
              }
            }
#pragma unroll
            for (int c = 0; c < C; ++c) zn[c * LDZ] = acc[c];
            continue;
          }
          const int i = q / DZ, z = q % DZ;
          const bool up_i = i < NU;
          // electrons of this channel: same spin (ch 0) or opposite spin (ch 1)
          const bool want_up = (ch == 0) == up_i;
          const int j_lo = want_up ? 0 : NU, j_hi = want_up ? NU : N;
          TN acc[C];
#pragma unroll
          for (int c = 0; c < C; ++c) acc[c] = 0;
          if (n > 0) {
            // Two partners per step; j = i contributes w = 0 (no branch).  All
            // of a step's LDS reads are issued before its first product (the
            // scheduling barriers keep the compiler from interleaving read,
            // wait, multiply per column, which would expose one LDS latency
            // per column).
            // (wide FP64 chunks take one partner per step: fewer live registers)
            constexpr bool kTwo = C * sizeof(TN) <= 48;
            int j = j_lo;
            for (; kTwo && j + 1 < j_hi; j += 2) {
              const int pa = max(pidx[i * N + j], 0), pb = max(pidx[i * N + j + 1], 0);
              const TN* hja = HT + j * C * LDZ + z;
              const TN* hjb = hja + C * LDZ;
              TN ha[C], hb[C];
#pragma unroll
              for (int c = 0; c < C; ++c) ha[c] = hja[c * LDZ];
#pragma unroll
              for (int c = 0; c < C; ++c) hb[c] = hjb[c * LDZ];
              const TN wa0 = STAGE ? wvs[pa * DZ + z] : fv[(int64_t)pa * DZ + z];
              const TN wb0 = STAGE ? wvs[pb * DZ + z] : fv[(int64_t)pb * DZ + z];
              __builtin_amdgcn_sched_barrier(0);
              const TN wa = j == i ? TN(0) : wa0, wb = j + 1 == i ? TN(0) : wb0;
#pragma unroll
              for (int c = 0; c < C; ++c) acc[c] += wa * ha[c];
#pragma unroll
              for (int c = 0; c < C; ++c) acc[c] += wb * hb[c];
              __builtin_amdgcn_sched_barrier(0);
            }
            for (; j < j_hi; ++j) {
              const int pa = max(pidx[i * N + j], 0);
              const TN* hja = HT + j * C * LDZ + z;
              TN ha[C];
#pragma unroll
              for (int c = 0; c < C; ++c) ha[c] = hja[c * LDZ];
              const TN wa0 = STAGE ? wvs[pa * DZ + z] : fv[(int64_t)pa * DZ + z];
              __builtin_amdgcn_sched_barrier(0);
              const TN wa = j == i ? TN(0) : wa0;
#pragma unroll
              for (int c = 0; c < C; ++c) acc[c] += wa * ha[c];
            }
          }
          TN* zi = ZT + (size_t)i * C * LDZ + z;
          TN lap = acc[LC];
          // sources from the coordinates of electron i itself
          if (i >= e_lo && i <= e_hi) {
            const TN* gi = cg + (size_t)(i - e_lo) * N * 4;  // r_j - r_i
            const int c0 = 3 * i - a0;
            // the chunk's columns of electron i: masks instead of branches, and
            // clamped column indices for the (masked) reads
            const TN m0 = (c0 >= 0 && c0 < Tc) ? TN(1) : TN(0);
            const TN m1 = (c0 + 1 >= 0 && c0 + 1 < Tc) ? TN(1) : TN(0);
            const TN m2 = (c0 + 2 >= 0 && c0 + 2 < Tc) ? TN(1) : TN(0);
            const int k0 = min(max(c0, 0), LC), k1 = min(max(c0 + 1, 0), LC), k2 = min(max(c0 + 2, 0), LC);
            TN sv0 = 0, sv1 = 0, sv2 = 0;
            // j = i adds nothing: its staged w'/d, w'' and 1/|r_i - r_j| are zero.
            // A partner's reads are issued together (FP32: two partners per step).
            struct Own {
              TN wd, w2, hj, g0, g1, g2, inv, h0, h1, h2;
            };
            auto load_own = [&](int j) {
              Own o;
              if constexpr (STAGE) {
                o.wd = wds[((i - e_lo) * NP + j) * DZ + z];
                o.w2 = w2s[((i - e_lo) * NP + j) * DZ + z];
              } else {
                const int64_t p = max(pidx[i * N + j], 0);
                o.wd = j == i ? TN(0) : fd[p * DZ + z];
                o.w2 = j == i ? TN(0) : f2[p * DZ + z];
              }
              o.hj = hvs[j * DZ + z];
              o.g0 = gi[4 * j];
              o.g1 = gi[4 * j + 1];
              o.g2 = gi[4 * j + 2];
              o.inv = gi[4 * j + 3];
              const TN* hjc = HT + j * C * LDZ + z;
              o.h0 = n > 0 ? hjc[k0 * LDZ] : TN(0);
              o.h1 = n > 0 ? hjc[k1 * LDZ] : TN(0);
              o.h2 = n > 0 ? hjc[k2 * LDZ] : TN(0);
              return o;
            };
            auto use_own = [&](const Own& o) {
              const TN u0 = -o.g0, u1 = -o.g1, u2 = -o.g2;  // (r_i - r_j)_alpha
              const TN r0 = u0 * o.inv, r1 = u1 * o.inv, r2 = u2 * o.inv;
              const TN d0 = m0 * o.wd * u0, d1 = m1 * o.wd * u1, d2 = m2 * o.wd * u2;
              sv0 += d0 * o.hj;
              sv1 += d1 * o.hj;
              sv2 += d2 * o.hj;
              lap += (m0 * (o.w2 * r0 * r0 + o.wd * (TN(1) - r0 * r0)) + m1 * (o.w2 * r1 * r1 + o.wd * (TN(1) - r1 * r1)) +
                      m2 * (o.w2 * r2 * r2 + o.wd * (TN(1) - r2 * r2))) * o.hj;
              lap += TN(2) * (d0 * o.h0 + d1 * o.h1 + d2 * o.h2);  // h tangents are zero at n = 0
            };
            int j = j_lo;
            for (; sizeof(TN) == 4 && j + 1 < j_hi; j += 2) {
              const Own oa = load_own(j), ob = load_own(j + 1);
              __builtin_amdgcn_sched_barrier(0);
              use_own(oa);
              use_own(ob);
              __builtin_amdgcn_sched_barrier(0);
            }
            for (; j < j_hi; ++j) {
              const Own oa = load_own(j);
              __builtin_amdgcn_sched_barrier(0);
              use_own(oa);
              __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
              const int al = c - c0;
              if (al == 0) acc[c] += sv0;
              if (al == 1) acc[c] += sv1;
              if (al == 2) acc[c] += sv2;
            }
          }
#pragma unroll
          for (int c = 0; c < LC; ++c) zi[c * LDZ] = acc[c];
          // sources from the coordinates of the chunk's other electrons k (read,
          // update, write the item's own Z entries; masked columns are left alone)
          for (int k = max(e_lo, j_lo); k <= min(e_hi, j_hi - 1); ++k) {
            if (k == i) continue;
            const TN* gk = cg + ((size_t)(k - e_lo) * N + i) * 4;  // r_i - r_k
            TN wd, w2;
            if constexpr (STAGE) {
              wd = wds[((k - e_lo) * NP + i) * DZ + z];
              w2 = w2s[((k - e_lo) * NP + i) * DZ + z];
            } else {
              const int64_t p = pidx[i * N + k];
              wd = fd[p * DZ + z];
              w2 = f2[p * DZ + z];
            }
            const TN hk = hvs[k * DZ + z];
            const TN* hkc = HT + (size_t)k * C * LDZ + z;
            const int cb = 3 * k - a0;
            int cc[3];
            TN ua[3], hc[3], zv[3];
            bool ok[3];
#pragma unroll
            for (int al = 0; al < 3; ++al) {
              ok[al] = cb + al >= 0 && cb + al < Tc;
              cc[al] = min(max(cb + al, 0), LC);
              ua[al] = gk[al];
              hc[al] = n > 0 ? hkc[cc[al] * LDZ] : TN(0);
              zv[al] = zi[cc[al] * LDZ];
            }
            const TN inv = gk[3];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int al = 0; al < 3; ++al) {
              const TN ur = ua[al] * inv;
              const TN dw = -wd * ua[al];  // d/dr_k of w(|r_i - r_k|)
              const TN m = ok[al] ? TN(1) : TN(0);
              lap += m * ((w2 * ur * ur + wd * (TN(1) - ur * ur)) * hk + TN(2) * dw * hc[al]);
              if (ok[al]) zi[cc[al] * LDZ] = zv[al] + dw * hk;
            }
          }
          zi[LC * LDZ] = lap;
        }
      } else {
        // Row blocks share each partner's global reads (below).
        // Items of a channel: (row block, feature z) for the pair sums, then
        // (channel 0) (chunk electron, z) for the nuclear messages, which only
        // rows of the chunk's own electrons have (their product joins channel
        // 0's).  A row block is RB consecutive rows of one spin; its item
        // reads each partner's h tangents once for all its rows.
        const int nbu = (NU + RB - 1) / RB, nbd = (N - NU + RB - 1) / RB;
        const int n_bulk = (nbu + nbd) * DZ;
        const int n_items = n_bulk + (ch == 0 ? NCE * DZ : 0);
        for (int q = threadIdx.x; q < n_items; q += blockDim.x) {
          if (q >= n_bulk) {
            const int i = e_lo + (q - n_bulk) / DZ, z = q % DZ;
            TN* zn = ZN + (i - e_lo) * C * LDZ + z;
            TN acc[C];
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c] = 0;
            const int c0 = 3 * i - a0;
            for (int I = 0; I < d.NN; ++I) {
              const TN* gn = cgn + ((i - e_lo) * d.NN + I) * 4;
              const TN y = P[pl.Y + I * DZ + z];
              TN wd, w2;
              if constexpr (STAGE) {
                wd = wds[((i - e_lo) * NP + N + I) * DZ + z];
                w2 = w2s[((i - e_lo) * NP + N + I) * DZ + z];
              } else {
                const int p = d.n_ee + i * d.NN + I;
                wd = fd[p * DZ + z];
                w2 = f2[p * DZ + z];
              }
#pragma unroll
              for (int c = 0; c < T; ++c) {
                const int al = c - c0;
                if (al < 0 || al > 2 || c >= Tc) continue;
                const TN ua = gn[al];
                const TN ur = ua * gn[3];
                acc[c] += wd * ua * y;
                acc[LC] += (w2 * ur * ur + wd * (TN(1) - ur * ur)) * y;
              }
            }
#pragma unroll
            for (int c = 0; c < C; ++c) zn[c * LDZ] = acc[c];
            continue;
          }
          // ---- pair sums of row block blk at feature z ----
          const int blk = q / DZ, z = q % DZ;
          const bool upb = blk < nbu;
          const int i0 = upb ? blk * RB : NU + (blk - nbu) * RB;
          const int nr = min(RB, (upb ? NU : N) - i0);
          // electrons of this channel: same spin (ch 0) or opposite spin (ch 1)
          const bool want_up = (ch == 0) == upb;
          const int j_lo = want_up ? 0 : NU, j_hi = want_up ? NU : N;
          // chunk electrons among the partners (their coordinates move w_ik)
          const int kk_lo = max(e_lo, j_lo), kk_hi = min(e_hi, j_hi - 1), nk = kk_hi - kk_lo + 1;
          TN acc[RB][C];
#pragma unroll
          for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < C; ++c) acc[r][c] = 0;
          // w'/d and w'' of the pairs (row, chunk electron k): requested first,
          // so their latency overlaps the sums (rows past nr and pairs with
          // k = i read clamped, valid entries that are never used)
          TN kwd[RB][KK], kw2[RB][KK];
          if (!kSplitK && nk > 0) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
              const int ir = i0 + min(r, nr - 1);
#pragma unroll
              for (int u = 0; u < KK; ++u) {
                const int k = kk_lo + min(u, nk - 1);
                if constexpr (STAGE) {
                  kwd[r][u] = wds[((k - e_lo) * NP + ir) * DZ + z];
                  kw2[r][u] = w2s[((k - e_lo) * NP + ir) * DZ + z];
                } else {
                  const int o = max(pidx[ir * N + k], 0) * DZ + z;
                  kwd[r][u] = fd[o];
                  kw2[r][u] = f2[o];
                }
              }
            }
          }
          // sum_j w_ij h_{j,c}: JB partners per step, their w for all RB rows
          // and their h tangents requested together, and the next step's
          // requested before this step's products; each h read serves RB rows
          if (n > 0) {
            auto fetch = [&](int j, TN (&wv)[JB][RB], TN (&hh)[JB][C]) {
#pragma unroll
              for (int jj = 0; jj < JB; ++jj) {
                const int jc = min(j + jj, j_hi - 1);
                if constexpr (kH4) {
                  const float4 h4 = *reinterpret_cast<const float4*>(HT + jc * SH4 + 4 * z);
                  hh[jj][0] = h4.x;
                  hh[jj][1] = h4.y;
                  hh[jj][2] = h4.z;
                  hh[jj][3] = h4.w;
                } else {
                  const TN* hj = HT + jc * C * LDZ + z;
#pragma unroll
                  for (int c = 0; c < C; ++c) hh[jj][c] = hj[c * LDZ];
                }
                const int4 p4 = *reinterpret_cast<const int4*>(prow + (blk * N + jc) * RB);
                const int po[4] = {p4.x, p4.y, p4.z, p4.w};
#pragma unroll
                for (int r = 0; r < RB; ++r) wv[jj][r] = fv[po[r] * DZ + z];
              }
            };
            auto sum = [&](int j, const TN (&wv)[JB][RB], const TN (&hh)[JB][C]) {
#pragma unroll
              for (int jj = 0; jj < JB; ++jj) {
                if (j + jj >= j_hi) break;  // wave-uniform
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                  const TN wr = j + jj == i0 + r ? TN(0) : wv[jj][r];  // w_ii = 0
#pragma unroll
                  for (int c = 0; c < C; ++c) acc[r][c] += wr * hh[jj][c];
                }
              }
            };
            TN wa[JB][RB], ha[JB][C], wb[JB][RB], hb[JB][C];
            if (j_lo < j_hi) fetch(j_lo, wa, ha);
            for (int j = j_lo; j < j_hi; j += 2 * JB) {
              if (j + JB < j_hi) fetch(j + JB, wb, hb);
              sum(j, wa, ha);
              if (j + JB >= j_hi) break;
              if (j + 2 * JB < j_hi) fetch(j + 2 * JB, wa, ha);
              sum(j + JB, wb, hb);
            }
          }
          // sources from the coordinates of chunk electron k != i: d_a w_ik for
          // the columns a of k, and their part of the Laplacian column (pair
          // coefficients g, A, B of (k, i) from the chunk's table)
          if (!kSplitK && nk > 0) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
              const int i = i0 + min(r, nr - 1);
#pragma unroll
              for (int u = 0; u < KK; ++u) {
                const int k = kk_lo + u;
                if (u >= nk) break;  // wave-uniform
                if (k == i) continue;
                const TN* gk = cg + ((k - e_lo) * N + i) * 8;
                const TN g0 = gk[0], g1 = gk[1], g2 = gk[2], A = gk[3], B = gk[4];
                const TN hk = hvs[k * DZ + z];
                const TN* hkc = kH4 ? HT + k * SH4 + 4 * z : HT + k * C * LDZ + z;
                const int cb = 3 * k - a0;
                const TN wd = kwd[r][u], w2 = kw2[r][u];
                TN hsum = 0;
                if (n > 0)
                  hsum = g0 * hkc[min(max(cb, 0), LC) * HCS] + g1 * hkc[min(max(cb + 1, 0), LC) * HCS] +
                         g2 * hkc[min(max(cb + 2, 0), LC) * HCS];
                acc[r][LC] += (w2 * A + wd * B) * hk + TN(2) * wd * hsum;
                const TN t = wd * hk;
#pragma unroll
                for (int c = 0; c < LC; ++c) {
                  const int al = c - cb;
                  if (al >= 0 && al <= 2 && c < Tc) acc[r][c] += (al == 0 ? g0 : (al == 1 ? g1 : g2)) * t;
                }
              }
            }
          }
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            if (r >= nr) break;
            TN* zi = ZT + (i0 + r) * C * LDZ + z;
#pragma unroll
            for (int c = 0; c < C; ++c) zi[c * LDZ] = acc[r][c];
          }
          // sources from the coordinates of electron i itself (rows of chunk
          // electrons only): added to the stored row
          for (int r = 0; r < nr; ++r) {
            if constexpr (kSplitOwn) break;  // below, over all waves
            const int i = i0 + r;
            if (i < e_lo || i > e_hi) continue;
            TN* zi = ZT + i * C * LDZ + z;
            TN lap = zi[LC * LDZ];
            const TN* gi = cg + (i - e_lo) * N * 8;  // coefficients of the pairs (i, j)
            const int c0 = 3 * i - a0;
            // clamped column indices for the reads (masked columns have g = 0)
            const int k0 = min(max(c0, 0), LC), k1 = min(max(c0 + 1, 0), LC), k2 = min(max(c0 + 2, 0), LC);
            TN sv0 = 0, sv1 = 0, sv2 = 0;
            // partner j != i: d_a w_ij = (w'/d) g_a, and its Laplacian terms
            auto own = [&](int j, TN wd, TN w2) {
              const TN* gj = gi + 8 * j;
              const TN g0 = gj[0], g1 = gj[1], g2 = gj[2], A = gj[3], B = gj[4];
              const TN hj = hvs[j * DZ + z];
              TN hsum = 0;
              if (n > 0) {
                const TN* hjc = kH4 ? HT + j * SH4 + 4 * z : HT + j * C * LDZ + z;
                hsum = g0 * hjc[k0 * HCS] + g1 * hjc[k1 * HCS] + g2 * hjc[k2 * HCS];
              }
              const TN t = wd * hj;
              sv0 += g0 * t;
              sv1 += g1 * t;
              sv2 += g2 * t;
              lap += (w2 * A + wd * B) * hj + TN(2) * wd * hsum;
            };
            const int np = j_hi - j_lo;
            if constexpr (STAGE) {
              for (int j = j_lo; j < j_hi; ++j)
                if (j != i) own(j, wds[((i - e_lo) * NP + j) * DZ + z], w2s[((i - e_lo) * NP + j) * DZ + z]);
            } else {
              // w'/d and w'' of the first KO partners requested together
              TN owd[KO], ow2[KO];
#pragma unroll
              for (int u = 0; u < KO; ++u) {
                const int o = max(pidx[i * N + j_lo + min(u, np - 1)], 0) * DZ + z;
                owd[u] = fd[o];
                ow2[u] = f2[o];
              }
#pragma unroll
              for (int u = 0; u < KO; ++u) {
                if (u >= np) break;  // wave-uniform
                if (j_lo + u != i) own(j_lo + u, owd[u], ow2[u]);
              }
              for (int j = j_lo + KO; j < j_hi; ++j) {
                if (j == i) continue;
                const int o = pidx[i * N + j] * DZ + z;
                own(j, fd[o], f2[o]);
              }
            }
#pragma unroll
            for (int c = 0; c < LC; ++c) {
              const int al = c - c0;
              if (al == 0) zi[c * LDZ] += sv0;
              if (al == 1) zi[c * LDZ] += sv1;
              if (al == 2) zi[c * LDZ] += sv2;
            }
            zi[LC * LDZ] = lap;
          }
        }
        if constexpr (kSplitOwn) {
          // The chunk electron i (the one electron of the chunk): thread
          // (group g, feature z) takes the partners j_lo + g, j_lo + g + G, ...
          // of i's channel and leaves its partial sums of d_a w_ij h_j (the
          // columns of i in the chunk) and of the Laplacian terms in ownp;
          // after the barrier the first DZ threads add the G partials, in
          // group order, to the row the item pass stored.
          const int i = e_lo;
          const int G = min((int)blockDim.x / DZ, kSplitG), g = (int)threadIdx.x / DZ, z = (int)threadIdx.x % DZ;
          const bool want_up = (ch == 0) == (i < NU);
          const int j_lo = want_up ? 0 : NU, j_hi = want_up ? NU : N;
          const TN* gi = cg;  // coefficients of the pairs (i, j)
          const int c0 = 3 * i - a0;
          const int k0 = min(max(c0, 0), LC), k1 = min(max(c0 + 1, 0), LC), k2 = min(max(c0 + 2, 0), LC);
          // (kSplitK) rows whose partners in this channel include i: thread
          // group gk takes rows kr_lo + gk, kr_lo + gk + GR, ... (the rotation
          // leaves group 0, which also adds the partials, one row fewer); the
          // slopes of its first two rows are requested now, ahead of the
          // partner pass and the barrier
          const bool krows_up = (ch == 0) == (i < NU);
          const int kr_lo = krows_up ? 0 : NU, kr_hi = krows_up ? NU : N;
          const int GR = (int)blockDim.x / DZ, gk = (g + GR - 1) % GR;
          TN kwdp[2], kw2p[2];
          if constexpr (kSplitK) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              const int ic = min(kr_lo + gk + u * GR, kr_hi - 1);
              const int o = max(pidx[ic * N + i], 0) * DZ + z;
              kwdp[u] = fd[o];
              kw2p[u] = f2[o];
            }
          }
          TN sv0 = 0, sv1 = 0, sv2 = 0, lap = 0;
          for (int j = j_lo + g; g < G && j < j_hi; j += G) {
            if (j == i) continue;
            const int o = pidx[i * N + j] * DZ + z;
            const TN wd = fd[o], w2 = f2[o];
            const TN* gj = gi + 8 * j;
            const TN g0 = gj[0], g1 = gj[1], g2 = gj[2], A = gj[3], B = gj[4];
            const TN hj = hvs[j * DZ + z];
            TN hsum = 0;
            if (n > 0) {
              const TN* hjc = kH4 ? HT + j * SH4 + 4 * z : HT + j * C * LDZ + z;
              hsum = g0 * hjc[k0 * HCS] + g1 * hjc[k1 * HCS] + g2 * hjc[k2 * HCS];
            }
            const TN t = wd * hj;
            sv0 += g0 * t;
            sv1 += g1 * t;
            sv2 += g2 * t;
            lap += (w2 * A + wd * B) * hj + TN(2) * wd * hsum;
          }
          if (g < G) {
            TN* pg = ownp + g * 4 * DZ + z;
            pg[0] = sv0;
            pg[DZ] = sv1;
            pg[2 * DZ] = sv2;
            pg[3 * DZ] = lap;
          }
          __syncthreads();
          if (g == 0) {
            TN s0 = 0, s1 = 0, s2 = 0, sl = 0;
            for (int q = 0; q < G; ++q) {
              const TN* pq = ownp + q * 4 * DZ + z;
              s0 += pq[0];
              s1 += pq[DZ];
              s2 += pq[2 * DZ];
              sl += pq[3 * DZ];
            }
            TN* zi = ZT + i * C * LDZ + z;
#pragma unroll
            for (int c = 0; c < LC; ++c) {
              const int al = c - c0;
              if (al == 0) zi[c * LDZ] += s0;
              if (al == 1) zi[c * LDZ] += s1;
              if (al == 2) zi[c * LDZ] += s2;
            }
            zi[LC * LDZ] += sl;
          }
          if constexpr (kSplitK) {
            // terms of the pairs (r, i) in the rows r != i stored by the item
            // pass: d_a w_ri for the columns of i, and their part of the
            // Laplacian column (coefficients g, A, B of (i, r))
            const TN hk = hvs[i * DZ + z];
            const TN* hkc = kH4 ? HT + i * SH4 + 4 * z : HT + i * C * LDZ + z;
            auto kterm = [&](int r, TN wd, TN w2) {
              const TN* gk8 = cg + r * 8;
              const TN g0 = gk8[0], g1 = gk8[1], g2 = gk8[2], A = gk8[3], B = gk8[4];
              TN hsum = 0;
              if (n > 0) hsum = g0 * hkc[k0 * HCS] + g1 * hkc[k1 * HCS] + g2 * hkc[k2 * HCS];
              TN* zr = ZT + r * C * LDZ + z;
              zr[LC * LDZ] += (w2 * A + wd * B) * hk + TN(2) * wd * hsum;
              const TN t = wd * hk;
#pragma unroll
              for (int c = 0; c < LC; ++c) {
                const int al = c - c0;
                if (al >= 0 && al <= 2 && c < Tc) zr[c * LDZ] += (al == 0 ? g0 : (al == 1 ? g1 : g2)) * t;
              }
            };
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              const int r = kr_lo + gk + u * GR;
              if (r < kr_hi && r != i) kterm(r, kwdp[u], kw2p[u]);
            }
            for (int r = kr_lo + gk + 2 * GR; r < kr_hi; r += GR) {
              if (r == i) continue;
              const int o = pidx[r * N + i] * DZ + z;
              kterm(r, fd[o], f2[o]);
            }
          }
        }
      }
      __syncthreads();
      // channel 0 with the nuclear rows in one pass over the tiles, both weight
      // slabs read up front (FP32 only: FP64 and BF16 spill with it)
      if (sizeof(TN) == 4 && !BF16 && ch == 0) {
        gemm_mfma_dual<TN, true>(ZT, LDZ, R, DZ, P + Lp.gW[0], DX, XT, LDX, ZN, LDZ, e_lo * C, NCE * C,
                                 P + Lp.gW[2], bf16);
      } else {
        gemm_mfma<TN, true>(ZT, LDZ, R, DZ, P + Lp.gW[ch], DX, XT, LDX, true, bf16);
        if (ch == 0) gemm_mfma_window<TN>(ZN, LDZ, R, e_lo * C, NCE * C, DZ, P + Lp.gW[2], DX, XT, LDX, bf16);
      }
      __syncthreads();
    }
  }
  if (xsave) {
    TN* xs = xsave + (((size_t)w * n_chunks + chunk) * d.L + (d.L - 1)) * R * DX;
    for (int q = threadIdx.x; q < R * DX; q += blockDim.x) xs[q] = XT[(q / DX) * LDX + q % DX];
  }
  // The heads' activation slopes (kappa [2][2][N][DX], then eta [2][2][DX])
  // go to the staging region, which the layers no longer need; the copy is
  // issued before the Jastrow sum so its latency overlaps that work.
  // chunks of three coordinates in FP32 layout apply the head activations in
  // the products' epilogues (slopes read from global memory, no staging)
  constexpr bool kFuse = C == 4 && sizeof(TN) == 4;
  const bool hstage = !kFuse && STAGE && d.n_ee * DZ + 2 * nce_max * NP * DZ >= 4 * N * DX + 4 * DX;
  if (hstage) {
    const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6, nwv = (int)blockDim.x >> 6;
    dma16(reinterpret_cast<uint4*>(wvs), reinterpret_cast<const uint4*>(kcoef + w * 4 * N * DX), 4 * N * DX / V, lane,
          wv, nwv);
    dma16(reinterpret_cast<uint4*>(wvs + 4 * N * DX), reinterpret_cast<const uint4*>(ecoef + w * 4 * DX), 4 * DX / V,
          lane, wv, nwv);
  }
  // ---- heads: Jastrow on sum_i x_i (rows = columns), backflow per row ----
  // The two heads are independent chains of products and activations; they
  // advance together, one step of each between barriers.  Without the
  // Jastrow factor J = 0, without the backflow f = 1 (no tangents).
  const bool do_j = !(d.flags & PN_NET_NO_JASTROW), do_k = !(d.flags & PN_NET_NO_BACKFLOW);
  double* jt = jtan + ((int64_t)w * n_chunks + chunk) * C;
  double* ft = ftan + ((int64_t)w * n_chunks + chunk) * N * C * M;
  TN* S0 = ES;             // [C][LDX]
  TN* S1 = ES + C * LDX;   // [C][LDX]
  // Jastrow activation in place: s1 v per column, s1 v_L + s2 sum_a v_a^2
  auto act_j = [&](TN* S, int lay) {
    const TN* ec = hstage ? wvs + 4 * N * DX + lay * 2 * DX : ecoef + (w * 2 + lay) * 2 * DX;
    for (int x = threadIdx.x; x < DX; x += blockDim.x) {
      const TN s1 = ec[x], s2 = ec[DX + x];
      TN v[LC];
#pragma unroll
      for (int col = 0; col < LC; ++col) v[col] = S[col * LDX + x];
      const TN vl = S[LC * LDX + x];
      TN sq = 0;
#pragma unroll
      for (int col = 0; col < LC; ++col) {
        sq += v[col] * v[col];
        S[col * LDX + x] = s1 * v[col];
      }
      S[LC * LDX + x] = s1 * vl + s2 * sq;
    }
  };
  // backflow activation in place, rows (i, column)
  auto act_k = [&](TN* A, int lay) {
    const TN* kc = hstage ? wvs + lay * 2 * N * DX : kcoef + (w * 2 + lay) * 2 * N * DX;
    for (int q = threadIdx.x; q < N * DX; q += blockDim.x) {
      const int i = q / DX, x = q % DX;
      const TN s1 = kc[i * DX + x], s2 = kc[N * DX + i * DX + x];
      TN* ai = A + i * C * LDX + x;
      TN v[LC];
#pragma unroll
      for (int col = 0; col < LC; ++col) v[col] = ai[col * LDX];
      const TN vl = ai[LC * LDX];
      TN sq = 0;
#pragma unroll
      for (int col = 0; col < LC; ++col) {
        sq += v[col] * v[col];
        ai[col * LDX] = s1 * v[col];
      }
      ai[LC * LDX] = s1 * vl + s2 * sq;
    }
  };
  if (do_j) {
    for (int q = threadIdx.x; q < C * DX; q += blockDim.x) {
      const int col = q / DX, x = q % DX;
      const TN* xc = XT + col * LDX + x;
      TN s = 0;
      int i = 0;
      for (; i + 3 < N; i += 4) {  // four reads in flight
        const TN a = xc[i * C * LDX], b = xc[(i + 1) * C * LDX];
        const TN e = xc[(i + 2) * C * LDX], f = xc[(i + 3) * C * LDX];
        __builtin_amdgcn_sched_barrier(0);
        s += a + b + e + f;
      }
      for (; i < N; ++i) s += xc[i * C * LDX];
      S0[col * LDX + x] = s;
    }
  } else {
    for (int col = threadIdx.x; col < C; col += blockDim.x) jt[col] = 0.0;
  }
  if constexpr (kFuse) {
    const HeadAct<TN> k0{kcoef + (w * 2 + 0) * 2 * N * DX, N, DX, true}, k1{kcoef + (w * 2 + 1) * 2 * N * DX, N, DX, true};
    const HeadAct<TN> j0{ecoef + (w * 2 + 0) * 2 * DX, 1, DX, false}, j1{ecoef + (w * 2 + 1) * 2 * DX, 1, DX, false};
    if (do_k)
      gemm_mfma<TN, true>(XT, LDX, R, DX, P + pl.kW1, DX, KT, LDX, false, bf16, k0);
    else
      for (int q = threadIdx.x; q < R * M; q += blockDim.x) ft[q] = 0.0;
    __syncthreads();
    if (do_j) gemm_mfma<TN, true>(S0, LDX, C, DX, P + pl.eW1, DX, S1, LDX, false, bf16, j0);
    if (do_k) gemm_mfma<TN, true>(KT, LDX, R, DX, P + pl.kW2, DX, XT, LDX, false, bf16, k1);
    __syncthreads();
    if (do_j) gemm_mfma<TN, true>(S1, LDX, C, DX, P + pl.eW2, DX, S0, LDX, false, bf16, j1);
    if (do_k) gemm_mfma_cols<TN>(XT, LDX, R, DX, P + pl.kW3, M, KT, LDX, false, bf16);
    __syncthreads();
  } else {
    if (do_k)
      gemm_mfma<TN, true>(XT, LDX, R, DX, P + pl.kW1, DX, KT, LDX, false, bf16);
    else
      for (int q = threadIdx.x; q < R * M; q += blockDim.x) ft[q] = 0.0;
    __builtin_amdgcn_s_waitcnt(0);  // the staged activation slopes have landed
    __syncthreads();
    if (do_j) gemm_mfma<TN, true>(S0, LDX, C, DX, P + pl.eW1, DX, S1, LDX, false, bf16);
    if (do_k) act_k(KT, 0);
    __syncthreads();
    if (do_j) act_j(S1, 0);
    if (do_k) gemm_mfma<TN, true>(KT, LDX, R, DX, P + pl.kW2, DX, XT, LDX, false, bf16);
    __syncthreads();
    if (do_j) gemm_mfma<TN, true>(S1, LDX, C, DX, P + pl.eW2, DX, S0, LDX, false, bf16);
    if (do_k) act_k(XT, 1);
    __syncthreads();
    if (do_j) act_j(S0, 1);
    if (do_k) gemm_mfma_cols<TN>(XT, LDX, R, DX, P + pl.kW3, M, KT, LDX, false, bf16);
    __syncthreads();
  }
  if (do_j) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int col = wv; col < C; col += (int)(blockDim.x >> 6)) {
      TN acc = 0;
      for (int x = lane; x < DX; x += 64)
        acc += maybe_bf16(S0[col * LDX + x], bf16) * maybe_bf16(P[pl.eW3 + x], bf16);
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if (lane == 0) jt[col] = (double)acc;
    }
  }
  if (do_k)
    for (int q = threadIdx.x; q < R * M; q += blockDim.x) {
      const int row = q / M, mu = q % M;
      ft[(int64_t)row * M + mu] = (double)KT[row * LDX + mu];
    }
}

template <typename TN, int C, bool STAGE>
void launch_c(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const TN* P, char* ws, const WsLayout& L,
              bool bf16, TN* xsave) {
  const int64_t nb = nw * L.n_chunks;
  int nt = kThreadsT;
  auto go = [&](auto kern) {
    if (L.lds_tangent > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)L.lds_tangent);
    hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(nt), L.lds_tangent, s, c->d, c->t, nw, L.n_chunks, r, P,
                       c->pl, reinterpret_cast<const TN*>(ws + L.filt), reinterpret_cast<const TN*>(ws + L.hval),
                       reinterpret_cast<const TN*>(ws + L.kcoef), reinterpret_cast<const TN*>(ws + L.ecoef),
                       reinterpret_cast<double*>(ws + L.ftan), reinterpret_cast<double*>(ws + L.jtan), xsave, false);
  };
  // one 512-thread block per CU where the planner gives a block all the LDS
  // (instantiated for the chunk sizes that rule produces)
  if constexpr (C <= 7) {
    if (L.tan_threads == 512) {
      nt = 512;
      if constexpr (sizeof(TN) == sizeof(float)) {
        if (bf16) {
          go(&k_net_tangent<TN, C, STAGE, true, 512>);
          return;
        }
      }
      go(&k_net_tangent<TN, C, STAGE, false, 512>);
      return;
    }
  }
  if constexpr (sizeof(TN) == sizeof(float)) {
    if (bf16) {
      go(&k_net_tangent<TN, C, STAGE, true, kThreadsT>);
      return;
    }
  }
  go(&k_net_tangent<TN, C, STAGE, false, kThreadsT>);
}

template <typename TN, bool STAGE>
void launch_t(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const TN* P, char* ws, const WsLayout& L,
              bool bf16, TN* xsave) {
  switch (L.T + 1) {
    case 2: launch_c<TN, 2, STAGE>(c, s, nw, r, P, ws, L, bf16, xsave); break;
    case 3: launch_c<TN, 3, STAGE>(c, s, nw, r, P, ws, L, bf16, xsave); break;
    case 4: launch_c<TN, 4, STAGE>(c, s, nw, r, P, ws, L, bf16, xsave); break;
    case 5: launch_c<TN, 5, STAGE>(c, s, nw, r, P, ws, L, bf16, xsave); break;
    case 6: launch_c<TN, 6, STAGE>(c, s, nw, r, P, ws, L, bf16, xsave); break;
    case 7: launch_c<TN, 7, STAGE>(c, s, nw, r, P, ws, L, bf16, xsave); break;
    case 9: launch_c<TN, 9, STAGE>(c, s, nw, r, P, ws, L, bf16, xsave); break;
    case 10: launch_c<TN, 10, STAGE>(c, s, nw, r, P, ws, L, bf16, xsave); break;
    case 11: launch_c<TN, 11, STAGE>(c, s, nw, r, P, ws, L, bf16, xsave); break;
    case 13: launch_c<TN, 13, STAGE>(c, s, nw, r, P, ws, L, bf16, xsave); break;
    case 16: launch_c<TN, 16, STAGE>(c, s, nw, r, P, ws, L, bf16, xsave); break;
    default: break;  // the planner only picks supported chunk sizes
  }
}

}  // namespace

template <typename TN>
void launch_net_tangent(const pn_ctx* c, hipStream_t s, int64_t nw, const double* r, const TN* P, char* ws,
                        const WsLayout& L, bool bf16, TN* xsave) {
  if (L.stage_filters)
    launch_t<TN, true>(c, s, nw, r, P, ws, L, bf16, xsave);
  else
    launch_t<TN, false>(c, s, nw, r, P, ws, L, bf16, xsave);
}

}  // namespace pn
