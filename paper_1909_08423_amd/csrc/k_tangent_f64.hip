// Network tangent pass, FP64 network; also the chunk planner helpers.
#include "k_tangent_impl.h"

namespace pn {

// Chunk sizes T the kernel is instantiated for (columns C = T + 1).
bool tangent_chunk_supported(int T) {
  switch (T) {
    case 1: case 2: case 3: case 4: case 5: case 6: case 8: case 9: case 10: case 12: case 15: return true;
    default: return false;
  }
}

template <typename TN>
size_t tangent_lds_bytes(const Dims& d, int T, int stage) {
  const int C = T + 1, R = d.N * C;
  const int LDX = ld_pad<TN>(d.DX), LDZ = ld_pad<TN>(d.DZ), LDHZ = std::max(2 * LDZ, LDX);
  const int NCE = chunk_elecs_max(d.N, T);  // electrons a chunk of T coordinates can touch
  size_t tn = (size_t)d.N * d.DZ + (size_t)R * (LDX + LDHZ) + std::max(2 * (size_t)C * LDX, (size_t)NCE * C * LDZ) + (size_t)NCE * ((stage == 0 && T <= 3 ? 8 : 4) * d.N + 4 * d.NN);
  // stage 2: all electron pairs' w and the chunk rows' w'/d, w'' in LDS
  if (stage >= 2) tn += (size_t)d.n_ee * d.DZ + 2 * (size_t)NCE * (d.N + d.NN) * d.DZ;
  // unstaged chunks of at most 3 coordinates: the row blocks' pair indices
  const size_t prow = stage == 0 && T <= 3 ? (size_t)((d.n_up + 3) / 4 + (d.n_dn + 3) / 4) * d.N * 4 * sizeof(int) : 0;
  // unstaged chunks of 1 or 3 coordinates: partial own-row sums, [groups][4][DZ]
  // (8 groups in FP32, 2 in FP64, at most one per DZ threads of 512)
  const int groups = std::min(512 / d.DZ, sizeof(TN) == 4 ? 8 : 2);
  const size_t ownp = stage == 0 && (T == 1 || T == 3) ? (size_t)groups * 4 * d.DZ * sizeof(TN) : 0;
  return 3 * kMaxElec * sizeof(double) + (size_t)((d.N * d.N + 3) & ~3) * sizeof(int) + tn * sizeof(TN) + prow + ownp;
}

template size_t tangent_lds_bytes<double>(const Dims&, int, int);
template size_t tangent_lds_bytes<float>(const Dims&, int, int);
template void launch_net_tangent<double>(const pn_ctx*, hipStream_t, int64_t, const double*, const double*, char*,
                                         const WsLayout&, bool, double*);
}  // namespace pn
