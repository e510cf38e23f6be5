// rswr_fused.hip -- the fused span kernel of one problem: one launch per
// span, one work-group per tile (device code in rswr_fused.h).
#include "rswr_fused.h"

namespace rswr {

// GEN: general tiles (node 0 inside the region), receivers recorded and
// sources injected.  EXT: a launch whose tiles may record receivers or
// inject interior sources; each work-group takes that code path only if its
// tile has any (a uniform branch), so the others run the plain step.
// Neither: the plain step only.
template <typename T, int NT, int MPT, bool GEN, bool EXT>
__global__ __launch_bounds__(NT) void k_fused(const UpdateArgs<T> p) {
  constexpr int NW = NT / 64;
  constexpr int TM = NT * MPT;
  constexpr int TMP = TM + (TM >> 5) + 1;
  __shared__ T st[TMP];
  __shared__ T edge[2][2][NW];
  const int slot = xcd_tile(blockIdx.x, gridDim.x);
  const Tile tl = p.tiles[p.tile_idx[slot]];
  const int S = p.span;
  if (S <= 0 || S > kMaxFusedSpan) return;
  if constexpr (GEN) {
    fused_tile<T, NT, MPT, true, true>(p, tl, slot, S, st, edge);
  } else if constexpr (EXT) {
    const int t3 = 3 * p.tile_idx[slot];
    if ((p.rec_ptr && p.rec_ptr[slot + 1] > p.rec_ptr[slot]) ||
        (p.src_ptr && p.src_ptr[t3 + 3] > p.src_ptr[t3]))
      fused_tile<T, NT, MPT, false, true>(p, tl, slot, S, st, edge);
    else
      fused_tile<T, NT, MPT, false, false>(p, tl, slot, S, st, edge);
  } else {
    fused_tile<T, NT, MPT, false, false>(p, tl, slot, S, st, edge);
  }
}

template <typename T>
hipError_t launch_fused(const UpdateArgs<T>& a, int threads, int per_thread, int kind,
                        hipStream_t s) {
  if (a.n_tiles <= 0) return hipSuccess;
#define RSWR_LAUNCH(NT_, MPT_)                                                        \
  if (threads == NT_ && per_thread == MPT_) {                                       \
    if constexpr (sizeof(T) == 8 && MPT_ > 22) return hipErrorInvalidValue;        \
    else {                                                                          \
      if (kind == kFusedGeneral)                                                    \
        hipLaunchKernelGGL((k_fused<T, NT_, MPT_, true, true>), dim3(a.n_tiles),    \
                           dim3(NT_), 0, s, a);                                     \
      else if (kind == kFusedExt)                                                   \
        hipLaunchKernelGGL((k_fused<T, NT_, MPT_, false, true>), dim3(a.n_tiles),   \
                           dim3(NT_), 0, s, a);                                     \
      else                                                                          \
        hipLaunchKernelGGL((k_fused<T, NT_, MPT_, false, false>), dim3(a.n_tiles),  \
                           dim3(NT_), 0, s, a);                                     \
      return hipGetLastError();                                                     \
    }                                                                               \
  }
  RSWR_SHAPES(RSWR_LAUNCH)
#undef RSWR_LAUNCH
  return hipErrorInvalidValue;
}

template hipError_t launch_fused<float>(const UpdateArgs<float>&, int, int, int,
                                        hipStream_t);
template hipError_t launch_fused<double>(const UpdateArgs<double>&, int, int, int,
                                         hipStream_t);

}  // namespace rswr
