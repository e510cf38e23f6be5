// rswr_fused_kernel.h -- the fused span kernel of one problem (one launch
// per span, one work-group per tile; device code in rswr_fused.h) and its
// launcher over the built shapes.  Each launch kind is instantiated in a
// translation unit of its own (rswr_fused_*.hip) so that they compile in
// parallel.
#pragma once

#include "rswr_fused.h"

namespace rswr {

// The kernel body.  kFusedGeneral: general tiles (node 0 inside the region),
// receivers recorded and sources injected.  kFusedExt: a launch whose tiles may
// record receivers or inject interior sources; each work-group takes the
// code path its tile needs (a uniform branch), the others run the plain
// step.  kFusedPlain: the plain step only.
template <typename T, int NT, int MPT, int KIND>
__device__ __forceinline__ void fused_kernel_body(const UpdateArgs<T>& p) {
  constexpr int NW = NT / 64;
  constexpr int TM = NT * MPT;
  constexpr int TMP = TM + (TM >> 5) + 1;
  __shared__ T st[TMP];
  __shared__ T edge[2][2][NW];
  const int slot = xcd_tile(blockIdx.x, gridDim.x);
  const Tile tl = p.tiles[p.tile_idx[slot]];
  const int S = p.span;
  if (S <= 0 || S > kMaxFusedSpan) return;
  if constexpr (KIND == kFusedGeneral) {
    fused_tile<T, NT, MPT, true, true, true>(p, tl, slot, S, st, edge);
  } else if constexpr (KIND == kFusedExt) {
    const int t3 = 3 * p.tile_idx[slot];
    if (p.src_ptr && p.src_ptr[t3 + 3] > p.src_ptr[t3])
      fused_tile<T, NT, MPT, false, true, true>(p, tl, slot, S, st, edge);
    else if (p.rec_ptr && p.rec_ptr[slot + 1] > p.rec_ptr[slot])
      fused_tile<T, NT, MPT, false, true, false>(p, tl, slot, S, st, edge);
    else
      fused_tile<T, NT, MPT, false, false, false>(p, tl, slot, S, st, edge);
  } else {
    fused_tile<T, NT, MPT, false, false, false>(p, tl, slot, S, st, edge);
  }
}

// BY: problem blockIdx.y of a same-shape batch (YStrides); its states,
// boundary samples and flux rows lie at fixed strides from problem 0's.
template <typename T, int NT, int MPT, int KIND, bool BY>
__global__ __launch_bounds__(NT) void k_fused(const UpdateArgs<T> p) {
  if constexpr (BY) {
    UpdateArgs<T> q = p;
    q.state_in = at_y(p.state_in, p.ys.ws);
    q.state_out = at_y(p.state_out, p.ys.ws);
    q.flux_out = at_y(p.flux_out, p.ys.ws);
    q.fa = at_y(p.fa, p.ys.src);
    q.fb = at_y(p.fb, p.ys.src);
    fused_kernel_body<T, NT, MPT, KIND>(q);
  } else {
    fused_kernel_body<T, NT, MPT, KIND>(p);
  }
}

template <typename T, int KIND>
hipError_t launch_fused_kind(const UpdateArgs<T>& a, int threads, int per_thread,
                             hipStream_t s) {
  if (a.n_tiles <= 0) return hipSuccess;
#define RSWR_LAUNCH(NT_, MPT_)                                                      \
  if (threads == NT_ && per_thread == MPT_) {                                     \
    if constexpr (sizeof(T) == 8 && MPT_ > 22) return hipErrorInvalidValue;      \
    else {                                                                        \
      if (a.ys.ny <= 1) {                                                         \
        hipLaunchKernelGGL((k_fused<T, NT_, MPT_, KIND, false>), dim3(a.n_tiles), \
                           dim3(NT_), 0, s, a);                                   \
      } else if constexpr (KIND != kFusedExt) {                                   \
        hipLaunchKernelGGL((k_fused<T, NT_, MPT_, KIND, true>),                   \
                           dim3(a.n_tiles, a.ys.ny), dim3(NT_), 0, s, a);         \
      } else {                                                                    \
        return hipErrorInvalidValue;                                              \
      }                                                                           \
      return hipGetLastError();                                                   \
    }                                                                             \
  }
  RSWR_SHAPES(RSWR_LAUNCH)
#undef RSWR_LAUNCH
  return hipErrorInvalidValue;
}

}  // namespace rswr
