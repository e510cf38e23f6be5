// rswr_batch.hip -- many independent problems in one recorded graph.
//
// Each problem advances span by span (Sec. 2.6) with its own grid, windows,
// wave speed and span.  Round r runs span r of every problem that still has
// spans left: per kernel shape, one persistent launch whose work-groups walk
// the round's tiles (every problem's, in one list) with a grid stride, so
// problems of very different sizes share the chip within a round.  The tile
// work itself is the fused span of rswr_fused.h.
#include "rswr_fused.h"

namespace rswr {

template <typename T, int NT, int MPT>
__global__ __launch_bounds__(NT) void k_fused_batch(const BatchArgs<T> b) {
  constexpr int NW = NT / 64;
  constexpr int TM = NT * MPT;
  constexpr int TMP = TM + (TM >> 5) + 1;
  __shared__ T st[TMP];
  __shared__ T edge[2][2][NW];
  // the round's items from the last one down: problems are ordered by span
  // count, longest first, so the prefix ends with the longest spans (the
  // dearest tiles), which go first
  for (int k = blockIdx.x; k < b.n_items; k += gridDim.x) {
    const int item = b.n_items - 1 - k;
    const Tile tl = b.items[item];
    const BatchInst<T> in = b.inst[tl.inst];
    const int64_t n0 = static_cast<int64_t>(b.round) * in.S;
    const int64_t left = in.n_steps - n0;
    const int S = left < in.S ? static_cast<int>(left) : in.S;
    if (S <= 0 || S > kMaxFusedSpan) continue;  // whole work-group: uniform
    UpdateArgs<T> p{};
    p.state_in = (b.round & 1) ? in.st_b : in.st_a;
    p.state_out = (b.round & 1) ? in.st_a : in.st_b;
    p.fa = in.fa;
    p.fb = in.fb;
    p.lo = in.lo;
    p.hi = in.hi;
    p.flux_out = nullptr;
    p.rec_ptr = nullptr;
    p.M = in.M;
    p.n0 = n0;
    p.span = S;
    p.c2 = in.c2;
    p.k = in.k;
    p.q = in.q;
    p.r = in.r;
    fused_tile<T, NT, MPT, false, false, false>(p, tl, item, S, st, edge);
  }
}

// Copies of several buffers in one launch: blockIdx.y picks the job.
template <typename T>
__global__ __launch_bounds__(256) void k_copy_many(const CopyJob<T>* jobs) {
  const CopyJob<T> j = jobs[blockIdx.y];
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < j.n;
       i += stride)
    j.dst[i] = j.src[i];
}

// Resident work-groups of one kernel on the whole device: the grid of a
// persistent launch.
template <typename K>
int resident_groups(K kernel, int threads) {
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess)
    return 1024;
  return per_cu > 0 ? per_cu * prop.multiProcessorCount : prop.multiProcessorCount;
}

template <typename T>
int fused_batch_capacity(int threads, int per_thread) {
#define RSWR_CAP(NT_, MPT_)                                                \
  if (threads == NT_ && per_thread == MPT_) {                            \
    if constexpr (sizeof(T) == 8 && MPT_ > 22) return 0;                 \
    else return resident_groups(k_fused_batch<T, NT_, MPT_>, NT_);       \
  }
  RSWR_SHAPES(RSWR_CAP)
#undef RSWR_CAP
  return 0;
}

template <typename T>
hipError_t launch_fused_batch(const BatchArgs<T>& a, int threads, int per_thread, int grid,
                              hipStream_t s) {
  if (a.n_items <= 0) return hipSuccess;
  if (grid > a.n_items) grid = a.n_items;
  if (grid < 1) grid = 1;
#define RSWR_LAUNCH(NT_, MPT_)                                                         \
  if (threads == NT_ && per_thread == MPT_) {                                        \
    if constexpr (sizeof(T) == 8 && MPT_ > 22) return hipErrorInvalidValue;         \
    else {                                                                           \
      hipLaunchKernelGGL((k_fused_batch<T, NT_, MPT_>), dim3(grid), dim3(NT_), 0, s, a); \
      return hipGetLastError();                                                      \
    }                                                                                \
  }
  RSWR_SHAPES(RSWR_LAUNCH)
#undef RSWR_LAUNCH
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_copy_many(const CopyJob<T>* jobs, int32_t n_jobs, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_many<T>, dim3(64, n_jobs), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

template int fused_batch_capacity<float>(int, int);
template int fused_batch_capacity<double>(int, int);
template hipError_t launch_fused_batch<float>(const BatchArgs<float>&, int, int, int,
                                              hipStream_t);
template hipError_t launch_fused_batch<double>(const BatchArgs<double>&, int, int, int,
                                               hipStream_t);
template hipError_t launch_copy_many<float>(const CopyJob<float>*, int32_t, hipStream_t);
template hipError_t launch_copy_many<double>(const CopyJob<double>*, int32_t, hipStream_t);

}  // namespace rswr
