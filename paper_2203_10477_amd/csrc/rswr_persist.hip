// rswr_persist.hip -- the redo loop of Sec. 2.6 in one launch: every
// work-group owns one tile of the fused span (rswr_fused.h) for all spans.
//
// Method: Wei & Zhao, arXiv 2203.10477.  A tile's span k reads the glued
// state of span k-1 over its region and its prediction frames (Sec. 2.3:
// the predicting neighbour's nodes around each input end), and writes its
// stored range.  Instead of a kernel boundary between spans, each tile waits
// only for the tiles it depends on: those whose stored ranges meet its
// region or frames, and those whose regions or frames meet its stored range
// (so a tile never overwrites a ping-pong buffer before every reader of the
// old contents has read it).  A tile announces a finished span with a
// counter in memory and polls its dependencies' counters.  The producer and
// the consumer may sit on different XCDs, each with its own L2: every state
// load and store of these tiles uses the device-coherent policy, and each
// wave waits for its stores to complete before the count is published, so
// no cache is written back or invalidated.  Tiles of one span run as soon
// as their neighbours allow, so spans overlap across the grid.
//
// The launch holds every tile at once (the host checks the resident
// capacity), so every wait ends once its producer runs.  Each wait is still
// bounded: a tile that times out records it and stops; the tiles waiting on
// it time out in turn, and the failed tiles fill their stored range of the
// final state with NaN, so a failure can never hang the device or pass as
// a result.
#include "rswr_fused.h"

namespace rswr {

// Polls of one dependency wait before it gives up: each poll is a load that
// bypasses the caches, plus a short sleep, so this is a few seconds, far
// beyond any span's time.
constexpr int kPersistSpin = 1 << 21;

template <typename T, int NT, int MPT>
__global__ __launch_bounds__(NT) void k_fused_persist(const UpdateArgs<T> p0,
                                                      const PersistArgs<T> q) {
  constexpr int NW = NT / 64;
  constexpr int TM = NT * MPT;
  constexpr int TMP = TM + (TM >> 5) + 1;
  __shared__ T st[TMP];
  __shared__ T edge[2][2][NW];
  __shared__ int s_fail;
  const int tid = threadIdx.x;
  const int slot = xcd_tile(blockIdx.x, gridDim.x);
  const int tix = p0.tile_idx[slot];
  const Tile tl = p0.tiles[tix];
  if (tid == 0) s_fail = 0;
  __syncthreads();
  int k = 0;
  for (; k < q.n_spans; ++k) {
    if (k > 0) {
      // every dependency has finished span k-1
      if (tid == 0) {
        int fail = 0;
        for (int d = q.dep_ptr[tix]; d < q.dep_ptr[tix + 1] && !fail; ++d) {
          const int32_t* f = q.flags + q.dep[d];
          int spins = 0;
          while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < k) {
            if (++spins > kPersistSpin) {
              fail = 1;
              break;
            }
            __builtin_amdgcn_s_sleep(2);
          }
        }
        if (fail) {
          __hip_atomic_store(q.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          s_fail = 1;
        }
      }
      __syncthreads();
      if (s_fail) break;  // uniform: read after the barrier
    }
    const int64_t n0 = q.n0 + static_cast<int64_t>(k) * q.S;
    const int64_t left = q.n_end - n0;
    const int S = left < q.S ? static_cast<int>(left) : q.S;
    UpdateArgs<T> p = p0;
    p.n0 = n0;
    p.span = S;
    if (q.ck) {
      p.state_in = q.ck + static_cast<int64_t>(k) * q.st_elems;
      p.state_out = q.ck + static_cast<int64_t>(k + 1) * q.st_elems;
      p.flux_out = q.ck_flux + static_cast<int64_t>(k) * q.fl_elems;
    } else {
      p.state_in = (k & 1) ? q.buf1 : q.buf0;
      p.state_out = (k & 1) ? q.buf0 : q.buf1;
      p.flux_out = nullptr;
    }
    fused_tile<T, NT, MPT, false, false, false, true>(p, tl, slot, S, st, edge);
    // every wave's device-coherent stores are complete before the barrier;
    // then one thread publishes the count
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0)
      __hip_atomic_store(q.flags + tix, k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (k < q.n_spans) {
    // failed: NaN over the stored range of the state the last span writes
    T* out = q.ck ? q.ck + static_cast<int64_t>(q.n_spans) * q.st_elems
                  : ((q.n_spans & 1) ? q.buf1 : q.buf0);
    const T nan = __builtin_nan("");
    for (int64_t j = tl.out_lo + tid; j <= tl.out_hi; j += NT) {
      out[j] = nan;
      out[p0.M + j] = nan;
    }
  }
}

template <typename T>
int persist_capacity(int threads, int per_thread) {
#define RSWR_CAP(NT_, MPT_)                                                      \
  if (threads == NT_ && per_thread == MPT_) {                                  \
    if constexpr (sizeof(T) == 8 && MPT_ > 22) return 0;                       \
    else {                                                                     \
      int dev = 0, per_cu = 0, cus = 0;                                        \
      if (hipGetDevice(&dev) != hipSuccess ||                                  \
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,  \
                                dev) != hipSuccess ||                          \
          hipOccupancyMaxActiveBlocksPerMultiprocessor(                        \
              &per_cu, k_fused_persist<T, NT_, MPT_>, NT_, 0) != hipSuccess)   \
        return 0;                                                              \
      return per_cu * cus;                                                     \
    }                                                                          \
  }
  RSWR_SHAPES(RSWR_CAP)
#undef RSWR_CAP
  return 0;
}

template <typename T>
hipError_t launch_fused_persist(const UpdateArgs<T>& a, const PersistArgs<T>& q, int threads,
                                int per_thread, hipStream_t s) {
  if (a.n_tiles <= 0 || q.n_spans <= 0) return hipSuccess;
#define RSWR_LAUNCH(NT_, MPT_)                                                         \
  if (threads == NT_ && per_thread == MPT_) {                                        \
    if constexpr (sizeof(T) == 8 && MPT_ > 22) return hipErrorInvalidValue;         \
    else {                                                                           \
      hipLaunchKernelGGL((k_fused_persist<T, NT_, MPT_>), dim3(a.n_tiles), dim3(NT_), \
                         0, s, a, q);                                                \
      return hipGetLastError();                                                      \
    }                                                                                \
  }
  RSWR_SHAPES(RSWR_LAUNCH)
#undef RSWR_LAUNCH
  return hipErrorInvalidValue;
}

template int persist_capacity<float>(int, int);
template int persist_capacity<double>(int, int);
template hipError_t launch_fused_persist<float>(const UpdateArgs<float>&,
                                                const PersistArgs<float>&, int, int,
                                                hipStream_t);
template hipError_t launch_fused_persist<double>(const UpdateArgs<double>&,
                                                 const PersistArgs<double>&, int, int,
                                                 hipStream_t);

}  // namespace rswr
