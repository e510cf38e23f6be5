// rswr_internal.h -- types shared by the host driver and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rswr {

// Largest span a kernel launch accepts (per-step boundary data is staged in
// LDS arrays of this length).
constexpr int kMaxSpan = 256;

// Sentinel for "no left-input ghost in this tile".
constexpr int64_t kNoNode = INT64_MIN;

// Treatment of the neighbour just outside a tile's register region.
enum : int32_t {
  kEndZero = 0,       // zero data: the host stores no node it can reach
  kEndGhost = 1,      // the region end is the window's input boundary: ghost
                      // value from that input's flux waveform
  kEndDirichlet = 2   // the neighbour is node 0 (left) or node M-1 (right):
                      // its Dirichlet value, Eq. (3)
};

// One update work-group: lanes hold the register region
// [a, a + threads*per_thread - 1] of window `window` for the whole span.  The
// tile stores the nodes out_lo..out_hi (clipped to the region, plus node 0 /
// node M-1 when the matching end is kEndDirichlet).  fl / fr: flux rows of
// the left / right input ([fl][0], [fr][1]).  General tiles hold the
// window's left input `lin` or node 0 strictly inside the region (small
// windows); they run the general kernel.
struct Tile {
  int64_t a;
  int64_t out_lo, out_hi;
  int64_t lin;
  int32_t fl, fr;
  int32_t lmode, rmode;
  int32_t window, general;
  int32_t pad[2];
};
static_assert(sizeof(Tile) == 64, "Tile layout");

template <typename T>
struct PredictArgs {
  const T* state;       // [2][M]
  const T* fa;
  const T* fb;
  T* flux;              // [N-1][2][ld]
  const int64_t* lo;    // [N]
  const int64_t* hi;    // [N]
  int64_t M, n0;
  int32_t N, shat, ld, pad;
  T c2, k, r, q;
};

template <typename T>
struct UpdateArgs {
  const T* state_in;    // [2][M]
  T* state_out;         // [2][M]
  const T* fa;
  const T* fb;
  const T* flux;        // [N-1][2][ld]
  const Tile* tiles;
  const int32_t* tile_idx;  // [n_tiles] entries of `tiles` this launch runs
  const int32_t* span_dev;  // nullable
  const int32_t* rec_ptr;   // [n_tiles+1] CSR over this launch, or nullptr
  const int64_t* rec_node;
  const int32_t* rec_id;
  T* traces;
  int64_t M, n0, trace_ld, trace_col0;
  int32_t n_tiles, span, ld, pad;
  T c2, k, q;
};

template <typename T>
struct SelectArgs {
  const T* flux;
  int32_t* span_dev;
  int32_t n_rows, shat, ld, cone, mode, fixed_span;
};

// Launchers (defined in rswr_kernels.hip).  They return hipGetLastError().
template <typename T>
hipError_t launch_predict(const PredictArgs<T>& a, int shmem_nodes,
                          hipStream_t s);
template <typename T>
hipError_t launch_update(const UpdateArgs<T>& a, int threads, int per_thread,
                         bool general, hipStream_t s);
template <typename T>
hipError_t launch_select(const SelectArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_copy(T* dst, const T* src, int64_t n, hipStream_t s);

// Kernel shapes compiled into the library: (threads, nodes per lane).
struct Shape {
  int threads, per_thread;
};
int n_shapes();
Shape shape_at(int i);
bool shape_built(int threads, int per_thread);

}  // namespace rswr
