// rswr_internal.h -- types shared by the host driver and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rswr {

// Largest span a kernel launch accepts (per-step boundary data is staged in
// LDS arrays of this length).
constexpr int kMaxSpan = 256;
// Prediction frame of the fused span: 2 * kFrameHalf nodes, two per lane.
constexpr int kFrameHalf = 64;
constexpr int kMaxFusedSpan = kFrameHalf - 1;
// Receivers one launched tile of the fused span records (the host repeats a
// tile holding more, one copy per group); adjoint sources held in registers.
constexpr int kRecSlots = 4;
// Interior sources a fused tile injects from registers: kSrcSlots in its
// region, kFrameSrc in each prediction frame; further ones are read from
// memory every step.
constexpr int kSrcSlots = 2;
constexpr int kFrameSrc = 1;

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
  int32_t inst;  // problem index in a batched launch (0 otherwise)
  int32_t pad;
};
static_assert(sizeof(Tile) == 64, "Tile layout");

// Problems of a same-shape batch along grid dimension y: problem y's
// buffers lie a fixed number of bytes after problem 0's.  ny <= 1: a
// single problem (every stride unused).
struct YStrides {
  int64_t ws;    // buffers in the batch workspace (states, fluxes, adjoint state, partials)
  int64_t src;   // boundary samples f_A, f_B
  int64_t gtr;   // dJ/dtrace
  int64_t grad;  // dJ/df outputs
  int32_t ny, pad;
};

template <typename T>
struct PredictArgs {
  const T* state;       // [2][M]
  const T* fa;
  const T* fb;
  T* flux;              // [N-1][2][ld]
  const int64_t* lo;    // [N]
  const int64_t* hi;    // [N]
  // nullable: read n0 / shat from the device (an adaptive solve recorded as
  // one graph); shat 0 there means the solve is done
  const int64_t* n0_dev;
  const int32_t* shat_dev;
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
  // fused span only: window bounds (for the predicting neighbours) and the
  // nullable destination of the predicted fluxes ([N-1][2][ld], the rows of
  // the tiles' input ends)
  const int64_t* lo;
  const int64_t* hi;
  T* flux_out;
  // interior point sources (nullable; fused span only): for tile number t,
  // entries src_ptr[3t] .. src_ptr[3t+3) of (src_node, src_id) in three runs
  // -- the tile's register region, its left frame, its right frame -- each
  // in source order; the step from level n adds src_amp[id * src_ld + n]
  const int32_t* src_ptr;
  const int64_t* src_node;
  const int32_t* src_id;
  const T* src_amp;
  int64_t src_ld;
  // nullable: the span starts at level *n0_dev instead of n0 (trace columns
  // shift by the same amount)
  const int64_t* n0_dev;
  YStrides ys;  // batch of same-shape problems (fused span: states, fa/fb, flux_out)
  int64_t M, n0, trace_ld, trace_col0;
  int32_t n_tiles, span, ld, pad;
  T c2, k, q, r;
};

// The whole span loop in one launch (rswr_persist.hip): span k reads
// buf0 (k even) or buf1 and writes the other, or, with checkpoints, reads
// ck[k] and writes ck[k+1] (and its flux rows to ck_flux[k]).  flags[t]
// counts the spans tile t has finished (zero on entry); dep_ptr / dep list,
// per tile, the tiles it waits for before each span; err is set if a wait
// gave up.
template <typename T>
struct PersistArgs {
  T* buf0;
  T* buf1;
  T* ck;
  T* ck_flux;
  int32_t* flags;
  int32_t* err;
  const int32_t* dep_ptr;
  const int32_t* dep;
  int64_t st_elems, fl_elems;
  int64_t n0, n_end;
  int32_t n_spans, S;
};

template <typename T>
struct SelectArgs {
  const T* flux;
  int32_t* span_dev;
  const int32_t* shat_dev;  // nullable: shat from the device (0: done)
  int32_t n_rows, shat, ld, cone, mode, fixed_span;
  // nullable (mode 1): the rows are scanned by many work-groups, one wave
  // per row, which take the minimum into *qmin (INT32_MAX on entry); the
  // last launch forms the span and restores *qmin to INT32_MAX
  int32_t* qmin;
};

// Device-side state of an adaptive (QUIET) solve recorded as one graph of a
// bounded number of predict -> select -> update rounds; rounds after the
// last span do nothing.
struct QuietCtl {
  int64_t n0;      // first level of the next span
  int64_t n_end;   // level the solve ends at
  int32_t shat;    // predictive span of the next span (0: done)
  int32_t span;    // span the select chose (0: done)
  int32_t parity;  // 1: the newest state is in the second buffer
  int32_t s_max;   // cap of the predictive span
  double beta;     // growth of Sec. 2.6
  int32_t qmin;    // the select's running minimum (INT32_MAX between rounds)
  int32_t pad;
};

// Adjoint of the receiver misfit (see rswr_adjoint.hip).  The adjoint field
// W runs backward in time: a span ending at level n_e starts from
// (W^{n_e+2}, W^{n_e+1}) and ends at (W^{n_k+2}, W^{n_k+1}).
template <typename T>
struct AdjPredictArgs {
  const T* w;           // [2][M]: row 0 = W^{n_e+2}, row 1 = W^{n_e+1}
  T* flux;              // [N-1][2][ld]; sample t is taken from W^{n_e+1-t}
  const int64_t* lo;
  const int64_t* hi;
  const int64_t* rec_node;  // all receivers, in receiver order
  const T* gtr;         // dJ/dtrace [n_rec][gtr_ld], column L-1 for level L
  YStrides ys;          // batch of same-shape problems (w, flux, gtr)
  int64_t gtr_ld, M, n_e;
  int32_t N, shat, ld, n_rec;
  T c2, k, r, q;
};

template <typename T>
struct AdjUpdateArgs {
  const T* w_in;        // [2][M] adjoint state at the span end
  T* w_out;             // [2][M] adjoint state at the span start
  const T* u_end;       // [2][M] forward state at the span end (levels n_e-1, n_e)
  const T* u_beg;       // [2][M] forward state at the span start (row 1 = level n_k)
  const T* ffl;         // forward fluxes of the span, sample m - n_k
  const T* afl;         // adjoint fluxes of the span, sample n_e - L
  const T* fa;
  const T* fb;
  const Tile* tiles;
  const int32_t* tile_idx;
  const int32_t* src_ptr;   // [n_tiles+1] CSR over this launch (general only)
  const int64_t* src_node;
  const int32_t* src_id;
  const T* gtr;
  int64_t gtr_ld;
  T* grad_fa;           // [n_steps+1]
  T* grad_fb;
  double* lam_part;     // one accumulator per tile (indexed by tile number)
  // fused update only: window bounds and every receiver's node (receiver
  // order), for the W frames the tiles carry at their input ends
  const int64_t* lo;
  const int64_t* hi;
  const int64_t* rec_all;
  YStrides ys;          // batch of same-shape problems (every pointer above but the tables)
  int64_t M, n_e, n_k;
  int32_t n_tiles, span, ld, n_rec_all;
  T c2, k, q, r;
};

// One problem of a batched launch.  Round r reads st_a (r even) or st_b
// and writes the other; n0 = r * S.
template <typename T>
struct BatchInst {
  T* st_a;
  T* st_b;
  const T* fa;
  const T* fb;
  const int64_t* lo;
  const int64_t* hi;
  int64_t M, n_steps;
  int32_t S, pad;
  T c2, k, q, r;
};

template <typename T>
struct BatchArgs {
  const Tile* items;  // tiles of every problem in this launch (Tile::inst set)
  const BatchInst<T>* inst;
  int32_t n_items, round;
};

template <typename T>
struct CopyJob {
  T* dst;
  const T* src;
  int64_t n;
};

// Launchers (defined in rswr_kernels.hip / rswr_fused.hip / rswr_batch.hip /
// rswr_adjoint.hip).  They return hipGetLastError().
template <typename T>
hipError_t launch_predict(const PredictArgs<T>& a, int shmem_nodes,
                          hipStream_t s);
template <typename T>
hipError_t launch_update(const UpdateArgs<T>& a, int threads, int per_thread,
                         bool general, hipStream_t s);
// Fused span (rswr_fused.hip dispatching to rswr_fused_kernel.h, one
// translation unit per launch kind): predict folded into the update; needs
// 1 <= span <= kMaxFusedSpan and inputs only at region ends.
// kFusedExt: a launch in which some tiles record receivers (CSR rec_ptr
// over its slots) or inject interior sources (src_ptr); kFusedGeneral:
// general tiles.
enum { kFusedPlain = 0, kFusedExt = 1, kFusedGeneral = 2 };
template <typename T>
hipError_t launch_fused(const UpdateArgs<T>& a, int threads, int per_thread, int kind,
                        hipStream_t s);
template <typename T, int KIND>
hipError_t launch_fused_kind(const UpdateArgs<T>& a, int threads, int per_thread,
                             hipStream_t s);
// Batched fused span: one persistent launch over the items with `grid`
// work-groups (at most the items); fused_batch_capacity gives the kernel's
// resident work-groups on the current device (0: shape not built).
template <typename T>
int fused_batch_capacity(int threads, int per_thread);
template <typename T>
hipError_t launch_fused_batch(const BatchArgs<T>& a, int threads, int per_thread, int grid,
                              hipStream_t s);
template <typename T>
hipError_t launch_copy_many(const CopyJob<T>* jobs, int32_t n_jobs, hipStream_t s);
// The whole loop in one launch (plain tiles of a fused plan, one work-group
// per tile, all resident): persist_capacity gives the resident work-groups
// of the shape's kernel on the current device (0: shape not built).
template <typename T>
int persist_capacity(int threads, int per_thread);
template <typename T>
hipError_t launch_fused_persist(const UpdateArgs<T>& a, const PersistArgs<T>& q, int threads,
                                int per_thread, hipStream_t s);
template <typename T>
hipError_t launch_select(const SelectArgs<T>& a, hipStream_t s);
// Adaptive solve on the device: set up the control block, advance it after
// each round, and copy the second buffer back when it holds the result.
hipError_t launch_quiet_init(QuietCtl* c, int64_t n0, int64_t n_end, int32_t shat0,
                             int32_t s_max, double beta, hipStream_t s);
hipError_t launch_quiet_next(QuietCtl* c, hipStream_t s);
template <typename T>
hipError_t launch_copy_if(T* dst, const T* src, int64_t n, const int32_t* flag,
                          hipStream_t s);
// n elements for each of ny problems, problem y at y * stride bytes
template <typename T>
hipError_t launch_copy_y(T* dst, const T* src, int64_t n, int32_t ny, int64_t stride,
                         hipStream_t s);
template <typename T>
hipError_t launch_fill_y(T* dst, T v, int64_t n, int32_t ny, int64_t stride, hipStream_t s);
template <typename T>
hipError_t launch_copy(T* dst, const T* src, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_fill(T* dst, T v, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_adj_predict(const AdjPredictArgs<T>& a, int shmem_nodes,
                              hipStream_t s);
// fused: the tiles predict their input ends' W fluxes themselves (plans
// that run the fused span; afl unused), else afl holds the predict
// kernel's rows.
template <typename T>
hipError_t launch_adj_update(const AdjUpdateArgs<T>& a, int threads,
                             int per_thread, bool general, bool fused, hipStream_t s);
// the fused update kernels of this shape run without scratch (the current
// device's code objects)
template <typename T>
bool adj_update_fused_fits(int threads, int per_thread);
template <typename T, bool FR>
hipError_t launch_adj_update_kind(const AdjUpdateArgs<T>& a, int threads, int per_thread,
                                  bool general, hipStream_t s);
// grad_fa[L] += dJ/dtrace of receivers on node 0 (grad_fb: node M-1), in
// receiver order, for L = 1..n_steps; grad_lam = 2 lam * sum(lam_part).
template <typename T>
hipError_t launch_adj_finish(T* grad_fa, T* grad_fb, const T* gtr, int64_t gtr_ld,
                             const int64_t* rec_node, int32_t n_rec, int64_t M,
                             int64_t n_steps, const double* lam_part,
                             int32_t n_part, double lam, double* grad_lam,
                             hipStream_t s);

// Kernel shapes compiled into the library: (threads, nodes per lane).
struct Shape {
  int threads, per_thread;
};
int n_shapes();
Shape shape_at(int i);
bool shape_built(int threads, int per_thread);

}  // namespace rswr
