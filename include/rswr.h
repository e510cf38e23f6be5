/*
 * rswr.h -- C-ABI of the RSWR hot path on AMD Instinct MI355X (gfx950).
 *
 * Method: Wei & Zhao, "A Non-iterative Overlapping Schwarz Waveform
 * Relaxation Algorithm for Wave Equation", arXiv 2203.10477.
 *
 * The library solves u_tt = a^2 u_xx on Omega = [X_A, X_B] (Sec. 2.1,
 * Eq. (1)) with Dirichlet data f_A, f_B at the ends (Eq. (3)) by splitting
 * Omega into N overlapping windows (Sec. 2.2 Eqs. (4)-(5), Sec. 3) and
 * advancing them span by span with the predict (Sec. 2.3), select (Sec. 2.4)
 * and update (Sec. 2.5) steps and the redo loop of Sec. 2.6.
 *
 * Discretisation (the paper fixes none): nodes x_j = X_A + j dx,
 * j = 0..M-1, dx = (X_B - X_A)/(M-1), dt = C dx / a_ref, lam = a dt/dx;
 * second-order leapfrog with per-node order s = ul + ur,
 * t = fma(k, u, -u_old), u_new = fma(lam^2, s, t), k = 2 - 2 lam^2;
 * output flux waveforms are centred differences (u_{o+1} - u_{o-1})/(2dx);
 * a Neumann input at a right window end b uses the ghost
 * u_{b+1} = u_{b-1} + 2dx F, at a left end u_{b-1} = u_{b+1} - 2dx F.
 * U^n_0 = f_A[n], U^n_{M-1} = f_B[n] for n >= 1; levels -1 and 0 are the
 * initial state (zero for the paper's Eq. (2)).
 *
 * Conventions
 *  - Every `void*` data argument is a DEVICE pointer owned by the caller
 *    (allocated, e.g., by PyTorch); the element type is the plan's dtype.
 *    Host pointers are marked (host).
 *  - A state is [2][M]: row 0 = level n0-1, row 1 = level n0.
 *  - Source arrays f_a, f_b are indexed by absolute level and must hold
 *    every level a call touches (n0 .. n0 + steps).
 *  - A flux buffer is [N-1][2][flux_ld] (flux_ld from rswr_plan_info):
 *    [i][0][s] = window i's output flux at lo_{i+1} (feeds window i+1's left
 *    input), [i][1][s] = window i+1's output flux at hi_i (feeds window i's
 *    right input), at level n0+s.  These are the corresponding waveforms of
 *    Sec. 2.2.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued asynchronously; argument errors are reported
 *    synchronously; asynchronous device faults surface at a later call or
 *    stream synchronisation as RSWR_ERR_HIP.
 *  - No function throws or aborts; each returns a status code and
 *    rswr_last_error() gives a thread-local description of the last error.
 *  - A plan is immutable after creation and may be used from several
 *    streams; it owns only its host tables and small device tables that it
 *    uploads on first use on each device.
 */
#ifndef RSWR_H
#define RSWR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rswr_plan_s* rswr_plan_t;
typedef struct rswr_batch_s* rswr_batch_t;

typedef enum {
  RSWR_OK = 0,
  RSWR_ERR_INVALID_ARG = 1, /* null pointer, bad size or flag */
  RSWR_ERR_UNSTABLE = 2,    /* Courant number outside (0, 1] */
  RSWR_ERR_LAYOUT = 3,      /* windows violate Eq. (4) or are too small */
  RSWR_ERR_SPAN = 4,        /* span beyond the light-cone limit */
  RSWR_ERR_NOMEM = 5,       /* host or device allocation failed, or the
                               workspace is too small */
  RSWR_ERR_HIP = 6,         /* HIP runtime error (launch or device fault) */
  /* 7 is not used */
  RSWR_ERR_UNSUPPORTED = 8  /* valid request outside the built kernels */
} rswr_status_t;

typedef enum { RSWR_F32 = 0, RSWR_F64 = 1 } rswr_dtype_t;

typedef enum {
  /* S = min(light-cone limit, Waveform Time Span Theorem, Sec. 2.4 Eq. (10))
   * every span; select needs no data. */
  RSWR_SPAN_FIXED = 0,
  /* adaptive: first predictive span = light-cone limit, then
   * Shat_k = ceil((1+beta) S_{k-1}) (Sec. 2.6); S_k = min(Shat_k,
   * min_b min(q_b, S_cone) + S_cone) with q_b the leading exact zeros of the
   * predicted flux feeding input b (a safe replacement for the agreement
   * test of Sec. 2.4, which is unsafe on mirror-symmetric data). */
  RSWR_SPAN_QUIET = 1
} rswr_span_mode_t;

typedef struct {
  double x_a, x_b;          /* Omega = [X_A, X_B], Sec. 2.1 */
  int64_t n_points;         /* M >= 3 grid nodes */
  double a;                 /* wave speed a > 0, Eq. (1) */
  double a_ref;             /* speed that fixes dt = courant dx / a_ref;
                               0 means a (then lam = courant) */
  double courant;           /* C in (0, 1] */
  int32_t courant_num;      /* optional exact C = num/den for the span rule; */
  int32_t courant_den;      /* must equal `courant` to rounding (else
                               INVALID_ARG); (0, 0) = use `courant` */
  int32_t n_sub;            /* N >= 1 windows, Sec. 3 */
  int32_t overlap;          /* P, overlap width in grid intervals, even,
                               Eq. (5); ignored with explicit windows */
  const int64_t* sub_lo;    /* (host) optional explicit windows [lo_i, hi_i], */
  const int64_t* sub_hi;    /* N entries each; NULL = uniform cores
                               round(i (M-1)/N) widened by P/2 each side */
  int32_t span;             /* 0 = default fixed span; else 1..light-cone
                               limit (FIXED mode) */
  int32_t span_mode;        /* rswr_span_mode_t */
  double beta;              /* span growth of Sec. 2.6; 0 means 0.1 */
  int32_t dtype;            /* rswr_dtype_t */
  int32_t tile_threads;     /* 0 = library choice; else a built kernel shape */
  int32_t tile_per_thread;  /* nodes per lane of that shape */
  int32_t no_fuse;          /* 1 = rswr_solve keeps predict and update as two
                               launches per span even where the fused span
                               applies (see rswr_plan_info_t.fused) */
  /* Interior point sources, the pulse sources of Sec. 4 (u_tt = a^2 u_xx +
   * s): the step from level n to n+1 adds src_amp[q][n] (the caller's
   * samples of dt^2 s at the node, dtype of the plan) to node src_node[q]
   * after the leapfrog update, sources in list order, in every window that
   * holds the node (prediction and update alike).  n_src = 0: none.  Nodes
   * must lie in 1..M-2.  Plans with sources must take the fused span
   * (rswr_plan_info_t.fused; else UNSUPPORTED) and run rswr_span and
   * rswr_solve only; the device array must stay valid while the plan is
   * used, and a call must end at a level <= src_ld. */
  int32_t n_src;
  const int64_t* src_node;  /* (host) copied by rswr_plan */
  const void* src_amp;      /* (device) [n_src][src_ld] */
  int64_t src_ld;
  /* 1: rswr_solve without receivers runs the whole loop of Sec. 2.6 as one
   * launch where the plan allows it (rswr_plan_info_t.one_launch) and its
   * tiles all fit on the device at once: each tile waits only for its
   * neighbours' previous span, with no launch boundary between spans.  The
   * results are identical; on one MI355X the span-by-span graph is the
   * faster form for the configurations measured, so 0 (span by span) is the
   * default. */
  int32_t one_launch;
} rswr_desc_t;

typedef struct {
  int64_t n_points;
  int32_t n_sub, dtype;
  int32_t span;             /* fixed span S (FIXED) or the cap 2*S_cone (QUIET) */
  int32_t span_cone;        /* light-cone limit: min distance input<->output */
  int32_t span_paper;       /* largest S with 2 S lam < P, Eq. (10) */
  int32_t flux_ld;          /* row stride of flux buffers */
  int32_t n_tiles;          /* update work-groups per span */
  int32_t tile_threads, tile_per_thread;
  double dx, dt, lambda;
  int32_t fused;            /* 1: rswr_solve runs each span as one launch, the
                               prediction of every input end carried by the
                               wave holding that end (fixed span S <= 63,
                               every input at a region end); results are
                               identical either way */
  int32_t one_launch;       /* 1: the plan asked for the one-launch loop
                               (rswr_desc_t.one_launch) and can run it (a
                               fused plan without general tiles or
                               sources) */
} rswr_plan_info_t;

/* (host) Kernel shapes built into the library: up to `cap` (threads per
 * work-group, nodes per lane) pairs and whether FP64 may use them
 * (fp64_ok[i] = 0 when the shape would not fit the register file in FP64).
 * Returns the number of shapes; any of them may be given to rswr_plan as
 * tile_threads / tile_per_thread. */
int32_t rswr_kernel_shapes(int32_t* threads, int32_t* per_thread,
                           int32_t* fp64_ok, int32_t cap);

/* Builds a plan from the problem statement of Sec. 2.1-2.2 and Sec. 3.
 * Host only: makes no HIP call.  Errors: INVALID_ARG, UNSTABLE, LAYOUT,
 * SPAN, UNSUPPORTED, NOMEM. */
rswr_status_t rswr_plan(const rswr_desc_t* desc, rswr_plan_t* out);
rswr_status_t rswr_plan_destroy(rswr_plan_t plan);
rswr_status_t rswr_plan_info(rswr_plan_t plan, rswr_plan_info_t* info);
/* (host) arrays of N entries each: windows and owned ranges (a node shared by
 * two windows belongs to the lower-indexed one, Sec. 2.5 Eq. (15)). */
rswr_status_t rswr_plan_layout(rswr_plan_t plan, int64_t* lo, int64_t* hi,
                               int64_t* own_lo, int64_t* own_hi);

/* (host) The update work-groups of one span, for inspection: for tile t,
 * tiles[8t..8t+7] = {first node of its register region, last node of the
 * region, first and last node it stores, window index, left end, right end
 * (0 zero data, 1 the window's input ghost, 2 the Dirichlet neighbour),
 * general flag}.  `tiles` holds 8 * n_tiles entries. */
rswr_status_t rswr_plan_tiles(rswr_plan_t plan, int64_t* tiles);

/* Predict, Sec. 2.3 Eqs. (8)-(9): every window advances `span_hat` levels
 * from `state` (level n0) with zero input flux; writes the output flux
 * waveforms at levels n0..n0+span_hat-1 into `flux`.  Only the light-cone
 * trapezoid around each output node is computed; it equals the whole-window
 * prediction exactly.  1 <= span_hat <= plan's span cap. */
rswr_status_t rswr_predict(rswr_plan_t plan, const void* state,
                           const void* f_a, const void* f_b, int64_t n0,
                           int32_t span_hat, void* flux, void* stream);

/* Select, Sec. 2.4 and Sec. 3 Eq. (19): writes the span for this step to the
 * device int32 `span_dev`.  FIXED: min(span_hat, S).  QUIET: the rule above,
 * evaluated on `flux` (span_hat samples per waveform). */
rswr_status_t rswr_select(rswr_plan_t plan, const void* flux, int32_t span_hat,
                          int32_t* span_dev, void* stream);

/* Update, Sec. 2.5 Eqs. (13)-(14), and gluing, Eq. (15): every window
 * advances S levels from `state_in` with its neighbours' predicted fluxes as
 * input fluxes; the owned ranges of levels n0+S-1 and n0+S are written to
 * `state_out` (which must not overlap `state_in`).  S is read from the device
 * int32 `span_dev` when it is not NULL, else it is `span`. */
rswr_status_t rswr_update(rswr_plan_t plan, const void* state_in,
                          const void* f_a, const void* f_b, int64_t n0,
                          const void* flux, const int32_t* span_dev,
                          int32_t span, void* state_out, void* stream);

/* One whole span of the redo loop (Sec. 2.6) with the fixed span: the
 * predict of Sec. 2.3 and the update and gluing of Sec. 2.5 over `span`
 * levels (1..S) from levels n0-1, n0 in `state_in` to levels n0+span-1,
 * n0+span in `state_out` (must not overlap `state_in`).  Plans with
 * rswr_plan_info_t.fused run it as one launch: then `flux` is optional and,
 * when given ([N-1][2][flux_ld], device), receives the predicted flux rows of
 * the input ends the tiles use.  Other plans predict into `flux` (required
 * when N > 1) and update from it, two launches.  f_a, f_b as for
 * rswr_predict.  The result is the same either way.  Errors: INVALID_ARG,
 * SPAN, UNSUPPORTED (QUIET plans), HIP. */
rswr_status_t rswr_span(rswr_plan_t plan, const void* state_in, const void* f_a,
                        const void* f_b, int64_t n0, int32_t span, void* flux,
                        void* state_out, void* stream);

/* Bytes of device workspace rswr_solve needs for n_rec receivers. */
rswr_status_t rswr_solve_workspace_size(rswr_plan_t plan, int32_t n_rec,
                                        size_t* bytes);

/* Bytes of a checkpoint buffer for an n_steps solve: the states at the
 * n_spans+1 span boundaries ([n_spans+1][2][M]) followed by the predicted
 * flux waveforms of every span ([n_spans][N-1][2][flux_ld]), n_spans =
 * ceil(n_steps / S).  This is what rswr_solve_adjoint reads. */
rswr_status_t rswr_checkpoint_size(rswr_plan_t plan, int64_t n_steps,
                                   size_t* bytes);

/* The redo loop of Sec. 2.6: n_steps levels from level n0, predict ->
 * select -> update per span, the last span shortened.  FIXED plans use the
 * plan's span.  QUIET plans choose every span on the device (first
 * predictive span S_cone, then ceil((1+beta) S_prev), capped by the plan's
 * span cap and the levels left; the select rule of rswr_span_mode_t); the
 * loop is recorded with enough rounds for spans of min(S_cone, cap) levels,
 * and rounds after the last span exit at once.  Checkpoints need FIXED.
 * `state` is read and overwritten with levels n0+n_steps-1 and n0+n_steps.
 * Receivers: `rec_idx` (host) holds n_rec node indices; `traces`
 * [n_rec][n_steps] receives U^{n0+s+1}[rec] at column s.  `checkpoints`
 * (optional, rswr_checkpoint_size bytes) receives the state at every span
 * boundary and every span's predicted fluxes.  The whole loop is recorded
 * once into a HIP graph per argument set and replayed. */
rswr_status_t rswr_solve(rswr_plan_t plan, void* state, const void* f_a,
                         const void* f_b, int64_t n0, int64_t n_steps,
                         const int64_t* rec_idx, int32_t n_rec, void* traces,
                         void* workspace, size_t ws_bytes, void* checkpoints,
                         void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the redo
 * loop of rswr_solve without receivers or checkpoints, whose workspace (the
 * second state buffer, the flux rows, the control block of a QUIET solve)
 * is a device array inside the library of RSWR_NOALLOC_SCRATCH_BYTES
 * (64 MiB) per GPU, held until the process ends.  The launches are
 * enqueued directly on `stream` (no graph of its own, so a capturing caller
 * records them); nothing is allocated or freed.  The plan's device tables
 * must already be on the current device: any earlier compute call of the
 * plan there (rswr_span, rswr_solve, ...) uploads them; else UNSUPPORTED.
 * Arguments as rswr_solve.  Every call on one GPU uses that GPU's one
 * array, which keeps the previous call's contents: calls that overlap in
 * time on one GPU (two streams, two host threads) race, and the caller must
 * order them.  Errors: INVALID_ARG, NOMEM (rswr_solve_workspace_size with no
 * receivers exceeds the array), UNSUPPORTED, HIP. */
#define RSWR_NOALLOC_SCRATCH_BYTES (64u << 20)
rswr_status_t rswr_solve_noalloc(rswr_plan_t plan, void* state, const void* f_a,
                                 const void* f_b, int64_t n0, int64_t n_steps,
                                 void* stream);

/* Bytes of device workspace rswr_solve_adjoint needs for n_rec receivers. */
rswr_status_t rswr_adjoint_workspace_size(rswr_plan_t plan, int32_t n_rec,
                                          size_t* bytes);

/* *fused = 1 if rswr_solve_adjoint of this plan runs the fused adjoint span
 * on the current device (the plan runs the fused span, and the fused update
 * kernels of its shape need no scratch memory there), else 0: then each
 * span is a predict launch and an update launch.  The results are the same
 * bit for bit either way.  Needs a device (reads the kernels' attributes);
 * no allocation. */
rswr_status_t rswr_adjoint_fused(rswr_plan_t plan, int32_t* fused);

/* Gradient of the receiver misfit J = sum_r sum_n (U^n[rec_r] - d_r^n)^2 of
 * an n_steps solve from level 0 (FIXED plan), given dJ/dtrace in
 * `grad_traces` [n_rec][n_steps] (2 (trace - d) for this J; any upstream
 * gradient works).  Reverse mode of the discrete solve: the adjoint field
 * obeys the same leapfrog backward in time with the trace gradients as point
 * sources, and is advanced span by span, last span first, with the method's
 * own predict / update exchange (Sec. 2.3-2.5) on the plan's windows (on
 * plans that run the fused span, one launch per span: the tiles holding an
 * input end advance its prediction themselves); the forward field is rebuilt
 * inside each span from the span-end checkpoint by running the leapfrog
 * backward.  `checkpoints` is the buffer filled by
 * rswr_solve over the same n_steps.  Writes dJ/df_A[n], dJ/df_B[n]
 * (n = 0..n_steps, entry 0 is 0) to grad_f_a / grad_f_b and dJ/dlam
 * (lam = a dt/dx at fixed dt) to the device double *grad_lambda; dJ/da is
 * dJ/dlam * lam / a. */
rswr_status_t rswr_solve_adjoint(rswr_plan_t plan, const void* checkpoints,
                                 const void* f_a, const void* f_b,
                                 int64_t n_steps, const int64_t* rec_idx,
                                 int32_t n_rec, const void* grad_traces,
                                 void* grad_f_a, void* grad_f_b,
                                 double* grad_lambda, void* workspace,
                                 size_t ws_bytes, void* stream);

/* A batch of adjoint solves of one plan: n_prob problems of the same shape,
 * receivers and span (a fused FIXED plan without sources), each the solve of
 * rswr_solve from rest (zero levels -1 and 0) driven by its own boundary
 * samples, with its own dJ/dtrace.  Per problem the result equals
 * rswr_solve (with checkpoints) followed by rswr_solve_adjoint, bit for bit.
 * Checkpoints are chunked, so a batch of large problems fits in memory: the
 * forward pass keeps the state at every seg-th span boundary, and the
 * backward sweep recomputes each segment's span states and fluxes (last
 * segment first) before running its adjoint spans; that is one extra forward
 * pass.  `group` problems share every launch (problem index in grid
 * dimension y) and the workspace (rswr_adjoint_batch_workspace_size) holds
 * one group; groups run one after another.  seg = 0 picks ceil(sqrt(spans)).
 * Device arrays: f_a, f_b [n_prob][src_ld] (src_ld >= n_steps+1),
 * grad_traces [n_prob][n_rec][n_steps], grad_f_a, grad_f_b
 * [n_prob][n_steps+1], grad_lambda [n_prob] (double).  rec_idx is host.
 * Errors: INVALID_ARG, NOMEM (workspace), UNSUPPORTED (plan), HIP. */
rswr_status_t rswr_adjoint_batch_workspace_size(rswr_plan_t plan, int64_t n_steps,
                                                int32_t n_rec, int32_t group, int32_t seg,
                                                size_t* bytes);
rswr_status_t rswr_solve_adjoint_batch(rswr_plan_t plan, int32_t n_prob, const void* f_a,
                                       const void* f_b, int64_t src_ld, int64_t n_steps,
                                       const int64_t* rec_idx, int32_t n_rec,
                                       const void* grad_traces, void* grad_f_a,
                                       void* grad_f_b, double* grad_lambda, int32_t group,
                                       int32_t seg, void* workspace, size_t ws_bytes,
                                       void* stream);

/* ---- Batched solve -------------------------------------------------------
 * Many independent problems (each with its own grid, windows, wave speed,
 * span, sources and length) advanced by the redo loop of Sec. 2.6 in one
 * recorded graph: round r runs span r of every problem that has one left,
 * one persistent launch per kernel shape walking all those problems' tiles.
 * Results are identical to rswr_solve of each problem alone (n0 = 0, no
 * receivers or checkpoints). */

/* (host) Groups n plans of one dtype.  Every plan must run the fused span
 * (rswr_plan_info_t.fused = 1; else UNSUPPORTED) and must outlive the batch;
 * each keeps its own kernel shape and span.  Errors: INVALID_ARG,
 * UNSUPPORTED, NOMEM. */
rswr_status_t rswr_batch_plan(const rswr_plan_t* plans, int32_t n,
                              rswr_batch_t* out);
rswr_status_t rswr_batch_destroy(rswr_batch_t batch);
/* Bytes of device workspace rswr_batch_solve needs: a second state buffer
 * per problem plus the launch tables. */
rswr_status_t rswr_batch_workspace_size(rswr_batch_t batch, size_t* bytes);
/* Advances problem i by n_steps[i] levels from level 0: states[i] (device,
 * [2][M_i], levels -1 and 0 on entry) is overwritten with levels
 * n_steps[i]-1 and n_steps[i]; f_a[i], f_b[i] (device, n_steps[i]+1
 * entries) are its boundary sources.  `states`, `f_a`, `f_b` and `n_steps`
 * are host arrays of n entries.  Calls with the same pointers and lengths
 * replay one recorded graph; the tables in the workspace are rewritten on
 * every call.  Problems must not share state buffers.  Errors: INVALID_ARG,
 * NOMEM (workspace too small), HIP. */
rswr_status_t rswr_batch_solve(rswr_batch_t batch, void* const* states,
                               const void* const* f_a, const void* const* f_b,
                               const int64_t* n_steps, void* workspace,
                               size_t ws_bytes, void* stream);

const char* rswr_status_string(rswr_status_t status);
const char* rswr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
