/*
 * rswr_oracle.h -- the CPU oracle of the RSWR hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing here is part of the product: only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or constant generator with the GPU
 * library.
 *
 * Method: Wei & Zhao, "A Non-iterative Overlapping Schwarz Waveform
 * Relaxation Algorithm for Wave Equation" (arXiv 2203.10477).
 *
 * Discrete reading (the paper fixes no grid, scheme or precision):
 *   nodes x_j = X_A + j dx, j = 0..M-1, dx = (X_B - X_A)/(M - 1);
 *   leapfrog U^{n+1}_j = (2 - 2 lam^2) U^n_j - U^{n-1}_j
 *                        + lam^2 (U^n_{j-1} + U^n_{j+1}),  lam = a dt/dx;
 *   floating-point order per node: s = ul + ur; t = fma(k, u, -u_old);
 *   u_new = fma(c2, s, t) with c2 = T(lam^2), k = T(2 - 2 lam^2) formed in
 *   double and rounded once;
 *   Dirichlet ends (Sec. 2.1, Eq. (3)): U^n_0 = f_A[n], U^n_{M-1} = f_B[n]
 *   for n >= 1; the zero initial condition (Eq. (2)) owns levels -1 and 0;
 *   centred flux F = (U_{o+1} - U_{o-1}) * r, r = T(1/(2dx)); a Neumann
 *   input at a right end b uses the ghost U_{b+1} = fma(q, F, U_{b-1}), at a
 *   left end U_{b-1} = fma(-q, F, U_{b+1}), q = T(2dx) (Sec. 2.2, Eqs.
 *   (6)-(7));
 *   interior point sources (the pulse sources of Sec. 4, u_tt = a^2 u_xx +
 *   s): the step from level n to n+1 adds amp[q][n] (the caller's samples of
 *   dt^2 s at node node[q]) to the updated value at node[q], after the
 *   leapfrog, sources in list order, in every window holding the node; the
 *   Dirichlet nodes 0 and M-1 take no source.
 *
 * Every real-valued function exists twice: suffix _f64 (double) and _f32
 * (float), compiled from the same source with -ffp-contract=off.
 * State arrays are [2][M]: row 0 holds level n0-1, row 1 level n0.
 * Flux arrays are [N-1][2][ld]: [i][0][s] is the output flux of window i at
 * lo_{i+1}, [i][1][s] that of window i+1 at hi_i, both at level n0+s.
 * Trace arrays are [n_rec][trace_ld]; the column for level L is
 * L - 1 - trace_level0 where trace_level0 is the start level of the run.
 */
#ifndef RSWR_ORACLE_H
#define RSWR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Layout of N overlapping windows (Sec. 2.2 Eqs. (4)-(5), Sec. 3).
 * Returns 0 on success, a negative code if the layout is invalid. */
int oracle_layout(int64_t M, int32_t N, int32_t P, int64_t* lo, int64_t* hi,
                  int64_t* own_lo, int64_t* own_hi);
/* Checks an explicit layout; fills the owned ranges (lowest index owns). */
int oracle_check_layout(int64_t M, int32_t N, const int64_t* lo,
                        const int64_t* hi, int64_t* own_lo, int64_t* own_hi);
/* Largest span (steps) for which every predicted output flux is exact: the
 * smallest distance between an input and an output boundary of one window.
 * Returns INT32_MAX for N = 1. */
int32_t oracle_span_cone(int32_t N, const int64_t* lo, const int64_t* hi);
/* Threads of the oracle's parallel loops from now on (n >= 1; n < 1 only
 * queries); returns the number in force. */
int oracle_threads(int n);
/* Waveform Time Span Theorem (Sec. 2.4, Eq. (10)) in steps: the largest S
 * with 2 S lam < P; exact integers when lam = num/den is given (num > 0). */
int32_t oracle_span_paper(int32_t P, double lam, int32_t num, int32_t den);

#define ORACLE_DECLARE(T, SUF)                                                 \
  void oracle_single##SUF(int64_t M, double lam, double dx, const T* fa,       \
                          const T* fb, int64_t n0, int64_t n_steps, T* state,  \
                          int32_t n_rec, const int64_t* rec, T* traces,        \
                          int64_t trace_ld, int32_t n_src,                     \
                          const int64_t* src_node, const T* src_amp,           \
                          int64_t src_ld);                                     \
  void oracle_predict##SUF(int64_t M, int32_t N, const int64_t* lo,            \
                           const int64_t* hi, double lam, double dx,           \
                           const T* fa, const T* fb, int64_t n0, int32_t Shat, \
                           const T* state, T* flux, int32_t ld, T* hist,       \
                           int32_t n_src, const int64_t* src_node,             \
                           const T* src_amp, int64_t src_ld);                  \
  void oracle_update##SUF(int64_t M, int32_t N, const int64_t* lo,             \
                          const int64_t* hi, const int64_t* own_lo,            \
                          const int64_t* own_hi, double lam, double dx,        \
                          const T* fa, const T* fb, int64_t n0, int32_t S,     \
                          const T* state_in, const T* flux, int32_t ld,        \
                          T* state_out, int32_t n_win_sel,                     \
                          const int32_t* win_sel, int32_t n_rec,               \
                          const int64_t* rec, T* traces, int64_t trace_ld,     \
                          int64_t trace_level0, int32_t n_src,                 \
                          const int64_t* src_node, const T* src_amp,           \
                          int64_t src_ld);                                     \
  int oracle_rswr##SUF(int64_t M, int32_t N, const int64_t* lo,                \
                       const int64_t* hi, const int64_t* own_lo,               \
                       const int64_t* own_hi, double lam, double dx,           \
                       const T* fa, const T* fb, int64_t n0, int64_t n_steps,  \
                       T* state, int32_t mode, int32_t S_fixed,                \
                       int32_t S_cone, int32_t tau_hat, double beta,           \
                       int32_t n_rec, const int64_t* rec, T* traces,           \
                       int64_t trace_ld, int32_t* spans, int32_t spans_cap,    \
                       int32_t n_src, const int64_t* src_node,                 \
                       const T* src_amp, int64_t src_ld);

ORACLE_DECLARE(double, _f64)
ORACLE_DECLARE(float, _f32)

/* oracle_rswr (FIXED span, from level 0, no receivers or sources) of n_prob
 * independent problems, spread over the threads; argument b of every array
 * belongs to problem b. */
#define ORACLE_DECLARE_MANY(T, SUF)                                            \
  void oracle_rswr_many##SUF(int32_t n_prob, const int64_t* M, const int32_t* N, \
                             const int64_t* const* lo, const int64_t* const* hi, \
                             const int64_t* const* own_lo,                     \
                             const int64_t* const* own_hi, const double* lam,  \
                             const double* dx, const T* const* fa,             \
                             const T* const* fb, const int64_t* n_steps,       \
                             const int32_t* S, T* const* state);

ORACLE_DECLARE_MANY(double, _f64)
ORACLE_DECLARE_MANY(float, _f32)

/* Reverse mode of oracle_single (same precision) from the zero initial
 * state, level 0, n_steps steps: given dJ/dtrace, returns dJ/df_A[n],
 * dJ/df_B[n] (n = 0..n_steps; entry 0 is 0 because the initial condition
 * owns level 0) and dJ/dlam, and (sum_abs, nullable) the sum of the
 * magnitudes of dJ/dlam's terms.  Forward states are kept every `ck` levels
 * and each segment is recomputed during the reverse sweep. */
#define ORACLE_DECLARE_ADJ(T, SUF)                                             \
  int oracle_adjoint##SUF(int64_t M, double lam, double dx, const T* fa,       \
                          const T* fb, int64_t n_steps, int32_t n_rec,         \
                          const int64_t* rec, const T* grad_traces,            \
                          int64_t trace_ld, int32_t ck, T* grad_fa,            \
                          T* grad_fb, double* grad_lam, double* sum_abs);

ORACLE_DECLARE_ADJ(double, _f64)
ORACLE_DECLARE_ADJ(float, _f32)

#ifdef __cplusplus
}
#endif
#endif
