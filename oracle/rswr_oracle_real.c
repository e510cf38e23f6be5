/*
 * rswr_oracle_real.c -- real-valued part of the CPU oracle of the RSWR hot
 * path.  TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the GPU library never does.
 *
 * Compiled twice with -ffp-contract=off: once as double (suffix _f64) and
 * once with -DORACLE_F32 as float (suffix _f32).  The discrete reading of
 * the paper that it follows is stated in rswr_oracle.h.
 *
 * Pins: tests/test_oracle_*.py check this file against d'Alembert's image
 * sum at Courant number 1, second-order convergence, discrete energy,
 * causality, mirror symmetry and linearity, "RSWR equals the single-domain
 * solve" for spans inside the light cone, a brute-force Jacobian for the
 * adjoint and central finite differences.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "rswr_oracle.h"

#ifdef ORACLE_F32
typedef float real;
#define SFX(name) name##_f32
#define FMA(a, b, c) fmaf((a), (b), (c))
#else
typedef double real;
#define SFX(name) name##_f64
#define FMA(a, b, c) fma((a), (b), (c))
#endif

typedef struct {
  real c2, k, r, q;
} coef_t;

/* Interior point sources (the pulse sources of Sec. 4): the step from level
 * n to n+1 adds amp[q*ld + n] to node node[q] after the leapfrog update, in
 * list order.  NULL or n == 0: no sources. */
typedef struct {
  int32_t n;
  const int64_t* node;
  const real* amp;
  int64_t ld;
} src_t;

/* Leapfrog and flux constants, formed in double and rounded once. */
static coef_t make_coef(double lam, double dx) {
  coef_t c;
  const double l2 = lam * lam;
  c.c2 = (real)l2;
  c.k = (real)(2.0 - 2.0 * l2);
  c.r = (real)(1.0 / (2.0 * dx));
  c.q = (real)(2.0 * dx);
  return c;
}

/* Second-order leapfrog for Eq. (1) at one node. */
static real leap(const coef_t* c, real ul, real u, real ur, real u_old) {
  const real s = ul + ur;
  const real t = FMA(c->k, u, -u_old);
  return FMA(c->c2, s, t);
}

/* Centred approximation of du/dx at local index i (the flux waveform of the
 * boundary output definitions in Sec. 2.2). */
static real flux_at(const coef_t* c, const real* u, int64_t i) {
  return (u[i + 1] - u[i - 1]) * c->r;
}

/*
 * One level of the sub-problem on the window [lo, hi] (Eqs. (6)-(7) for a
 * split window, Eq. (1)-(3) when the window is the whole domain).
 * Arrays are local (index i = j - lo): u_old = level n-1, u = level n; the
 * result (level n+1) goes to u_new.  Node 0 and node M-1 take the Dirichlet
 * data of Eq. (3); any other window end is a Neumann input whose flux at
 * level n is fin_l (left end) or fin_r (right end).
 */
static void window_step(const coef_t* c, int64_t M, int64_t lo, int64_t hi,
                        const real* u_old, const real* u, real* u_new,
                        real fin_l, real fin_r, real fa_next, real fb_next,
                        const src_t* src, int64_t level) {
  const int64_t n = hi - lo + 1;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t j = lo + i;
    if (j == 0) {
      u_new[i] = fa_next;
      continue;
    }
    if (j == M - 1) {
      u_new[i] = fb_next;
      continue;
    }
    const real ul = (i == 0) ? FMA(-c->q, fin_l, u[1]) : u[i - 1];
    const real ur = (i == n - 1) ? FMA(c->q, fin_r, u[n - 2]) : u[i + 1];
    u_new[i] = leap(c, ul, u[i], ur, u_old[i]);
  }
  /* sources of the PDE inside this window (every window holding the node
   * carries them); the Dirichlet nodes keep their data */
  if (src)
    for (int32_t q = 0; q < src->n; ++q) {
      const int64_t j = src->node[q];
      if (j >= lo && j <= hi && j > 0 && j < M - 1)
        u_new[j - lo] = u_new[j - lo] + src->amp[(int64_t)q * src->ld + level];
    }
}

static int64_t trace_col(int64_t level, int64_t level0) {
  return level - 1 - level0;
}

/* ------------------------------------------------------------------------ */
/* Single-domain solve: the "true solution" of Sec. 2.1 (Definition after   */
/* Eq. (3)) in the discrete reading.                                         */
/* ------------------------------------------------------------------------ */
void SFX(oracle_single)(int64_t M, double lam, double dx, const real* fa,
                        const real* fb, int64_t n0, int64_t n_steps,
                        real* state, int32_t n_rec, const int64_t* rec,
                        real* traces, int64_t trace_ld, int32_t n_src,
                        const int64_t* src_node, const real* src_amp,
                        int64_t src_ld) {
  const coef_t c = make_coef(lam, dx);
  const src_t src = {n_src, src_node, src_amp, src_ld};
  real* b0 = (real*)malloc(sizeof(real) * (size_t)M);
  real* b1 = (real*)malloc(sizeof(real) * (size_t)M);
  real* b2 = (real*)malloc(sizeof(real) * (size_t)M);
  memcpy(b0, state, sizeof(real) * (size_t)M);
  memcpy(b1, state + M, sizeof(real) * (size_t)M);
  for (int64_t s = 0; s < n_steps; ++s) {
    const int64_t n = n0 + s;
    window_step(&c, M, 0, M - 1, b0, b1, b2, 0, 0, fa[n + 1], fb[n + 1], &src, n);
    real* t = b0;
    b0 = b1;
    b1 = b2;
    b2 = t;
    for (int32_t r = 0; r < n_rec; ++r)
      traces[(int64_t)r * trace_ld + trace_col(n + 1, n0)] = b1[rec[r]];
  }
  memcpy(state, b0, sizeof(real) * (size_t)M);
  memcpy(state + M, b1, sizeof(real) * (size_t)M);
  free(b0);
  free(b1);
  free(b2);
}

/* ------------------------------------------------------------------------ */
/* Prediction (Sec. 2.3, Eqs. (8)-(9)): every window starts from the common  */
/* state, assumes zero input flux and runs Shat levels.  Its output fluxes    */
/* at levels n0..n0+Shat-1 are recorded.  When hist != NULL the predictive    */
/* solution on each overlap is kept for the literal selection of Sec. 2.4:   */
/* hist[((i*2 + side)*(Shat+1) + s)*hld + (j - lo[i+1])], side 0 = window i, */
/* side 1 = window i+1, s = 0..Shat.                                         */
/* ------------------------------------------------------------------------ */
static void predict_impl(int64_t M, int32_t N, const int64_t* lo,
                         const int64_t* hi, double lam, double dx,
                         const real* fa, const real* fb, int64_t n0,
                         int32_t Shat, const real* state, real* flux,
                         int32_t ld, real* hist, int64_t hld, const src_t* src) {
  const coef_t c = make_coef(lam, dx);
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t w = 0; w < N; ++w) {
    const int64_t nw = hi[w] - lo[w] + 1;
    real* b0 = (real*)malloc(sizeof(real) * (size_t)nw);
    real* b1 = (real*)malloc(sizeof(real) * (size_t)nw);
    real* b2 = (real*)malloc(sizeof(real) * (size_t)nw);
    memcpy(b0, state + lo[w], sizeof(real) * (size_t)nw);
    memcpy(b1, state + M + lo[w], sizeof(real) * (size_t)nw);
    for (int32_t s = 0; s <= Shat; ++s) {
      if (s < Shat) {
        if (w < N - 1)
          flux[(int64_t)(2 * w + 0) * ld + s] = flux_at(&c, b1, lo[w + 1] - lo[w]);
        if (w > 0)
          flux[(int64_t)(2 * (w - 1) + 1) * ld + s] =
              flux_at(&c, b1, hi[w - 1] - lo[w]);
      }
      if (hist) {
        if (w < N - 1)
          for (int64_t j = lo[w + 1]; j <= hi[w]; ++j)
            hist[((int64_t)(w * 2 + 0) * (Shat + 1) + s) * hld + (j - lo[w + 1])] =
                b1[j - lo[w]];
        if (w > 0)
          for (int64_t j = lo[w]; j <= hi[w - 1]; ++j)
            hist[((int64_t)((w - 1) * 2 + 1) * (Shat + 1) + s) * hld + (j - lo[w])] =
                b1[j - lo[w]];
      }
      if (s == Shat) break;
      const int64_t n = n0 + s;
      window_step(&c, M, lo[w], hi[w], b0, b1, b2, (real)0, (real)0, fa[n + 1],
                  fb[n + 1], src, n);
      real* t = b0;
      b0 = b1;
      b1 = b2;
      b2 = t;
    }
    free(b0);
    free(b1);
    free(b2);
  }
}

void SFX(oracle_predict)(int64_t M, int32_t N, const int64_t* lo,
                         const int64_t* hi, double lam, double dx,
                         const real* fa, const real* fb, int64_t n0,
                         int32_t Shat, const real* state, real* flux,
                         int32_t ld, real* hist, int32_t n_src,
                         const int64_t* src_node, const real* src_amp,
                         int64_t src_ld) {
  const src_t src = {n_src, src_node, src_amp, src_ld};
  int64_t hld = 1;
  for (int32_t i = 0; i + 1 < N; ++i)
    if (hi[i] - lo[i + 1] + 1 > hld) hld = hi[i] - lo[i + 1] + 1;
  predict_impl(M, N, lo, hi, lam, dx, fa, fb, n0, Shat, state, flux, ld, hist,
               hld, &src);
}

/* ------------------------------------------------------------------------ */
/* Update (Sec. 2.5, Eqs. (13)-(14)) and gluing (Eq. (15)): every window     */
/* re-runs S levels with the neighbours' predicted output fluxes as its      */
/* input fluxes and writes its owned range of the two newest levels.  Only  */
/* the windows listed in win_sel are processed when win_sel != NULL.        */
/* ------------------------------------------------------------------------ */
void SFX(oracle_update)(int64_t M, int32_t N, const int64_t* lo,
                        const int64_t* hi, const int64_t* own_lo,
                        const int64_t* own_hi, double lam, double dx,
                        const real* fa, const real* fb, int64_t n0, int32_t S,
                        const real* state_in, const real* flux, int32_t ld,
                        real* state_out, int32_t n_win_sel,
                        const int32_t* win_sel, int32_t n_rec,
                        const int64_t* rec, real* traces, int64_t trace_ld,
                        int64_t trace_level0, int32_t n_src,
                        const int64_t* src_node, const real* src_amp,
                        int64_t src_ld) {
  const coef_t c = make_coef(lam, dx);
  const src_t src = {n_src, src_node, src_amp, src_ld};
  const int32_t nsel = win_sel ? n_win_sel : N;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t ws = 0; ws < nsel; ++ws) {
    const int32_t w = win_sel ? win_sel[ws] : ws;
    const int64_t nw = hi[w] - lo[w] + 1;
    real* b0 = (real*)malloc(sizeof(real) * (size_t)nw);
    real* b1 = (real*)malloc(sizeof(real) * (size_t)nw);
    real* b2 = (real*)malloc(sizeof(real) * (size_t)nw);
    memcpy(b0, state_in + lo[w], sizeof(real) * (size_t)nw);
    memcpy(b1, state_in + M + lo[w], sizeof(real) * (size_t)nw);
    for (int32_t s = 0; s < S; ++s) {
      const int64_t n = n0 + s;
      /* corresponding waveforms (Sec. 2.2): the left input of window w is
       * fed by window w-1's output at lo_w, the right input by window w+1's
       * output at hi_w */
      const real fin_l = (w > 0) ? flux[(int64_t)(2 * (w - 1) + 0) * ld + s] : (real)0;
      const real fin_r = (w < N - 1) ? flux[(int64_t)(2 * w + 1) * ld + s] : (real)0;
      window_step(&c, M, lo[w], hi[w], b0, b1, b2, fin_l, fin_r, fa[n + 1],
                  fb[n + 1], &src, n);
      real* t = b0;
      b0 = b1;
      b1 = b2;
      b2 = t;
      for (int32_t r = 0; r < n_rec; ++r)
        if (rec[r] >= own_lo[w] && rec[r] <= own_hi[w])
          traces[(int64_t)r * trace_ld + trace_col(n + 1, trace_level0)] =
              b1[rec[r] - lo[w]];
    }
    for (int64_t j = own_lo[w]; j <= own_hi[w]; ++j) {
      state_out[j] = b0[j - lo[w]];
      state_out[M + j] = b1[j - lo[w]];
    }
    free(b0);
    free(b1);
    free(b2);
  }
}

/* ------------------------------------------------------------------------ */
/* The span loop (Sec. 2.6, Eqs. (16)-(17); Sec. 3 for N > 2).               */
/* mode 0 FIXED: S = min(S_fixed, remaining) every span.                     */
/* mode 1 QUIET: Shat_1 = tau_hat (S_cone when tau_hat = 0),               */
/*   Shat_k = ceil((1+beta) S_{k-1}) (Sec. 2.6); with q_b                    */
/*   the number of leading exact zeros of the predicted flux that feeds      */
/*   input b, S_k = min(Shat_k, min_b min(q_b, S_cone) + S_cone).            */
/* mode 2 PAPER: the literal rule of Sec. 2.4 (Definition of the maximum     */
/*   waveform time span) and Eq. (19): per interface the largest number of   */
/*   leading levels at which the two predictions agree exactly at some       */
/*   overlap node, minus one; the minimum over interfaces; Shat as QUIET.    */
/* Returns the number of spans; spans[k] holds S_k for k < spans_cap.        */
/* ------------------------------------------------------------------------ */
int SFX(oracle_rswr)(int64_t M, int32_t N, const int64_t* lo,
                     const int64_t* hi, const int64_t* own_lo,
                     const int64_t* own_hi, double lam, double dx,
                     const real* fa, const real* fb, int64_t n0,
                     int64_t n_steps, real* state, int32_t mode,
                     int32_t S_fixed, int32_t S_cone, int32_t tau_hat,
                     double beta, int32_t n_rec, const int64_t* rec,
                     real* traces, int64_t trace_ld, int32_t* spans,
                     int32_t spans_cap, int32_t n_src,
                     const int64_t* src_node, const real* src_amp,
                     int64_t src_ld) {
  const src_t src = {n_src, src_node, src_amp, src_ld};
  if (mode < 0 || mode > 2) return -1;
  if (mode == 0 && S_fixed < 1) return -2;
  int64_t hld = 1;
  for (int32_t i = 0; i + 1 < N; ++i)
    if (hi[i] - lo[i + 1] + 1 > hld) hld = hi[i] - lo[i + 1] + 1;
  real* other = (real*)malloc(sizeof(real) * 2 * (size_t)M);
  real* flux = NULL;
  real* hist = NULL;
  const int64_t level0 = n0;
  int64_t done = 0;
  int32_t k = 0, S_prev = 0;
  while (done < n_steps) {
    const int64_t rem = n_steps - done;
    int64_t shat;
    if (mode == 0)
      shat = S_fixed;
    else if (k == 0)
      shat = (tau_hat > 0) ? tau_hat : S_cone; /* tau-hat of Sec. 2.3 */
    else
      shat = (int64_t)ceil((1.0 + beta) * (double)S_prev);
    if (shat > rem) shat = rem;
    if (shat < 1) shat = 1;
    const int32_t Shat = (int32_t)shat;
    const int32_t ld = Shat;
    const int64_t nfl = (N > 1) ? (int64_t)(N - 1) * 2 * ld : 1;
    flux = (real*)realloc(flux, sizeof(real) * (size_t)nfl);
    if (mode == 2 && N > 1)
      hist = (real*)realloc(hist, sizeof(real) * (size_t)((int64_t)(N - 1) * 2 *
                                                          (Shat + 1) * hld));
    predict_impl(M, N, lo, hi, lam, dx, fa, fb, n0, Shat, state, flux, ld,
                 (mode == 2 && N > 1) ? hist : NULL, hld, &src);

    int64_t S = Shat;
    if (mode == 1 && N > 1) {
      int64_t qmin = INT64_MAX;
      for (int32_t i = 0; i + 1 < N; ++i)
        for (int side = 0; side < 2; ++side) {
          const real* f = flux + (int64_t)(2 * i + side) * ld;
          int64_t q = 0;
          while (q < Shat && f[q] == (real)0) ++q;
          if (q > S_cone) q = S_cone;
          if (q < qmin) qmin = q;
        }
      if (qmin + S_cone < S) S = qmin + S_cone;
    } else if (mode == 2 && N > 1) {
      int64_t gmin = INT64_MAX;
      for (int32_t i = 0; i + 1 < N; ++i) {
        const int64_t nov = hi[i] - lo[i + 1] + 1;
        int64_t best = 0;
        for (int64_t x = 0; x < nov; ++x) {
          int64_t m = 0;
          while (m <= Shat) {
            const real p1 = hist[((int64_t)(i * 2 + 0) * (Shat + 1) + m) * hld + x];
            const real p2 = hist[((int64_t)(i * 2 + 1) * (Shat + 1) + m) * hld + x];
            if (!(p1 == p2)) break;
            ++m;
          }
          if (m - 1 > best) best = m - 1;
        }
        if (best < gmin) gmin = best;
      }
      if (gmin < S) S = gmin;
      if (S < 1) S = 1;
    }

    SFX(oracle_update)(M, N, lo, hi, own_lo, own_hi, lam, dx, fa, fb, n0,
                       (int32_t)S, state, flux, ld, other, 0, NULL, n_rec, rec,
                       traces, trace_ld, level0, n_src, src_node, src_amp,
                       src_ld);
    memcpy(state, other, sizeof(real) * 2 * (size_t)M);
    if (k < spans_cap && spans) spans[k] = (int32_t)S;
    S_prev = (int32_t)S;
    n0 += S;
    done += S;
    ++k;
  }
  free(other);
  free(flux);
  free(hist);
  return k;
}

/* ------------------------------------------------------------------------ */
/* Many independent FIXED-span problems (a batch): oracle_rswr of each, the   */
/* problems spread over the threads (each problem's own loops then run on     */
/* one thread).  Problem b: M[b] nodes, N[b] windows lo[b]/hi[b]/own_lo[b]/   */
/* own_hi[b], lam[b], dx[b], span S[b], n_steps[b] levels from the state in  */
/* state[b] (level 0 start), sources fa[b], fb[b].                            */
/* ------------------------------------------------------------------------ */
void SFX(oracle_rswr_many)(int32_t n_prob, const int64_t* M, const int32_t* N,
                           const int64_t* const* lo, const int64_t* const* hi,
                           const int64_t* const* own_lo,
                           const int64_t* const* own_hi, const double* lam,
                           const double* dx, const real* const* fa,
                           const real* const* fb, const int64_t* n_steps,
                           const int32_t* S, real* const* state) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t b = 0; b < n_prob; ++b)
    SFX(oracle_rswr)(M[b], N[b], lo[b], hi[b], own_lo[b], own_hi[b], lam[b], dx[b],
                     fa[b], fb[b], 0, n_steps[b], state[b], 0, S[b], 0, 0, 0.1, 0,
                     NULL, NULL, 1, NULL, 0, 0, NULL, NULL, 0);
}

/* ------------------------------------------------------------------------ */
/* Reverse mode of the single-domain solve.  The forward map is the leapfrog */
/* of oracle_single from U^{-1} = U^0 = 0; the adjoint W^n = dJ/dU^n obeys,  */
/* on interior nodes,                                                        */
/*   W^n_j = g^n_j + k W^{n+1}_j + lam^2 (W^{n+1}_{j-1} + W^{n+1}_{j+1})      */
/*           - W^{n+2}_j,                                                    */
/* with W taken as zero on the two Dirichlet nodes and beyond level N_t,     */
/* g^n_j = dJ/dtrace at receivers on node j.  Then dJ/df_A[n] = g^n_0 +       */
/* lam^2 W^{n+1}_1, dJ/df_B[n] likewise at the right end, and                */
/* dJ/dlam = 2 lam sum_{n,j} W^n_j (U^{n-1}_{j-1} - 2 U^{n-1}_j + U^{n-1}_{j+1}).*/
/* W and the Laplacian are formed in the working precision (the pinned       */
/* per-node order); each product W * Lap and every sum is taken in double    */
/* (a float product is exact there), pairwise.  sum_abs (nullable) receives  */
/* 2 |lam| sum_{n,j} |W^n_j Lap_j|: the scale against which the rounding of  */
/* this long, cancelling sum is judged.                                      */
/* ------------------------------------------------------------------------ */
static double pairwise_sum(const double* x, int64_t n) {
  if (n <= 16) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += x[i];
    return s;
  }
  const int64_t h = n / 2;
  return pairwise_sum(x, h) + pairwise_sum(x + h, n - h);
}

int SFX(oracle_adjoint)(int64_t M, double lam, double dx, const real* fa,
                        const real* fb, int64_t n_steps, int32_t n_rec,
                        const int64_t* rec, const real* grad_traces,
                        int64_t trace_ld, int32_t ck, real* grad_fa,
                        real* grad_fb, double* grad_lam, double* sum_abs) {
  if (ck < 1 || M < 3) return -1;
  for (int32_t r = 0; r < n_rec; ++r)
    if (rec[r] < 0 || rec[r] > M - 1) return -3;
  const coef_t c = make_coef(lam, dx);
  const int64_t nck = n_steps / ck + 1;
  /* checkpoint m holds levels m*ck - 1 and m*ck */
  real* ckpt = (real*)calloc((size_t)(nck * 2 * M), sizeof(real));
  real* seg = (real*)malloc(sizeof(real) * (size_t)((ck + 1) * M));
  real* w0 = (real*)calloc((size_t)M, sizeof(real)); /* W^{n+2} */
  real* w1 = (real*)calloc((size_t)M, sizeof(real)); /* W^{n+1} */
  real* w2 = (real*)calloc((size_t)M, sizeof(real)); /* W^n */
  double* term = (double*)malloc(sizeof(double) * (size_t)M);
  double* aterm = (double*)malloc(sizeof(double) * (size_t)M);
  double* lev_sum = (double*)calloc((size_t)(n_steps + 1), sizeof(double));
  double* lev_abs = (double*)calloc((size_t)(n_steps + 1), sizeof(double));
  if (!ckpt || !seg || !w0 || !w1 || !w2 || !term || !aterm || !lev_sum || !lev_abs)
    return -2;

  /* forward sweep storing checkpoints */
  {
    real* b0 = (real*)calloc((size_t)M, sizeof(real));
    real* b1 = (real*)calloc((size_t)M, sizeof(real));
    real* b2 = (real*)calloc((size_t)M, sizeof(real));
    for (int64_t n = 0; n < n_steps; ++n) {
      if (n % ck == 0) {
        memcpy(ckpt + (n / ck) * 2 * M, b0, sizeof(real) * (size_t)M);
        memcpy(ckpt + (n / ck) * 2 * M + M, b1, sizeof(real) * (size_t)M);
      }
      window_step(&c, M, 0, M - 1, b0, b1, b2, 0, 0, fa[n + 1], fb[n + 1], NULL, n);
      real* t = b0;
      b0 = b1;
      b1 = b2;
      b2 = t;
    }
    free(b0);
    free(b1);
    free(b2);
  }

  grad_fa[0] = 0;
  grad_fb[0] = 0;
  int64_t seg_base = -1; /* level held by seg[1] */
  for (int64_t n = n_steps; n >= 1; --n) {
    /* W^n from W^{n+1} (w1) and W^{n+2} (w0) */
    for (int64_t j = 1; j <= M - 2; ++j) {
      const real wl = (j - 1 >= 1) ? w1[j - 1] : (real)0;
      const real wr = (j + 1 <= M - 2) ? w1[j + 1] : (real)0;
      w2[j] = leap(&c, wl, w1[j], wr, w0[j]);
    }
    w2[0] = 0;
    w2[M - 1] = 0;
    real ga = c.c2 * w1[1];
    real gb = c.c2 * w1[M - 2];
    for (int32_t r = 0; r < n_rec; ++r) {
      const real g = grad_traces[(int64_t)r * trace_ld + (n - 1)];
      const int64_t j = rec[r];
      if (j == 0)
        ga = ga + g;
      else if (j == M - 1)
        gb = gb + g;
      else
        w2[j] = w2[j] + g;
    }
    grad_fa[n] = ga;
    grad_fb[n] = gb;

    /* dJ/dlam term of the step n-1 -> n: W^n . Lap(U^{n-1}) */
    const int64_t m = n - 1;
    const int64_t cidx = m / ck;
    if (seg_base < 0 || cidx * ck != seg_base) {
      seg_base = cidx * ck;
      memcpy(seg, ckpt + cidx * 2 * M, sizeof(real) * 2 * (size_t)M);
      const int64_t top = (seg_base + ck - 1 < n_steps) ? seg_base + ck - 1 : n_steps;
      for (int64_t L = seg_base; L < top; ++L) {
        const int64_t t = L - seg_base + 1; /* seg[t] = U^L */
        window_step(&c, M, 0, M - 1, seg + (t - 1) * M, seg + t * M,
                    seg + (t + 1) * M, 0, 0, fa[L + 1], fb[L + 1], NULL, L);
      }
    }
    const real* U = seg + (m - seg_base + 1) * M;
    term[0] = term[M - 1] = 0.0;
    aterm[0] = aterm[M - 1] = 0.0;
    for (int64_t j = 1; j <= M - 2; ++j) {
      const real lap = (U[j - 1] + U[j + 1]) - (real)2 * U[j];
      term[j] = (double)w2[j] * (double)lap;
      aterm[j] = fabs(term[j]);
    }
    lev_sum[n] = pairwise_sum(term, M);
    lev_abs[n] = pairwise_sum(aterm, M);

    real* t = w0;
    w0 = w1;
    w1 = w2;
    w2 = t;
  }
  *grad_lam = 2.0 * lam * pairwise_sum(lev_sum, n_steps + 1);
  if (sum_abs) *sum_abs = 2.0 * fabs(lam) * pairwise_sum(lev_abs, n_steps + 1);
  free(ckpt);
  free(seg);
  free(w0);
  free(w1);
  free(w2);
  free(term);
  free(aterm);
  free(lev_sum);
  free(lev_abs);
  return 0;
}
