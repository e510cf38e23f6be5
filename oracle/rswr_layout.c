/*
 * rswr_layout.c -- integer part of the CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Decomposition of Omega into N overlapping windows (Sec. 2.2, Eqs. (4)-(5);
 * Sec. 3 for N > 2) and the two span limits used by the select step.
 */
#include <stdint.h>
#include <stdlib.h>

#include "rswr_oracle.h"

/* Owned ranges follow the gluing rule of Sec. 2.5, Eq. (15): a node that two
 * windows share belongs to the lower-indexed one. */
static void owned_ranges(int64_t M, int32_t N, const int64_t* hi,
                         int64_t* own_lo, int64_t* own_hi) {
  for (int32_t i = 0; i < N; ++i) {
    own_lo[i] = (i == 0) ? 0 : hi[i - 1] + 1;
    own_hi[i] = (i == N - 1) ? M - 1 : hi[i];
  }
}

int oracle_check_layout(int64_t M, int32_t N, const int64_t* lo,
                        const int64_t* hi, int64_t* own_lo, int64_t* own_hi) {
  if (M < 3 || N < 1) return -1;
  if (lo[0] != 0 || hi[N - 1] != M - 1) return -2;
  for (int32_t i = 0; i < N; ++i)
    if (hi[i] - lo[i] < 2) return -3;
  for (int32_t i = 0; i + 1 < N; ++i) {
    /* X_{iA} < X_{(i+1)A} < X_{iB} < X_{(i+1)B}, Eq. (4) */
    if (!(lo[i] < lo[i + 1] && lo[i + 1] < hi[i] && hi[i] < hi[i + 1]))
      return -4;
    /* each output boundary is an interior node of the window that predicts
     * it, so its centred flux has both neighbours inside that window */
    if (!(lo[i + 1] - 1 >= lo[i] && lo[i + 1] + 1 <= hi[i])) return -5;
    if (!(hi[i] - 1 >= lo[i + 1] && hi[i] + 1 <= hi[i + 1])) return -5;
    /* an input boundary must not be a Dirichlet node */
    if (lo[i + 1] == 0 || hi[i] == M - 1) return -6;
  }
  owned_ranges(M, N, hi, own_lo, own_hi);
  for (int32_t i = 0; i < N; ++i)
    if (own_hi[i] < own_lo[i]) return -8;
  return 0;
}

int oracle_layout(int64_t M, int32_t N, int32_t P, int64_t* lo, int64_t* hi,
                  int64_t* own_lo, int64_t* own_hi) {
  if (M < 3 || N < 1) return -1;
  if (N > 1 && (P < 2 || (P % 2) != 0)) return -9;
  const int64_t h = P / 2;
  /* cores c_i = round(i (M-1) / N), rounding halves up */
  int64_t* c = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N + 1));
  if (!c) return -10;
  for (int32_t i = 0; i <= N; ++i)
    c[i] = (2 * (int64_t)i * (M - 1) + N) / (2 * (int64_t)N);
  int rc = 0;
  for (int32_t i = 0; i < N; ++i) {
    if (c[i + 1] - c[i] < 1) rc = -11;
    lo[i] = (i == 0) ? 0 : c[i] - h;
    hi[i] = (i == N - 1) ? M - 1 : c[i + 1] + h;
  }
  if (N > 1 && (c[1] - c[0] < h + 1 || c[N] - c[N - 1] < h + 1)) rc = -12;
  free(c);
  if (rc) return rc;
  return oracle_check_layout(M, N, lo, hi, own_lo, own_hi);
}

static int64_t dist(int64_t x, int64_t y) { return x > y ? x - y : y - x; }

int32_t oracle_span_cone(int32_t N, const int64_t* lo, const int64_t* hi) {
  /* For each window: inputs are lo_w (w > 0) and hi_w (w < N-1); outputs
   * are hi_{w-1} (w > 0) and lo_{w+1} (w < N-1).  A zero-flux error entering
   * at an input first changes the node itself one level later and then moves
   * one node per level, so an output at distance d keeps an exact centred
   * flux for d levels. */
  int64_t best = INT32_MAX;
  for (int32_t w = 0; w < N; ++w) {
    int64_t in[2], out[2];
    int ni = 0, no = 0;
    if (w > 0) { in[ni++] = lo[w]; out[no++] = hi[w - 1]; }
    if (w < N - 1) { in[ni++] = hi[w]; out[no++] = lo[w + 1]; }
    for (int a = 0; a < ni; ++a)
      for (int b = 0; b < no; ++b) {
        int64_t d = dist(in[a], out[b]);
        if (d < best) best = d;
      }
  }
  return (int32_t)best;
}

int32_t oracle_span_paper(int32_t P, double lam, int32_t num, int32_t den) {
  if (num > 0 && den > 0) {
    /* 2 S num/den < P  <=>  2 S num < P den  <=>  S <= (P den - 1) / (2 num) */
    int64_t s = ((int64_t)P * den - 1) / (2 * (int64_t)num);
    return (int32_t)s;
  }
  int64_t s = 0;
  while (2.0 * (double)(s + 1) * lam < (double)P) ++s;
  return (int32_t)s;
}

/* Threads the oracle's parallel loops use from now on (n >= 1); returns the
 * number in force.  For timing the oracle on one core or on all. */
#include <omp.h>
int oracle_threads(int n) {
  if (n >= 1) omp_set_num_threads(n);
  return omp_get_max_threads();
}
