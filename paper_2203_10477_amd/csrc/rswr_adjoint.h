// rswr_adjoint.h -- device code of the adjoint of the RSWR solve (the
// adjoint predict frame and the adjoint update kernel; launchers and the
// other kernels in rswr_adjoint.hip).
//
// Misfit J = sum_r sum_n (U^n[j_r] - d_r^n)^2; its reverse mode (the
// transposed leapfrog) is W^n_j = g^n_j + k W^{n+1}_j - W^{n+2}_j +
// c2 (W^{n+1}_{j-1} + W^{n+1}_{j+1}) on interior nodes, W = 0 on the two
// Dirichlet nodes, g = dJ/dtrace on receiver nodes.  It is the same
// self-adjoint wave equation run backward in time with point sources, so
// each span of it is advanced with the method's own predict / update
// exchange (Sec. 2.3-2.5 of Wei & Zhao, arXiv 2203.10477) on the forward
// plan's windows.  dJ/df_A[n] = c2 W^{n+1}_1 (+ g^n_0), and
// dJ/dlam = 2 lam sum_n sum_j W^n_j (U^{n-1}_{j-1} - 2 U^{n-1}_j + U^{n-1}_{j+1});
// the forward field is rebuilt span by span by running the leapfrog
// backward from the span-end checkpoint (it is time-reversible), with the
// stored forward flux waveforms as ghost data.
#pragma once

#include <type_traits>

#include "rswr_device.h"

namespace rswr {

// ---------------------------------------------------------------------------
// Adjoint predict: W's flux at each output node over shat levels, zero input
// flux at the window's own inputs, receiver sources injected in receiver
// order after each level (the order the single-domain reverse sweep uses).
// One wave per (interface, side) carries a 128-node frame around the output
// node o, two nodes per lane, in registers: the sample at o over shat <=
// light-cone-limit levels reads only [o-shat, o+shat] (the window's input
// ends lie farther away), so the frame runs the plain stencil with the data
// mirrored into the window, W = 0 on nodes 0 and M-1, and the sources of
// [o-shat, o+shat] inside the window: the same samples as the whole-window
// prediction, bit for bit.  Each source's samples for the span sit one per
// lane (kAdjFrameSrc of them in registers, further ones read each step).
// ---------------------------------------------------------------------------
constexpr int kAdjFrameSrc = 8;
// Frame receivers a wave of the fused update holds in registers.
constexpr int kAdjFuseSrc = 2;


// Problem blockIdx.y of a same-shape batch (YStrides); the arguments as they
// are for a single problem.
template <typename T>
__device__ __forceinline__ AdjPredictArgs<T> batch_problem(const AdjPredictArgs<T>& a) {
  AdjPredictArgs<T> p = a;
  if (a.ys.ny > 1) {
    p.w = at_y(a.w, a.ys.ws);
    p.flux = at_y(a.flux, a.ys.ws);
    p.gtr = at_y(a.gtr, a.ys.gtr);
  }
  return p;
}

template <typename T>
__device__ __forceinline__ AdjUpdateArgs<T> batch_problem(const AdjUpdateArgs<T>& a) {
  AdjUpdateArgs<T> p = a;
  if (a.ys.ny > 1) {
    p.w_in = at_y(a.w_in, a.ys.ws);
    p.w_out = at_y(a.w_out, a.ys.ws);
    p.u_end = at_y(a.u_end, a.ys.ws);
    p.u_beg = at_y(a.u_beg, a.ys.ws);
    p.ffl = at_y(a.ffl, a.ys.ws);
    p.afl = at_y(a.afl, a.ys.ws);
    p.lam_part = at_y(a.lam_part, a.ys.ws);
    p.fa = at_y(a.fa, a.ys.src);
    p.fb = at_y(a.fb, a.ys.src);
    p.gtr = at_y(a.gtr, a.ys.gtr);
    p.grad_fa = at_y(a.grad_fa, a.ys.grad);
    p.grad_fb = at_y(a.grad_fb, a.ys.grad);
  }
  return p;
}

inline unsigned ny(const YStrides& y) { return y.ny > 1 ? static_cast<unsigned>(y.ny) : 1u; }

// W's frame around output node o of window `win`, used by the predict
// kernel (one wave per interface side) and by the fused update (the wave
// holding a tile's input end): lane l holds nodes base + 2l + e, base =
// o - kFrameHalf, mirrored into the window; W = 0 on nodes 0 and M-1; the
// receivers of [o - shat, o + shat] inside the window add their dJ/dtrace
// samples after each level in receiver order: the first NS from registers
// (lane s: level n_e - s), the rest read each step.
template <typename T, int NS>
struct AdjFrame {
  bool dir[2];  // element e is node 0 or M-1 (W = 0)
  int nsrc, first_extra;
  int64_t A, B, base;
  int sx[NS];
  T sg[NS];
};

template <typename T, int NS>
__device__ __forceinline__ void adj_frame_load(const T* w, const int64_t* lo,
                                               const int64_t* hi, const int64_t* rec_node,
                                               int n_rec, const T* gtr, int64_t gtr_ld,
                                               int64_t M, int64_t n_e, int64_t o, int win,
                                               int shat, int lane, T (&cur)[2], T (&old)[2],
                                               AdjFrame<T, NS>& f) {
  const int64_t wlo = lo[win], whi = hi[win];
  f.A = (o - shat > wlo) ? o - shat : wlo;
  f.B = (o + shat < whi) ? o + shat : whi;
  f.base = o - kFrameHalf;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int64_t x = f.base + 2 * lane + e;
    int64_t j = (x < wlo) ? 2 * wlo - x : ((x > whi) ? 2 * whi - x : x);
    j = j < wlo ? wlo : (j > whi ? whi : j);
    cur[e] = w[M + j];
    old[e] = w[j];
    f.dir[e] = (x == 0) || (x == M - 1);
  }
  // sources in [A, B] (interior nodes), in receiver order: frame offset and
  // the span's samples (lane s: level n_e - s, column n_e - s - 1); 64
  // receivers checked at once, one per lane, the hits taken in order
  f.nsrc = 0;
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    f.sx[q] = 0;
    f.sg[q] = T(0);
  }
  f.first_extra = n_rec;
  for (int r0 = 0; r0 < n_rec && f.first_extra == n_rec; r0 += 64) {
    const int r = r0 + lane;
    const int64_t j = (r < n_rec) ? rec_node[r] : int64_t(-1);
    const bool hit = j > 0 && j < M - 1 && j >= f.A && j <= f.B;
    uint64_t m = __ballot(hit);
    while (m != 0) {
      const int b = __builtin_ctzll(m);
      m &= m - 1;
      if (f.nsrc == NS) {
        f.first_extra = r0 + b;
        break;
      }
      const int x = __builtin_amdgcn_readlane(static_cast<int>(j - f.base), b);
      const T* g = gtr + static_cast<int64_t>(r0 + b) * gtr_ld + (n_e - 1);
      const T gs = (lane < shat) ? g[-lane] : T(0);
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        if (q == f.nsrc) {
          f.sx[q] = x;
          f.sg[q] = gs;
        }
      }
      ++f.nsrc;
    }
  }
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    cur[e] = in_vgpr(cur[e]);
    old[e] = in_vgpr(old[e]);
  }
#pragma unroll
  for (int q = 0; q < NS; ++q) f.sg[q] = in_vgpr(f.sg[q]);
}

// Step s of the frame (cur = W^{L+1}, old = W^{L+2}, L = n_e - s): returns
// the centred flux at o (wave-uniform); if `adv`, writes W^L over old with
// the sources held in registers added; adj_frame_extra then adds the rest.
// The register sources of the fused update (NS = kAdjFuseSrc) are added by
// selects only, so a step of the frame is straight-line code that the
// compiler can interleave with the tile's own step.
template <typename T, int NS>
__device__ __forceinline__ T adj_frame_step(const T (&cur)[2], T (&old)[2],
                                            const AdjFrame<T, NS>& f, T c2, T k, T r, int s,
                                            int lane, bool adv) {
  const T l1 = lane_shift_z<kWaveShr1>(cur[1]);
  const T r0 = lane_shift_z<kWaveShl1>(cur[0]);
  const T F = rd_lane((cur[1] - l1) * r, kFrameHalf / 2);
  if (adv) {
    T n0 = leap(c2, k, l1, cur[0], cur[1], old[0]);
    T n1 = leap(c2, k, cur[0], cur[1], r0, old[1]);
    n0 = f.dir[0] ? T(0) : n0;
    n1 = f.dir[1] ? T(0) : n1;
    const int ns = NS > kAdjFuseSrc ? uni(f.nsrc) : f.nsrc;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      if (NS <= kAdjFuseSrc || q < ns) {
        // the source's lane for each of the two elements (-1: none)
        const T g = rd_lane(f.sg[q], s);
        const int x = f.sx[q];
        const int t1 = (q < ns && (x & 1)) ? (x >> 1) : -1;
        const int t0 = (q < ns && !(x & 1)) ? (x >> 1) : -1;
        n1 = (lane == t1) ? n1 + g : n1;
        n0 = (lane == t0) ? n0 + g : n0;
      }
    }
    old[0] = n0;
    old[1] = n1;
  }
  return F;
}

// The frame's sources beyond those in registers, read from memory and added
// to W^L (in old) in receiver order after a step of adj_frame_step.
template <typename T, int NS>
__device__ __forceinline__ void adj_frame_extra(T (&old)[2], const AdjFrame<T, NS>& f,
                                                const int64_t* rec_node, int n_rec,
                                                const T* gtr, int64_t gtr_ld, int64_t M,
                                                int64_t n_e, int s, int lane) {
  if (uni(f.first_extra) < n_rec) {
    const int64_t L = n_e - s;  // level just computed
    T n0 = old[0], n1 = old[1];
    for (int r = f.first_extra; r < n_rec; ++r) {
      const int64_t j = rec_node[r];
      if (j > 0 && j < M - 1 && j >= f.A && j <= f.B) {
        const T g = gtr[static_cast<int64_t>(r) * gtr_ld + (L - 1)];
        const int x = static_cast<int>(j - f.base);
        if (x & 1)
          n1 = (lane == (x >> 1)) ? n1 + g : n1;
        else
          n0 = (lane == (x >> 1)) ? n0 + g : n0;
      }
    }
    old[0] = n0;
    old[1] = n1;
  }
}

// ---------------------------------------------------------------------------
// Adjoint update.  Per lane MPT consecutive nodes of four register arrays:
// W^{L+1}, W^{L+2} (adjoint) and U^{L-1}, U^L (forward, rebuilt backward).
// One step: exchange lane-end values (DPP inside a wave, LDS across waves),
// W^L by the leapfrog (+ sources, general tiles), the dJ/dlam terms of the
// stored interior nodes, then U^{L-2} by the reversed leapfrog.
// ---------------------------------------------------------------------------
// A lane's counted elements (stored interior nodes, whose dJ/dlam terms
// count): one run lo .. lo + n - 1 of its MPT consecutive nodes, since the
// nodes counted are those of the intersection of two node ranges.  On long
// rows the test is made per step on values re-read through an empty asm
// statement: a mask per element hoisted out of the step loop would need a
// register pair each (with 33 nodes per lane, more than the scalar file
// holds); short rows keep the hoisted masks.
struct ElemRun {
  int lo, n;
};

// The first kRecSlots sources [b, e) of a tile's list: the loads go out
// together (indices clamped into the list), one wait for all.
__device__ __forceinline__ RecSlots adj_slots(const int64_t* node, const int32_t* id, int b,
                                              int e) {
  RecSlots r;
  r.n = (e - b < kRecSlots) ? e - b : kRecSlots;
#pragma unroll
  for (int q = 0; q < kRecSlots; ++q) {
    r.node[q] = kNoNode;
    r.id[q] = 0;
  }
  if (r.n > 0) {
#pragma unroll
    for (int q = 0; q < kRecSlots; ++q) {
      const int i = b + (q < r.n ? q : r.n - 1);
      const int64_t nd = node[i];
      const int32_t d = id[i];
      r.node[q] = q < r.n ? nd : kNoNode;
      r.id[q] = q < r.n ? d : 0;
    }
  }
  return r;
}

// A load through a global (not generic) address: it counts only against
// the vector memory counter, so waits for scalar loads do not wait for it.
template <typename T>
__device__ __forceinline__ T gload(const T* ptr) {
  typedef const __attribute__((address_space(1))) T* GPtr;
  return *(GPtr)(ptr);
}

template <typename T, int NT, int MPT>
struct AdjCtx {
  T (*edge)[4][NT / 64];
  const T* sRw;
  const T* sLw;
  const T* sRu;
  const T* sLu;
  const T* sAu;
  const T* sBu;
  int64_t base;
  int dl, d0, dM, d1, dM2;
  int sb, se, lane, wv, lmode, rmode;
  ElemRun cnt;  // elements stored and interior (enter dJ/dlam)
  bool gen, wr_fa, wr_fb;
  RecSlots rs;          // the tile's first sources (GEN, SRC)
  const T (*sg)[kMaxSpan];  // their dJ/dtrace samples of this span, by step
  // SRC, all wave-uniform: the slot sources' wave, lane and element, and
  // those of nodes 1 and M-2 (index 0 / 1; wave -1: not in this tile)
  int swv[kRecSlots], slane[kRecSlots], selem[kRecSlots];
  int gwv[2], glane[2], gelem[2];
  // fused update (span <= 64): lane s holds sample s of the forward flux at
  // the left / right input and of nodes 0 / M-1 (the staged rows, read with
  // readlane); wvu: the wave index as a scalar
  T vLu, vRu, vAu, vBu;
  int wvu;
  // fused update of short rows: the slot sources' dJ/dtrace samples (lane
  // s: step s) and the element each lane adds them to (-1: none)
  T vsg[kRecSlots];
  int vse[kRecSlots];
};

// W (or a reversed U) one level: old <- leap(cur) with the general tile's
// treatments (ghost at element dl, Dirichlet value at d0 / dM).
template <typename T, int MPT, bool GEN>
__device__ __forceinline__ void adj_chunk(const T (&cur)[MPT], T (&old)[MPT], T L,
                                          T R, T c2, T k, int dl, int d0, int dM,
                                          T ghost, T pin0, T pinM) {
#pragma unroll
  for (int e = 0; e < MPT; ++e) {
    T ul = (e == 0) ? L : cur[e - 1];
    const T ur = (e == MPT - 1) ? R : cur[e + 1];
    if (GEN) ul = (e == dl) ? ghost : ul;
    T v = leap(c2, k, ul, cur[e], ur, old[e]);
    if (GEN) {
      v = (e == d0) ? pin0 : v;
      v = (e == dM) ? pinM : v;
    }
    old[e] = v;
  }
}

// dJ/dlam terms W^L_j (U_{j-1} + U_{j+1} - 2 U_j) of the counted elements,
// accumulated in double (FP32: a step's terms of this lane summed in FP32,
// at most MPT of them, then added in double); then (if rev) U^{L-2} into
// uold.
template <typename T, int MPT, bool GEN>
__device__ __forceinline__ void lap_and_reverse(const T (&wn)[MPT], const T (&ucur)[MPT],
                                                T (&uold)[MPT], T L, T R, T c2, T k,
                                                int dl, int d0, int dM, T ghost, T pin0,
                                                T pinM, const ElemRun& cnt, bool rev,
                                                double& acc) {
  T step = T(0);
  int clo = cnt.lo, cn = cnt.n;
  if constexpr (MPT * sizeof(T) > 64) asm volatile("" : "+v"(clo), "+v"(cn));
#pragma unroll
  for (int e = 0; e < MPT; ++e) {
    T ul = (e == 0) ? L : ucur[e - 1];
    const T ur = (e == MPT - 1) ? R : ucur[e + 1];
    if (GEN) ul = (e == dl) ? ghost : ul;
    const T s = ul + ur;
    // s - 2u in one rounding: 2u is exact, so the fused form rounds the same
    const T lap = fma_(T(-2), ucur[e], s);
    const bool counted = static_cast<unsigned>(e - clo) < static_cast<unsigned>(cn);
    const T lapm = counted ? lap : T(0);
    if constexpr (sizeof(T) == 4)
      step = fma_(wn[e], lapm, step);
    else
      acc = __builtin_fma(static_cast<double>(wn[e]), static_cast<double>(lapm), acc);
    if (rev) {
      T v = fma_(c2, s, fma_(k, ucur[e], -uold[e]));
      if (GEN) {
        v = (e == d0) ? pin0 : v;
        v = (e == dM) ? pinM : v;
      }
      uold[e] = v;
    }
  }
  if constexpr (sizeof(T) == 4) acc += static_cast<double>(step);
}

// GEN: general tiles (per-element treatments at the window's own ends).
// SRC: plain tiles holding sources or storing nodes 1 / M-2.  Both inject
// the sources and write dJ/df; neither: the plain step.
// FR: fused update; fwL / fwR are this step's samples of the W frames the
// wave carries (used only by a wave whose region end is an input ghost).
// ENDS >= 0: which of those frames the wave carries (bit 0 left, bit 1
// right) is fixed at compile time; -1: read from the tile's end modes.
// REV >= 0: whether the step rebuilds U^{L-2} (1) or not (0, the span's
// last step), fixed at compile time; -1: from tau.
template <typename T, int NT, int MPT, bool GEN, bool SRC, bool FR, int ENDS = -1,
          int REV = -1>
__device__ __forceinline__ void adj_step(const AdjUpdateArgs<T>& p,
                                         const AdjCtx<T, NT, MPT>& c,
                                         const T (&wc)[MPT], T (&wp)[MPT],
                                         const T (&uc)[MPT], T (&up)[MPT], T (&gf)[2],
                                         int tau, int S, double& acc, T fwL, T fwR) {
  constexpr int NW = NT / 64;
  const int par = tau & 1;
  const int64_t L = p.n_e - tau;  // adjoint level computed now
  const int mi = S - 1 - tau;     // sample of the forward level m = L-1
  T Lw, Rw, Lu, Ru;
  if constexpr (FR) {
    // the neighbours of lane 0 and lane 63, computed on every lane (the
    // branches are wave-uniform) and put in place by the lane shifts
    if constexpr (NW > 1) {
      if (c.lane == 63) {
        c.edge[par][1][c.wvu] = wc[MPT - 1];
        c.edge[par][3][c.wvu] = uc[MPT - 1];
      }
      if (c.lane == 0) {
        c.edge[par][0][c.wvu] = wc[0];
        c.edge[par][2][c.wvu] = uc[0];
      }
      __syncthreads();
    }
    // a wave at the tile's left (right) end carries that end's frame
    // exactly when the end is an input ghost, so with ENDS fixed only the
    // Dirichlet case is left to test
    T Lw0, Lu0, Rw0, Ru0;
    if (NW > 1 && c.wvu > 0) {
      Lw0 = c.edge[par][1][c.wvu - 1];
      Lu0 = c.edge[par][3][c.wvu - 1];
    } else {
      const int m = uni(c.lmode);
      Lw0 = T(0);
      Lu0 = T(0);
      if ((ENDS >= 0) ? (ENDS & 1) != 0 : m == kEndGhost) {
        Lw0 = fma_(-p.q, fwL, wc[1]);
        Lu0 = fma_(-p.q, rd_lane(c.vLu, mi), uc[1]);
      } else if (ENDS >= 0) {
        const T d = rd_lane(c.vAu, mi);
        Lu0 = (m == kEndDirichlet) ? d : T(0);
      } else if (m == kEndDirichlet) {
        Lu0 = rd_lane(c.vAu, mi);
      }
    }
    if (NW > 1 && c.wvu < NW - 1) {
      Rw0 = c.edge[par][0][c.wvu + 1];
      Ru0 = c.edge[par][2][c.wvu + 1];
    } else {
      const int m = uni(c.rmode);
      Rw0 = T(0);
      Ru0 = T(0);
      if ((ENDS >= 0) ? (ENDS & 2) != 0 : m == kEndGhost) {
        Rw0 = fma_(p.q, fwR, wc[MPT - 2]);
        Ru0 = fma_(p.q, rd_lane(c.vRu, mi), uc[MPT - 2]);
      } else if (ENDS >= 0) {
        const T d = rd_lane(c.vBu, mi);
        Ru0 = (m == kEndDirichlet) ? d : T(0);
      } else if (m == kEndDirichlet) {
        Ru0 = rd_lane(c.vBu, mi);
      }
    }
    Lw = lane_shift_old<kWaveShr1>(Lw0, wc[MPT - 1]);
    Rw = lane_shift_old<kWaveShl1>(Rw0, wc[0]);
    Lu = lane_shift_old<kWaveShr1>(Lu0, uc[MPT - 1]);
    Ru = lane_shift_old<kWaveShl1>(Ru0, uc[0]);
  } else {
    Lw = lane_shift<kWaveShr1>(wc[MPT - 1]);
    Rw = lane_shift<kWaveShl1>(wc[0]);
    Lu = lane_shift<kWaveShr1>(uc[MPT - 1]);
    Ru = lane_shift<kWaveShl1>(uc[0]);
    if constexpr (NW > 1) {
      if (c.lane == 63) {
        c.edge[par][1][c.wv] = wc[MPT - 1];
        c.edge[par][3][c.wv] = uc[MPT - 1];
      }
      if (c.lane == 0) {
        c.edge[par][0][c.wv] = wc[0];
        c.edge[par][2][c.wv] = uc[0];
      }
      __syncthreads();
    }
    if (c.lane == 0) {
      if (c.wv > 0) {
        Lw = c.edge[par][1][c.wv - 1];
        Lu = c.edge[par][3][c.wv - 1];
      } else {
        Lw = end_value(c.lmode, fma_(-p.q, c.sLw[tau], wc[1]), T(0));
        Lu = end_value(c.lmode, fma_(-p.q, c.sLu[mi], uc[1]), c.sAu[mi]);
      }
    }
    if (c.lane == 63) {
      if (c.wv < NW - 1) {
        Rw = c.edge[par][0][c.wv + 1];
        Ru = c.edge[par][2][c.wv + 1];
      } else {
        Rw = end_value(c.rmode, fma_(p.q, c.sRw[tau], wc[MPT - 2]), T(0));
        Ru = end_value(c.rmode, fma_(p.q, c.sRu[mi], uc[MPT - 2]), c.sBu[mi]);
      }
    }
  }
  // dJ/df at level L from W^{L+1} next to the Dirichlet nodes
  if (GEN) {
    if (c.wr_fa && c.d1 >= 0 && c.d1 < MPT) p.grad_fa[L] = p.c2 * pick<T, MPT>(wc, c.d1);
    if (c.wr_fb && c.dM2 >= 0 && c.dM2 < MPT) p.grad_fb[L] = p.c2 * pick<T, MPT>(wc, c.dM2);
  } else if (SRC) {  // into lane tau of gf, stored after the loop
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      if (c.gwv[g] == c.wvu) {
        const T x = rd_lane(elem_at(wc, c.gelem[g]), c.glane[g]);
        gf[g] = wr_lane(p.c2 * x, tau, gf[g], c.lane);
      }
    }
  }
  const bool rev = REV >= 0 ? REV != 0 : tau < S - 1;
  if (GEN && c.gen) {
    const int rn = c.dl + 1;
    const T rw = (rn == MPT) ? Rw : pick<T, MPT>(wc, rn);
    const T gw = fma_(-p.q, c.sLw[tau], rw);
    adj_chunk<T, MPT, true>(wc, wp, Lw, Rw, p.c2, p.k, c.dl, c.d0, c.dM, gw, T(0), T(0));
  } else {
    adj_chunk<T, MPT, false>(wc, wp, Lw, Rw, p.c2, p.k, 0, 0, 0, T(0), T(0), T(0));
  }
  if (GEN || SRC) {
    // receiver sources in list order: the slots (samples staged in LDS),
    // then any further ones from memory
    auto inject = [&](int64_t node, T g) {
      const int64_t d = node - c.base;
      if (d >= 0 && d < MPT) {
#pragma unroll
        for (int e = 0; e < MPT; ++e) wp[e] = (d == e) ? wp[e] + g : wp[e];
      }
    };
#pragma unroll
    for (int q = 0; q < kRecSlots; ++q) {
      if (GEN) {
        if (q < c.rs.n) inject(c.rs.node[q], c.sg[q][tau]);
      } else if (q < c.rs.n && c.swv[q] == c.wvu) {
        if constexpr (FR && MPT * sizeof(T) <= 32) {
          // short rows (fused update): the sample from a lane, a compare per
          // element, no select over the array to fetch and put back the one
          // element
          const T g = rd_lane(c.vsg[q], tau);
#pragma unroll
          for (int e = 0; e < MPT; ++e) wp[e] = (c.vse[q] == e) ? wp[e] + g : wp[e];
        } else {
          add_at(wp, c.selem[q], c.sg[q][tau], c.lane == c.slane[q]);
        }
      }
    }
    for (int r = c.sb + kRecSlots; r < c.se; ++r)
      inject(p.src_node[r], p.gtr[static_cast<int64_t>(p.src_id[r]) * p.gtr_ld + (L - 1)]);
  }
  if (GEN && c.gen) {
    const int rn = c.dl + 1;
    const T ru = (rn == MPT) ? Ru : pick<T, MPT>(uc, rn);
    const T gu = fma_(-p.q, c.sLu[mi], ru);
    const T p0 = rev ? c.sAu[mi - 1] : T(0);
    const T pM = rev ? c.sBu[mi - 1] : T(0);
    lap_and_reverse<T, MPT, true>(wp, uc, up, Lu, Ru, p.c2, p.k, c.dl, c.d0, c.dM, gu, p0,
                                  pM, c.cnt, rev, acc);
  } else {
    lap_and_reverse<T, MPT, false>(wp, uc, up, Lu, Ru, p.c2, p.k, 0, 0, 0, T(0), T(0),
                                   T(0), c.cnt, rev, acc);
  }
}

// Which input-end frames wave wv of tile tl carries in the fused update
// (bit 0 left, bit 1 right): the tile's ends that are input ghosts, held
// by its first and last wave.  Wave-uniform.
template <int NT>
__device__ __forceinline__ int adj_ends(int wv, const Tile& tl) {
  constexpr int NW = NT / 64;
  return __builtin_amdgcn_readfirstlane(((wv == 0 && tl.lmode == kEndGhost) ? 1 : 0) |
                                        ((wv == NW - 1 && tl.rmode == kEndGhost) ? 2 : 0));
}

// The span's S steps; returns tau (tau < S: the last step left W^{n_k+1}
// in wp, else in wc).  FR (fused update): a wave holding the tile's left
// (hl) or right (hr) input end advances that end's W frame with the tile
// (the arithmetic of k_adj_predict_frame, so the same samples bit for bit)
// and takes each step's ghost flux from it; hl / hr are wave-uniform.
// ENDS >= 0: the caller has read hl / hr (bits 0 / 1) and each is fixed at
// compile time; -1: read here.
template <typename T, int NT, int MPT, bool GEN, bool SRC, bool FR, int ENDS = -1>
__device__ __forceinline__ int adj_run(const AdjUpdateArgs<T>& p, const AdjCtx<T, NT, MPT>& c,
                                       const Tile& tl, T (&wc)[MPT], T (&wp)[MPT],
                                       T (&uc)[MPT], T (&up)[MPT], T (&flc)[2], T (&flo)[2],
                                       T (&frc)[2], T (&fro)[2],
                                       const AdjFrame<T, kAdjFuseSrc>& fa,
                                       const AdjFrame<T, kAdjFuseSrc>& fb, int S,
                                       double& acc) {
  T gf[2] = {T(0), T(0)};
  bool hl, hr;
  if constexpr (ENDS >= 0) {
    hl = FR && (ENDS & 1) != 0;
    hr = FR && (ENDS & 2) != 0;
  } else {
    const int ends = adj_ends<NT>(c.wv, tl);
    hl = FR && (uni(ends) & 1) != 0;
    hr = FR && (uni(ends) & 2) != 0;
  }
  // flc / flo, frc / fro: the frames' two levels (loaded by the caller where
  // hl / hr hold), swapped each step
  // rev: whether the step also rebuilds the forward level two back (every
  // step but the span's last), fixed per call so a step has no test on it;
  // the frames' sources beyond the registers come after the tile's step,
  // off its dependence chain (the frames' new level is needed next step)
  auto step = [&](auto rev, T (&w0)[MPT], T (&w1)[MPT], T (&u0)[MPT], T (&u1)[MPT],
                  T (&lc)[2], T (&lo)[2], T (&rc)[2], T (&ro)[2], int t) {
    T fwL = T(0), fwR = T(0);
    if (hl) fwL = adj_frame_step(lc, lo, fa, p.c2, p.k, p.r, t, c.lane, true);
    if (hr) fwR = adj_frame_step(rc, ro, fb, p.c2, p.k, p.r, t, c.lane, true);
    adj_step<T, NT, MPT, GEN, SRC, FR, ENDS, decltype(rev)::value>(p, c, w0, w1, u0, u1, gf, t,
                                                                   S, acc, fwL, fwR);
    if (hl)
      adj_frame_extra(lo, fa, p.rec_all, p.n_rec_all, p.gtr, p.gtr_ld, p.M, p.n_e, t, c.lane);
    if (hr)
      adj_frame_extra(ro, fb, p.rec_all, p.n_rec_all, p.gtr, p.gtr_ld, p.M, p.n_e, t, c.lane);
  };
  using Rev = std::integral_constant<int, 1>;
  using Last = std::integral_constant<int, 0>;
  int tau = 0;
  for (; tau + 2 < S; tau += 2) {
    step(Rev{}, wc, wp, uc, up, flc, flo, frc, fro, tau);
    step(Rev{}, wp, wc, up, uc, flo, flc, fro, frc, tau + 1);
  }
  if (tau + 1 < S) {  // the last two steps
    step(Rev{}, wc, wp, uc, up, flc, flo, frc, fro, tau);
    step(Last{}, wp, wc, up, uc, flo, flc, fro, frc, tau + 1);
    tau += 2;
  } else {  // the last step (S odd): W^{n_k+1} is left in wp
    step(Last{}, wc, wp, uc, up, flc, flo, frc, fro, tau);
  }
  if (SRC && c.lane < S) {  // dJ/df of levels n_e - lane
    if (c.gwv[0] == c.wv) p.grad_fa[p.n_e - c.lane] = gf[0];
    if (c.gwv[1] == c.wv) p.grad_fb[p.n_e - c.lane] = gf[1];
  }
  return tau;
}

// GEN: general tiles.  MIX: every other tile; those holding sources or
// nodes 1 / M-2 take the SRC step, the rest the plain one (a uniform branch
// per work-group).  FR: fused update (no adjoint flux rows: the tiles
// predict their input ends themselves; fused plans only).
// PART (MIX only): 0 every tile; 1 the tiles without sources and not
// holding nodes 1 / M-2; 2 the others.  Launched as parts 1 and 2, each
// kernel is allocated the registers of its own path: on long rows the
// source path needs more than the registers that keep two waves per SIMD.
template <typename T, int MPT>
constexpr bool adj_split_mix() {
  return MPT * sizeof(T) > 64;
}

template <typename T, int NT, int MPT, bool GEN, bool MIX, bool FR, int PART = 0>
__global__ __launch_bounds__(NT) void k_adj_update(const AdjUpdateArgs<T> p0) {
  const AdjUpdateArgs<T> p = batch_problem(p0);
  constexpr int NW = NT / 64;
  constexpr int TM = NT * MPT;
  constexpr int TMP = TM + (TM >> 5) + 1;
  __shared__ T st[TMP];
  __shared__ T sRw[kMaxSpan], sLw[kMaxSpan], sRu[kMaxSpan], sLu[kMaxSpan];
  __shared__ T sAu[kMaxSpan], sBu[kMaxSpan];
  __shared__ T edge[2][4][NW];
  __shared__ double red[NW];
  __shared__ T sg[(GEN || MIX) ? kRecSlots : 1][kMaxSpan];

  const int tid = threadIdx.x;
  const int slot = xcd_tile(blockIdx.x, gridDim.x);
  const int tix = p.tile_idx[slot];
  const Tile tl = p.tiles[tix];
  int S = p.span < kMaxSpan ? p.span : kMaxSpan;
  if (S <= 0) return;
  const int64_t M = p.M;
  const int lane = tid & 63;
  // short rows: the four levels and the frames are read at once
  constexpr bool kEarlyLoads = MPT * sizeof(T) <= 32;

  // The tile's reads that depend on the tile alone go out together, so one
  // memory latency covers them: the source list range, the fused update's
  // lane-staged rows, this tile's dJ/dlam partial, the four levels; then
  // the LDS rows (two-launch update and general tiles) and the transposes.
  const int sb = ((GEN || MIX) && p.src_ptr) ? p.src_ptr[slot] : 0;
  const int se = ((GEN || MIX) && p.src_ptr) ? p.src_ptr[slot + 1] : 0;
  if constexpr (MIX && PART != 0) {
    const bool src = se > sb || (tl.out_lo <= 1 && 1 <= tl.out_hi) ||
                     (tl.out_lo <= M - 2 && M - 2 <= tl.out_hi);
    if (src != (PART == 2)) return;  // the other part's tile
  }
  T vLu = T(0), vRu = T(0), vAu = T(0), vBu = T(0);
  if (FR && lane < S) {
    if (tl.fl >= 0) vLu = gload(p.ffl + static_cast<int64_t>(2 * tl.fl + 0) * p.ld + lane);
    if (tl.fr >= 0) vRu = gload(p.ffl + static_cast<int64_t>(2 * tl.fr + 1) * p.ld + lane);
    vAu = (lane == 0) ? gload(p.u_beg + M) : gload(p.fa + p.n_k + lane);
    vBu = (lane == 0) ? gload(p.u_beg + 2 * M - 1) : gload(p.fb + p.n_k + lane);
  }
  // (short rows: this tile's dJ/dlam partial is read now, not at the end)
  const double lam0 = (kEarlyLoads && tid == 0) ? gload(p.lam_part + tix) : 0.0;
  auto stage_rows = [&]() {
    for (int s = tid; s < S; s += NT) {
      const int64_t rr = static_cast<int64_t>(2 * tl.fr + 1) * p.ld + s;
      const int64_t rl = static_cast<int64_t>(2 * tl.fl + 0) * p.ld + s;
      const T a = (!FR && tl.fr >= 0) ? gload(p.afl + rr) : T(0);
      const T b = (!FR && tl.fl >= 0) ? gload(p.afl + rl) : T(0);
      const T cr = (tl.fr >= 0) ? gload(p.ffl + rr) : T(0);
      const T cl = (tl.fl >= 0) ? gload(p.ffl + rl) : T(0);
      const T da = (s == 0) ? gload(p.u_beg + M) : gload(p.fa + p.n_k + s);
      const T db = (s == 0) ? gload(p.u_beg + 2 * M - 1) : gload(p.fb + p.n_k + s);
      sRw[s] = a;
      sLw[s] = b;
      sRu[s] = cr;
      sLu[s] = cl;
      sAu[s] = da;
      sBu[s] = db;
    }
  };
  // the fused update of a plain tile reads none of the LDS rows
  constexpr bool kRows = !FR || GEN;
  // fused update: the W frames of the tile's input ends, carried by its
  // first (left) and last (right) wave
  T flc[2], flo[2], frc[2], fro[2];
  AdjFrame<T, kAdjFuseSrc> fa, fb;
  auto load_frames = [&]() {
    if constexpr (FR) {
      const int ends = adj_ends<NT>(tid >> 6, tl);
      if (ends & 1)
        adj_frame_load(p.w_in, p.lo, p.hi, p.rec_all, p.n_rec_all, p.gtr, p.gtr_ld, M, p.n_e,
                       p.lo[tl.fl + 1], tl.fl, S, lane, flc, flo, fa);
      if (ends & 2)
        adj_frame_load(p.w_in, p.lo, p.hi, p.rec_all, p.n_rec_all, p.gtr, p.gtr_ld, M, p.n_e,
                       p.hi[tl.fr], tl.fr + 1, S, lane, frc, fro, fb);
    }
  };

  T wc[MPT], wp[MPT], uc[MPT], up[MPT];
  if constexpr (kEarlyLoads) {
    T t0[MPT], t1[MPT], t2[MPT], t3[MPT];
    load_level<T, NT, MPT>(p.w_in + M, tl.a, M, t0);
    load_level<T, NT, MPT>(p.w_in, tl.a, M, t1);
    load_level<T, NT, MPT>(p.u_end, tl.a, M, t2);
    load_level<T, NT, MPT>(p.u_end + M, tl.a, M, t3);
    if constexpr (kRows) stage_rows();
    load_frames();
    transpose_in<T, NT, MPT>(t0, st, wc);  // W^{n_e+1}
    transpose_in<T, NT, MPT>(t1, st, wp);  // W^{n_e+2}
    transpose_in<T, NT, MPT>(t2, st, uc);  // U^{n_e-1}
    transpose_in<T, NT, MPT>(t3, st, up);  // U^{n_e}
  } else {
    // (longer rows: one level in flight at a time and the frames after the
    // levels, to bound the registers)
    if constexpr (kRows) stage_rows();
    T t[MPT];
    load_level<T, NT, MPT>(p.w_in + M, tl.a, M, t);
    transpose_in<T, NT, MPT>(t, st, wc);
    load_level<T, NT, MPT>(p.w_in, tl.a, M, t);
    transpose_in<T, NT, MPT>(t, st, wp);
    load_level<T, NT, MPT>(p.u_end, tl.a, M, t);
    transpose_in<T, NT, MPT>(t, st, uc);
    load_level<T, NT, MPT>(p.u_end + M, tl.a, M, t);
    transpose_in<T, NT, MPT>(t, st, up);
    load_frames();
  }

  AdjCtx<T, NT, MPT> c;
  c.edge = edge;
  c.sRw = sRw;
  c.sLw = sLw;
  c.sRu = sRu;
  c.sLu = sLu;
  c.sAu = sAu;
  c.sBu = sBu;
  c.base = tl.a + static_cast<int64_t>(tid) * MPT;
  c.lane = tid & 63;
  c.wv = tid >> 6;
  c.wvu = __builtin_amdgcn_readfirstlane(tid >> 6);
  c.lmode = __builtin_amdgcn_readfirstlane(tl.lmode);
  c.rmode = __builtin_amdgcn_readfirstlane(tl.rmode);
  c.vLu = vLu;
  c.vRu = vRu;
  c.vAu = vAu;
  c.vBu = vBu;
  auto rel = [](int64_t node, int64_t base) -> int {
    const int64_t d = node - base;
    return (d < -2 || d > MPT + 1) ? -1000 : static_cast<int>(d);
  };
  c.dl = (tl.lin == kNoNode) ? -1000 : rel(tl.lin, c.base);
  c.d0 = rel(0, c.base);
  c.dM = rel(M - 1, c.base);
  c.d1 = rel(1, c.base);
  c.dM2 = rel(M - 2, c.base);
  c.wr_fa = tl.out_lo <= 1 && 1 <= tl.out_hi;
  c.wr_fb = tl.out_lo <= M - 2 && M - 2 <= tl.out_hi;
  {
    const bool mine = (c.dl >= 0 && c.dl < MPT) || (c.d0 >= 0 && c.d0 < MPT) ||
                      (c.dM >= 0 && c.dM < MPT);
    c.gen = GEN && (__any(mine) != 0);
  }
  c.sb = sb;
  c.se = se;
  c.rs = (GEN || MIX) ? adj_slots(p.src_node, p.src_id, c.sb, c.se) : RecSlots{0, {}, {}};
  c.sg = sg;
  {
    // wave-uniform positions: tile offset x lies in thread x / MPT,
    // element x % MPT
    auto place = [&](bool use, int64_t node, int& w, int& l, int& e) {
      const int64_t x = node - tl.a;
      const bool in = use && x >= 0 && x < TM;
      const int th = in ? static_cast<int>(x) / MPT : 0;
      w = __builtin_amdgcn_readfirstlane(in ? th >> 6 : -1);
      l = __builtin_amdgcn_readfirstlane(th & 63);
      e = __builtin_amdgcn_readfirstlane(in ? static_cast<int>(x) % MPT : 0);
    };
#pragma unroll
    for (int q = 0; q < kRecSlots; ++q)
      place(q < c.rs.n, c.rs.node[q], c.swv[q], c.slane[q], c.selem[q]);
    place(c.wr_fa, 1, c.gwv[0], c.glane[0], c.gelem[0]);
    place(c.wr_fb, M - 2, c.gwv[1], c.glane[1], c.gelem[1]);
  }
  // dJ/dtrace of the slot sources at levels n_e-1-tau, tau = 0..S-1: one
  // per lane for the fused update of a plain tile with short rows, in LDS
  // otherwise
  constexpr bool kLaneSrc = FR && MIX && kEarlyLoads;
#pragma unroll
  for (int q = 0; q < kRecSlots; ++q) {
    c.vsg[q] = T(0);
    c.vse[q] = (kLaneSrc && q < c.rs.n && c.swv[q] == c.wv && c.lane == c.slane[q])
                   ? c.selem[q]
                   : -1;
  }
  if constexpr (kLaneSrc) {
#pragma unroll
    for (int q = 0; q < kRecSlots; ++q) {
      if (q < c.rs.n && c.lane < S)
        c.vsg[q] = gload(p.gtr + static_cast<int64_t>(c.rs.id[q]) * p.gtr_ld + (p.n_e - 1) -
                         c.lane);
    }
  } else if constexpr (GEN || MIX) {
#pragma unroll
    for (int q = 0; q < kRecSlots; ++q) {
      if (q < c.rs.n) {
        const T* g = p.gtr + static_cast<int64_t>(c.rs.id[q]) * p.gtr_ld + (p.n_e - 1);
        for (int tau = tid; tau < S; tau += NT) sg[q][tau] = g[-tau];
      }
    }
    __syncthreads();
  }
  {
    // nodes max(out_lo, 1) .. min(out_hi, M-2), as this lane's elements
    const int64_t first = (tl.out_lo > 1 ? tl.out_lo : 1) - c.base;
    const int64_t last = (tl.out_hi < M - 2 ? tl.out_hi : M - 2) - c.base;
    const int64_t lo = first > 0 ? first : 0;
    const int64_t hi = last < MPT - 1 ? last : MPT - 1;
    c.cnt.lo = static_cast<int>(lo < MPT ? lo : MPT);
    c.cnt.n = hi >= lo ? static_cast<int>(hi - lo + 1) : 0;
  }

  double acc = 0.0;
  // run<SRC, ENDS>: the span's steps on the path for those (GEN: ENDS -1)
  auto run = [&](auto src, auto ends) -> int {
    return adj_run<T, NT, MPT, GEN, decltype(src)::value, FR, decltype(ends)::value>(
        p, c, tl, wc, wp, uc, up, flc, flo, frc, fro, fa, fb, S, acc);
  };
  using Plain = std::false_type;
  using Src = std::true_type;
  int tau;
  if constexpr (GEN) {
    tau = run(Plain{}, std::integral_constant<int, -1>{});
  } else if constexpr (MIX && FR) {
    // a code path per carried frame, so the steps test for none; a wave
    // carrying both (a window no wider than a tile), and on longer rows one
    // with sources, take the path that tests for them, which needs fewer
    // registers than both fixed
    const bool src = c.se > c.sb || c.wr_fa || c.wr_fb;
    const int ends = adj_ends<NT>(c.wv, tl);
    using Any = std::integral_constant<int, -1>;
    using E0 = std::integral_constant<int, 0>;
    using E1 = std::integral_constant<int, 1>;
    using E2 = std::integral_constant<int, 2>;
    if constexpr (MPT * sizeof(T) <= 32) {
      if (ends == 3) {
        tau = src ? run(Src{}, Any{}) : run(Plain{}, Any{});
      } else if (ends == 0) {
        tau = src ? run(Src{}, E0{}) : run(Plain{}, E0{});
      } else if (ends == 1) {
        tau = src ? run(Src{}, E1{}) : run(Plain{}, E1{});
      } else {
        tau = src ? run(Src{}, E2{}) : run(Plain{}, E2{});
      }
    } else if constexpr (MPT * sizeof(T) <= 64) {
      if (src) {
        tau = run(Src{}, Any{});
      } else if (ends == 3) {
        tau = run(Plain{}, Any{});
      } else if (ends == 0) {
        tau = run(Plain{}, E0{});
      } else if (ends == 1) {
        tau = run(Plain{}, E1{});
      } else {
        tau = run(Plain{}, E2{});
      }
    } else if constexpr (PART == 1) {
      // rows above 64 bytes: one path that tests for the frames (fewest
      // registers; the state itself fills most of them)
      tau = run(Plain{}, Any{});
    } else if constexpr (PART == 2) {
      tau = run(Src{}, Any{});
    } else {
      tau = src ? run(Src{}, Any{}) : run(Plain{}, Any{});
    }
  } else if constexpr (MIX && PART == 1) {
    tau = run(Plain{}, std::integral_constant<int, -1>{});
  } else if constexpr (MIX && PART == 2) {
    tau = run(Src{}, std::integral_constant<int, -1>{});
  } else if constexpr (MIX) {
    if (c.se > c.sb || c.wr_fa || c.wr_fb)
      tau = run(Src{}, std::integral_constant<int, -1>{});
    else
      tau = run(Plain{}, std::integral_constant<int, -1>{});
  } else {
    tau = run(Plain{}, std::integral_constant<int, -1>{});
  }
  const int64_t rlo = tl.out_lo > tl.a ? tl.out_lo : tl.a;
  const int64_t rhi = tl.out_hi < tl.a + TM - 1 ? tl.out_hi : tl.a + TM - 1;
  const int xlo = static_cast<int>(rlo - tl.a);
  const int xhi = static_cast<int>(rhi - tl.a);
  if (tau < S) {
    stage_out<T, NT, MPT>(p.w_out, tl.a, xlo, xhi, st, wc);      // W^{n_k+2}
    stage_out<T, NT, MPT>(p.w_out + M, tl.a, xlo, xhi, st, wp);  // W^{n_k+1}
  } else {
    stage_out<T, NT, MPT>(p.w_out, tl.a, xlo, xhi, st, wp);
    stage_out<T, NT, MPT>(p.w_out + M, tl.a, xlo, xhi, st, wc);
  }
  // Dirichlet nodes next to the region: W = 0
  if (tid == 0 && tl.lmode == kEndDirichlet) {
    p.w_out[0] = T(0);
    p.w_out[M] = T(0);
  }
  if (tid == NT - 1 && tl.rmode == kEndDirichlet) {
    p.w_out[M - 1] = T(0);
    p.w_out[2 * M - 1] = T(0);
  }
  // fixed-order reduction of the dJ/dlam partial of this tile
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (c.lane == 0) red[c.wv] = acc;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < NW; ++w) t += red[w];
    p.lam_part[tix] = (kEarlyLoads ? lam0 : p.lam_part[tix]) + t;
  }
}

// Launch of the update kernels of one kind (FR: fused update); the library
// instantiates FR = false in rswr_adjoint.hip and FR = true in
// rswr_adjoint_fused_*.hip, one translation unit each.  Plain (not general)
// tiles of long rows go out as two launches, the parts of k_adj_update.
template <typename T, int NT, int MPT, bool FR>
hipError_t launch_adj_update_shape(const AdjUpdateArgs<T>& a, bool general, hipStream_t s) {
  const dim3 grid(a.n_tiles, ny(a.ys));
  if (general) {
    hipLaunchKernelGGL((k_adj_update<T, NT, MPT, true, false, FR>), grid, dim3(NT), 0, s, a);
  } else if constexpr (adj_split_mix<T, MPT>()) {
    hipLaunchKernelGGL((k_adj_update<T, NT, MPT, false, true, FR, 1>), grid, dim3(NT), 0, s, a);
    hipLaunchKernelGGL((k_adj_update<T, NT, MPT, false, true, FR, 2>), grid, dim3(NT), 0, s, a);
  } else {
    hipLaunchKernelGGL((k_adj_update<T, NT, MPT, false, true, FR>), grid, dim3(NT), 0, s, a);
  }
  return hipGetLastError();
}

template <typename T, bool FR>
hipError_t launch_adj_update_kind(const AdjUpdateArgs<T>& a, int threads, int per_thread,
                                  bool general, hipStream_t s) {
  if (a.n_tiles <= 0) return hipSuccess;
#define RSWR_ADJ_LAUNCH(NT_, MPT_)              \
  if (threads == NT_ && per_thread == MPT_)   \
    return launch_adj_update_shape<T, NT_, MPT_, FR>(a, general, s);
  RSWR_SHAPES(RSWR_ADJ_LAUNCH)
#undef RSWR_ADJ_LAUNCH
  return hipErrorInvalidValue;
}

// Whether the fused update kernels of a shape keep their state in
// registers (no scratch): the fused adjoint runs only there.
template <typename T, int NT, int MPT>
bool adj_update_fused_fits_shape() {
  auto no_scratch = [](const void* f) {
    hipFuncAttributes at{};
    return hipFuncGetAttributes(&at, f) == hipSuccess && at.localSizeBytes == 0;
  };
  if (!no_scratch(reinterpret_cast<const void*>(k_adj_update<T, NT, MPT, true, false, true>)))
    return false;
  if constexpr (adj_split_mix<T, MPT>())
    return no_scratch(reinterpret_cast<const void*>(
               k_adj_update<T, NT, MPT, false, true, true, 1>)) &&
           no_scratch(reinterpret_cast<const void*>(
               k_adj_update<T, NT, MPT, false, true, true, 2>));
  else
    return no_scratch(reinterpret_cast<const void*>(k_adj_update<T, NT, MPT, false, true, true>));
}

template <typename T>
bool adj_update_fused_fits(int threads, int per_thread) {
#define RSWR_ADJ_FIT(NT_, MPT_) \
  if (threads == NT_ && per_thread == MPT_) return adj_update_fused_fits_shape<T, NT_, MPT_>();
  RSWR_SHAPES(RSWR_ADJ_FIT)
#undef RSWR_ADJ_FIT
  return false;
}

}  // namespace rswr
