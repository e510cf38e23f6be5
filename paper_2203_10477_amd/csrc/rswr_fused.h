// rswr_fused.h -- device code of the fused span: the predict of Sec. 2.3
// folded into the update of Sec. 2.5 (used by the single-problem and the
// batched kernels).
//
// Method: Wei & Zhao, arXiv 2203.10477.  The flux a window receives at an
// input end is predicted by the neighbouring window at that node (Eqs.
// (8)-(9)).  Over S levels that sample depends only on the state within S
// nodes of the end (one node per level, Sec. 2.4), so the wave holding the
// tile's input end carries the prediction itself: a frame of 2*kFrameHalf
// nodes centred on the end, two nodes per lane, advanced in lockstep with
// the tile; F[s] is read across lanes with readlane and feeds the ghost
// node of Eqs. (6)-(7) in the same step.  No flux passes through memory
// (it is written only when the caller keeps the span's fluxes).
//
// Over S levels the flux at o reads the state in [o-S, o+S] and nothing
// else: the predicting window's input ends lie at least the light-cone
// limit >= S nodes from o.  So the frame runs the plain stencil everywhere,
// except at node 0 or M-1 (Dirichlet, Eq. (3)) where a frame holds one; what
// lies outside [o-S, o+S] (the state mirrored at the window's ends, the
// frame's cut ends, which reach o +- 1 only after kFrameHalf - 1 >= S
// levels) cannot reach the sample in time, and F[s] equals the
// whole-window prediction bit for bit.
//
// Dirichlet values of nodes 0 and M-1 for the span's levels sit one per
// lane and are read with readlane, so a step waits on LDS only for the
// values crossing between waves.
#pragma once

#include "rswr_device.h"

namespace rswr {

template <typename T, int NT, int MPT>
struct FusedCtx {
  T (*edge)[2][NT / 64];
  T vA, vB;      // lane s: node 0 / node M-1 at level n0+s (or 0 where unused)
  T nq, pq;      // -2 dx and 2 dx, in vector registers
  int64_t base;  // this lane's first node
  int64_t a;     // the region's first node
  int tid;
  int d0, lane, wv;
  // receivers this tile records (all wave-uniform): trace row, the wave
  // and lane holding the node (wave -1: none), and its element (-1: node
  // 0's value, -2: node M-1's value)
  // work bits of this wave (wave-uniform): kW* below
  int work;
  int nrec;
  T* rdst[kRecSlots];
  int rwv[kRecSlots], rlane[kRecSlots], relem[kRecSlots];
  // interior sources this tile injects (all but the samples wave-uniform):
  // region slots as (wave << 16) | (lane << 8) | element, frame slots as the
  // frame offset 2 lane + element; samp / famp hold the span's samples, one
  // per lane; [sfb, sfe) and [ffb, ffe) are the sources read from memory
  int nsrc, sfb, sfe;
  int scode[kSrcSlots];
  T samp[kSrcSlots];
  int nfs[2], ffb[2], ffe[2];
  int fcode[2][kFrameSrc];
  T famp[2][kFrameSrc];
  bool gen;
  bool dirL, dirR;    // this wave's lane 0 / lane 63 borders a Dirichlet node
  bool fdirL, fdirR;  // this wave's left frame holds node 0 / right frame node M-1
  bool fmL[2], fmR[2];  // which of this lane's frame elements is that node
  bool fmLc[2], fmRc[2];  // the same in the compact frame (one node per lane)
  bool keep;          // the caller keeps the predicted fluxes
};

// Frame around output node o of window [wlo, whi]: lane l holds nodes
// o - kFrameHalf + 2l and the next one (j[0], j[1]); nodes beyond the window
// take their mirror image (clamped into the window), a value the sample
// never sees.
__device__ __forceinline__ void frame_index(int64_t o, int64_t wlo, int64_t whi, int lane,
                                            int64_t (&j)[2]) {
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    int64_t x = o - kFrameHalf + 2 * lane + e;
    x = (x < wlo) ? 2 * wlo - x : ((x > whi) ? 2 * whi - x : x);
    j[e] = x < wlo ? wlo : (x > whi ? whi : x);
  }
}

// The frame's nodes j at the span's first level (cur) and the one before
// (old).  COH: device-coherent loads (the one-launch loop).
template <typename T, bool COH = false>
__device__ __forceinline__ void frame_load(const UpdateArgs<T>& p, const int64_t (&j)[2],
                                           T (&cur)[2], T (&old)[2]) {
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    if constexpr (COH) {
      cur[e] = ld_coh<T>(state_row(p.state_in, p.M, 1), j[e]);
      old[e] = ld_coh<T>(state_row(p.state_in, p.M, 0), j[e]);
    } else {
      cur[e] = p.state_in[p.M + j[e]];
      old[e] = p.state_in[j[e]];
    }
  }
}

// One level of a frame: returns the centred flux at the output node (lane
// kFrameHalf/2, element 0) at the current level and writes the next level
// over `old`.
template <typename T>
__device__ __forceinline__ T frame_step(const T (&cur)[2], T (&old)[2], T c2, T k, T r) {
  const T l1 = lane_shift_z<kWaveShr1>(cur[1]);
  const T r0 = lane_shift_z<kWaveShl1>(cur[0]);
  const T f = rd_lane((cur[1] - l1) * r, kFrameHalf / 2);
  old[0] = leap(c2, k, l1, cur[0], cur[1], old[0]);
  old[1] = leap(c2, k, cur[0], cur[1], r0, old[1]);
  return f;
}

// The compact frame: once at most 31 levels are left, the samples need only
// the nodes within 31 of o, so lane l keeps node o - 32 + l alone (its cut
// ends reach o +- 1 after 31 levels).  One level: the same samples and the
// same stencil as frame_step.
template <typename T>
__device__ __forceinline__ T frame_step1(const T (&cur)[2], T (&old)[2], T c2, T k, T r) {
  const T l = lane_shift_z<kWaveShr1>(cur[0]);
  const T rr = lane_shift_z<kWaveShl1>(cur[0]);
  const T f = rd_lane((rr - l) * r, 32);  // o + 1 is lane 33, o - 1 lane 31
  old[0] = leap(c2, k, l, cur[0], rr, old[0]);
  return f;
}

// v in lane `src` (per lane), through the lane permute (no LDS storage).
__device__ __forceinline__ float lane_gather(float v, int src) {
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_ds_bpermute(src << 2, __builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double lane_gather(double v, int src) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint64_t lo = static_cast<uint32_t>(
      __builtin_amdgcn_ds_bpermute(src << 2, static_cast<int>(static_cast<uint32_t>(b))));
  const uint64_t hi = static_cast<uint32_t>(
      __builtin_amdgcn_ds_bpermute(src << 2, static_cast<int>(static_cast<uint32_t>(b >> 32))));
  return __builtin_bit_cast(double, lo | (hi << 32));
}

// Two nodes per lane (node o - 64 + 2l + e) -> one (node o - 32 + l, in v[0]).
template <typename T>
__device__ __forceinline__ void frame_compact(T (&v)[2], int lane) {
  const int src = 16 + (lane >> 1);
  const T a = lane_gather(v[0], src), b = lane_gather(v[1], src);
  v[0] = (lane & 1) ? b : a;
}

// A frame of window 0 may hold node 0, one of window N-1 node M-1: those
// nodes take the Dirichlet value of the new level (Eq. (3)) instead of the
// stencil.  `dir` is wave-uniform; `d` is the value, `m` marks the element.
template <typename T>
__device__ __forceinline__ void frame_dirichlet(bool dir, const bool (&m)[2], T d,
                                                T (&lvl)[2]) {
  if (dir) {
    lvl[0] = m[0] ? d : lvl[0];
    lvl[1] = m[1] ? d : lvl[1];
  }
}

// Work bits of a wave in a tile with receivers or sources.
constexpr int kWSrc = 1 << 0;      // region source slot q: bit q (4 bits)
constexpr int kWSrcMem = 1 << 4;   // region sources read from memory
constexpr int kWFrame = 1 << 5;    // frame side sd has sources: bit 5 + sd
constexpr int kWRec = 1 << 8;      // receiver slot q recorded by this wave: bit 8 + q
constexpr int kWSrcAny = 0x1f;
constexpr int kWRecAny = 0xf00;

// Sources of the frame on side `sd` (0 left, 1 right) into its new level
// (after the frame's step, as every window adds its sources after the
// leapfrog): slots from registers, the rest from memory.  o0 is the frame's
// first node.
template <typename T, int NT, int MPT>
__device__ __forceinline__ void frame_sources(const UpdateArgs<T>& p,
                                             const FusedCtx<T, NT, MPT>& c, int sd,
                                             int64_t o0, int s, T (&lvl)[2]) {
  const int nfs = uni(c.nfs[sd]);
#pragma unroll
  for (int q = 0; q < kFrameSrc; ++q) {
    if (q < nfs) {
      const int x = uni(c.fcode[sd][q]);
      const T g = rd_lane(c.famp[sd][q], s);
      const bool mine = c.lane == (x >> 1);
      if (x & 1)
        lvl[1] = mine ? lvl[1] + g : lvl[1];
      else
        lvl[0] = mine ? lvl[0] + g : lvl[0];
    }
  }
  for (int r = uni(c.ffb[sd]); r < c.ffe[sd]; ++r) {
    const int64_t x = p.src_node[r] - o0 - 2 * c.lane;
    const T g = p.src_amp[static_cast<int64_t>(p.src_id[r]) * p.src_ld + p.n0 + s];
    lvl[0] = (x == 0) ? lvl[0] + g : lvl[0];
    lvl[1] = (x == 1) ? lvl[1] + g : lvl[1];
  }
}

// One step of the tile (cur = level n, old = level n-1 on entry, old = level
// n+1 on exit) and of the frames this wave carries (HL: the left input,
// HR: the right input).  fl / fr collect F[s] in lane s when the caller
// keeps the fluxes.  The lane shifts fill the wave's ends with zero: the
// zero data of a cut region end; input ghosts, Dirichlet values and the
// neighbouring wave's node replace it where they apply.
template <typename T, int NT, int MPT, bool GEN, bool REC, bool SRC, bool HL, bool HR,
          int FK = 2>
__device__ __forceinline__ void fused_step(const UpdateArgs<T>& p,
                                           const FusedCtx<T, NT, MPT>& c,
                                           const T (&cur)[MPT], T (&old)[MPT],
                                           const T (&lc)[2], T (&lo)[2], const T (&rc)[2],
                                           T (&ro)[2], T& fl, T& fr, T (&tr)[kRecSlots],
                                           int s) {
  constexpr int NW = NT / 64;
  const int par = s & 1;
  // the left neighbour of lane 0 and the right neighbour of lane 63: zero
  // data at a cut end, else the input ghost, the Dirichlet value or the
  // neighbouring wave's node; the lane shifts below put them in place
  T L0 = T(0), R0 = T(0);
  if constexpr (HL) {
    const T F = (FK == 2) ? frame_step(lc, lo, p.c2, p.k, p.r)
                          : frame_step1(lc, lo, p.c2, p.k, p.r);
    if (c.fdirL) {
      const T d = rd_lane(c.vA, s + 1);
      frame_dirichlet(true, FK == 2 ? c.fmL : c.fmLc, d, lo);
    }
    if (SRC && (uni(c.work) & (kWFrame << 0)))
      frame_sources(p, c, 0, c.a - kFrameHalf, s, lo);
    if (c.keep) fl = wr_lane(F, s, fl, c.lane);
    L0 = fma_(c.nq, F, cur[1]);
  }
  if constexpr (HR) {
    const T F = (FK == 2) ? frame_step(rc, ro, p.c2, p.k, p.r)
                          : frame_step1(rc, ro, p.c2, p.k, p.r);
    if (c.fdirR) {
      const T d = rd_lane(c.vB, s + 1);
      frame_dirichlet(true, FK == 2 ? c.fmR : c.fmRc, d, ro);
    }
    if (SRC && (uni(c.work) & (kWFrame << 1)))
      frame_sources(p, c, 1, c.a + NT * MPT - 1 - kFrameHalf, s, ro);
    if (c.keep) fr = wr_lane(F, s, fr, c.lane);
    R0 = fma_(c.pq, F, cur[MPT - 2]);
  }
  if constexpr (NW > 1) {
    if (c.lane == 63) c.edge[par][1][c.wv] = cur[MPT - 1];
    if (c.lane == 0) c.edge[par][0][c.wv] = cur[0];
    __syncthreads();
    if (!HL && c.wv > 0) L0 = c.edge[par][1][c.wv - 1];
    if (!HR && c.wv < NW - 1) R0 = c.edge[par][0][c.wv + 1];
  }
  // readlane reads another lane, so it runs with the whole wave active (a
  // wave-uniform branch)
  if (!HL && c.dirL) L0 = rd_lane(c.vA, s);
  if (!HR && c.dirR) R0 = rd_lane(c.vB, s);
  const T L = lane_shift_old<kWaveShr1>(L0, cur[MPT - 1]);
  const T R = lane_shift_old<kWaveShl1>(R0, cur[0]);
  if (GEN && c.gen)
    step_chunk<T, MPT, true>(cur, old, L, R, p.c2, p.k, -1000, c.d0, T(0),
                             rd_lane(c.vA, s + 1));
  else
    step_chunk<T, MPT, false>(cur, old, L, R, p.c2, p.k, 0, 0, T(0), T(0));
  const int w = (REC || SRC) ? uni(c.work) : 0;
  if (SRC && (w & kWSrcAny)) {
    // interior sources of level n+1, in source order
#pragma unroll
    for (int q = 0; q < kSrcSlots; ++q) {
      if (w & (kWSrc << q)) {
        const int code = uni(c.scode[q]);
        add_at(old, code & 255, rd_lane(c.samp[q], s), c.lane == ((code >> 8) & 255));
      }
    }
    if (w & kWSrcMem)
      for (int r = uni(c.sfb); r < c.sfe; ++r) {
        const int64_t d = p.src_node[r] - c.base;
        const T g = p.src_amp[static_cast<int64_t>(p.src_id[r]) * p.src_ld + p.n0 + s];
#pragma unroll
        for (int e = 0; e < MPT; ++e) old[e] = (d == e) ? old[e] + g : old[e];
      }
  }
  if (REC && (w & kWRecAny)) {
    // receivers: the sample of level n+1 goes to lane s of tr[q] (all
    // branches wave-uniform)
#pragma unroll
    for (int q = 0; q < kRecSlots; ++q) {
      if (w & (kWRec << q)) {
        const int e = uni(c.relem[q]);
        T x;
        if (e >= 0)
          x = rd_lane(elem_at(old, e), uni(c.rlane[q]));
        else if (e == -1)
          x = rd_lane(c.vA, s + 1);
        else
          x = rd_lane(c.vB, s + 1);
        tr[q] = wr_lane(x, s, tr[q], c.lane);
      }
    }
  }
}

// The S steps of one tile and of the frames its wave carries (lc / lo: the
// left frame's levels n0 / n0-1, rc / ro: the right frame's), then the
// per-span results the caller keeps.
template <typename T, int NT, int MPT, bool GEN, bool REC, bool SRC, bool HL, bool HR>
__device__ __forceinline__ void fused_run(const UpdateArgs<T>& p, const Tile& tl,
                                          const FusedCtx<T, NT, MPT>& c, int S,
                                          T (&u)[MPT], T (&uo)[MPT], T (&lc)[2], T (&lo)[2],
                                          T (&rc)[2], T (&ro)[2]) {
  T fl = T(0), fr = T(0);
  T tr[kRecSlots];
#pragma unroll
  for (int q = 0; q < kRecSlots; ++q) tr[q] = T(0);
  int s = 0;
  if constexpr (!GEN && !REC && !SRC && (HL || HR)) {
    // the full frame while more than 31 levels are left (from an even step,
    // so the level roles are the entry ones), then the compact frame
    const int s0 = S > 31 ? (S - 30) & ~1 : 0;
    for (; s < s0; s += 2) {
      fused_step<T, NT, MPT, GEN, REC, SRC, HL, HR>(p, c, u, uo, lc, lo, rc, ro, fl, fr, tr, s);
      fused_step<T, NT, MPT, GEN, REC, SRC, HL, HR>(p, c, uo, u, lo, lc, ro, rc, fl, fr, tr,
                                                    s + 1);
    }
    if constexpr (HL) {
      frame_compact(lc, c.lane);
      frame_compact(lo, c.lane);
    }
    if constexpr (HR) {
      frame_compact(rc, c.lane);
      frame_compact(ro, c.lane);
    }
    for (; s + 1 < S; s += 2) {
      fused_step<T, NT, MPT, GEN, REC, SRC, HL, HR, 1>(p, c, u, uo, lc, lo, rc, ro, fl, fr, tr,
                                                       s);
      fused_step<T, NT, MPT, GEN, REC, SRC, HL, HR, 1>(p, c, uo, u, lo, lc, ro, rc, fl, fr, tr,
                                                       s + 1);
    }
    if (s < S)
      fused_step<T, NT, MPT, GEN, REC, SRC, HL, HR, 1>(p, c, u, uo, lc, lo, rc, ro, fl, fr, tr,
                                                       s);
  } else {
    for (; s + 1 < S; s += 2) {
      fused_step<T, NT, MPT, GEN, REC, SRC, HL, HR>(p, c, u, uo, lc, lo, rc, ro, fl, fr, tr, s);
      fused_step<T, NT, MPT, GEN, REC, SRC, HL, HR>(p, c, uo, u, lo, lc, ro, rc, fl, fr, tr,
                                                    s + 1);
    }
    if (s < S)
      fused_step<T, NT, MPT, GEN, REC, SRC, HL, HR>(p, c, u, uo, lc, lo, rc, ro, fl, fr, tr, s);
  }
  // per-span results, one value per lane and step: no stores in the loop
  if (p.flux_out != nullptr && c.lane < S) {
    if constexpr (HL) p.flux_out[static_cast<int64_t>(2 * tl.fl) * p.ld + c.lane] = fl;
    if constexpr (HR) p.flux_out[static_cast<int64_t>(2 * tl.fr + 1) * p.ld + c.lane] = fr;
  }
  if (REC && c.nrec > 0) {
#pragma unroll
    for (int q = 0; q < kRecSlots; ++q)
      if (q < c.nrec && c.rwv[q] == c.wv && c.lane < S) c.rdst[q][c.lane] = tr[q];
  }
}

// Which ends of tile tl touch node 0 / M-1, and whether its frames (the
// predicting neighbours' states around its input ends, each spanning
// [o - kFrameHalf, o + kFrameHalf - 1]) hold node 0 or M-1.
struct TileEnds {
  bool dirL, dirR, fA, fB;
};

template <typename T, int NT, int MPT>
__device__ __forceinline__ TileEnds tile_ends(const UpdateArgs<T>& p, const Tile& tl) {
  constexpr int TM = NT * MPT;
  const int64_t oL = tl.a, oR = tl.a + TM - 1;
  TileEnds e;
  e.dirL = tl.lmode == kEndDirichlet;
  e.dirR = tl.rmode == kEndDirichlet;
  e.fA = tl.lmode == kEndGhost && tl.window == 1 && oL - kFrameHalf <= 0;
  e.fB = tl.rmode == kEndGhost && oR + kFrameHalf - 1 >= p.M - 1 &&
         p.hi[tl.window + 1] == p.M - 1;
  return e;
}

// Everything a tile reads before its first step: both levels of the region
// (unit stride: t1[it] and t0[it] hold node a + it*NT + tid at levels n0 and
// n0-1), the frames of the input ends this wave carries, and nodes 0 / M-1
// at levels n0..n0+S, one level per lane.  Every load is issued before the
// first wait.
template <typename T, int NT, int MPT>
struct TileInput {
  T t1[MPT], t0[MPT];
  T lc[2], lo[2], rc[2], ro[2];
  T vA, vB;
  TileEnds ends;
};

// The bulk of a tile's reads, all issued without a wait: the two levels of
// the region, the frames (nodes jl / jr, frame_index) of the input ends this
// wave carries (carryL / carryR), and the values of nodes 0 / M-1.
// COH: device-coherent loads (the one-launch loop).
template <typename T, int NT, int MPT, bool GEN, bool COH>
__device__ __forceinline__ void tile_fetch_at(const UpdateArgs<T>& p, const Tile& tl,
                                              const TileEnds& e, bool carryL, bool carryR,
                                              const int64_t (&jl)[2], const int64_t (&jr)[2],
                                              int S, TileInput<T, NT, MPT>& in) {
  const int lane = threadIdx.x & 63;
  in.ends = e;
  if constexpr (COH) {
    load_level_coh<T, NT, MPT>(state_row(p.state_in, p.M, 1), tl.a, in.t1);  // level n0
    load_level_coh<T, NT, MPT>(state_row(p.state_in, p.M, 0), tl.a, in.t0);  // level n0-1
  } else {
    load_level<T, NT, MPT>(p.state_in + p.M, tl.a, p.M, in.t1);  // level n0
    load_level<T, NT, MPT>(p.state_in, tl.a, p.M, in.t0);        // level n0-1
  }
  if (carryL) frame_load<T, COH>(p, jl, in.lc, in.lo);
  if (carryR) frame_load<T, COH>(p, jr, in.rc, in.ro);
  // node 0 / M-1 at level n0 (from the state) and n0+1.. (from f_A, f_B)
  T a = T(0), b = T(0);
  if constexpr (COH) {
    if ((e.dirL || e.fA) && lane <= S)
      a = (lane == 0) ? ld_coh<T>(state_row(p.state_in, p.M, 1), 0) : p.fa[p.n0 + lane];
    if ((e.dirR || e.fB) && lane <= S)
      b = (lane == 0) ? ld_coh<T>(state_row(p.state_in, p.M, 1), p.M - 1) : p.fb[p.n0 + lane];
  } else {
    if ((GEN || e.dirL || e.fA) && lane <= S)
      a = (lane == 0) ? p.state_in[p.M] : p.fa[p.n0 + lane];
    if ((GEN || e.dirR || e.fB) && lane <= S)
      b = (lane == 0) ? p.state_in[2 * p.M - 1] : p.fb[p.n0 + lane];
  }
  in.vA = a;
  in.vB = b;
}

// Every read of a tile before its first step, for a wave that carries the
// left (HL) / right (HR) input's frame.  The reads whose values address
// other reads (the frames' window bounds, the window right of the tile) come
// first and are consumed before a scheduling barrier, so no wait for them
// waits for the bulk.
template <typename T, int NT, int MPT, bool GEN, bool COH, bool HL, bool HR>
__device__ __forceinline__ void tile_fetch(const UpdateArgs<T>& p, const Tile& tl, int S,
                                           TileInput<T, NT, MPT>& in) {
  constexpr int TM = NT * MPT;
  const int lane = threadIdx.x & 63;
  int64_t jl[2] = {0, 0}, jr[2] = {0, 0};
  if constexpr (HL) frame_index(tl.a, p.lo[tl.window - 1], p.hi[tl.window - 1], lane, jl);
  if constexpr (HR)
    frame_index(tl.a + TM - 1, p.lo[tl.window + 1], p.hi[tl.window + 1], lane, jr);
  const TileEnds e = tile_ends<T, NT, MPT>(p, tl);
  asm volatile("" : "+v"(jl[0]), "+v"(jl[1]), "+v"(jr[0]), "+v"(jr[1]));
  int flags = (e.dirL ? 1 : 0) | (e.dirR ? 2 : 0) | (e.fA ? 4 : 0) | (e.fB ? 8 : 0);
  asm volatile("" : "+v"(flags));
  __builtin_amdgcn_sched_barrier(0);
  tile_fetch_at<T, NT, MPT, GEN, COH>(p, tl, e, HL, HR, jl, jr, S, in);
}

// The steps of a tile whose input is in registers: u / uo hold this lane's
// MPT consecutive nodes at levels n0 / n0-1 on entry and n0+S / n0+S-1 (S
// even) or n0+S-1 / n0+S (S odd) on exit; lc .. ro are the frames of the
// left (HL) / right (HR) input this wave carries, vA / vB the values of
// nodes 0 / M-1 (tile_fetch).  `edge`: the cross-wave slots.
// GEN: node 0 may lie inside the region (per-element Dirichlet treatment).
// REC: the tile may record receivers.  SRC: the tile and its frames may
// inject interior sources.
template <typename T, int NT, int MPT, bool GEN, bool REC, bool SRC, bool HL, bool HR>
__device__ __forceinline__ void tile_run(const UpdateArgs<T>& p, const Tile& tl, int slot,
                                         int S, T (*edge)[2][NT / 64], T (&u)[MPT],
                                         T (&uo)[MPT], T (&lc)[2], T (&lo)[2], T (&rc)[2],
                                         T (&ro)[2], T vA, T vB, const TileEnds& ends) {
  constexpr int NW = NT / 64;
  constexpr int TM = NT * MPT;
  const int tid = threadIdx.x;
  FusedCtx<T, NT, MPT> c;
  c.edge = edge;
  c.lane = tid & 63;
  c.wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  c.base = tl.a + static_cast<int64_t>(tid) * MPT;
  c.a = tl.a;
  c.tid = tid;
  const bool dirL = ends.dirL, dirR = ends.dirR;
  c.dirL = dirL && c.wv == 0;
  c.dirR = dirR && c.wv == NW - 1;
  // frames around the input ends (left: o = a, right: o = a + TM - 1)
  const int64_t oL = tl.a, oR = tl.a + TM - 1;
  c.fdirL = ends.fA && c.wv == 0;
  c.fdirR = ends.fB && c.wv == NW - 1;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    c.fmL[e] = oL - kFrameHalf + 2 * c.lane + e == 0;
    c.fmR[e] = oR - kFrameHalf + 2 * c.lane + e == p.M - 1;
  }
  c.fmLc[0] = oL - kFrameHalf / 2 + c.lane == 0;
  c.fmRc[0] = oR - kFrameHalf / 2 + c.lane == p.M - 1;
  c.fmLc[1] = c.fmRc[1] = false;
  c.keep = p.flux_out != nullptr;
  c.nq = in_vgpr(-p.q);
  c.pq = in_vgpr(p.q);
  c.vA = vA;
  c.vB = vB;
  c.d0 = -1000;
  c.gen = false;
  if (GEN) {
    const int64_t d = -c.base;
    c.d0 = (d < -2 || d > MPT + 1) ? -1000 : static_cast<int>(d);
    c.gen = __any(c.d0 >= 0 && c.d0 < MPT) != 0;
  }
  // receivers this tile records (REC instantiations; at most kRecSlots)
  c.nrec = 0;
  if (REC && p.rec_ptr) {
    const int rb = p.rec_ptr[slot], re = p.rec_ptr[slot + 1];
    c.nrec = re - rb < kRecSlots ? re - rb : kRecSlots;
#pragma unroll
    for (int q = 0; q < kRecSlots; ++q) {
      const bool h = q < c.nrec;
      const int64_t x = h ? p.rec_node[rb + q] - tl.a : -1000;
      const int32_t id = h ? p.rec_id[rb + q] : 0;
      c.rdst[q] = p.traces + static_cast<int64_t>(id) * p.trace_ld + p.trace_col0;
      int th = -1, el = -1;  // thread of the tile holding the node, element
      if (x >= 0 && x < TM) {
        th = static_cast<int>(x) / MPT;
        el = static_cast<int>(x) % MPT;
      } else if (x == -1 && dirL) {
        th = 0;
        el = -1;
      } else if (x == TM && dirR) {
        th = NT - 1;
        el = -2;
      }
      c.rwv[q] = __builtin_amdgcn_readfirstlane(th < 0 ? -1 : th >> 6);
      c.rlane[q] = __builtin_amdgcn_readfirstlane(th & 63);
      c.relem[q] = __builtin_amdgcn_readfirstlane(el);
    }
    c.nrec = __builtin_amdgcn_readfirstlane(c.nrec);
  }
  // interior sources (SRC instantiations)
  c.nsrc = 0;
  c.sfb = c.sfe = 0;
#pragma unroll
  for (int sd = 0; sd < 2; ++sd) c.nfs[sd] = c.ffb[sd] = c.ffe[sd] = 0;
  if (SRC && p.src_ptr) {
    const int t3 = 3 * p.tile_idx[slot];
    const int b0 = p.src_ptr[t3], b1 = p.src_ptr[t3 + 1];
    const int b2 = p.src_ptr[t3 + 2], b3 = p.src_ptr[t3 + 3];
    auto sample = [&](int r) -> T {
      return (c.lane < S)
                 ? p.src_amp[static_cast<int64_t>(p.src_id[r]) * p.src_ld + p.n0 + c.lane]
                 : T(0);
    };
    c.nsrc = __builtin_amdgcn_readfirstlane(b1 - b0 < kSrcSlots ? b1 - b0 : kSrcSlots);
    c.sfb = __builtin_amdgcn_readfirstlane(b0 + kSrcSlots < b1 ? b0 + kSrcSlots : b1);
    c.sfe = __builtin_amdgcn_readfirstlane(b1);
#pragma unroll
    for (int q = 0; q < kSrcSlots; ++q) {
      const bool h = q < c.nsrc;
      const int x = h ? static_cast<int>(p.src_node[b0 + q] - tl.a) : 0;
      const int th = x / MPT;
      c.scode[q] = __builtin_amdgcn_readfirstlane(h ? ((th >> 6) << 16) | ((th & 63) << 8) |
                                                          (x % MPT)
                                                    : -1);
      c.samp[q] = h ? sample(b0 + q) : T(0);
    }
    const int fb[2] = {b1, b2}, fe[2] = {b2, b3};
    const int64_t o0[2] = {tl.a - kFrameHalf, tl.a + TM - 1 - kFrameHalf};
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const int n = fe[sd] - fb[sd];
      c.nfs[sd] = __builtin_amdgcn_readfirstlane(n < kFrameSrc ? n : kFrameSrc);
      c.ffb[sd] = __builtin_amdgcn_readfirstlane(n > kFrameSrc ? fb[sd] + kFrameSrc : fe[sd]);
      c.ffe[sd] = __builtin_amdgcn_readfirstlane(fe[sd]);
#pragma unroll
      for (int q = 0; q < kFrameSrc; ++q) {
        const bool h = q < c.nfs[sd];
        c.fcode[sd][q] = __builtin_amdgcn_readfirstlane(
            h ? static_cast<int>(p.src_node[fb[sd] + q] - o0[sd]) : 0);
        c.famp[sd][q] = h ? sample(fb[sd] + q) : T(0);
      }
    }
  }
  {
    int w = 0;
#pragma unroll
    for (int q = 0; q < kRecSlots; ++q)
      if (REC && q < c.nrec && c.rwv[q] == c.wv) w |= kWRec << q;
#pragma unroll
    for (int q = 0; q < kSrcSlots; ++q)
      if (SRC && q < c.nsrc && (c.scode[q] >> 16) == c.wv) w |= kWSrc << q;
    if (SRC && c.sfe > c.sfb) w |= kWSrcMem;
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
      if (SRC && (c.nfs[sd] > 0 || c.ffe[sd] > c.ffb[sd])) w |= kWFrame << sd;
    c.work = __builtin_amdgcn_readfirstlane(w);
  }

  fused_run<T, NT, MPT, GEN, REC, SRC, HL, HR>(p, tl, c, S, u, uo, lc, lo, rc, ro);
}

// A tile's stored range as offsets from its region start.
template <int TM>
__device__ __forceinline__ void stored_range(const Tile& tl, int& xlo, int& xhi) {
  const int64_t rlo = tl.out_lo > tl.a ? tl.out_lo : tl.a;
  const int64_t rhi = tl.out_hi < tl.a + TM - 1 ? tl.out_hi : tl.a + TM - 1;
  xlo = static_cast<int>(rlo - tl.a);
  xhi = static_cast<int>(rhi - tl.a);
}

// Node 0 / M-1 at the span's last two levels (a1, a2 / b1, b2), written by
// lane 0 of the first wave / the last lane of the last wave of a tile whose
// region borders it.  COH: device-coherent stores.
template <typename T, int NT, bool COH>
__device__ __forceinline__ void dirichlet_put(const UpdateArgs<T>& p, bool dirL, bool dirR,
                                              T a1, T a2, T b1, T b2) {
  constexpr int AUX = COH ? kCohAux : 0;
  auto put = [&](int64_t j, T v) {
    if constexpr (COH)
      range_store<AUX>(v, range_rsrc(p.state_out + j, static_cast<int>(sizeof(T))), 0);
    else
      p.state_out[j] = v;
  };
  const int tid = threadIdx.x;
  if (dirL && tid == 0) {
    put(0, a1);
    put(p.M, a2);
  }
  if (dirR && tid == NT - 1) {
    put(p.M - 1, b1);
    put(2 * p.M - 1, b2);
  }
}

// The steps and the stores of a tile whose input is in registers
// (tile_run, then the stored range of both levels through the LDS buffer
// `st`, and the Dirichlet nodes next to the region).  COH: device-coherent
// stores (the one-launch loop, where tiles exchange the state within one
// launch).
template <typename T, int NT, int MPT, bool GEN, bool REC, bool SRC, bool COH, bool HL,
          bool HR>
__device__ __forceinline__ void tile_steps(const UpdateArgs<T>& p, const Tile& tl, int slot,
                                           int S, T* st, T (*edge)[2][NT / 64], T (&u)[MPT],
                                           T (&uo)[MPT], T (&lc)[2], T (&lo)[2], T (&rc)[2],
                                           T (&ro)[2], T vA, T vB, const TileEnds& ends) {
  constexpr int NW = NT / 64;
  constexpr int TM = NT * MPT;
  tile_run<T, NT, MPT, GEN, REC, SRC, HL, HR>(p, tl, slot, S, edge, u, uo, lc, lo, rc, ro,
                                              vA, vB, ends);
  int xlo, xhi;
  stored_range<TM>(tl, xlo, xhi);
  constexpr int AUX = COH ? kCohAux : 0;
  if (S & 1) {  // uo = level n0+S, u = n0+S-1
    stage_out<T, NT, MPT, AUX>(p.state_out, tl.a, xlo, xhi, st, u);
    stage_out<T, NT, MPT, AUX>(p.state_out + p.M, tl.a, xlo, xhi, st, uo);
  } else {
    stage_out<T, NT, MPT, AUX>(p.state_out, tl.a, xlo, xhi, st, uo);
    stage_out<T, NT, MPT, AUX>(p.state_out + p.M, tl.a, xlo, xhi, st, u);
  }
  // Dirichlet nodes next to the region (readlane in wave-uniform flow)
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  T a1 = T(0), a2 = T(0), b1 = T(0), b2 = T(0);
  const bool pl = ends.dirL && wv == 0, pr = ends.dirR && wv == NW - 1;
  if (pl) {
    a1 = rd_lane(vA, S - 1);
    a2 = rd_lane(vA, S);
  }
  if (pr) {
    b1 = rd_lane(vB, S - 1);
    b2 = rd_lane(vB, S);
  }
  dirichlet_put<T, NT, COH>(p, pl, pr, a1, a2, b1, b2);
}

// One tile over S levels for a wave that carries the left (HL) / right (HR)
// input's frame: load, step, store.
template <typename T, int NT, int MPT, bool GEN, bool REC, bool SRC, bool COH, bool HL,
          bool HR>
__device__ __forceinline__ void fused_tile_v(const UpdateArgs<T>& p, const Tile& tl, int slot,
                                             int S, T* st, T (*edge)[2][NT / 64]) {
  TileInput<T, NT, MPT> in;
  tile_fetch<T, NT, MPT, GEN, COH, HL, HR>(p, tl, S, in);
  T u[MPT], uo[MPT];
  transpose_in<T, NT, MPT>(in.t1, st, u);
  transpose_in<T, NT, MPT>(in.t0, st, uo);
  tile_steps<T, NT, MPT, GEN, REC, SRC, COH, HL, HR>(p, tl, slot, S, st, edge, u, uo, in.lc,
                                                     in.lo, in.rc, in.ro, in.vA, in.vB,
                                                     in.ends);
}

// One tile over S levels: load, step (with the frames its waves carry),
// store.  The frames a wave carries (wave-uniform) pick one of four whole
// code paths, chosen before the first load: each path's registers are
// allocated on their own, where four step loops after one shared load
// would hold the values of every path at once.
template <typename T, int NT, int MPT, bool GEN, bool REC, bool SRC, bool COH = false>
__device__ __forceinline__ void fused_tile(const UpdateArgs<T>& p, const Tile& tl, int slot,
                                           int S, T* st, T (*edge)[2][NT / 64]) {
  constexpr int NW = NT / 64;
  static_assert(NT % 64 == 0 && MPT >= 2, "shape");
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool hl = wv == 0 && tl.lmode == kEndGhost;
  const bool hr = wv == NW - 1 && tl.rmode == kEndGhost;
  if (hl) {
    if (hr)
      fused_tile_v<T, NT, MPT, GEN, REC, SRC, COH, true, true>(p, tl, slot, S, st, edge);
    else
      fused_tile_v<T, NT, MPT, GEN, REC, SRC, COH, true, false>(p, tl, slot, S, st, edge);
  } else {
    if (hr)
      fused_tile_v<T, NT, MPT, GEN, REC, SRC, COH, false, true>(p, tl, slot, S, st, edge);
    else
      fused_tile_v<T, NT, MPT, GEN, REC, SRC, COH, false, false>(p, tl, slot, S, st, edge);
  }
}

}  // namespace rswr
