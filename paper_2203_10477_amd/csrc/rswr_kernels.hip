// rswr_kernels.hip -- gfx950 kernels of the RSWR hot path.
//
// Method: Wei & Zhao, arXiv 2203.10477.  Stencil arithmetic per node (the
// same operation order everywhere): s = ul + ur; t = fma(k, u, -u_old);
// u_new = fma(c2, s, t).  No packed FP32 (built with -packed-fp32-ops) and
// no contraction (-ffp-contract=off), so every result is one fixed sequence
// of correctly rounded IEEE operations.
#include "rswr_device.h"

namespace rswr {

// ---------------------------------------------------------------------------
// Predict (Sec. 2.3, Eqs. (8)-(9)).  One wave per (interface i, side): side 0
// is window i's output node lo_{i+1}, side 1 is window i+1's output node hi_i.
// The flux at the output node over shat levels depends only on the state in
// [o - shat, o + shat] (one node per level), clipped to the window; the
// window's own ends inside that range keep their exact treatment (Dirichlet
// data, or the zero-flux ghost of the prediction), the cut ends carry zero
// data that cannot reach o +- 1 in time.  So this trapezoid reproduces the
// whole-window prediction bit for bit; so does the register frame below,
// which k_predict uses for spans up to 159 levels.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void predict_trapezoid(const PredictArgs<T>& p, int i, int side) {
  extern __shared__ unsigned char smem_raw[];
  T* const sm = reinterpret_cast<T*>(smem_raw);
  __shared__ T sda[kMaxSpan], sdb[kMaxSpan];
  const int w = i + side;
  const int64_t o = (side == 0) ? p.lo[i + 1] : p.hi[i];
  const int64_t wlo = p.lo[w], whi = p.hi[w];
  const int shat = p.shat;
  const int64_t A = (o - shat > wlo) ? o - shat : wlo;
  const int64_t B = (o + shat < whi) ? o + shat : whi;
  const int n = static_cast<int>(B - A + 1);
  const int cap = 2 * shat + 1;
  T* u0 = sm;        // level n-1, overwritten with level n+1
  T* u1 = sm + cap;  // level n
  const int tid = threadIdx.x;
  for (int s = tid; s + 1 < shat; s += 64) {
    sda[s] = p.fa[p.n0 + s + 1];
    sdb[s] = p.fb[p.n0 + s + 1];
  }
  for (int x = tid; x < n; x += 64) {
    u0[x] = p.state[A + x];
    u1[x] = p.state[p.M + A + x];
  }
  __syncthreads();
  const bool lex = (A == wlo), rex = (B == whi);
  const T zero = T(0);
  T* const row = p.flux + static_cast<int64_t>(2 * i + side) * p.ld;
  const int oi = static_cast<int>(o - A);
  for (int s = 0; s < shat; ++s) {
    if (tid == 0) row[s] = (u1[oi + 1] - u1[oi - 1]) * p.r;
    if (s == shat - 1) break;
    const T da = sda[s], db = sdb[s];
    for (int x = tid; x < n; x += 64) {
      const int64_t j = A + x;
      T v;
      if (j == 0) {
        v = da;
      } else if (j == p.M - 1) {
        v = db;
      } else {
        const T ul = (x == 0) ? (lex ? fma_(-p.q, zero, u1[1]) : zero) : u1[x - 1];
        const T ur = (x == n - 1) ? (rex ? fma_(p.q, zero, u1[n - 2]) : zero) : u1[x + 1];
        v = leap(p.c2, p.k, ul, u1[x], ur, u0[x]);
      }
      u0[x] = v;
    }
    __syncthreads();
    T* t = u0;
    u0 = u1;
    u1 = t;
  }
}

// Element e (wave-uniform) of a frame's K nodes in this lane, and frame node
// `at` := x: bit masks, not an index (an indexed access, or a select chain
// the compiler folds into one, would move the frame to scratch memory).
template <typename T, int K>
__device__ __forceinline__ T frame_elem(const T (&v)[K], int e) {
  return pick<T, K>(v, e);
}

template <typename T, int K>
__device__ __forceinline__ void frame_put(T (&v)[K], int at, T x, int lane) {
  using U = typename Bits<T>::U;
  const int l = at / K, e = at % K;
  const U xb = __builtin_bit_cast(U, x);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const U m = static_cast<U>(0) - static_cast<U>(lane == l && k == e);
    v[k] = __builtin_bit_cast(T, (__builtin_bit_cast(U, v[k]) & ~m) | (xb & m));
  }
}

// The ghost node g (frame offset, -1: none) := fma(sq, 0, node src).
template <typename T, int K>
__device__ __forceinline__ void frame_ghost(T (&v)[K], int g, int src, T sq, int lane) {
  if (g >= 0) {
    const T x = rd_lane(frame_elem<T, K>(v, src % K), src / K);
    frame_put<T, K>(v, g, fma_(sq, T(0), x), lane);
  }
}

// Where a predict frame's nodes need their own treatment (frame offsets,
// -1: not in the frame) and the Dirichlet data of levels n0+1.. (lane s of
// register s / 64).
template <typename T>
struct FrameEnds {
  int gl, gr, d0, d1;
  T dA[3], dB[3];
};

// One level of a predict frame: records F[s] (lane s % 64 of fr[s / 64]),
// then, unless it is the last sample, writes level n+1 over `old`.
template <typename T, int K>
__device__ __forceinline__ bool frame_level(const PredictArgs<T>& p, const FrameEnds<T>& fe,
                                            const T (&cur)[K], T (&old)[K], T (&fr)[3], int s,
                                            int lane) {
  const T l1 = lane_shift_z<kWaveShr1>(cur[K - 1]);
  // o + 1: lane 32, element 1; o - 1: lane 31, element K-1
  const T F = rd_lane((cur[1] - l1) * p.r, 32);
  const int r = s >> 6, l = s & 63;
  frame_put<T, 3>(fr, 3 * l + r, F, lane);  // sample s: fr[s / 64] in lane s % 64
  if (s == p.shat - 1) return false;
  const T r0 = lane_shift_z<kWaveShl1>(cur[0]);
#pragma unroll
  for (int e = 0; e < K; ++e) {
    const T ul = (e == 0) ? l1 : cur[e - 1];
    const T ur = (e == K - 1) ? r0 : cur[e + 1];
    old[e] = leap(p.c2, p.k, ul, cur[e], ur, old[e]);
  }
  if (fe.d0 >= 0) frame_put<T, K>(old, fe.d0, rd_lane(pick<T, 3>(fe.dA, r), l), lane);
  if (fe.d1 >= 0) frame_put<T, K>(old, fe.d1, rd_lane(pick<T, 3>(fe.dB, r), l), lane);
  frame_ghost<T, K>(old, fe.gl, fe.gl + 2, -p.q, lane);
  frame_ghost<T, K>(old, fe.gr, fe.gr - 2, p.q, lane);
  return true;
}

// The same prediction on a register frame: one wave, K nodes per lane, the
// 64K nodes o - 32K .. o + 32K - 1 around the output node o; nodes beyond
// the predicting window load their mirror image (clamped into the window).
// The window's nodes step exactly as in the whole-window prediction: node 0
// / M-1 take the Dirichlet data, and the ghost node outside an input end is
// set every level to the zero-flux ghost of Eqs. (6)-(7), fma(-+q, 0, u)
// of the node two inside, so whatever the nodes beyond it hold never
// reaches the window.  The frame's own cut ends (zero data) reach o +- 1
// only after 32K - 1 levels, so 32K >= shat + 1 makes every sample equal
// to the whole-window prediction bit for bit.  No LDS and no barrier: a
// level is three operations per node and two lane shifts.
template <typename T, int K>
__device__ __forceinline__ void predict_frame(const PredictArgs<T>& p, int i, int side) {
  constexpr int H = 32 * K;
  static_assert(K >= 2, "the output node's neighbours lie in lanes 31 and 32");
  const int lane = threadIdx.x;
  const int w = i + side;
  const int64_t o = (side == 0) ? p.lo[i + 1] : p.hi[i];
  const int64_t wlo = p.lo[w], whi = p.hi[w];
  const int64_t f0 = o - H;  // the frame's first node
  T ca[K], cb[K];  // levels n, n-1 (their roles alternate)
#pragma unroll
  for (int e = 0; e < K; ++e) {
    int64_t x = f0 + K * lane + e;
    x = (x < wlo) ? 2 * wlo - x : ((x > whi) ? 2 * whi - x : x);
    x = x < wlo ? wlo : (x > whi ? whi : x);
    ca[e] = p.state[p.M + x];
    cb[e] = p.state[x];
  }
  auto pos = [&](int64_t j) -> int {
    const int64_t d = j - f0;
    return (d >= 0 && d < 64 * K) ? static_cast<int>(d) : -1;
  };
  FrameEnds<T> fe;
  fe.gl = (w > 0) ? pos(wlo - 1) : -1;
  fe.gr = (w < p.N - 1) ? pos(whi + 1) : -1;
  fe.d0 = (w == 0) ? pos(0) : -1;
  fe.d1 = (w == p.N - 1) ? pos(p.M - 1) : -1;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int s = lane + 64 * r;
    fe.dA[r] = (fe.d0 >= 0 && s + 1 < p.shat) ? p.fa[p.n0 + 1 + s] : T(0);
    fe.dB[r] = (fe.d1 >= 0 && s + 1 < p.shat) ? p.fb[p.n0 + 1 + s] : T(0);
  }
  frame_ghost<T, K>(ca, fe.gl, fe.gl + 2, -p.q, lane);
  frame_ghost<T, K>(ca, fe.gr, fe.gr - 2, p.q, lane);
  T fr[3] = {T(0), T(0), T(0)};
  for (int s = 0; s < p.shat; s += 2) {
    if (!frame_level<T, K>(p, fe, ca, cb, fr, s, lane)) break;
    if (!frame_level<T, K>(p, fe, cb, ca, fr, s + 1, lane)) break;
  }
  T* const row = p.flux + static_cast<int64_t>(2 * i + side) * p.ld;
#pragma unroll
  for (int r = 0; r < 3; ++r)
    if (lane + 64 * r < p.shat) row[lane + 64 * r] = fr[r];
}

// One wave per (interface i, side): the frame for spans up to 159 levels,
// the LDS trapezoid beyond.
template <typename T>
__global__ __launch_bounds__(64) void k_predict(const PredictArgs<T> p0) {
  PredictArgs<T> p = p0;
  if (p0.n0_dev) p.n0 = *p0.n0_dev;
  if (p0.shat_dev) p.shat = *p0.shat_dev;
  const int shat = p.shat;
  if (shat <= 0) return;
  const int i = blockIdx.x >> 1, side = blockIdx.x & 1;
  if (shat <= 63)
    predict_frame<T, 2>(p, i, side);
  else if (shat <= 95)
    predict_frame<T, 3>(p, i, side);
  else if (shat <= 127)
    predict_frame<T, 4>(p, i, side);
  else if (shat <= 159)
    predict_frame<T, 5>(p, i, side);
  else
    predict_trapezoid<T>(p, i, side);
}

// ---------------------------------------------------------------------------
// Update (Sec. 2.5, Eqs. (13)-(14)) and gluing (Eq. (15)).
//
// A tile is NT*MPT consecutive nodes; lane t of the work-group keeps nodes
// a + t*MPT .. a + t*MPT + MPT-1 of both levels in registers for all S
// steps.  Per step a lane needs one value from each neighbouring lane: inside
// a wave by a DPP lane shift, across waves through a double-buffered LDS slot
// (one barrier per step).  The region's ends take the window's right
// input ghost (last lane) or zero data; zero data moves one node per step,
// and the host only stores nodes it cannot reach.  Waves holding node 0,
// node M-1 or the window's left input run the general step with those
// treatments; all other waves run the plain stencil.
// Loads and stores go through an LDS staging buffer so global accesses are
// unit-stride across lanes.
// ---------------------------------------------------------------------------
template <typename T, int NT, int MPT>
struct UpdateCtx {
  T (*edge)[2][NT / 64];
  const T* sR;
  const T* sL;
  const T* sA;
  const T* sB;
  int64_t base;
  int dl, d0;
  int rb, re, lane, wv;
  RecSlots rs;  // the tile's first receivers (GEN)
  int lmode, rmode;
  bool gen;
};

template <typename T, int NT, int MPT, bool GEN>
__device__ __forceinline__ void one_step(const UpdateArgs<T>& p,
                                         const UpdateCtx<T, NT, MPT>& c,
                                         const T (&cur)[MPT], T (&old)[MPT],
                                         int s) {
  constexpr int NW = NT / 64;
  const int par = s & 1;
  T L = lane_shift<kWaveShr1>(cur[MPT - 1]);
  T R = lane_shift<kWaveShl1>(cur[0]);
  if constexpr (NW > 1) {
    if (c.lane == 63) c.edge[par][1][c.wv] = cur[MPT - 1];
    if (c.lane == 0) c.edge[par][0][c.wv] = cur[0];
    __syncthreads();
  }
  if (c.lane == 0)
    L = (c.wv > 0) ? c.edge[par][1][c.wv - 1]
                   : end_value(c.lmode, fma_(-p.q, c.sL[s], cur[1]), c.sA[s]);
  if (c.lane == 63)
    R = (c.wv < NW - 1) ? c.edge[par][0][c.wv + 1]
                        : end_value(c.rmode, fma_(p.q, c.sR[s], cur[MPT - 2]), c.sB[s]);
  if (GEN && c.gen) {
    // the left-input ghost u_{lin-1} = u_{lin+1} - 2dx F; its right
    // neighbour may sit in the next lane
    const int rn = c.dl + 1;
    const T right = (rn == MPT) ? R : pick<T, MPT>(cur, rn);
    const T ghost = fma_(-p.q, c.sL[s], right);
    step_chunk<T, MPT, true>(cur, old, L, R, p.c2, p.k, c.dl, c.d0, ghost, c.sA[s + 1]);
  } else {
    step_chunk<T, MPT, false>(cur, old, L, R, p.c2, p.k, 0, 0, T(0), T(0));
  }
  if (GEN) {
    auto record = [&](int64_t node, int32_t id) {
      const int64_t d = node - c.base;
      T* dst = p.traces + static_cast<int64_t>(id) * p.trace_ld + p.trace_col0 + s;
      if (d >= 0 && d < MPT)
        *dst = pick<T, MPT>(old, d);
      else if (d == -1 && c.lane == 0 && c.wv == 0 && c.lmode == kEndDirichlet)
        *dst = c.sA[s + 1];
      else if (d == MPT && c.lane == 63 && c.wv == NW - 1 && c.rmode == kEndDirichlet)
        *dst = c.sB[s + 1];
    };
#pragma unroll
    for (int q = 0; q < kRecSlots; ++q)
      if (q < c.rs.n) record(c.rs.node[q], c.rs.id[q]);
    for (int r = c.rb + kRecSlots; r < c.re; ++r) record(p.rec_node[r], p.rec_id[r]);
  }
}

template <typename T, int NT, int MPT, bool GEN>
__global__ __launch_bounds__(NT) void k_update(const UpdateArgs<T> p0) {
  UpdateArgs<T> p = p0;
  if (p0.n0_dev) {
    const int64_t dn = *p0.n0_dev - p0.n0;
    p.n0 += dn;
    p.trace_col0 += dn;
  }
  constexpr int NW = NT / 64;
  constexpr int TM = NT * MPT;
  constexpr int TMP = TM + (TM >> 5) + 1;
  static_assert(NT % 64 == 0 && MPT >= 2, "shape");
  __shared__ T st[TMP];
  __shared__ T sR[kMaxSpan], sL[kMaxSpan], sA[kMaxSpan + 1], sB[kMaxSpan + 1];
  __shared__ T edge[2][2][NW];

  const int tid = threadIdx.x;
  const int slot = xcd_tile(blockIdx.x, gridDim.x);
  const int tix = p.tile_idx[slot];
  const Tile tl = p.tiles[tix];
  int S = p.span_dev ? *p.span_dev : p.span;
  S = S < kMaxSpan ? S : kMaxSpan;
  if (S <= 0) return;

  // per-step boundary data: input flux waveforms, and the Dirichlet values of
  // nodes 0 and M-1 (level n0 from the state, later levels from f_A, f_B)
  for (int s = tid; s < S; s += NT) {
    sR[s] = (tl.fr >= 0) ? p.flux[static_cast<int64_t>(2 * tl.fr + 1) * p.ld + s] : T(0);
    sL[s] = (tl.fl >= 0) ? p.flux[static_cast<int64_t>(2 * tl.fl + 0) * p.ld + s] : T(0);
  }
  for (int s = tid; s <= S; s += NT) {
    sA[s] = (s == 0) ? p.state_in[p.M] : p.fa[p.n0 + s];
    sB[s] = (s == 0) ? p.state_in[2 * p.M - 1] : p.fb[p.n0 + s];
  }

  T u[MPT], uo[MPT];
  {
    T t1[MPT], t0[MPT];
    load_level<T, NT, MPT>(p.state_in + p.M, tl.a, p.M, t1);  // level n0
    load_level<T, NT, MPT>(p.state_in, tl.a, p.M, t0);        // level n0-1
    transpose_in<T, NT, MPT>(t1, st, u);
    transpose_in<T, NT, MPT>(t0, st, uo);
  }

  UpdateCtx<T, NT, MPT> c;
  c.edge = edge;
  c.sR = sR;
  c.sL = sL;
  c.sA = sA;
  c.sB = sB;
  c.base = tl.a + static_cast<int64_t>(tid) * MPT;
  c.lane = tid & 63;
  c.wv = tid >> 6;
  c.lmode = tl.lmode;
  c.rmode = tl.rmode;
  c.dl = -1000;
  c.d0 = -1000;
  c.gen = false;
  c.rb = 0;
  c.re = 0;
  if (GEN) {
    // offsets of the special nodes from this lane's first node, clamped so
    // that far-away nodes match no element
    auto rel = [](int64_t node, int64_t base) -> int {
      const int64_t d = node - base;
      return (d < -2 || d > MPT + 1) ? -1000 : static_cast<int>(d);
    };
    c.dl = (tl.lin == kNoNode) ? -1000 : rel(tl.lin, c.base);
    c.d0 = rel(0, c.base);
    const bool mine = (c.dl >= 0 && c.dl < MPT) || (c.d0 >= 0 && c.d0 < MPT);
    c.gen = __any(mine) != 0;
    c.rb = p.rec_ptr ? p.rec_ptr[slot] : 0;
    c.re = p.rec_ptr ? p.rec_ptr[slot + 1] : 0;
  }
  c.rs = GEN ? load_slots(p.rec_node, p.rec_id, c.rb, c.re) : RecSlots{0, {}, {}};
  const int64_t rlo = tl.out_lo > tl.a ? tl.out_lo : tl.a;
  const int64_t rhi = tl.out_hi < tl.a + TM - 1 ? tl.out_hi : tl.a + TM - 1;
  const int xlo = static_cast<int>(rlo - tl.a);
  const int xhi = static_cast<int>(rhi - tl.a);

  int s = 0;
  for (; s + 1 < S; s += 2) {
    one_step<T, NT, MPT, GEN>(p, c, u, uo, s);      // uo <- level n0+s+1
    one_step<T, NT, MPT, GEN>(p, c, uo, u, s + 1);  // u  <- level n0+s+2
  }
  if (s < S) {
    one_step<T, NT, MPT, GEN>(p, c, u, uo, s);  // uo = level n0+S, u = n0+S-1
    stage_out<T, NT, MPT>(p.state_out, tl.a, xlo, xhi, st, u);
    stage_out<T, NT, MPT>(p.state_out + p.M, tl.a, xlo, xhi, st, uo);
  } else {
    stage_out<T, NT, MPT>(p.state_out, tl.a, xlo, xhi, st, uo);
    stage_out<T, NT, MPT>(p.state_out + p.M, tl.a, xlo, xhi, st, u);
  }
  // Dirichlet nodes next to the region
  if (tid == 0 && tl.lmode == kEndDirichlet) {
    p.state_out[0] = sA[S - 1];
    p.state_out[p.M] = sA[S];
  }
  if (tid == NT - 1 && tl.rmode == kEndDirichlet) {
    p.state_out[p.M - 1] = sB[S - 1];
    p.state_out[2 * p.M - 1] = sB[S];
  }
}

// ---------------------------------------------------------------------------
// Select (Sec. 2.4, Sec. 3 Eq. (19)).  mode 0: min(shat, fixed_span).
// mode 1: S = min(shat, min_rows min(q_row, cone) + cone), q_row = leading
// exact zeros of a predicted flux waveform (shat samples).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_select(const SelectArgs<T> a0) {
  SelectArgs<T> a = a0;
  if (a0.shat_dev) a.shat = *a0.shat_dev;
  if (a.shat <= 0) {
    if (threadIdx.x == 0) *a.span_dev = 0;
    return;
  }
  __shared__ int smin;
  if (threadIdx.x == 0) smin = 0x7fffffff;
  __syncthreads();
  if (a.mode == 1) {
    int local = 0x7fffffff;
    for (int r = threadIdx.x; r < a.n_rows; r += 256) {
      const T* f = a.flux + static_cast<int64_t>(r) * a.ld;
      int q = 0;
      while (q < a.shat && f[q] == T(0)) ++q;
      q = q < a.cone ? q : a.cone;
      local = q < local ? q : local;
    }
    atomicMin(&smin, local);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int S;
    if (a.mode == 0) {
      S = a.shat < a.fixed_span ? a.shat : a.fixed_span;
    } else {
      S = a.shat;
      if (a.n_rows > 0) {
        const long long lim = static_cast<long long>(smin) + a.cone;
        if (lim < S) S = static_cast<int>(lim);
      }
    }
    *a.span_dev = S;
  }
}

// The same select for many rows: one wave per row finds the row's first
// nonzero sample with a ballot over 64 samples at a time (the leading exact
// zeros, capped by shat and the cone, as above) and the waves' minimum goes
// to *qmin; k_select_final then forms the span and restores *qmin.
template <typename T>
__global__ __launch_bounds__(256) void k_select_rows(const SelectArgs<T> a) {
  const int shat = a.shat_dev ? *a.shat_dev : a.shat;
  if (shat <= 0) return;
  const int lane = threadIdx.x & 63;
  const int wave = static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int n_waves = static_cast<int>((gridDim.x * blockDim.x) >> 6);
  int wmin = 0x7fffffff;
  for (int r = wave; r < a.n_rows; r += n_waves) {
    const T* f = a.flux + static_cast<int64_t>(r) * a.ld;
    int q = shat;
    for (int s0 = 0; s0 < shat; s0 += 64) {
      const int s = s0 + lane;
      const bool nz = s < shat && !(f[s] == T(0));
      const uint64_t m = __ballot(nz);
      if (m != 0) {
        q = s0 + __builtin_ctzll(m);
        break;
      }
    }
    q = q < a.cone ? q : a.cone;
    wmin = q < wmin ? q : wmin;
  }
  // one atomic per work-group (the waves' minimum through LDS): the atomics
  // of one address serialise
  __shared__ int gmin[4];
  if (lane == 0) gmin[threadIdx.x >> 6] = wmin;
  __syncthreads();
  if (threadIdx.x == 0) {
    int m = gmin[0];
    for (int w = 1; w < 4; ++w) m = gmin[w] < m ? gmin[w] : m;
    if (m != 0x7fffffff) atomicMin(a.qmin, m);
  }
}

template <typename T>
__global__ __launch_bounds__(64) void k_select_final(const SelectArgs<T> a) {
  if (threadIdx.x == 0) {
    const int shat = a.shat_dev ? *a.shat_dev : a.shat;
    int S = shat > 0 ? shat : 0;
    if (S > 0 && a.n_rows > 0) {
      const long long lim = static_cast<long long>(*a.qmin) + a.cone;
      if (lim < S) S = static_cast<int>(lim);
    }
    *a.span_dev = S;
    *a.qmin = 0x7fffffff;
  }
}

// Control block of the adaptive solve (Sec. 2.6): the first predictive span
// is given; after each round the level advances by the chosen span and the
// next predictive span is ceil((1 + beta) S), capped by s_max and the
// levels left (0 once the solve is done).
__global__ __launch_bounds__(64) void k_quiet_init(QuietCtl* c, int64_t n0, int64_t n_end,
                                                   int32_t shat0, int32_t s_max,
                                                   double beta) {
  if (threadIdx.x == 0) {
    c->n0 = n0;
    c->n_end = n_end;
    c->shat = n_end > n0 ? shat0 : 0;
    c->span = 0;
    c->parity = 0;
    c->s_max = s_max;
    c->beta = beta;
    c->qmin = 0x7fffffff;
  }
}

__global__ __launch_bounds__(64) void k_quiet_next(QuietCtl* c) {
  if (threadIdx.x == 0) {
    const int32_t S = c->span;
    if (S > 0) {
      c->n0 += S;
      c->parity ^= 1;
    }
    const int64_t rem = c->n_end - c->n0;
    int64_t sh = static_cast<int64_t>(ceil((1.0 + c->beta) * static_cast<double>(S)));
    if (sh > c->s_max) sh = c->s_max;
    if (sh > rem) sh = rem;
    if (sh < 1) sh = 1;
    c->shat = (S > 0 && rem > 0) ? static_cast<int32_t>(sh) : 0;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy_if(T* __restrict__ dst, const T* __restrict__ src,
                                                 int64_t n, const int32_t* flag) {
  if (*flag == 0) return;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride)
    dst[i] = src[i];
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy(T* __restrict__ dst, const T* __restrict__ src,
                                             int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride)
    dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_predict(const PredictArgs<T>& a, int shmem_nodes, hipStream_t s) {
  if (a.N < 2) return hipSuccess;
  const size_t shm = static_cast<size_t>(2 * shmem_nodes) * sizeof(T);
  hipLaunchKernelGGL(k_predict<T>, dim3(2 * (a.N - 1)), dim3(64), shm, s, a);
  return hipGetLastError();
}

static const Shape kShapes[] = {
#define RSWR_SHAPE_ENTRY(a, b) {a, b},
    RSWR_SHAPES(RSWR_SHAPE_ENTRY)
#undef RSWR_SHAPE_ENTRY
};

int n_shapes() { return static_cast<int>(sizeof(kShapes) / sizeof(kShapes[0])); }
Shape shape_at(int i) { return kShapes[i]; }
bool shape_built(int threads, int per_thread) {
  for (const Shape& s : kShapes)
    if (s.threads == threads && s.per_thread == per_thread) return true;
  return false;
}

template <typename T>
hipError_t launch_update(const UpdateArgs<T>& a, int threads, int per_thread,
                         bool general, hipStream_t s) {
  if (a.n_tiles <= 0) return hipSuccess;
#define RSWR_LAUNCH(NT_, MPT_)                                                    \
  if (threads == NT_ && per_thread == MPT_) {                                   \
    if (general)                                                                \
      hipLaunchKernelGGL((k_update<T, NT_, MPT_, true>), dim3(a.n_tiles),       \
                         dim3(NT_), 0, s, a);                                   \
    else                                                                        \
      hipLaunchKernelGGL((k_update<T, NT_, MPT_, false>), dim3(a.n_tiles),      \
                         dim3(NT_), 0, s, a);                                   \
    return hipGetLastError();                                                   \
  }
  RSWR_SHAPES(RSWR_LAUNCH)
#undef RSWR_LAUNCH
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_select(const SelectArgs<T>& a, hipStream_t s) {
  if (a.mode == 1 && a.qmin) {
    // at least four rows per wave, at most 512 work-groups of four waves
    // (grid-stride)
    if (a.n_rows > 0) {
      const int64_t groups = std::min<int64_t>((int64_t(a.n_rows) + 15) / 16, 512);
      hipLaunchKernelGGL(k_select_rows<T>, dim3(static_cast<unsigned>(groups)), dim3(256), 0,
                         s, a);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_select_final<T>, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_select<T>, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_quiet_init(QuietCtl* c, int64_t n0, int64_t n_end, int32_t shat0,
                             int32_t s_max, double beta, hipStream_t s) {
  hipLaunchKernelGGL(k_quiet_init, dim3(1), dim3(64), 0, s, c, n0, n_end, shat0, s_max, beta);
  return hipGetLastError();
}

hipError_t launch_quiet_next(QuietCtl* c, hipStream_t s) {
  hipLaunchKernelGGL(k_quiet_next, dim3(1), dim3(64), 0, s, c);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy_if(T* dst, const T* src, int64_t n, const int32_t* flag,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_copy_if<T>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                     dst, src, n, flag);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy_y(T* dst, const T* src, int64_t n,
                                                int64_t stride) {
  T* const d = at_y(dst, stride);
  const T* const x = at_y(src, stride);
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += step)
    d[i] = x[i];
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill_y(T* dst, T v, int64_t n, int64_t stride) {
  T* const d = at_y(dst, stride);
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += step)
    d[i] = v;
}

template <typename T>
hipError_t launch_copy_y(T* dst, const T* src, int64_t n, int32_t ny, int64_t stride,
                         hipStream_t s) {
  if (n <= 0 || ny <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_copy_y<T>, dim3(static_cast<unsigned>(blocks), ny), dim3(256), 0, s,
                     dst, src, n, stride);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_y(T* dst, T v, int64_t n, int32_t ny, int64_t stride, hipStream_t s) {
  if (n <= 0 || ny <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_fill_y<T>, dim3(static_cast<unsigned>(blocks), ny), dim3(256), 0, s,
                     dst, v, n, stride);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(T* dst, const T* src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_copy<T>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                     dst, src, n);
  return hipGetLastError();
}

template hipError_t launch_predict<float>(const PredictArgs<float>&, int, hipStream_t);
template hipError_t launch_predict<double>(const PredictArgs<double>&, int, hipStream_t);
template hipError_t launch_update<float>(const UpdateArgs<float>&, int, int, bool,
                                         hipStream_t);
template hipError_t launch_update<double>(const UpdateArgs<double>&, int, int, bool,
                                          hipStream_t);
template hipError_t launch_select<float>(const SelectArgs<float>&, hipStream_t);
template hipError_t launch_select<double>(const SelectArgs<double>&, hipStream_t);
template hipError_t launch_copy<float>(float*, const float*, int64_t, hipStream_t);
template hipError_t launch_copy<double>(double*, const double*, int64_t, hipStream_t);
template hipError_t launch_copy_if<float>(float*, const float*, int64_t, const int32_t*,
                                          hipStream_t);
template hipError_t launch_copy_y<float>(float*, const float*, int64_t, int32_t, int64_t,
                                         hipStream_t);
template hipError_t launch_copy_y<double>(double*, const double*, int64_t, int32_t, int64_t,
                                          hipStream_t);
template hipError_t launch_fill_y<float>(float*, float, int64_t, int32_t, int64_t,
                                         hipStream_t);
template hipError_t launch_fill_y<double>(double*, double, int64_t, int32_t, int64_t,
                                          hipStream_t);
template hipError_t launch_copy_if<double>(double*, const double*, int64_t, const int32_t*,
                                           hipStream_t);

}  // namespace rswr
