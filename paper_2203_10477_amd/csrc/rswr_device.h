// rswr_device.h -- device helpers shared by the forward and adjoint kernels.
#pragma once

#include "rswr_internal.h"

namespace rswr {

__device__ __forceinline__ float fma_(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}
__device__ __forceinline__ double fma_(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}

// Whole-wave lane shifts (DPP wave_shr:1 / wave_shl:1): a VALU move, no LDS
// round trip.  Lane l receives lane l-1's (prev) or lane l+1's (next) value;
// the lane at the wave's end receives its own value and is overwritten by
// the caller.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
  return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(
      static_cast<int>(v), static_cast<int>(v), CTRL, 0xf, 0xf, false));
}
constexpr int kWaveShr1 = 0x138;
constexpr int kWaveShl1 = 0x130;

// The same shifts with zero fill: the lane at the wave's end receives 0
// (bound_ctrl), so every lane is written and no copy of the source is made.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32z(uint32_t v) {
  return static_cast<uint32_t>(
      __builtin_amdgcn_mov_dpp(static_cast<int>(v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ float lane_shift_z(float v) {
  return __builtin_bit_cast(float, dpp32z<CTRL>(__builtin_bit_cast(uint32_t, v)));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift_z(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint64_t lo = dpp32z<CTRL>(static_cast<uint32_t>(b));
  const uint64_t hi = dpp32z<CTRL>(static_cast<uint32_t>(b >> 32));
  return __builtin_bit_cast(double, lo | (hi << 32));
}

// Lane shift whose lane without a source (lane 0 for a right shift, lane 63
// for a left shift) takes `old` instead: one DPP move sets a wave's end value
// together with the shift.
template <int CTRL>
__device__ __forceinline__ float lane_shift_old(float old, float v) {
  return __builtin_bit_cast(
      float, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(
                 __builtin_bit_cast(int, old), __builtin_bit_cast(int, v), CTRL, 0xf, 0xf,
                 false)));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift_old(double old, double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint64_t o = __builtin_bit_cast(uint64_t, old);
  const uint64_t lo = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(
      static_cast<int>(static_cast<uint32_t>(o)), static_cast<int>(static_cast<uint32_t>(b)),
      CTRL, 0xf, 0xf, false));
  const uint64_t hi = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(
      static_cast<int>(static_cast<uint32_t>(o >> 32)),
      static_cast<int>(static_cast<uint32_t>(b >> 32)), CTRL, 0xf, 0xf, false));
  return __builtin_bit_cast(double, lo | (hi << 32));
}

// A wave-uniform value kept in a vector register, so an instruction may
// combine it with a scalar operand (one scalar source per VALU instruction).
template <typename T>
__device__ __forceinline__ T in_vgpr(T v) {
  asm("" : "+v"(v));
  return v;
}

// Problem y's copy of a batched buffer: `stride` bytes per problem.
template <typename P>
__device__ __forceinline__ P* at_y(P* ptr, int64_t stride) {
  return ptr ? reinterpret_cast<P*>(reinterpret_cast<uintptr_t>(ptr) +
                                    static_cast<uintptr_t>(blockIdx.y * stride))
             : ptr;
}

// A wave-uniform integer re-read in every loop iteration: tests on it stay
// scalar compares and branches inside the loop instead of being hoisted out
// as per-lane masks that occupy (and spill) scalar register pairs.
__device__ __forceinline__ int uni(int x) {
  asm volatile("" : "+s"(x));
  return x;
}

template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
  return __builtin_bit_cast(float, dpp32<CTRL>(__builtin_bit_cast(uint32_t, v)));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint64_t lo = dpp32<CTRL>(static_cast<uint32_t>(b));
  const uint64_t hi = dpp32<CTRL>(static_cast<uint32_t>(b >> 32));
  return __builtin_bit_cast(double, lo | (hi << 32));
}

// Value of lane l (wave-uniform l) in every lane: v_readlane, no LDS round
// trip.
__device__ __forceinline__ float rd_lane(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double rd_lane(double v, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint64_t lo = static_cast<uint32_t>(
      __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(b)), l));
  const uint64_t hi = static_cast<uint32_t>(
      __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(b >> 32)), l));
  return __builtin_bit_cast(double, lo | (hi << 32));
}
// v with lane l's element replaced by the wave-uniform x.
template <typename T>
__device__ __forceinline__ T wr_lane(T x, int l, T v, int lane) {
  return lane == l ? x : v;
}

// Second-order leapfrog for Eq. (1) at one node.
template <typename T>
__device__ __forceinline__ T leap(T c2, T k, T ul, T u, T ur, T u_old) {
  const T s = ul + ur;
  const T t = fma_(k, u, -u_old);
  return fma_(c2, s, t);
}

// Work-groups are dispatched to the 8 XCDs round-robin by block id.  Give
// each XCD a contiguous run of tiles, so neighbouring tiles (which share
// overlap nodes) meet in the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = bid & 7, i = bid >> 3;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

__device__ __forceinline__ int pad32(int x) { return x + (x >> 5); }

// LDS slot of tile node x in the staging buffer.  With an odd number of
// nodes per lane, lane t's elements (stride MPT) already fall in distinct
// banks, so the plain layout is conflict-free and every address is a
// per-lane base plus a compile-time offset; even MPT pads one slot per 32.
template <int MPT>
__device__ __forceinline__ int lds_slot(int x) {
  if constexpr (MPT % 2 == 1)
    return x;
  else
    return pad32(x);
}

// Issue every load of a level before the first wait: node a + it*NT + tid
// into tmp[it], through a range resource over the region's nodes that lie
// in [0, M) -- 32-bit offsets from the first of them, and every node outside
// the range (before node 0, after node M-1) reads as zero in hardware, with
// no clamp, select or branch.  The offsets may be negative (regions that
// start before node 0): as unsigned values they lie far beyond the range.
template <typename T, int NT, int MPT>
__device__ __forceinline__ void load_level(const T* __restrict__ src, int64_t a,
                                           int64_t M, T (&tmp)[MPT]) {
  constexpr int TM = NT * MPT;
  const int tid = static_cast<int>(threadIdx.x);
  const int64_t lo = a < 0 ? 0 : a;
  const int64_t hi = a + TM < M ? a + TM : M;
  const int n = hi > lo ? static_cast<int>(hi - lo) : 0;
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(src) + lo, 0, n * sizeof(T), 0x00020000);
  const int shift = static_cast<int>(a - lo);  // <= 0
#pragma unroll
  for (int it = 0; it < MPT; ++it) {
    int off = (shift + it * NT + tid) * static_cast<int>(sizeof(T));
    // the whole offset in the vector operand: a part folded into the
    // instruction or scalar offset would escape the range check
    asm("" : "+v"(off));
    if constexpr (sizeof(T) == 4)
      tmp[it] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    else
      tmp[it] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  }
}

// Unit-stride (coalesced) values -> LDS -> this lane's MPT consecutive nodes.
template <typename T, int NT, int MPT>
__device__ __forceinline__ void transpose_in(const T (&tmp)[MPT], T* st, T (&v)[MPT]) {
#pragma unroll
  for (int it = 0; it < MPT; ++it)
    st[lds_slot<MPT>(it * NT + static_cast<int>(threadIdx.x))] = tmp[it];
  __syncthreads();
#pragma unroll
  for (int e = 0; e < MPT; ++e) v[e] = st[lds_slot<MPT>(static_cast<int>(threadIdx.x) * MPT + e)];
  __syncthreads();
}

// Raw buffer stores (vector memory) through a resource that covers exactly
// [base, base + bytes): the hardware drops every store whose offset falls
// outside (a negative offset reads as a huge unsigned one).  Dword 3 of the
// descriptor: 32-bit data format, as gfx9-family buffer accesses need.
constexpr int kBufDword3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t range_rsrc(void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(base, 0, bytes, kBufDword3);
}

// Cache policy of the state loads and stores that the tiles of one launch
// exchange with each other (the one-launch span loop): device scope (sc1),
// so a value stored on one XCD is seen by a load on another without writing
// back or invalidating the XCDs' separate L2 caches.  0: the default policy.
constexpr int kCohAux = 16;

template <int AUX = 0>
__device__ __forceinline__ void range_store(float v, __amdgpu_buffer_rsrc_t r, int off) {
  // the whole offset sits in the vector operand (no folded instruction
  // offset), so the range check sees exactly this value
  asm("" : "+v"(off));
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, AUX);
}
template <int AUX = 0>
__device__ __forceinline__ void range_store(double v, __amdgpu_buffer_rsrc_t r, int off) {
  typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
  asm("" : "+v"(off));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, AUX);
}

// Device-coherent load of element idx of a row seen through `r` (a range
// resource over the row): indices outside the row read 0.
template <typename T>
__device__ __forceinline__ T ld_coh(__amdgpu_buffer_rsrc_t r, int64_t idx);
template <>
__device__ __forceinline__ float ld_coh<float>(__amdgpu_buffer_rsrc_t r, int64_t idx) {
  int off = static_cast<int>(idx * 4);
  asm("" : "+v"(off));
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kCohAux));
}
template <>
__device__ __forceinline__ double ld_coh<double>(__amdgpu_buffer_rsrc_t r, int64_t idx) {
  int off = static_cast<int>(idx * 8);
  asm("" : "+v"(off));
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kCohAux));
}

// A range resource over row `row` (0 or 1) of a [2][M] state.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t state_row(const T* st, int64_t M, int row) {
  return range_rsrc(const_cast<T*>(st) + row * M, static_cast<int>(M * sizeof(T)));
}

// load_level through a range resource over the row with the device-coherent
// policy; nodes outside [0, M) read 0.
template <typename T, int NT, int MPT>
__device__ __forceinline__ void load_level_coh(__amdgpu_buffer_rsrc_t r, int64_t a,
                                               T (&tmp)[MPT]) {
  const int tid = static_cast<int>(threadIdx.x);
#pragma unroll
  for (int it = 0; it < MPT; ++it) tmp[it] = ld_coh<T>(r, a + it * NT + tid);
}

// This lane's nodes -> LDS -> unit-stride stores of the stored range
// [a + xlo, a + xhi] (offsets relative to the region start).  Every row of
// NT nodes stores unmasked through a resource covering exactly that range;
// nodes outside it are dropped by the range check.
template <typename T, int NT, int MPT, int AUX = 0>
__device__ __forceinline__ void stage_out(T* __restrict__ dst, int64_t a, int xlo,
                                          int xhi, T* st, const T (&v)[MPT]) {
  const int tid = static_cast<int>(threadIdx.x);
#pragma unroll
  for (int e = 0; e < MPT; ++e) st[lds_slot<MPT>(tid * MPT + e)] = v[e];
  __syncthreads();
  if (xlo <= xhi) {
    const __amdgpu_buffer_rsrc_t r =
        range_rsrc(dst + a + xlo, (xhi - xlo + 1) * static_cast<int>(sizeof(T)));
    const int base = (tid - xlo) * static_cast<int>(sizeof(T));
    T tmp[MPT];
#pragma unroll
    for (int it = 0; it < MPT; ++it) tmp[it] = st[lds_slot<MPT>(it * NT + tid)];
#pragma unroll
    for (int it = 0; it < MPT; ++it)
      range_store<AUX>(tmp[it], r, base + it * NT * static_cast<int>(sizeof(T)));
  }
  __syncthreads();
}

// Value of element d of a register array without indexing it: an indexed
// read (or a select chain the compiler folds into one) would move the whole
// array to scratch memory.
template <typename T> struct Bits;
template <> struct Bits<float> { using U = uint32_t; };
template <> struct Bits<double> { using U = uint64_t; };

template <typename T, int MPT>
__device__ __forceinline__ T pick(const T (&v)[MPT], int64_t d) {
  using U = typename Bits<T>::U;
  U acc = 0;
#pragma unroll
  for (int e = 0; e < MPT; ++e) {
    const U m = static_cast<U>(0) - static_cast<U>(d == e);
    acc |= __builtin_bit_cast(U, v[e]) & m;
  }
  return __builtin_bit_cast(T, acc);
}

// Up to kRecSlots receivers (or adjoint sources) of one tile, held in
// wave-uniform registers for the whole span; any further ones are read from
// memory each step.  Slots keep the list order.
struct RecSlots {
  int n;
  int64_t node[kRecSlots];
  int32_t id[kRecSlots];
};

__device__ __forceinline__ RecSlots load_slots(const int64_t* node, const int32_t* id, int b,
                                               int e) {
  RecSlots r;
  r.n = (e - b < kRecSlots) ? e - b : kRecSlots;
#pragma unroll
  for (int q = 0; q < kRecSlots; ++q) {
    const bool h = q < r.n;
    r.node[q] = h ? node[b + q] : kNoNode;
    r.id[q] = h ? id[b + q] : 0;
  }
  return r;
}

// Element access with a wave-uniform runtime index e.  The array is viewed
// as a vector of registers and read or written in the GPU's register
// indexing mode (a few instructions, no branches, no scratch memory).  A
// vector longer than 32 dwords cannot be indexed that way, so longer arrays
// split into halves first (one uniform branch per level; each leaf ends in
// an empty asm statement naming its range, which keeps the compiler from
// merging the leaves into one runtime-indexed access to the array).
template <typename T, int N>
struct RegVec {
  typedef T type __attribute__((ext_vector_type(N)));
};

template <int OFF, int LEN, typename T, int MPT>
__device__ __forceinline__ T elem_range(const T (&v)[MPT], int e) {
  if constexpr (LEN * sizeof(T) <= 128) {
    typename RegVec<T, LEN>::type t;
#pragma unroll
    for (int i = 0; i < LEN; ++i) t[i] = v[OFF + i];
    const T x = t[e - OFF];
    asm volatile("; elem %0" ::"n"(OFF));
    return x;
  } else {
    constexpr int H = LEN / 2;
    if (e < OFF + H) return elem_range<OFF, H>(v, e);
    return elem_range<OFF + H, LEN - H>(v, e);
  }
}

template <int OFF, int LEN, typename T, int MPT>
__device__ __forceinline__ void add_range(T (&v)[MPT], int e, T g, bool mine) {
  if constexpr (LEN * sizeof(T) <= 128) {
    typename RegVec<T, LEN>::type t;
#pragma unroll
    for (int i = 0; i < LEN; ++i) t[i] = v[OFF + i];
    const T x = t[e - OFF];
    t[e - OFF] = mine ? x + g : x;
#pragma unroll
    for (int i = 0; i < LEN; ++i) v[OFF + i] = t[i];
    asm volatile("; add %0" ::"n"(OFF));
  } else {
    constexpr int H = LEN / 2;
    if (e < OFF + H)
      add_range<OFF, H>(v, e, g, mine);
    else
      add_range<OFF + H, LEN - H>(v, e, g, mine);
  }
}

// v[e], e wave-uniform in [0, MPT).
template <typename T, int MPT>
__device__ __forceinline__ T elem_at(const T (&v)[MPT], int e) {
  return elem_range<0, MPT>(v, e);
}

// v[e] += g in the lanes where `mine` holds, e wave-uniform in [0, MPT).
template <typename T, int MPT>
__device__ __forceinline__ void add_at(T (&v)[MPT], int e, T g, bool mine) {
  add_range<0, MPT>(v, e, g, mine);
}

// Value just outside the region: zero data, the input ghost (Eqs. (6)-(7)
// with a centred flux), or the Dirichlet value of Eq. (3).
template <typename T>
__device__ __forceinline__ T end_value(int mode, T ghost, T dir) {
  return (mode == kEndGhost) ? ghost : ((mode == kEndDirichlet) ? dir : T(0));
}

// One leapfrog step of this lane's nodes.
// cur = level n, old = level n-1 on entry; old = level n+1 on exit.
// GEN: element dl takes the left-input ghost as its left neighbour and
// element d0 is the Dirichlet node 0 (offsets relative to this lane's first
// node; out-of-range offsets match no element).
template <typename T, int MPT, bool GEN>
__device__ __forceinline__ void step_chunk(const T (&cur)[MPT], T (&old)[MPT],
                                           T L, T R, T c2, T k, int dl, int d0,
                                           T ghost, T da) {
#pragma unroll
  for (int e = 0; e < MPT; ++e) {
    T ul = (e == 0) ? L : cur[e - 1];
    const T ur = (e == MPT - 1) ? R : cur[e + 1];
    if (GEN) ul = (e == dl) ? ghost : ul;
    T v = leap(c2, k, ul, cur[e], ur, old[e]);
    if (GEN) v = (e == d0) ? da : v;
    old[e] = v;
  }
}

// Kernel shapes (threads per work-group, nodes per lane) built into the
// library; the update and adjoint launchers dispatch over this list.
#define RSWR_SHAPES(X) \
  X(64, 2)             \
  X(64, 4)             \
  X(64, 8)             \
  X(64, 16)            \
  X(64, 33)            \
  X(64, 65)            \
  X(128, 8)            \
  X(128, 33)           \
  X(192, 22)           \
  X(256, 8)            \
  X(256, 16)           \
  X(320, 13)           \
  X(512, 8)            \
  X(512, 12)

}  // namespace rswr
