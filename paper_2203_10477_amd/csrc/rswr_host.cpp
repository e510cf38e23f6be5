// rswr_host.cpp -- plan construction and host driver of the RSWR C-ABI.
//
// Method: Wei & Zhao, arXiv 2203.10477.  The plan holds the decomposition
// (Sec. 2.2 Eqs. (4)-(5), Sec. 3), the span rules (Sec. 2.4 Eq. (10) and the
// light-cone limit of the discrete scheme) and the update tiles; the driver
// runs the redo loop of Sec. 2.6 as predict -> select -> update per span and
// records it into a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <utility>
#include <vector>

#include "../../include/rswr.h"
#include "rswr_internal.h"

using rswr::Tile;

namespace {

thread_local std::string g_last_error;

rswr_status_t fail(rswr_status_t st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

rswr_status_t hip_fail(hipError_t e, const char* what) {
  return fail(RSWR_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define RSWR_HIP(call)                                  \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #call);   \
  } while (0)

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

struct DevTables {
  Tile* tiles = nullptr;
  int32_t* idx = nullptr;  // general tiles first, then the plain ones
  int64_t* lo = nullptr;
  int64_t* hi = nullptr;
  int32_t* src_ptr = nullptr;  // per-tile interior sources (plans with sources)
  int64_t* src_node = nullptr;
  int32_t* src_id = nullptr;
  int32_t* dep_ptr = nullptr;  // waits of the one-launch loop (plans with persist_ok)
  int32_t* dep = nullptr;
  hipStream_t capture = nullptr;
};

// Everything a recorded graph depends on: the entry point and its pointer
// and size arguments.
using GraphKey = std::vector<int64_t>;

struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec;
};

// Workspace of rswr_solve_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never names it directly: its
// device address on each GPU comes from hipGetSymbolAddress (scratch_on).
constexpr size_t kScratchBytes = RSWR_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

}  // namespace

struct rswr_plan_s {
  int64_t M = 0;
  int32_t N = 0, P = 0, dtype = 0, mode = 0;
  double dx = 0, dt = 0, lam = 0, beta = 0.1;
  std::vector<int64_t> lo, hi, own_lo, own_hi;
  int32_t S_cone = 0, S_paper = 0, S = 0, S_max = 0, flux_ld = 0;
  int32_t threads = 0, per_thread = 0;
  std::vector<Tile> tiles;
  std::vector<int32_t> idx;  // tile order of the launches: general ones first
  int32_t n_gen = 0;
  bool fused = false;  // rswr_solve runs one fused launch per span
  // interior point sources (the pulse sources of Sec. 4): nodes, the
  // caller's device samples [n][src_ld], and per tile three runs of
  // (node, source id) -- register region, left frame, right frame
  std::vector<int64_t> src_node;
  const void* src_amp = nullptr;
  int64_t src_ld = 0;
  std::vector<int32_t> src_ptr;  // [3 * n_tiles + 1]
  std::vector<int64_t> src_tnode;
  std::vector<int32_t> src_tid;
  // the one-launch loop (rswr_persist.hip): plain fused plans; per tile the
  // tiles it waits for before each span (CSR)
  bool persist_ok = false;
  std::vector<int32_t> dep_ptr, dep;
  std::mutex mu;
  std::map<int, DevTables> dev;
  std::vector<GraphEntry> graphs;
};

namespace {

// ---------------------------------------------------------------------------
// Decomposition (Sec. 2.2, Sec. 3).
// ---------------------------------------------------------------------------
rswr_status_t check_windows(rswr_plan_s& p) {
  const int64_t M = p.M;
  const int32_t N = p.N;
  if (p.lo[0] != 0 || p.hi[N - 1] != M - 1)
    return fail(RSWR_ERR_LAYOUT, "windows must start at node 0 and end at node M-1");
  for (int32_t i = 0; i < N; ++i)
    if (p.hi[i] - p.lo[i] < 2) return fail(RSWR_ERR_LAYOUT, "window narrower than 3 nodes");
  for (int32_t i = 0; i + 1 < N; ++i) {
    // X_{iA} < X_{(i+1)A} < X_{iB} < X_{(i+1)B}  (Eq. (4))
    if (!(p.lo[i] < p.lo[i + 1] && p.lo[i + 1] < p.hi[i] && p.hi[i] < p.hi[i + 1]))
      return fail(RSWR_ERR_LAYOUT, "windows " + std::to_string(i) + " and " +
                                       std::to_string(i + 1) + " do not overlap in order");
  }
  p.own_lo.resize(N);
  p.own_hi.resize(N);
  for (int32_t i = 0; i < N; ++i) {
    // gluing, Eq. (15): a shared node belongs to the lower-indexed window
    p.own_lo[i] = (i == 0) ? 0 : p.hi[i - 1] + 1;
    p.own_hi[i] = (i == N - 1) ? M - 1 : p.hi[i];
    if (p.own_hi[i] < p.own_lo[i]) return fail(RSWR_ERR_LAYOUT, "empty owned range");
  }
  return RSWR_OK;
}

rswr_status_t uniform_windows(rswr_plan_s& p) {
  const int64_t M = p.M;
  const int32_t N = p.N;
  if (N > 1 && (p.P < 2 || (p.P & 1)))
    return fail(RSWR_ERR_LAYOUT, "overlap must be an even number >= 2 of grid intervals");
  const int64_t h = p.P / 2;
  std::vector<int64_t> c(N + 1);
  for (int32_t i = 0; i <= N; ++i) c[i] = (2 * int64_t(i) * (M - 1) + N) / (2 * int64_t(N));
  p.lo.resize(N);
  p.hi.resize(N);
  for (int32_t i = 0; i < N; ++i) {
    if (c[i + 1] - c[i] < 1) return fail(RSWR_ERR_LAYOUT, "more windows than grid intervals");
    p.lo[i] = (i == 0) ? 0 : c[i] - h;
    p.hi[i] = (i == N - 1) ? M - 1 : c[i + 1] + h;
  }
  if (N > 1 && (c[1] - c[0] < h + 1 || c[N] - c[N - 1] < h + 1))
    return fail(RSWR_ERR_LAYOUT, "end cores must be at least overlap/2 + 1 nodes");
  return check_windows(p);
}

// Smallest distance between an input boundary and an output boundary of the
// same window: a zero-flux error entering at the input reaches an output at
// distance d after d levels, so predicted output fluxes are exact for that
// many levels (the discrete form of the Prediction Validation Theorem).
int32_t light_cone_span(const rswr_plan_s& p) {
  int64_t best = std::numeric_limits<int32_t>::max();
  for (int32_t w = 0; w < p.N; ++w) {
    int64_t in[2], out[2];
    int ni = 0, no = 0;
    if (w > 0) {
      in[ni++] = p.lo[w];
      out[no++] = p.hi[w - 1];
    }
    if (w < p.N - 1) {
      in[ni++] = p.hi[w];
      out[no++] = p.lo[w + 1];
    }
    for (int a = 0; a < ni; ++a)
      for (int b = 0; b < no; ++b) best = std::min<int64_t>(best, in[a] > out[b] ? in[a] - out[b] : out[b] - in[a]);
  }
  return static_cast<int32_t>(best);
}

// Waveform Time Span Theorem (Sec. 2.4, Eq. (10)) in steps: S dt < dX/(2a)
// <=> 2 S lam < P with P the narrowest overlap in grid intervals.
int32_t paper_span(const rswr_plan_s& p, int32_t num, int32_t den, bool exact) {
  int64_t P = std::numeric_limits<int32_t>::max();
  for (int32_t i = 0; i + 1 < p.N; ++i) P = std::min(P, p.hi[i] - p.lo[i + 1]);
  if (exact) return static_cast<int32_t>((P * den - 1) / (2 * int64_t(num)));
  int64_t s = 0;
  while (2.0 * double(s + 1) * p.lam < double(P)) ++s;
  return static_cast<int32_t>(s);
}

// ---------------------------------------------------------------------------
// Update tiles.  Window i is covered right to left.  Its first tile ends at
// the window's exact right end -- the right input hi_i (ghost from the flux
// waveform) or, for the last window, node M-2 next to the Dirichlet node
// M-1.  Further tiles end S nodes past the part they store, since zero data
// entering at a cut end moves one node per level.  A tile that would reach
// past the window's exact left end -- the left input lo_i, or node 1 next to
// the Dirichlet node 0 -- starts exactly there instead.  Only a window
// smaller than one tile leaves its left end strictly inside the region; that
// tile is "general" (handled by the general kernel).
// ---------------------------------------------------------------------------
bool build_tiles(const rswr_plan_s& p, int TM, int S, std::vector<Tile>& out) {
  out.clear();
  for (int32_t i = 0; i < p.N; ++i) {
    const int64_t lo = p.lo[i], hi = p.hi[i];
    const int64_t Olo = p.own_lo[i], Ohi = p.own_hi[i];
    const bool last = (i == p.N - 1);
    const int64_t rb0 = last ? p.M - 2 : hi;
    const int32_t rmode0 = last ? rswr::kEndDirichlet : rswr::kEndGhost;
    const int64_t lb0 = (i == 0) ? 1 : lo;
    const int32_t lmode0 = (i == 0) ? rswr::kEndDirichlet : rswr::kEndGhost;
    auto base_tile = [&]() {
      Tile t{};
      t.lin = rswr::kNoNode;
      t.fl = -1;
      t.fr = -1;
      t.window = i;
      return t;
    };
    if (rb0 - lb0 + 1 < TM) {
      // The window is narrower than one region.  A tile ending at the exact
      // right end treats the window's left end as a plain stencil node: node
      // w0 (node 0, or the left input) is wrong from the first level on, so
      // it stores only nodes >= w0 + S.  If that misses part of the owned
      // range, a second tile starting at the exact left end stores it; it
      // treats the right end w1 (node M-1, or the right input) as a plain
      // node and so stores only nodes <= w1 - S.  If the two cannot cover the
      // owned range, one general tile.
      const int64_t w0 = (i == 0) ? 0 : lo;
      const int64_t w1 = last ? p.M - 1 : hi;
      const int64_t split_lo = w0 + S;
      const int64_t split_hi = w1 - S;
      Tile r = base_tile();
      r.a = rb0 - TM + 1;
      r.rmode = rmode0;
      if (!last) r.fr = i;
      r.lmode = rswr::kEndZero;
      r.out_hi = Ohi;
      if (split_lo <= Olo) {
        r.out_lo = Olo;
        out.push_back(r);
        continue;
      }
      if (split_lo - 1 <= split_hi && split_lo <= Ohi) {
        r.out_lo = split_lo;
        Tile l = base_tile();
        l.a = lb0;
        l.lmode = lmode0;
        if (i > 0) l.fl = i - 1;
        l.rmode = rswr::kEndZero;
        l.out_lo = Olo;
        l.out_hi = split_lo - 1;
        out.push_back(r);
        out.push_back(l);
        continue;
      }
      r.general = 1;
      if (i > 0) {
        r.lin = lo;
        r.fl = i - 1;
      }
      r.out_lo = Olo;
      out.push_back(r);
      continue;
    }
    int64_t cur = Ohi;
    bool first = true;
    while (cur >= Olo) {
      Tile t = base_tile();
      int64_t rb;
      if (first) {
        rb = rb0;
        t.rmode = rmode0;
        if (!last) t.fr = i;
      } else {
        rb = cur + S;
        t.rmode = rswr::kEndZero;
        if (rb >= rb0) return false;
      }
      t.a = rb - TM + 1;
      t.lmode = rswr::kEndZero;
      bool exact_left = false;
      if (t.a <= lb0) {
        // only non-first tiles get here (the window is at least one region
        // wide): start exactly at the window's left end
        exact_left = true;
        t.a = lb0;
        t.lmode = lmode0;
        if (i > 0) t.fl = i - 1;
      }
      t.out_hi = cur;
      t.out_lo = exact_left ? Olo : std::max(t.a + S, Olo);
      const int64_t b = t.a + TM - 1;
      if (t.rmode == rswr::kEndZero && t.out_hi > b - S) return false;
      if (t.out_lo > t.out_hi) return false;
      out.push_back(t);
      cur = t.out_lo - 1;
      first = false;
    }
  }
  return true;
}

// FP64 keeps two levels of MPT doubles per lane in registers; beyond 22
// nodes per lane that no longer fits without spilling.
bool shape_fits_fp64(const rswr::Shape& sh) { return sh.per_thread <= 22; }

// The fused span (predict folded into the update) takes the fixed span, at
// most kMaxFusedSpan levels, and inputs only at region ends (no interior
// left input).
bool fuse_eligible(const rswr_plan_s& p) {
  if (p.mode != RSWR_SPAN_FIXED || p.S < 1 || p.S > rswr::kMaxFusedSpan) return false;
  const int64_t TM = int64_t(p.threads) * p.per_thread;
  auto frame_ok = [&](int64_t o, int32_t w) {
    if (w < 0 || w >= p.N) return false;
    return o > p.lo[w] && o < p.hi[w];
  };
  for (const Tile& t : p.tiles) {
    if (t.lin != rswr::kNoNode) return false;
    if (t.lmode == rswr::kEndGhost &&
        (t.fl != t.window - 1 || t.a != p.lo[t.window] || !frame_ok(t.a, t.window - 1)))
      return false;
    if (t.rmode == rswr::kEndGhost &&
        (t.fr != t.window || t.a + TM - 1 != p.hi[t.window] ||
         !frame_ok(t.a + TM - 1, t.window + 1)))
      return false;
  }
  return true;
}

// Default kernel shape: the least padded work, penalising launches too small
// to give every one of the 256 compute units a couple of work-groups.
bool choose_shape(rswr_plan_s& p) {
  double best = 0;
  bool found = false;
  std::vector<Tile> tiles;
  for (int s = 0; s < rswr::n_shapes(); ++s) {
    const rswr::Shape sh = rswr::shape_at(s);
    if (p.dtype == RSWR_F64 && (sh.threads * sh.per_thread > 6144 || !shape_fits_fp64(sh)))
      continue;
    const int TM = sh.threads * sh.per_thread;
    if (TM < 2 * p.S_max + 2) continue;
    if (!build_tiles(p, TM, p.S_max, tiles)) continue;
    double nt = 0;
    for (const Tile& t : tiles) nt += t.general ? 2.0 : 1.0;
    // beyond 33 nodes per lane (FP32) or 16 (FP64) a lane's two levels take
    // so many registers that a SIMD holds two waves or fewer; a tile of
    // several waves exchanges its inner ends through LDS with a barrier every
    // step.  Either runs a span 15-25 % slower than a one-wave shape of
    // about the same work (2^24-node FP32 case: 64x33 68 us, 128x33 77,
    // 64x65 80, 320x13 85).
    const bool wide = sh.per_thread > (p.dtype == RSWR_F64 ? 16 : 33);
    const double cost = nt * TM * std::max(1.0, 512.0 / double(tiles.size())) *
                        (wide ? 1.25 : 1.0) * (sh.threads > 64 ? 1.25 : 1.0);
    if (!found || cost < best) {
      best = cost;
      found = true;
      p.threads = sh.threads;
      p.per_thread = sh.per_thread;
    }
  }
  return found;
}

// Interior point sources of a plan: checked, then listed per tile in three
// runs -- sources of the tile's window inside its register region, sources
// of the left neighbour window inside the left prediction frame, those of
// the right neighbour inside the right frame -- each in source order (the
// order of the additions at one node).  Sources run on the fused span only.
rswr_status_t plan_sources(rswr_plan_s& p, const rswr_desc_t& D) {
  if (D.n_src < 0) return fail(RSWR_ERR_INVALID_ARG, "n_src < 0");
  if (D.n_src == 0) return RSWR_OK;
  if (!D.src_node || !D.src_amp || D.src_ld < 1)
    return fail(RSWR_ERR_INVALID_ARG, "sources need src_node, src_amp and src_ld >= 1");
  if (!p.fused)
    return fail(RSWR_ERR_UNSUPPORTED,
                "interior sources run on the fused span (FIXED mode, span <= " +
                    std::to_string(rswr::kMaxFusedSpan) + ", fusion not disabled)");
  for (int32_t q = 0; q < D.n_src; ++q)
    if (D.src_node[q] < 1 || D.src_node[q] > p.M - 2)
      return fail(RSWR_ERR_INVALID_ARG, "source node outside 1..M-2");
  p.src_node.assign(D.src_node, D.src_node + D.n_src);
  p.src_amp = D.src_amp;
  p.src_ld = D.src_ld;
  const int64_t TM = int64_t(p.threads) * p.per_thread;
  const int64_t H = rswr::kFrameHalf;
  p.src_ptr.assign(1, 0);
  auto run = [&](int32_t w, int64_t a, int64_t b) {
    if (w >= 0 && w < p.N) {
      a = std::max({a, p.lo[w], int64_t(1)});
      b = std::min({b, p.hi[w], p.M - 2});
      for (int32_t q = 0; q < D.n_src; ++q)
        if (p.src_node[q] >= a && p.src_node[q] <= b) {
          p.src_tnode.push_back(p.src_node[q]);
          p.src_tid.push_back(q);
        }
    }
    p.src_ptr.push_back(static_cast<int32_t>(p.src_tnode.size()));
  };
  for (const Tile& x : p.tiles) {
    run(x.window, x.a, x.a + TM - 1);
    const bool fl = x.lmode == rswr::kEndGhost, fr = x.rmode == rswr::kEndGhost;
    run(fl ? x.window - 1 : -1, x.a - H, x.a + H - 1);
    run(fr ? x.window + 1 : -1, x.a + TM - 1 - H, x.a + TM - 1 + H - 1);
  }
  return RSWR_OK;
}

// Waits of the one-launch loop.  Tile t reads the glued state over its
// region and, at an input end, over the prediction frame around it
// ([o - kFrameHalf, o + kFrameHalf - 1]); it writes its stored range and the
// Dirichlet node next to a Dirichlet end.  Before span k, t waits for every
// tile whose written nodes it reads (they must have finished span k-1) and
// for every tile that reads t's written nodes (they must have read the
// buffer t is about to overwrite).  The written ranges are disjoint and
// cover the grid, so each read range meets a contiguous run of them.
void build_deps(rswr_plan_s& p) {
  const int64_t TM = int64_t(p.threads) * p.per_thread;
  const int64_t H = rswr::kFrameHalf;
  const int32_t n = static_cast<int32_t>(p.tiles.size());
  std::vector<int64_t> rlo(n), rhi(n), wlo(n), whi(n);
  for (int32_t t = 0; t < n; ++t) {
    const Tile& x = p.tiles[t];
    rlo[t] = std::max<int64_t>(0, x.lmode == rswr::kEndGhost ? x.a - H : x.a);
    rhi[t] = std::min<int64_t>(p.M - 1, x.rmode == rswr::kEndGhost ? x.a + TM - 1 + H - 1
                                                                     : x.a + TM - 1);
    wlo[t] = x.lmode == rswr::kEndDirichlet ? 0 : x.out_lo;
    whi[t] = x.rmode == rswr::kEndDirichlet ? p.M - 1 : x.out_hi;
  }
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return wlo[x] < wlo[y]; });
  std::vector<std::vector<int32_t>> adj(n);
  for (int32_t t = 0; t < n; ++t) {
    // first written range that may end at or after rlo[t]
    auto it = std::lower_bound(order.begin(), order.end(), rlo[t],
                               [&](int32_t u, int64_t v) { return whi[u] < v; });
    for (; it != order.end() && wlo[*it] <= rhi[t]; ++it) {
      const int32_t u = *it;
      if (u == t || whi[u] < rlo[t]) continue;
      adj[t].push_back(u);
      adj[u].push_back(t);
    }
  }
  p.dep_ptr.assign(1, 0);
  p.dep.clear();
  for (int32_t t = 0; t < n; ++t) {
    std::sort(adj[t].begin(), adj[t].end());
    adj[t].erase(std::unique(adj[t].begin(), adj[t].end()), adj[t].end());
    p.dep.insert(p.dep.end(), adj[t].begin(), adj[t].end());
    p.dep_ptr.push_back(static_cast<int32_t>(p.dep.size()));
  }
}

// Whether a solve without receivers runs as one launch: plans that asked
// for it and can, when their tiles all fit on the device at once.
bool use_persist(const rswr_plan_s& p) {
  if (!p.persist_ok) return false;
  const int cap = p.dtype == RSWR_F64 ? rswr::persist_capacity<double>(p.threads, p.per_thread)
                                      : rswr::persist_capacity<float>(p.threads, p.per_thread);
  return int64_t(p.tiles.size()) <= int64_t(cap);
}

rswr_status_t ensure_device(rswr_plan_s* p, DevTables** out, int* device) {
  int dev = 0;
  RSWR_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(p->mu);
  auto it = p->dev.find(dev);
  if (it == p->dev.end()) {
    DevTables t;
    const size_t nt = std::max<size_t>(p->tiles.size(), 1);
    RSWR_HIP(hipMalloc(&t.tiles, nt * sizeof(Tile)));
    RSWR_HIP(hipMalloc(&t.idx, nt * sizeof(int32_t)));
    RSWR_HIP(hipMalloc(&t.lo, p->N * sizeof(int64_t)));
    RSWR_HIP(hipMalloc(&t.hi, p->N * sizeof(int64_t)));
    if (!p->tiles.empty()) {
      RSWR_HIP(hipMemcpy(t.tiles, p->tiles.data(), p->tiles.size() * sizeof(Tile),
                         hipMemcpyHostToDevice));
      RSWR_HIP(hipMemcpy(t.idx, p->idx.data(), p->idx.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice));
    }
    RSWR_HIP(hipMemcpy(t.lo, p->lo.data(), p->N * sizeof(int64_t), hipMemcpyHostToDevice));
    RSWR_HIP(hipMemcpy(t.hi, p->hi.data(), p->N * sizeof(int64_t), hipMemcpyHostToDevice));
    if (!p->src_node.empty()) {
      const size_t ne = std::max<size_t>(p->src_tnode.size(), 1);
      RSWR_HIP(hipMalloc(&t.src_ptr, p->src_ptr.size() * sizeof(int32_t)));
      RSWR_HIP(hipMalloc(&t.src_node, ne * sizeof(int64_t)));
      RSWR_HIP(hipMalloc(&t.src_id, ne * sizeof(int32_t)));
      RSWR_HIP(hipMemcpy(t.src_ptr, p->src_ptr.data(), p->src_ptr.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice));
      if (!p->src_tnode.empty()) {
        RSWR_HIP(hipMemcpy(t.src_node, p->src_tnode.data(),
                           p->src_tnode.size() * sizeof(int64_t), hipMemcpyHostToDevice));
        RSWR_HIP(hipMemcpy(t.src_id, p->src_tid.data(), p->src_tid.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice));
      }
    }
    if (p->persist_ok) {
      RSWR_HIP(hipMalloc(&t.dep_ptr, p->dep_ptr.size() * sizeof(int32_t)));
      RSWR_HIP(hipMalloc(&t.dep, std::max<size_t>(p->dep.size(), 1) * sizeof(int32_t)));
      RSWR_HIP(hipMemcpy(t.dep_ptr, p->dep_ptr.data(), p->dep_ptr.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice));
      if (!p->dep.empty())
        RSWR_HIP(hipMemcpy(t.dep, p->dep.data(), p->dep.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice));
    }
    RSWR_HIP(hipStreamCreateWithFlags(&t.capture, hipStreamNonBlocking));
    it = p->dev.emplace(dev, t).first;
  }
  *out = &it->second;
  if (device) *device = dev;
  return RSWR_OK;
}

template <typename T>
rswr::PredictArgs<T> predict_args(const rswr_plan_s& p, const DevTables& d,
                                  const void* state, const void* fa, const void* fb,
                                  int64_t n0, int32_t shat, void* flux) {
  rswr::PredictArgs<T> a{};
  a.state = static_cast<const T*>(state);
  a.fa = static_cast<const T*>(fa);
  a.fb = static_cast<const T*>(fb);
  a.flux = static_cast<T*>(flux);
  a.lo = d.lo;
  a.hi = d.hi;
  a.M = p.M;
  a.n0 = n0;
  a.N = p.N;
  a.shat = shat;
  a.ld = p.flux_ld;
  const double c2 = p.lam * p.lam;
  a.c2 = T(c2);
  a.k = T(2.0 - 2.0 * c2);
  a.r = T(1.0 / (2.0 * p.dx));
  a.q = T(2.0 * p.dx);
  return a;
}

template <typename T>
rswr::UpdateArgs<T> update_args(const rswr_plan_s& p, const DevTables& d,
                                const void* state_in, const void* fa, const void* fb,
                                int64_t n0, const void* flux, const int32_t* span_dev,
                                int32_t span, void* state_out) {
  rswr::UpdateArgs<T> a{};
  a.state_in = static_cast<const T*>(state_in);
  a.state_out = static_cast<T*>(state_out);
  a.fa = static_cast<const T*>(fa);
  a.fb = static_cast<const T*>(fb);
  a.flux = static_cast<const T*>(flux);
  a.tiles = d.tiles;
  a.span_dev = span_dev;
  a.M = p.M;
  a.n0 = n0;
  a.span = span;
  a.ld = p.flux_ld;
  const double c2 = p.lam * p.lam;
  a.c2 = T(c2);
  a.k = T(2.0 - 2.0 * c2);
  a.q = T(2.0 * p.dx);
  a.r = T(1.0 / (2.0 * p.dx));
  a.lo = d.lo;
  a.hi = d.hi;
  if (!p.src_node.empty()) {
    a.src_ptr = d.src_ptr;
    a.src_node = d.src_node;
    a.src_id = d.src_id;
    a.src_amp = static_cast<const T*>(p.src_amp);
    a.src_ld = p.src_ld;
  }
  return a;
}

// The two update launches of one span on the two-launch path: general
// tiles (and, in a solve, the tiles holding receivers) through the general
// kernel, the rest through the plain one.
template <typename T>
hipError_t launch_update_pair(const rswr_plan_s& p, rswr::UpdateArgs<T> a,
                              const int32_t* gen_idx, int32_t n_gen,
                              const int32_t* fast_idx, int32_t n_fast, hipStream_t s) {
  if (n_gen > 0) {
    a.tile_idx = gen_idx;
    a.n_tiles = n_gen;
    hipError_t e = rswr::launch_update<T>(a, p.threads, p.per_thread, true, s);
    if (e != hipSuccess) return e;
  }
  if (n_fast > 0) {
    a.tile_idx = fast_idx;
    a.n_tiles = n_fast;
    a.rec_ptr = nullptr;
    return rswr::launch_update<T>(a, p.threads, p.per_thread, false, s);
  }
  return hipSuccess;
}

// One fused span: the general tiles, then every other tile in one launch
// (`a.rec_ptr`: CSR over the general list then the plain list; tiles with
// receivers or interior sources take the extended path inside that launch).
template <typename T>
hipError_t launch_fused_span(const rswr_plan_s& p, rswr::UpdateArgs<T> a,
                             const int32_t* gen_idx, int32_t n_gen, const int32_t* fast_idx,
                             int32_t n_fast, hipStream_t s) {
  const int32_t* rec_ptr = a.rec_ptr;
  hipError_t e = hipSuccess;
  if (n_gen > 0) {
    a.tile_idx = gen_idx;
    a.n_tiles = n_gen;
    if ((e = rswr::launch_fused<T>(a, p.threads, p.per_thread, rswr::kFusedGeneral, s)) !=
        hipSuccess)
      return e;
  }
  if (n_fast > 0) {
    a.tile_idx = fast_idx;
    a.n_tiles = n_fast;
    a.rec_ptr = rec_ptr ? rec_ptr + n_gen : nullptr;
    return rswr::launch_fused<T>(a, p.threads, p.per_thread,
                                 (rec_ptr || a.src_ptr) ? rswr::kFusedExt
                                                        : rswr::kFusedPlain,
                                 s);
  }
  return hipSuccess;
}

size_t elem_size(const rswr_plan_s& p) { return p.dtype == RSWR_F64 ? 8 : 4; }

struct WsLayout {
  size_t state = 0, flux = 0, gen_idx = 0, fast_idx = 0, rec_ptr = 0, rec_node = 0,
         rec_id = 0, ctl = 0, flags = 0, total = 0;
};

WsLayout ws_layout(const rswr_plan_s& p, int32_t n_rec) {
  WsLayout w;
  const size_t b = elem_size(p);
  const size_t nt = p.tiles.size();
  size_t off = 0;
  w.state = off;
  off += round_up(2 * size_t(p.M) * b, 256);
  w.flux = off;
  off += round_up(size_t(std::max(p.N - 1, 1)) * 2 * p.flux_ld * b, 256);
  // launch lists: a tile may be listed once per group of receivers, so up
  // to nt + n_rec entries
  const size_t nl = nt + size_t(std::max(n_rec, 0));
  w.gen_idx = off;
  off += round_up(std::max<size_t>(nl, 1) * sizeof(int32_t), 256);
  w.fast_idx = off;
  off += round_up(std::max<size_t>(nl, 1) * sizeof(int32_t), 256);
  w.rec_ptr = off;
  off += round_up((nl + 1) * sizeof(int32_t), 256);
  w.rec_node = off;
  off += round_up(size_t(std::max(n_rec, 1)) * sizeof(int64_t), 256);
  w.rec_id = off;
  off += round_up(size_t(std::max(n_rec, 1)) * sizeof(int32_t), 256);
  w.ctl = off;  // control block of an adaptive solve
  off += round_up(sizeof(rswr::QuietCtl), 256);
  w.flags = off;  // one-launch loop: spans finished per tile, then the error word
  off += round_up((nt + 1) * sizeof(int32_t), 256);
  w.total = off;
  return w;
}

// Launch lists of one solve: where the lists live and how long they are.
struct Lists {
  const int32_t* gen = nullptr;
  const int32_t* fast = nullptr;
  int32_t n_gen = 0, n_fast = 0;
  const int32_t* rec_ptr = nullptr;
  const int64_t* rec_node = nullptr;
  const int32_t* rec_id = nullptr;
};

template <typename T>
rswr_status_t enqueue_solve(rswr_plan_s* p, const DevTables& d, void* state,
                            const void* fa, const void* fb, int64_t n0, int64_t n_steps,
                            const Lists& lists, void* traces, char* ws, const WsLayout& L,
                            void* ckpt, bool persist, hipStream_t s) {
  const int64_t M = p->M;
  const int64_t K = (n_steps + p->S - 1) / p->S;
  T* const user = static_cast<T*>(state);
  T* const buf = reinterpret_cast<T*>(ws + L.state);
  T* const flux = reinterpret_cast<T*>(ws + L.flux);
  T* const ck = static_cast<T*>(ckpt);
  const size_t st_elems = 2 * size_t(M);
  // checkpoint buffer: [K+1][2][M] span-boundary states, then [K][flux]
  // predicted fluxes of every span
  const size_t fl_elems = size_t(std::max(p->N - 1, 1)) * 2 * p->flux_ld;
  T* const ck_flux = ck ? ck + (K + 1) * st_elems : nullptr;
  T* x = user;
  T* y = buf;
  if (ck) {
    RSWR_HIP(rswr::launch_copy<T>(ck, user, 2 * M, s));
  } else if (K & 1) {
    RSWR_HIP(rswr::launch_copy<T>(buf, user, 2 * M, s));
    x = buf;
    y = user;
  }
  if (persist) {
    // the whole loop in one launch: the tiles wait on each other's counters
    const int32_t n_all = static_cast<int32_t>(p->tiles.size());
    int32_t* flags = reinterpret_cast<int32_t*>(ws + L.flags);
    RSWR_HIP(rswr::launch_fill<int32_t>(flags, 0, n_all + 1, s));
    rswr::UpdateArgs<T> ua =
        update_args<T>(*p, d, nullptr, fa, fb, n0, nullptr, nullptr, p->S, nullptr);
    ua.tile_idx = d.idx;
    ua.n_tiles = n_all;
    rswr::PersistArgs<T> q{};
    q.buf0 = x;
    q.buf1 = y;
    q.ck = ck;
    q.ck_flux = ck_flux;
    q.flags = flags;
    q.err = flags + n_all;
    q.dep_ptr = d.dep_ptr;
    q.dep = d.dep;
    q.st_elems = static_cast<int64_t>(st_elems);
    q.fl_elems = static_cast<int64_t>(fl_elems);
    q.n0 = n0;
    q.n_end = n0 + n_steps;
    q.n_spans = static_cast<int32_t>(K);
    q.S = p->S;
    RSWR_HIP(rswr::launch_fused_persist<T>(ua, q, p->threads, p->per_thread, s));
    if (ck) RSWR_HIP(rswr::launch_copy<T>(user, ck + K * st_elems, 2 * M, s));
    return RSWR_OK;
  }
  int64_t lev = n0;
  for (int64_t k = 0; k < K; ++k) {
    const int32_t S = static_cast<int32_t>(std::min<int64_t>(p->S, n0 + n_steps - lev));
    const T* in = ck ? ck + k * st_elems : x;
    T* out = ck ? ck + (k + 1) * st_elems : y;
    T* const fl = ck ? ck_flux + k * fl_elems : flux;
    if (!p->fused) {
      rswr::PredictArgs<T> pa = predict_args<T>(*p, d, in, fa, fb, lev, S, fl);
      RSWR_HIP(rswr::launch_predict<T>(pa, 2 * p->S_max + 1, s));
    }
    rswr::UpdateArgs<T> ua =
        update_args<T>(*p, d, in, fa, fb, lev, fl, nullptr, S, out);
    if (p->fused) {
      ua.flux = nullptr;
      ua.flux_out = ck ? fl : nullptr;  // the adjoint reads the span's fluxes
    }
    if (lists.rec_ptr) {
      ua.rec_ptr = lists.rec_ptr;
      ua.rec_node = lists.rec_node;
      ua.rec_id = lists.rec_id;
      ua.traces = static_cast<T*>(traces);
      ua.trace_ld = n_steps;
      ua.trace_col0 = lev - n0;
    }
    if (p->fused)
      RSWR_HIP(launch_fused_span<T>(*p, ua, lists.gen, lists.n_gen, lists.fast, lists.n_fast,
                                    s));
    else
      RSWR_HIP(launch_update_pair<T>(*p, ua, lists.gen, lists.n_gen, lists.fast, lists.n_fast,
                                     s));
    lev += S;
    std::swap(x, y);
  }
  if (ck) RSWR_HIP(rswr::launch_copy<T>(user, ck + K * st_elems, 2 * M, s));
  return RSWR_OK;
}

// The adaptive (QUIET) loop of Sec. 2.6 recorded as one graph: every span
// is at least min(S_cone, cap) levels (or the levels left), which bounds
// the rounds; each round predicts over the device's predictive span,
// selects on the device, updates over the chosen span and advances the
// control block, and rounds after the last span exit at once.  The result
// ends in the caller's buffer or the workspace copy, as the device parity
// says; a last conditional copy brings it to the caller's buffer.
template <typename T>
rswr_status_t enqueue_solve_quiet(rswr_plan_s* p, const DevTables& d, void* state,
                                  const void* fa, const void* fb, int64_t n0,
                                  int64_t n_steps, const Lists& lists, void* traces, char* ws,
                                  const WsLayout& L, hipStream_t s) {
  const int64_t M = p->M;
  T* const user = static_cast<T*>(state);
  T* const buf = reinterpret_cast<T*>(ws + L.state);
  T* const flux = reinterpret_cast<T*>(ws + L.flux);
  auto* const ctl = reinterpret_cast<rswr::QuietCtl*>(ws + L.ctl);
  const int32_t cap = p->S_max;
  const int32_t lo_span = std::max(1, std::min(p->S_cone, cap));
  const int64_t rounds = (n_steps + lo_span - 1) / lo_span;
  const int32_t shat0 =
      static_cast<int32_t>(std::min<int64_t>({int64_t(p->S_cone), int64_t(cap), n_steps}));
  RSWR_HIP(rswr::launch_quiet_init(ctl, n0, n0 + n_steps, shat0, cap, p->beta, s));
  for (int64_t k = 0; k < rounds; ++k) {
    T* in = (k & 1) ? buf : user;
    T* out = (k & 1) ? user : buf;
    rswr::PredictArgs<T> pa = predict_args<T>(*p, d, in, fa, fb, n0, cap, flux);
    pa.n0_dev = &ctl->n0;
    pa.shat_dev = &ctl->shat;
    RSWR_HIP(rswr::launch_predict<T>(pa, 2 * cap + 1, s));
    rswr::SelectArgs<T> sa{};
    sa.flux = flux;
    sa.span_dev = &ctl->span;
    sa.shat_dev = &ctl->shat;
    sa.qmin = &ctl->qmin;
    sa.n_rows = 2 * (p->N - 1);
    sa.shat = cap;
    sa.ld = p->flux_ld;
    sa.cone = p->S_cone;
    sa.mode = 1;
    sa.fixed_span = p->S;
    RSWR_HIP(rswr::launch_select<T>(sa, s));
    rswr::UpdateArgs<T> ua = update_args<T>(*p, d, in, fa, fb, n0, flux, &ctl->span, 0, out);
    ua.n0_dev = &ctl->n0;
    if (lists.rec_ptr) {
      ua.rec_ptr = lists.rec_ptr;
      ua.rec_node = lists.rec_node;
      ua.rec_id = lists.rec_id;
      ua.traces = static_cast<T*>(traces);
      ua.trace_ld = n_steps;
      ua.trace_col0 = 0;  // plus the span's offset from n0, read on the device
    }
    RSWR_HIP(launch_update_pair<T>(*p, ua, lists.gen, lists.n_gen, lists.fast, lists.n_fast,
                                   s));
    RSWR_HIP(rswr::launch_quiet_next(ctl, s));
  }
  RSWR_HIP(rswr::launch_copy_if<T>(user, buf, 2 * M, &ctl->parity, s));
  return RSWR_OK;
}

// Records `enqueue` into a HIP graph once per key (on the capture stream
// `cap`, kept in `graphs`, at most 8) and replays it on `s`.
template <typename F>
rswr_status_t run_graph_in(std::mutex& mu, std::vector<GraphEntry>& graphs, hipStream_t cap,
                           const GraphKey& key, F&& enqueue, hipStream_t s) {
  if (std::getenv("RSWR_NO_GRAPH") != nullptr) return enqueue(s);
  hipGraphExec_t exec = nullptr;
  {
    std::lock_guard<std::mutex> g(mu);
    for (auto& e : graphs)
      if (e.key == key) exec = e.exec;
  }
  if (!exec) {
    hipGraph_t graph = nullptr;
    RSWR_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    rswr_status_t cst = enqueue(cap);
    hipError_t ee = hipStreamEndCapture(cap, &graph);
    if (cst != RSWR_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return cst;
    }
    if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
    ee = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ee != hipSuccess) return hip_fail(ee, "hipGraphInstantiate");
    std::lock_guard<std::mutex> g(mu);
    if (graphs.size() >= 8) {
      (void)hipGraphExecDestroy(graphs.front().exec);
      graphs.erase(graphs.begin());
    }
    graphs.push_back({key, exec});
  }
  RSWR_HIP(hipGraphLaunch(exec, s));
  return RSWR_OK;
}

template <typename F>
rswr_status_t run_graph(rswr_plan_s* p, DevTables* d, const GraphKey& key, F&& enqueue,
                        hipStream_t s) {
  return run_graph_in(p->mu, p->graphs, d->capture, key, std::forward<F>(enqueue), s);
}

// ---------------------------------------------------------------------------
// Adjoint driver.
// ---------------------------------------------------------------------------
struct AdjWs {
  size_t w0 = 0, w1 = 0, afl = 0, lam = 0, gen_idx = 0, fast_idx = 0, src_ptr = 0,
         src_node = 0, src_id = 0, rec_node = 0, total = 0;
};

AdjWs adj_ws_layout(const rswr_plan_s& p, int32_t n_rec) {
  AdjWs w;
  const size_t b = elem_size(p);
  const size_t nt = std::max<size_t>(p.tiles.size(), 1);
  const size_t nr = size_t(std::max(n_rec, 1));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += round_up(bytes, 256);
    return at;
  };
  w.w0 = take(2 * size_t(p.M) * b);
  w.w1 = take(2 * size_t(p.M) * b);
  w.afl = take(size_t(std::max(p.N - 1, 1)) * 2 * p.flux_ld * b);
  w.lam = take(nt * sizeof(double));
  w.gen_idx = take(nt * sizeof(int32_t));
  w.fast_idx = take(nt * sizeof(int32_t));
  w.src_ptr = take((nt + 1) * sizeof(int32_t));
  w.src_node = take(nt * nr * sizeof(int64_t));
  w.src_id = take(nt * nr * sizeof(int32_t));
  w.rec_node = take(nr * sizeof(int64_t));
  w.total = off;
  return w;
}

struct AdjLists {
  int32_t n_gen = 0, n_fast = 0;
  // the update tiles carry the W frames of their input ends (fused plans
  // whose fused update kernels fit in registers); else a predict launch
  bool fused = false;
};

bool adj_fused_fits(const rswr_plan_s& p) {
  return p.dtype == RSWR_F64 ? rswr::adj_update_fused_fits<double>(p.threads, p.per_thread)
                             : rswr::adj_update_fused_fits<float>(p.threads, p.per_thread);
}

// Device tables of an adjoint run, shared by every problem of a batch: the
// general and plain tile lists and the receiver sources as one CSR over both
// (general first).  `W` is a layout with the offsets gen_idx, fast_idx,
// src_ptr, src_node, src_id and rec_node.
template <typename W>
rswr_status_t upload_adj_lists(const rswr_plan_s& p, const int64_t* rec_idx, int32_t n_rec,
                               char* ws, const W& L, hipStream_t s, AdjLists* al) {
  const int64_t TM = int64_t(p.threads) * p.per_thread;
  const int32_t n_all = static_cast<int32_t>(p.tiles.size());
  std::vector<int32_t> gen, fast, ptr(1, 0), id;
  std::vector<int64_t> node;
  for (int32_t t = 0; t < n_all; ++t) (p.tiles[t].general ? gen : fast).push_back(t);
  for (const std::vector<int32_t>* list : {&gen, &fast}) {
    for (int32_t t : *list) {
      const Tile& x = p.tiles[t];
      for (int32_t r = 0; r < n_rec; ++r) {
        const int64_t j = rec_idx[r];
        if (j > 0 && j < p.M - 1 && j >= x.a && j <= x.a + TM - 1) {
          id.push_back(r);
          node.push_back(rec_idx[r]);
        }
      }
      ptr.push_back(static_cast<int32_t>(id.size()));
    }
  }
  std::vector<int64_t> recs(rec_idx, rec_idx + n_rec);
  auto up = [&](size_t off, const void* src, size_t bytes) -> rswr_status_t {
    if (bytes) RSWR_HIP(hipMemcpyAsync(ws + off, src, bytes, hipMemcpyHostToDevice, s));
    return RSWR_OK;
  };
  rswr_status_t st;
  if ((st = up(L.gen_idx, gen.data(), gen.size() * 4)) != RSWR_OK) return st;
  if ((st = up(L.fast_idx, fast.data(), fast.size() * 4)) != RSWR_OK) return st;
  if ((st = up(L.src_ptr, ptr.data(), ptr.size() * 4)) != RSWR_OK) return st;
  if ((st = up(L.src_node, node.data(), node.size() * 8)) != RSWR_OK) return st;
  if ((st = up(L.src_id, id.data(), id.size() * 4)) != RSWR_OK) return st;
  if ((st = up(L.rec_node, recs.data(), recs.size() * 8)) != RSWR_OK) return st;
  al->n_gen = static_cast<int32_t>(gen.size());
  al->n_fast = static_cast<int32_t>(fast.size());
  return RSWR_OK;
}

// Buffers of one backward span k (levels n_e = n_k + S down to n_k).
template <typename T>
struct AdjSpanIO {
  T* w_cur;         // adjoint state at the span end (in)
  T* w_nxt;         // at the span start (out)
  T* afl;           // adjoint fluxes of the span
  const T* u_beg;   // forward state at the span start
  const T* u_end;   // and at its end
  const T* ffl;     // forward fluxes of the span
  double* lam;      // dJ/dlam partials, one per tile
};

// The adjoint predict and update of one span (last span first), all tiles;
// `ys` batches same-shape problems along grid dimension y.
template <typename T, typename W>
rswr_status_t enqueue_adj_span(const rswr_plan_s* p, const DevTables& d, char* ws,
                               const W& L, const AdjLists& al, int64_t k, int64_t n_steps,
                               const AdjSpanIO<T>& io, const void* fa, const void* fb,
                               const void* gtr, void* gfa, void* gfb, int32_t n_rec,
                               const rswr::YStrides& ys, hipStream_t s) {
  const int64_t M = p->M;
  const int64_t n_k = k * p->S;
  const int32_t S = static_cast<int32_t>(std::min<int64_t>(p->S, n_steps - n_k));
  const int64_t n_e = n_k + S;
  const double c2 = p->lam * p->lam;
  rswr::AdjPredictArgs<T> pa{};
  pa.w = io.w_cur;
  pa.flux = io.afl;
  pa.lo = d.lo;
  pa.hi = d.hi;
  pa.rec_node = reinterpret_cast<const int64_t*>(ws + L.rec_node);
  pa.gtr = static_cast<const T*>(gtr);
  pa.ys = ys;
  pa.gtr_ld = n_steps;
  pa.M = M;
  pa.n_e = n_e;
  pa.N = p->N;
  pa.shat = S;
  pa.ld = p->flux_ld;
  pa.n_rec = n_rec;
  pa.c2 = T(c2);
  pa.k = T(2.0 - 2.0 * c2);
  pa.r = T(1.0 / (2.0 * p->dx));
  pa.q = T(2.0 * p->dx);
  const bool fused = al.fused;
  if (!fused) RSWR_HIP(rswr::launch_adj_predict<T>(pa, 2 * p->S_max + 1, s));
  rswr::AdjUpdateArgs<T> ua{};
  ua.w_in = io.w_cur;
  ua.w_out = io.w_nxt;
  ua.u_end = io.u_end;
  ua.u_beg = io.u_beg;
  ua.ffl = io.ffl;
  ua.afl = io.afl;
  ua.fa = static_cast<const T*>(fa);
  ua.fb = static_cast<const T*>(fb);
  ua.tiles = d.tiles;
  ua.gtr = static_cast<const T*>(gtr);
  ua.gtr_ld = n_steps;
  ua.grad_fa = static_cast<T*>(gfa);
  ua.grad_fb = static_cast<T*>(gfb);
  ua.lam_part = io.lam;
  ua.ys = ys;
  ua.M = M;
  ua.n_e = n_e;
  ua.n_k = n_k;
  ua.span = S;
  ua.ld = p->flux_ld;
  ua.c2 = T(c2);
  ua.k = T(2.0 - 2.0 * c2);
  ua.q = T(2.0 * p->dx);
  ua.src_ptr = reinterpret_cast<const int32_t*>(ws + L.src_ptr);
  ua.src_node = reinterpret_cast<const int64_t*>(ws + L.src_node);
  ua.src_id = reinterpret_cast<const int32_t*>(ws + L.src_id);
  ua.lo = d.lo;
  ua.hi = d.hi;
  ua.rec_all = pa.rec_node;
  ua.n_rec_all = n_rec;
  ua.r = pa.r;
  if (al.n_gen > 0) {
    rswr::AdjUpdateArgs<T> g = ua;
    g.tile_idx = reinterpret_cast<const int32_t*>(ws + L.gen_idx);
    g.n_tiles = al.n_gen;
    RSWR_HIP(rswr::launch_adj_update<T>(g, p->threads, p->per_thread, true, fused, s));
  }
  if (al.n_fast > 0) {
    rswr::AdjUpdateArgs<T> f = ua;
    f.tile_idx = reinterpret_cast<const int32_t*>(ws + L.fast_idx);
    f.n_tiles = al.n_fast;
    f.src_ptr = ua.src_ptr + al.n_gen;
    RSWR_HIP(rswr::launch_adj_update<T>(f, p->threads, p->per_thread, false, fused, s));
  }
  return RSWR_OK;
}

template <typename T>
rswr_status_t enqueue_adjoint(rswr_plan_s* p, const DevTables& d, const void* ckpt,
                              const void* fa, const void* fb, int64_t n_steps,
                              const AdjLists& al, const void* gtr, void* gfa, void* gfb,
                              double* glam, char* ws, const AdjWs& L, int32_t n_rec,
                              hipStream_t s) {
  const int64_t M = p->M;
  const int64_t K = (n_steps + p->S - 1) / p->S;
  const size_t st_elems = 2 * size_t(M);
  const size_t fl_elems = size_t(std::max(p->N - 1, 1)) * 2 * p->flux_ld;
  const T* ck = static_cast<const T*>(ckpt);
  const T* ck_flux = ck + (K + 1) * st_elems;
  T* w_cur = reinterpret_cast<T*>(ws + L.w0);
  T* w_nxt = reinterpret_cast<T*>(ws + L.w1);
  T* afl = reinterpret_cast<T*>(ws + L.afl);
  double* lam = reinterpret_cast<double*>(ws + L.lam);
  const int32_t n_all = static_cast<int32_t>(p->tiles.size());
  RSWR_HIP(rswr::launch_fill<T>(w_cur, T(0), 2 * M, s));
  RSWR_HIP(rswr::launch_fill<double>(lam, 0.0, std::max(n_all, 1), s));
  RSWR_HIP(rswr::launch_fill<T>(static_cast<T*>(gfa), T(0), n_steps + 1, s));
  RSWR_HIP(rswr::launch_fill<T>(static_cast<T*>(gfb), T(0), n_steps + 1, s));
  const rswr::YStrides one{};
  for (int64_t k = K - 1; k >= 0; --k) {
    const AdjSpanIO<T> io{w_cur, w_nxt, afl, ck + k * st_elems, ck + (k + 1) * st_elems,
                          ck_flux + k * fl_elems, lam};
    const rswr_status_t st = enqueue_adj_span<T>(p, d, ws, L, al, k, n_steps, io, fa, fb,
                                                 gtr, gfa, gfb, n_rec, one, s);
    if (st != RSWR_OK) return st;
    std::swap(w_cur, w_nxt);
  }
  RSWR_HIP(rswr::launch_adj_finish<T>(
      static_cast<T*>(gfa), static_cast<T*>(gfb), static_cast<const T*>(gtr), n_steps,
      reinterpret_cast<const int64_t*>(ws + L.rec_node), n_rec, M, n_steps, lam, n_all,
      p->lam, glam, s));
  return RSWR_OK;
}

// A batch of adjoint solves of one plan (same shape, receivers and span),
// each from rest, processed `group` problems at a time with chunked
// checkpoints: the forward pass keeps the state at every C-th span boundary
// (C spans per segment); the backward sweep recomputes each segment's span
// states and fluxes, last segment first, and runs its adjoint spans.  All
// problems of a group share every launch (grid dimension y).
struct AdjBatchWs {
  // shared tables (as AdjWs)
  size_t gen_idx = 0, fast_idx = 0, src_ptr = 0, src_node = 0, src_id = 0, rec_node = 0;
  // one block per problem of a group; offsets inside a block
  size_t coarse = 0, seg_st = 0, seg_fl = 0, w0 = 0, w1 = 0, afl = 0, lam = 0;
  size_t blocks = 0, block = 0, total = 0;
  int64_t K = 0, C = 0, n_seg = 0;
};

AdjBatchWs adj_batch_layout(const rswr_plan_s& p, int64_t n_steps, int32_t n_rec,
                            int32_t group, int32_t seg) {
  AdjBatchWs w;
  const size_t b = elem_size(p);
  const size_t nt = std::max<size_t>(p.tiles.size(), 1);
  const size_t nr = size_t(std::max(n_rec, 1));
  w.K = (n_steps + p.S - 1) / p.S;
  w.C = seg > 0 ? seg : static_cast<int64_t>(std::ceil(std::sqrt(double(w.K))));
  w.C = std::max<int64_t>(1, std::min(w.C, w.K));
  w.n_seg = (w.K + w.C - 1) / w.C;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += round_up(bytes, 256);
    return at;
  };
  w.gen_idx = take(nt * sizeof(int32_t));
  w.fast_idx = take(nt * sizeof(int32_t));
  w.src_ptr = take((nt + 1) * sizeof(int32_t));
  w.src_node = take(nt * nr * sizeof(int64_t));
  w.src_id = take(nt * nr * sizeof(int32_t));
  w.rec_node = take(nr * sizeof(int64_t));
  w.blocks = off;
  const size_t st = 2 * size_t(p.M) * b;
  const size_t fl = size_t(std::max(p.N - 1, 1)) * 2 * p.flux_ld * b;
  off = 0;
  w.coarse = take(size_t(w.n_seg) * st);
  w.seg_st = take(size_t(w.C + 1) * st);
  w.seg_fl = take(size_t(w.C) * fl);
  w.w0 = take(st);
  w.w1 = take(st);
  w.afl = take(fl);
  w.lam = take(nt * sizeof(double));
  w.block = off;
  w.total = w.blocks + size_t(std::max(group, 1)) * w.block;
  return w;
}

template <typename T>
rswr_status_t enqueue_adjoint_batch(rswr_plan_s* p, const DevTables& d, int32_t n_prob,
                                    const void* fa, const void* fb, int64_t src_ld,
                                    int64_t n_steps, const AdjLists& al, const void* gtr,
                                    void* gfa, void* gfb, double* glam, char* ws,
                                    const AdjBatchWs& L, int32_t n_rec, int32_t group,
                                    hipStream_t s) {
  const int64_t M = p->M;
  const size_t stE = 2 * size_t(M);
  const size_t flE = size_t(std::max(p->N - 1, 1)) * 2 * p->flux_ld;
  const int32_t n_all = static_cast<int32_t>(p->tiles.size());
  char* const blk = ws + L.blocks;
  T* const coarse = reinterpret_cast<T*>(blk + L.coarse);
  T* const seg_st = reinterpret_cast<T*>(blk + L.seg_st);
  T* const seg_fl = reinterpret_cast<T*>(blk + L.seg_fl);
  T* const w0 = reinterpret_cast<T*>(blk + L.w0);
  T* const w1 = reinterpret_cast<T*>(blk + L.w1);
  T* const afl = reinterpret_cast<T*>(blk + L.afl);
  double* const lam = reinterpret_cast<double*>(blk + L.lam);
  const int64_t B = static_cast<int64_t>(L.block);
  const int64_t gstride = int64_t(n_rec) * n_steps;
  for (int32_t g0 = 0; g0 < n_prob; g0 += group) {
    const int32_t G = std::min(group, n_prob - g0);
    rswr::YStrides ys{};
    ys.ws = B;
    ys.src = src_ld * int64_t(sizeof(T));
    ys.gtr = gstride * int64_t(sizeof(T));
    ys.grad = (n_steps + 1) * int64_t(sizeof(T));
    ys.ny = G;
    const T* fa0 = static_cast<const T*>(fa) + int64_t(g0) * src_ld;
    const T* fb0 = static_cast<const T*>(fb) + int64_t(g0) * src_ld;
    const T* gtr0 = static_cast<const T*>(gtr) + int64_t(g0) * gstride;
    T* gfa0 = static_cast<T*>(gfa) + int64_t(g0) * (n_steps + 1);
    T* gfb0 = static_cast<T*>(gfb) + int64_t(g0) * (n_steps + 1);
    // one forward span of every problem of the group: in -> out (+ fluxes)
    auto fwd = [&](int64_t k, const T* in, T* out, T* flux_out) -> rswr_status_t {
      const int64_t n0 = k * p->S;
      const int32_t S = static_cast<int32_t>(std::min<int64_t>(p->S, n_steps - n0));
      rswr::UpdateArgs<T> ua = update_args<T>(*p, d, in, fa0, fb0, n0, nullptr, nullptr, S, out);
      ua.flux = nullptr;
      ua.flux_out = flux_out;
      ua.ys = ys;
      RSWR_HIP(launch_fused_span<T>(*p, ua, d.idx, p->n_gen, d.idx + p->n_gen,
                                    n_all - p->n_gen, s));
      return RSWR_OK;
    };
    rswr_status_t st;
    // forward from rest, keeping the state at every C-th span boundary
    RSWR_HIP(rswr::launch_fill_y<T>(coarse, T(0), int64_t(stE), G, B, s));
    const T* cur = coarse;
    for (int64_t k = 0; k < L.K; ++k) {
      T* out;
      if ((k + 1) % L.C == 0 && (k + 1) / L.C < L.n_seg)
        out = coarse + ((k + 1) / L.C) * stE;
      else
        out = (cur == seg_st) ? seg_st + stE : seg_st;
      if ((st = fwd(k, cur, out, nullptr)) != RSWR_OK) return st;
      cur = out;
    }
    // backward: segments last first; each recomputed, then swept in reverse
    RSWR_HIP(rswr::launch_fill_y<T>(w0, T(0), int64_t(stE), G, B, s));
    RSWR_HIP(rswr::launch_fill_y<double>(lam, 0.0, std::max(n_all, 1), G, B, s));
    RSWR_HIP(rswr::launch_fill<T>(gfa0, T(0), int64_t(G) * (n_steps + 1), s));
    RSWR_HIP(rswr::launch_fill<T>(gfb0, T(0), int64_t(G) * (n_steps + 1), s));
    T* w_cur = w0;
    T* w_nxt = w1;
    for (int64_t j = L.n_seg - 1; j >= 0; --j) {
      const int64_t k0 = j * L.C, k1 = std::min(L.K, k0 + L.C);
      // state at boundary k0 + i of the segment: the coarse checkpoint, then
      // the recomputed ones
      auto bnd = [&](int64_t i) { return i == 0 ? coarse + j * stE : seg_st + i * stE; };
      for (int64_t k = k0; k < k1; ++k)
        if ((st = fwd(k, bnd(k - k0), bnd(k - k0 + 1), seg_fl + (k - k0) * flE)) != RSWR_OK)
          return st;
      for (int64_t k = k1 - 1; k >= k0; --k) {
        const AdjSpanIO<T> io{w_cur, w_nxt, afl, bnd(k - k0), bnd(k - k0 + 1),
                              seg_fl + (k - k0) * flE, lam};
        if ((st = enqueue_adj_span<T>(p, d, ws, L, al, k, n_steps, io, fa0, fb0, gtr0, gfa0,
                                      gfb0, n_rec, ys, s)) != RSWR_OK)
          return st;
        std::swap(w_cur, w_nxt);
      }
    }
    for (int32_t y = 0; y < G; ++y)
      RSWR_HIP(rswr::launch_adj_finish<T>(
          gfa0 + int64_t(y) * (n_steps + 1), gfb0 + int64_t(y) * (n_steps + 1),
          gtr0 + int64_t(y) * gstride, n_steps,
          reinterpret_cast<const int64_t*>(ws + L.rec_node), n_rec, M, n_steps,
          reinterpret_cast<const double*>(reinterpret_cast<const char*>(lam) + y * B), n_all,
          p->lam, glam + g0 + y, s));
  }
  return RSWR_OK;
}

}  // namespace

extern "C" {

const char* rswr_last_error(void) { return g_last_error.c_str(); }

const char* rswr_status_string(rswr_status_t s) {
  switch (s) {
    case RSWR_OK: return "ok";
    case RSWR_ERR_INVALID_ARG: return "invalid argument";
    case RSWR_ERR_UNSTABLE: return "Courant number outside (0, 1]";
    case RSWR_ERR_LAYOUT: return "invalid window layout";
    case RSWR_ERR_SPAN: return "span beyond the light-cone limit";
    case RSWR_ERR_NOMEM: return "out of memory or workspace too small";
    case RSWR_ERR_HIP: return "HIP runtime error";
    case RSWR_ERR_UNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

int32_t rswr_kernel_shapes(int32_t* threads, int32_t* per_thread, int32_t* fp64_ok,
                           int32_t cap) {
  const int n = rswr::n_shapes();
  for (int i = 0; i < n && i < cap; ++i) {
    const rswr::Shape sh = rswr::shape_at(i);
    if (threads) threads[i] = sh.threads;
    if (per_thread) per_thread[i] = sh.per_thread;
    if (fp64_ok) fp64_ok[i] = shape_fits_fp64(sh) ? 1 : 0;
  }
  return n;
}

rswr_status_t rswr_plan(const rswr_desc_t* desc, rswr_plan_t* out) {
  if (!desc || !out) return fail(RSWR_ERR_INVALID_ARG, "null descriptor or output");
  *out = nullptr;
  const rswr_desc_t& D = *desc;
  if (D.n_points < 3) return fail(RSWR_ERR_INVALID_ARG, "n_points must be >= 3");
  if (D.n_sub < 1) return fail(RSWR_ERR_INVALID_ARG, "n_sub must be >= 1");
  if (!(D.x_b > D.x_a)) return fail(RSWR_ERR_INVALID_ARG, "x_b must exceed x_a");
  if (!(D.a > 0)) return fail(RSWR_ERR_INVALID_ARG, "wave speed must be positive");
  if (!(D.a_ref >= 0)) return fail(RSWR_ERR_INVALID_ARG, "a_ref must be >= 0");
  if (D.dtype != RSWR_F32 && D.dtype != RSWR_F64)
    return fail(RSWR_ERR_INVALID_ARG, "dtype must be RSWR_F32 or RSWR_F64");
  if (D.span_mode != RSWR_SPAN_FIXED && D.span_mode != RSWR_SPAN_QUIET)
    return fail(RSWR_ERR_INVALID_ARG, "unknown span mode");
  if (D.span < 0) return fail(RSWR_ERR_INVALID_ARG, "span must be >= 0");
  if ((D.courant_num > 0) != (D.courant_den > 0))
    return fail(RSWR_ERR_INVALID_ARG, "courant_num and courant_den go together");
  if (D.courant_num > 0 &&
      !(std::fabs(double(D.courant_num) / double(D.courant_den) - D.courant) <=
        4 * std::numeric_limits<double>::epsilon() * std::fabs(D.courant)))
    return fail(RSWR_ERR_INVALID_ARG, "courant_num / courant_den differs from courant");
  const double a_ref = D.a_ref > 0 ? D.a_ref : D.a;
  const double lam = D.courant * (D.a / a_ref);
  if (!(D.courant > 0) || !(lam <= 1.0))
    return fail(RSWR_ERR_UNSTABLE, "a dt/dx must lie in (0, 1]");
  if ((D.sub_lo == nullptr) != (D.sub_hi == nullptr))
    return fail(RSWR_ERR_INVALID_ARG, "sub_lo and sub_hi go together");

  rswr_plan_s* p = new (std::nothrow) rswr_plan_s;
  if (!p) return fail(RSWR_ERR_NOMEM, "plan allocation");
  p->M = D.n_points;
  p->N = D.n_sub;
  p->P = D.overlap;
  p->dtype = D.dtype;
  p->mode = D.span_mode;
  p->beta = D.beta > 0 ? D.beta : 0.1;
  p->dx = (D.x_b - D.x_a) / double(D.n_points - 1);
  p->dt = D.courant * p->dx / a_ref;
  p->lam = lam;

  rswr_status_t st;
  if (D.sub_lo) {
    p->lo.assign(D.sub_lo, D.sub_lo + D.n_sub);
    p->hi.assign(D.sub_hi, D.sub_hi + D.n_sub);
    st = check_windows(*p);
  } else {
    st = uniform_windows(*p);
  }
  if (st != RSWR_OK) {
    delete p;
    return st;
  }

  if (p->N == 1) {
    p->S_cone = rswr::kMaxSpan;
    p->S_paper = rswr::kMaxSpan;
  } else {
    p->S_cone = light_cone_span(*p);
    const bool exact = D.courant_num > 0 && D.a == a_ref;
    p->S_paper = paper_span(*p, D.courant_num, D.courant_den, exact);
  }
  if (p->mode == RSWR_SPAN_FIXED) {
    if (D.span > 0) {
      if (D.span > p->S_cone) {
        const std::string msg = "span " + std::to_string(D.span) +
                                " exceeds the light-cone limit " + std::to_string(p->S_cone);
        delete p;
        return fail(RSWR_ERR_SPAN, msg);
      }
      p->S = D.span;
    } else {
      p->S = (p->N == 1) ? 32 : std::min(p->S_cone, p->S_paper);
    }
    if (p->S < 1) {
      delete p;
      return fail(RSWR_ERR_SPAN, "no admissible span (overlap too narrow)");
    }
    if (p->S > rswr::kMaxSpan) {
      if (D.span > 0) {
        delete p;
        return fail(RSWR_ERR_UNSUPPORTED, "span above the kernels' limit of " +
                                              std::to_string(rswr::kMaxSpan));
      }
      p->S = rswr::kMaxSpan;
    }
    p->S_max = p->S;
  } else {
    p->S = std::min(p->S_cone, rswr::kMaxSpan);
    p->S_max = std::min<int64_t>(2 * int64_t(p->S_cone), rswr::kMaxSpan);
  }
  p->flux_ld = static_cast<int32_t>(round_up(p->S_max, 16));

  if (D.tile_threads > 0 || D.tile_per_thread > 0) {
    if (!rswr::shape_built(D.tile_threads, D.tile_per_thread) ||
        (p->dtype == RSWR_F64 &&
         !shape_fits_fp64(rswr::Shape{D.tile_threads, D.tile_per_thread}))) {
      delete p;
      return fail(RSWR_ERR_UNSUPPORTED, "tile shape not built for this dtype");
    }
    const int TM = D.tile_threads * D.tile_per_thread;
    if (TM < 2 * p->S_max + 2 || !build_tiles(*p, TM, p->S_max, p->tiles)) {
      delete p;
      return fail(RSWR_ERR_UNSUPPORTED, "tile shape too small for the span");
    }
    p->threads = D.tile_threads;
    p->per_thread = D.tile_per_thread;
  } else {
    if (!choose_shape(*p)) {
      delete p;
      return fail(RSWR_ERR_UNSUPPORTED, "no built kernel shape fits this span");
    }
    build_tiles(*p, p->threads * p->per_thread, p->S_max, p->tiles);
  }
  for (size_t t = 0; t < p->tiles.size(); ++t)
    if (p->tiles[t].general) p->idx.push_back(static_cast<int32_t>(t));
  p->n_gen = static_cast<int32_t>(p->idx.size());
  for (size_t t = 0; t < p->tiles.size(); ++t)
    if (!p->tiles[t].general) p->idx.push_back(static_cast<int32_t>(t));
  p->fused = D.no_fuse == 0 && fuse_eligible(*p);
  if ((st = plan_sources(*p, D)) != RSWR_OK) {
    delete p;
    return st;
  }
  p->persist_ok = D.one_launch != 0 && p->fused && p->n_gen == 0 && p->src_node.empty() &&
                  2 * p->M * int64_t(elem_size(*p)) < (int64_t(1) << 31);
  if (p->persist_ok) build_deps(*p);
  *out = p;
  return RSWR_OK;
}

rswr_status_t rswr_plan_destroy(rswr_plan_t p) {
  if (!p) return RSWR_OK;
  if (p->dev.empty()) {  // never touched a device: no HIP call at all
    delete p;
    return RSWR_OK;
  }
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto& kv : p->dev) {
    (void)hipSetDevice(kv.first);
    (void)hipFree(kv.second.tiles);
    (void)hipFree(kv.second.idx);
    (void)hipFree(kv.second.src_ptr);
    (void)hipFree(kv.second.src_node);
    (void)hipFree(kv.second.src_id);
    (void)hipFree(kv.second.lo);
    (void)hipFree(kv.second.hi);
    (void)hipFree(kv.second.dep_ptr);
    (void)hipFree(kv.second.dep);
    if (kv.second.capture) (void)hipStreamDestroy(kv.second.capture);
  }
  for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.exec);
  (void)hipSetDevice(cur);
  delete p;
  return RSWR_OK;
}

rswr_status_t rswr_plan_info(rswr_plan_t p, rswr_plan_info_t* info) {
  if (!p || !info) return fail(RSWR_ERR_INVALID_ARG, "null plan or info");
  info->n_points = p->M;
  info->n_sub = p->N;
  info->dtype = p->dtype;
  info->span = p->mode == RSWR_SPAN_FIXED ? p->S : p->S_max;
  info->span_cone = p->S_cone;
  info->span_paper = p->S_paper;
  info->flux_ld = p->flux_ld;
  info->n_tiles = static_cast<int32_t>(p->tiles.size());
  info->tile_threads = p->threads;
  info->tile_per_thread = p->per_thread;
  info->dx = p->dx;
  info->dt = p->dt;
  info->lambda = p->lam;
  info->fused = p->fused ? 1 : 0;
  info->one_launch = p->persist_ok ? 1 : 0;
  return RSWR_OK;
}

rswr_status_t rswr_plan_layout(rswr_plan_t p, int64_t* lo, int64_t* hi, int64_t* own_lo,
                               int64_t* own_hi) {
  if (!p) return fail(RSWR_ERR_INVALID_ARG, "null plan");
  for (int32_t i = 0; i < p->N; ++i) {
    if (lo) lo[i] = p->lo[i];
    if (hi) hi[i] = p->hi[i];
    if (own_lo) own_lo[i] = p->own_lo[i];
    if (own_hi) own_hi[i] = p->own_hi[i];
  }
  return RSWR_OK;
}

rswr_status_t rswr_plan_tiles(rswr_plan_t p, int64_t* out) {
  if (!p || !out) return fail(RSWR_ERR_INVALID_ARG, "null plan or output");
  const int64_t TM = int64_t(p->threads) * p->per_thread;
  for (size_t t = 0; t < p->tiles.size(); ++t) {
    const Tile& x = p->tiles[t];
    int64_t* o = out + 8 * t;
    o[0] = x.a;
    o[1] = x.a + TM - 1;
    o[2] = x.out_lo;
    o[3] = x.out_hi;
    o[4] = x.window;
    o[5] = x.lmode;
    o[6] = x.rmode;
    o[7] = x.general;
  }
  return RSWR_OK;
}

rswr_status_t rswr_predict(rswr_plan_t p, const void* state, const void* f_a,
                           const void* f_b, int64_t n0, int32_t span_hat, void* flux,
                           void* stream) {
  if (!p || !state || !f_a || !f_b || !flux)
    return fail(RSWR_ERR_INVALID_ARG, "null pointer");
  if (!p->src_node.empty())
    return fail(RSWR_ERR_UNSUPPORTED, "plans with interior sources run rswr_span / rswr_solve");
  if (n0 < 0) return fail(RSWR_ERR_INVALID_ARG, "n0 must be >= 0");
  if (span_hat < 1 || span_hat > p->S_max)
    return fail(RSWR_ERR_SPAN, "span_hat outside 1.." + std::to_string(p->S_max));
  DevTables* d = nullptr;
  rswr_status_t st = ensure_device(p, &d, nullptr);
  if (st != RSWR_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (p->dtype == RSWR_F64)
    e = rswr::launch_predict<double>(
        predict_args<double>(*p, *d, state, f_a, f_b, n0, span_hat, flux), 2 * span_hat + 1, s);
  else
    e = rswr::launch_predict<float>(
        predict_args<float>(*p, *d, state, f_a, f_b, n0, span_hat, flux), 2 * span_hat + 1, s);
  if (e != hipSuccess) return hip_fail(e, "predict launch");
  return RSWR_OK;
}

rswr_status_t rswr_select(rswr_plan_t p, const void* flux, int32_t span_hat,
                          int32_t* span_dev, void* stream) {
  if (!p || !span_dev || (!flux && p->N > 1))
    return fail(RSWR_ERR_INVALID_ARG, "null pointer");
  if (span_hat < 1 || span_hat > p->S_max)
    return fail(RSWR_ERR_SPAN, "span_hat outside 1.." + std::to_string(p->S_max));
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (p->dtype == RSWR_F64) {
    rswr::SelectArgs<double> a{static_cast<const double*>(flux), span_dev, nullptr,
                               2 * (p->N - 1), span_hat, p->flux_ld, p->S_cone, p->mode,
                               p->S};
    e = rswr::launch_select<double>(a, s);
  } else {
    rswr::SelectArgs<float> a{static_cast<const float*>(flux), span_dev, nullptr,
                              2 * (p->N - 1), span_hat, p->flux_ld, p->S_cone, p->mode,
                              p->S};
    e = rswr::launch_select<float>(a, s);
  }
  if (e != hipSuccess) return hip_fail(e, "select launch");
  return RSWR_OK;
}

rswr_status_t rswr_update(rswr_plan_t p, const void* state_in, const void* f_a,
                          const void* f_b, int64_t n0, const void* flux,
                          const int32_t* span_dev, int32_t span, void* state_out,
                          void* stream) {
  if (!p || !state_in || !f_a || !f_b || !state_out || (!flux && p->N > 1))
    return fail(RSWR_ERR_INVALID_ARG, "null pointer");
  if (!p->src_node.empty())
    return fail(RSWR_ERR_UNSUPPORTED, "plans with interior sources run rswr_span / rswr_solve");
  if (n0 < 0) return fail(RSWR_ERR_INVALID_ARG, "n0 must be >= 0");
  if (state_in == state_out) return fail(RSWR_ERR_INVALID_ARG, "state_out aliases state_in");
  if (!span_dev && (span < 1 || span > p->S_max))
    return fail(RSWR_ERR_SPAN, "span outside 1.." + std::to_string(p->S_max));
  DevTables* d = nullptr;
  rswr_status_t st = ensure_device(p, &d, nullptr);
  if (st != RSWR_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int32_t n_all = static_cast<int32_t>(p->tiles.size());
  hipError_t e;
  if (p->dtype == RSWR_F64)
    e = launch_update_pair<double>(
        *p, update_args<double>(*p, *d, state_in, f_a, f_b, n0, flux, span_dev, span,
                                state_out),
        d->idx, p->n_gen, d->idx + p->n_gen, n_all - p->n_gen, s);
  else
    e = launch_update_pair<float>(
        *p, update_args<float>(*p, *d, state_in, f_a, f_b, n0, flux, span_dev, span,
                               state_out),
        d->idx, p->n_gen, d->idx + p->n_gen, n_all - p->n_gen, s);
  if (e != hipSuccess) return hip_fail(e, "update launch");
  return RSWR_OK;
}

rswr_status_t rswr_span(rswr_plan_t p, const void* state_in, const void* f_a, const void* f_b,
                        int64_t n0, int32_t span, void* flux, void* state_out,
                        void* stream) {
  if (!p || !state_in || !f_a || !f_b || !state_out)
    return fail(RSWR_ERR_INVALID_ARG, "null pointer");
  if (!p->fused && !flux && p->N > 1)
    return fail(RSWR_ERR_INVALID_ARG, "this plan predicts through `flux`: pass a buffer");
  if (p->mode != RSWR_SPAN_FIXED)
    return fail(RSWR_ERR_UNSUPPORTED, "rswr_span runs FIXED plans");
  if (n0 < 0) return fail(RSWR_ERR_INVALID_ARG, "n0 must be >= 0");
  if (state_in == state_out) return fail(RSWR_ERR_INVALID_ARG, "state_out aliases state_in");
  if (span < 1 || span > p->S)
    return fail(RSWR_ERR_SPAN, "span outside 1.." + std::to_string(p->S));
  if (!p->src_node.empty() && n0 + span > p->src_ld)
    return fail(RSWR_ERR_INVALID_ARG, "the span runs past the source samples (src_ld)");
  DevTables* d = nullptr;
  rswr_status_t st = ensure_device(p, &d, nullptr);
  if (st != RSWR_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int32_t n_all = static_cast<int32_t>(p->tiles.size());
  auto run = [&](auto tag) -> hipError_t {
    using T = decltype(tag);
    if (!p->fused && p->N > 1) {
      hipError_t e = rswr::launch_predict<T>(
          predict_args<T>(*p, *d, state_in, f_a, f_b, n0, span, flux), 2 * p->S_max + 1, s);
      if (e != hipSuccess) return e;
    }
    rswr::UpdateArgs<T> ua =
        update_args<T>(*p, *d, state_in, f_a, f_b, n0, flux, nullptr, span, state_out);
    if (p->fused) {
      ua.flux = nullptr;
      ua.flux_out = static_cast<T*>(flux);
    }
    if (p->fused)
      return launch_fused_span<T>(*p, ua, d->idx, p->n_gen, d->idx + p->n_gen,
                                  n_all - p->n_gen, s);
    return launch_update_pair<T>(*p, ua, d->idx, p->n_gen, d->idx + p->n_gen,
                                 n_all - p->n_gen, s);
  };
  const hipError_t e = p->dtype == RSWR_F64 ? run(double{}) : run(float{});
  if (e != hipSuccess) return hip_fail(e, "span launch");
  return RSWR_OK;
}

rswr_status_t rswr_checkpoint_size(rswr_plan_t p, int64_t n_steps, size_t* bytes) {
  if (!p || !bytes || n_steps < 0) return fail(RSWR_ERR_INVALID_ARG, "bad argument");
  const int64_t K = (n_steps + p->S - 1) / p->S;
  const size_t st = 2 * size_t(p->M);
  const size_t fl = size_t(std::max(p->N - 1, 1)) * 2 * p->flux_ld;
  *bytes = (size_t(K + 1) * st + size_t(K) * fl) * elem_size(*p);
  return RSWR_OK;
}

rswr_status_t rswr_solve_workspace_size(rswr_plan_t p, int32_t n_rec, size_t* bytes) {
  if (!p || !bytes || n_rec < 0) return fail(RSWR_ERR_INVALID_ARG, "bad argument");
  *bytes = ws_layout(*p, n_rec).total;
  return RSWR_OK;
}

rswr_status_t rswr_solve(rswr_plan_t p, void* state, const void* f_a, const void* f_b,
                         int64_t n0, int64_t n_steps, const int64_t* rec_idx,
                         int32_t n_rec, void* traces, void* workspace, size_t ws_bytes,
                         void* checkpoints, void* stream) {
  if (!p || !state || !f_a || !f_b) return fail(RSWR_ERR_INVALID_ARG, "null pointer");
  if (p->mode != RSWR_SPAN_FIXED && checkpoints)
    return fail(RSWR_ERR_UNSUPPORTED, "checkpoints need a FIXED plan");
  if (n0 < 0 || n_steps < 0 || n_rec < 0)
    return fail(RSWR_ERR_INVALID_ARG, "negative n0, n_steps or n_rec");
  if (n_rec > 0 && (!rec_idx || !traces))
    return fail(RSWR_ERR_INVALID_ARG, "receivers need rec_idx and traces");
  if (!p->src_node.empty() && n0 + n_steps > p->src_ld)
    return fail(RSWR_ERR_INVALID_ARG, "the solve runs past the source samples (src_ld)");
  if (n_steps == 0) return RSWR_OK;
  const WsLayout L = ws_layout(*p, n_rec);
  if (!workspace || ws_bytes < L.total)
    return fail(RSWR_ERR_NOMEM, "workspace needs " + std::to_string(L.total) + " bytes");
  for (int32_t r = 0; r < n_rec; ++r)
    if (rec_idx[r] < 0 || rec_idx[r] >= p->M)
      return fail(RSWR_ERR_INVALID_ARG, "receiver index out of range");
  DevTables* d = nullptr;
  int device = 0;
  rswr_status_t st = ensure_device(p, &d, &device);
  if (st != RSWR_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);

  Lists lists;
  const int32_t n_all = static_cast<int32_t>(p->tiles.size());
  if (n_rec == 0) {
    lists.gen = d->idx;
    lists.n_gen = p->n_gen;
    lists.fast = d->idx + p->n_gen;
    lists.n_fast = n_all - p->n_gen;
  } else {
    // receiver r is recorded by the tile whose stored range holds its node;
    // such tiles run through the general kernel, which records traces
    std::vector<std::vector<int32_t>> per(n_all);
    for (int32_t r = 0; r < n_rec; ++r)
      for (int32_t t = 0; t < n_all; ++t)
        if (rec_idx[r] >= p->tiles[t].out_lo && rec_idx[r] <= p->tiles[t].out_hi) {
          per[t].push_back(r);
          break;
        }
    std::vector<int32_t> gen, fast, ptr(1, 0), id;
    std::vector<int64_t> node;
    // two-launch path: receiver tiles run general, the CSR covers the
    // general list.  Fused path: general tiles, then all others; the CSR
    // covers both lists.
    // a fused-path tile records at most kRecSlots receivers per launched
    // copy: a tile holding more is listed once per group (the copies store
    // the same state bits).  On a grid that leaves SIMDs idle (at most two
    // waves per SIMD even with one copy per receiver; 4 SIMDs per CU) each
    // copy records one receiver: there the recording tiles set the span's
    // time, and their copies run side by side.
    size_t rg = rswr::kRecSlots;
    if (p->fused) {
      int dev = 0, cus = 0;
      if (hipGetDevice(&dev) == hipSuccess &&
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) ==
              hipSuccess) {
        const int64_t waves = (int64_t(n_all) + n_rec) * (p->threads / 64);
        if (cus > 0 && waves <= 2 * 4 * int64_t(cus)) rg = 1;
      }
    }
    auto add = [&](std::vector<int32_t>& list, int32_t t) {
      const size_t n = per[t].size();
      const size_t g = p->fused ? rg : std::max<size_t>(n, 1);
      for (size_t b = 0; b == 0 || b < n; b += g) {
        list.push_back(t);
        for (size_t r = b; r < std::min(n, b + g); ++r) {
          id.push_back(per[t][r]);
          node.push_back(rec_idx[per[t][r]]);
        }
        ptr.push_back(static_cast<int32_t>(id.size()));
      }
    };
    for (int32_t t = 0; t < n_all; ++t)
      if (p->tiles[t].general || (!p->fused && !per[t].empty())) add(gen, t);
    for (int32_t t = 0; t < n_all; ++t) {
      if (p->tiles[t].general) continue;
      if (p->fused)
        add(fast, t);
      else if (per[t].empty())
        fast.push_back(t);
    }
    if (!gen.empty())
      RSWR_HIP(hipMemcpyAsync(ws + L.gen_idx, gen.data(), gen.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, s));
    if (!fast.empty())
      RSWR_HIP(hipMemcpyAsync(ws + L.fast_idx, fast.data(), fast.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, s));
    RSWR_HIP(hipMemcpyAsync(ws + L.rec_ptr, ptr.data(), ptr.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, s));
    RSWR_HIP(hipMemcpyAsync(ws + L.rec_node, node.data(), node.size() * sizeof(int64_t),
                            hipMemcpyHostToDevice, s));
    RSWR_HIP(hipMemcpyAsync(ws + L.rec_id, id.data(), id.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, s));
    lists.n_gen = static_cast<int32_t>(gen.size());
    lists.gen = reinterpret_cast<const int32_t*>(ws + L.gen_idx);
    lists.fast = reinterpret_cast<const int32_t*>(ws + L.fast_idx);
    lists.n_fast = static_cast<int32_t>(fast.size());
    lists.rec_ptr = reinterpret_cast<const int32_t*>(ws + L.rec_ptr);
    lists.rec_node = reinterpret_cast<const int64_t*>(ws + L.rec_node);
    lists.rec_id = reinterpret_cast<const int32_t*>(ws + L.rec_id);
  }

  const bool persist = n_rec == 0 && use_persist(*p);
  auto enqueue = [&](hipStream_t q) {
    if (p->mode == RSWR_SPAN_QUIET)
      return p->dtype == RSWR_F64
                 ? enqueue_solve_quiet<double>(p, *d, state, f_a, f_b, n0, n_steps, lists,
                                               traces, ws, L, q)
                 : enqueue_solve_quiet<float>(p, *d, state, f_a, f_b, n0, n_steps, lists,
                                              traces, ws, L, q);
    return p->dtype == RSWR_F64
               ? enqueue_solve<double>(p, *d, state, f_a, f_b, n0, n_steps, lists,
                                       traces, ws, L, checkpoints, persist, q)
               : enqueue_solve<float>(p, *d, state, f_a, f_b, n0, n_steps, lists,
                                      traces, ws, L, checkpoints, persist, q);
  };
  const GraphKey key{1,
                     device,
                     reinterpret_cast<int64_t>(state),
                     reinterpret_cast<int64_t>(f_a),
                     reinterpret_cast<int64_t>(f_b),
                     n0,
                     n_steps,
                     reinterpret_cast<int64_t>(traces),
                     reinterpret_cast<int64_t>(workspace),
                     reinterpret_cast<int64_t>(checkpoints),
                     n_rec > 0,
                     lists.n_gen,
                     lists.n_fast,
                     persist};
  return run_graph(p, d, key, enqueue, s);
}

}  // extern "C"

namespace {

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
rswr_status_t scratch_on(int dev, char** out) {
  static std::mutex mu;
  static std::map<int, char*> addr;
  std::lock_guard<std::mutex> g(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                      "hipGetSymbolAddress(scratch)");
    it = addr.emplace(dev, static_cast<char*>(ptr)).first;
  }
  *out = it->second;
  return RSWR_OK;
}

}  // namespace

extern "C" {

rswr_status_t rswr_solve_noalloc(rswr_plan_t p, void* state, const void* f_a, const void* f_b,
                                 int64_t n0, int64_t n_steps, void* stream) {
  if (!p || !state || !f_a || !f_b) return fail(RSWR_ERR_INVALID_ARG, "null pointer");
  if (n0 < 0 || n_steps < 0) return fail(RSWR_ERR_INVALID_ARG, "negative n0 or n_steps");
  if (!p->src_node.empty() && n0 + n_steps > p->src_ld)
    return fail(RSWR_ERR_INVALID_ARG, "the solve runs past the source samples (src_ld)");
  const WsLayout L = ws_layout(*p, 0);
  if (L.total > kScratchBytes)
    return fail(RSWR_ERR_NOMEM, "rswr_solve_noalloc: this plan needs " +
                                    std::to_string(L.total) + " bytes of workspace, beyond "
                                    "the library's scratch of " +
                                    std::to_string(kScratchBytes) + " bytes per GPU");
  if (n_steps == 0) return RSWR_OK;
  int dev = 0;
  RSWR_HIP(hipGetDevice(&dev));
  DevTables* d = nullptr;
  {
    std::lock_guard<std::mutex> g(p->mu);
    auto it = p->dev.find(dev);
    if (it == p->dev.end())
      return fail(RSWR_ERR_UNSUPPORTED,
                  "rswr_solve_noalloc: the plan's tables are not on this device yet (they "
                  "are uploaded by the plan's first other compute call here)");
    d = &it->second;
  }
  char* ws = nullptr;
  rswr_status_t st = scratch_on(dev, &ws);
  if (st != RSWR_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Lists lists;
  const int32_t n_all = static_cast<int32_t>(p->tiles.size());
  lists.gen = d->idx;
  lists.n_gen = p->n_gen;
  lists.fast = d->idx + p->n_gen;
  lists.n_fast = n_all - p->n_gen;
  if (p->mode == RSWR_SPAN_QUIET)
    return p->dtype == RSWR_F64
               ? enqueue_solve_quiet<double>(p, *d, state, f_a, f_b, n0, n_steps, lists,
                                             nullptr, ws, L, s)
               : enqueue_solve_quiet<float>(p, *d, state, f_a, f_b, n0, n_steps, lists,
                                            nullptr, ws, L, s);
  const bool persist = use_persist(*p);
  return p->dtype == RSWR_F64
             ? enqueue_solve<double>(p, *d, state, f_a, f_b, n0, n_steps, lists, nullptr, ws,
                                     L, nullptr, persist, s)
             : enqueue_solve<float>(p, *d, state, f_a, f_b, n0, n_steps, lists, nullptr, ws,
                                    L, nullptr, persist, s);
}

rswr_status_t rswr_adjoint_fused(rswr_plan_t p, int32_t* fused) {
  if (!p || !fused) return fail(RSWR_ERR_INVALID_ARG, "null pointer");
  *fused = (p->fused && adj_fused_fits(*p)) ? 1 : 0;
  return RSWR_OK;
}

rswr_status_t rswr_adjoint_workspace_size(rswr_plan_t p, int32_t n_rec, size_t* bytes) {
  if (!p || !bytes || n_rec < 0) return fail(RSWR_ERR_INVALID_ARG, "bad argument");
  *bytes = adj_ws_layout(*p, n_rec).total;
  return RSWR_OK;
}

rswr_status_t rswr_solve_adjoint(rswr_plan_t p, const void* checkpoints, const void* f_a,
                                 const void* f_b, int64_t n_steps, const int64_t* rec_idx,
                                 int32_t n_rec, const void* grad_traces, void* grad_f_a,
                                 void* grad_f_b, double* grad_lambda, void* workspace,
                                 size_t ws_bytes, void* stream) {
  if (!p || !checkpoints || !f_a || !f_b || !grad_f_a || !grad_f_b || !grad_lambda)
    return fail(RSWR_ERR_INVALID_ARG, "null pointer");
  if (p->mode != RSWR_SPAN_FIXED)
    return fail(RSWR_ERR_UNSUPPORTED, "rswr_solve_adjoint runs FIXED plans");
  if (!p->src_node.empty())
    return fail(RSWR_ERR_UNSUPPORTED, "rswr_solve_adjoint: plans with interior sources");
  if (n_steps < 1 || n_rec < 0 || (n_rec > 0 && (!rec_idx || !grad_traces)))
    return fail(RSWR_ERR_INVALID_ARG, "bad n_steps, receivers or grad_traces");
  for (int32_t r = 0; r < n_rec; ++r)
    if (rec_idx[r] < 0 || rec_idx[r] >= p->M)
      return fail(RSWR_ERR_INVALID_ARG, "receiver index out of range");
  const AdjWs L = adj_ws_layout(*p, n_rec);
  if (!workspace || ws_bytes < L.total)
    return fail(RSWR_ERR_NOMEM, "workspace needs " + std::to_string(L.total) + " bytes");
  DevTables* d = nullptr;
  int device = 0;
  rswr_status_t st = ensure_device(p, &d, &device);
  if (st != RSWR_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  AdjLists al;
  if ((st = upload_adj_lists(*p, rec_idx, n_rec, ws, L, s, &al)) != RSWR_OK) return st;
  al.fused = p->fused && adj_fused_fits(*p);

  auto enqueue = [&](hipStream_t q) {
    return p->dtype == RSWR_F64
               ? enqueue_adjoint<double>(p, *d, checkpoints, f_a, f_b, n_steps, al,
                                         grad_traces, grad_f_a, grad_f_b, grad_lambda, ws,
                                         L, n_rec, q)
               : enqueue_adjoint<float>(p, *d, checkpoints, f_a, f_b, n_steps, al,
                                        grad_traces, grad_f_a, grad_f_b, grad_lambda, ws,
                                        L, n_rec, q);
  };
  const GraphKey key{2,
                     device,
                     reinterpret_cast<int64_t>(checkpoints),
                     reinterpret_cast<int64_t>(f_a),
                     reinterpret_cast<int64_t>(f_b),
                     n_steps,
                     n_rec,
                     reinterpret_cast<int64_t>(grad_traces),
                     reinterpret_cast<int64_t>(grad_f_a),
                     reinterpret_cast<int64_t>(grad_f_b),
                     reinterpret_cast<int64_t>(grad_lambda),
                     reinterpret_cast<int64_t>(workspace),
                     al.n_gen,
                     al.n_fast};
  return run_graph(p, d, key, enqueue, s);
}

rswr_status_t rswr_adjoint_batch_workspace_size(rswr_plan_t p, int64_t n_steps, int32_t n_rec,
                                                int32_t group, int32_t seg, size_t* bytes) {
  if (!p || !bytes || n_steps < 1 || n_rec < 0 || group < 1 || seg < 0)
    return fail(RSWR_ERR_INVALID_ARG, "bad argument");
  *bytes = adj_batch_layout(*p, n_steps, n_rec, group, seg).total;
  return RSWR_OK;
}

rswr_status_t rswr_solve_adjoint_batch(rswr_plan_t p, int32_t n_prob, const void* f_a,
                                       const void* f_b, int64_t src_ld, int64_t n_steps,
                                       const int64_t* rec_idx, int32_t n_rec,
                                       const void* grad_traces, void* grad_f_a,
                                       void* grad_f_b, double* grad_lambda, int32_t group,
                                       int32_t seg, void* workspace, size_t ws_bytes,
                                       void* stream) {
  if (!p || !f_a || !f_b || !grad_f_a || !grad_f_b || !grad_lambda || n_prob < 1)
    return fail(RSWR_ERR_INVALID_ARG, "null pointer or no problems");
  if (p->mode != RSWR_SPAN_FIXED || !p->fused || !p->src_node.empty())
    return fail(RSWR_ERR_UNSUPPORTED,
                "rswr_solve_adjoint_batch runs fused FIXED plans without sources");
  if (n_steps < 1 || n_rec < 0 || (n_rec > 0 && (!rec_idx || !grad_traces)) || group < 1 ||
      seg < 0 || src_ld < n_steps + 1)
    return fail(RSWR_ERR_INVALID_ARG, "bad n_steps, receivers, group, seg or src_ld");
  for (int32_t r = 0; r < n_rec; ++r)
    if (rec_idx[r] < 0 || rec_idx[r] >= p->M)
      return fail(RSWR_ERR_INVALID_ARG, "receiver index out of range");
  const AdjBatchWs L = adj_batch_layout(*p, n_steps, n_rec, group, seg);
  if (!workspace || ws_bytes < L.total)
    return fail(RSWR_ERR_NOMEM, "workspace needs " + std::to_string(L.total) + " bytes");
  DevTables* d = nullptr;
  int device = 0;
  rswr_status_t st = ensure_device(p, &d, &device);
  if (st != RSWR_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  AdjLists al;
  if ((st = upload_adj_lists(*p, rec_idx, n_rec, ws, L, s, &al)) != RSWR_OK) return st;
  al.fused = p->fused && adj_fused_fits(*p);
  auto enqueue = [&](hipStream_t q) {
    return p->dtype == RSWR_F64
               ? enqueue_adjoint_batch<double>(p, *d, n_prob, f_a, f_b, src_ld, n_steps, al,
                                               grad_traces, grad_f_a, grad_f_b, grad_lambda,
                                               ws, L, n_rec, group, q)
               : enqueue_adjoint_batch<float>(p, *d, n_prob, f_a, f_b, src_ld, n_steps, al,
                                              grad_traces, grad_f_a, grad_f_b, grad_lambda,
                                              ws, L, n_rec, group, q);
  };
  const GraphKey key{7,
                     device,
                     n_prob,
                     reinterpret_cast<int64_t>(f_a),
                     reinterpret_cast<int64_t>(f_b),
                     src_ld,
                     n_steps,
                     n_rec,
                     reinterpret_cast<int64_t>(grad_traces),
                     reinterpret_cast<int64_t>(grad_f_a),
                     reinterpret_cast<int64_t>(grad_f_b),
                     reinterpret_cast<int64_t>(grad_lambda),
                     group,
                     seg,
                     reinterpret_cast<int64_t>(workspace),
                     al.n_gen,
                     al.n_fast};
  return run_graph(p, d, key, enqueue, s);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched solve: many independent problems (each a fused-span plan) advanced
// together.  Round r runs span r of every problem with spans left; per
// kernel shape one persistent launch walks the round's tiles.  Problems are
// ordered by span count, longest first, so a round's tiles are a prefix of
// each shape's list.  The whole run is recorded into one HIP graph.
// ---------------------------------------------------------------------------
struct rswr_batch_s {
  std::vector<rswr_plan_s*> plans;
  int32_t dtype = 0;
  std::vector<std::pair<int32_t, int32_t>> shapes;  // (threads, nodes per lane)
  std::vector<int32_t> shape_of;                    // per problem
  std::mutex mu;
  std::vector<GraphEntry> graphs;
  std::map<int, hipStream_t> capture;
  std::map<int, std::vector<hipStream_t>> lanes;  // per device: one stream per shape
  std::map<int, std::vector<hipEvent_t>> events;  // per device: fork + one per shape
  std::map<int, std::vector<int32_t>> grid;  // per device: resident groups per shape
};

namespace {

struct BatchWs {
  size_t inst = 0, items = 0, jobs = 0, total = 0;
  std::vector<size_t> state;  // per problem: its second state buffer
};

BatchWs batch_ws_layout(const rswr_batch_s& b) {
  BatchWs w;
  const size_t e = b.dtype == RSWR_F64 ? 8 : 4;
  const size_t n = b.plans.size();
  const size_t inst_bytes = b.dtype == RSWR_F64 ? sizeof(rswr::BatchInst<double>)
                                                : sizeof(rswr::BatchInst<float>);
  size_t n_tiles = 0;
  for (const rswr_plan_s* p : b.plans) n_tiles += p->tiles.size();
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += round_up(std::max<size_t>(bytes, 1), 256);
    return at;
  };
  w.inst = take(n * inst_bytes);
  w.items = take(n_tiles * sizeof(Tile));
  w.jobs = take(n * (2 * sizeof(void*) + sizeof(int64_t)));
  for (const rswr_plan_s* p : b.plans) w.state.push_back(take(2 * size_t(p->M) * e));
  w.total = off;
  return w;
}

template <typename T>
rswr_status_t batch_solve(rswr_batch_s* b, void* const* states, const void* const* f_a,
                          const void* const* f_b, const int64_t* n_steps, char* ws,
                          const BatchWs& L, hipStream_t s) {
  const int32_t n = static_cast<int32_t>(b->plans.size());
  int device = 0;
  std::vector<DevTables*> dt(n);
  for (int32_t i = 0; i < n; ++i) {
    rswr_status_t st = ensure_device(b->plans[i], &dt[i], &device);
    if (st != RSWR_OK) return st;
  }
  hipStream_t cap = nullptr;
  std::vector<int32_t> grid;
  {
    std::lock_guard<std::mutex> g(b->mu);
    auto it = b->capture.find(device);
    if (it == b->capture.end()) {
      hipStream_t c = nullptr;
      RSWR_HIP(hipStreamCreateWithFlags(&c, hipStreamNonBlocking));
      it = b->capture.emplace(device, c).first;
      std::vector<int32_t> gr;
      std::vector<hipStream_t> ln;
      std::vector<hipEvent_t> ev;
      hipEvent_t e = nullptr;
      RSWR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      ev.push_back(e);
      for (const auto& sh : b->shapes) {
        gr.push_back(std::max(1, rswr::fused_batch_capacity<T>(sh.first, sh.second)));
        hipStream_t q = nullptr;
        RSWR_HIP(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
        ln.push_back(q);
        RSWR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ev.push_back(e);
      }
      b->grid[device] = gr;
      b->lanes[device] = ln;
      b->events[device] = ev;
    }
    cap = it->second;
    grid = b->grid[device];
  }
  const std::vector<hipStream_t> lanes = b->lanes[device];
  const std::vector<hipEvent_t> events = b->events[device];

  // spans per problem, longest first
  std::vector<int64_t> K(n);
  for (int32_t i = 0; i < n; ++i) K[i] = (n_steps[i] + b->plans[i]->S - 1) / b->plans[i]->S;
  std::vector<int32_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return K[x] > K[y]; });
  const int64_t rounds = n > 0 ? K[order[0]] : 0;

  std::vector<rswr::BatchInst<T>> inst(n);
  std::vector<rswr::CopyJob<T>> jobs;
  for (int32_t i = 0; i < n; ++i) {
    const rswr_plan_s& p = *b->plans[i];
    T* user = static_cast<T*>(states[i]);
    T* other = reinterpret_cast<T*>(ws + L.state[i]);
    // an odd number of spans starts from a copy, so the last span writes
    // the caller's buffer
    const bool odd = K[i] & 1;
    rswr::BatchInst<T>& in = inst[i];
    in.st_a = odd ? other : user;
    in.st_b = odd ? user : other;
    if (odd) jobs.push_back({other, user, 2 * p.M});
    in.fa = static_cast<const T*>(f_a[i]);
    in.fb = static_cast<const T*>(f_b[i]);
    in.lo = dt[i]->lo;
    in.hi = dt[i]->hi;
    in.M = p.M;
    in.n_steps = n_steps[i];
    in.S = p.S;
    const double c2 = p.lam * p.lam;
    in.c2 = T(c2);
    in.k = T(2.0 - 2.0 * c2);
    in.q = T(2.0 * p.dx);
    in.r = T(1.0 / (2.0 * p.dx));
  }
  // tiles per shape in problem order; active[c][r]: tiles of round r
  const size_t n_shapes = b->shapes.size();
  std::vector<std::vector<Tile>> items(n_shapes);
  std::vector<std::vector<int32_t>> active(n_shapes, std::vector<int32_t>(rounds, 0));
  for (int32_t i : order) {
    const int32_t c = b->shape_of[i];
    for (Tile t : b->plans[i]->tiles) {
      t.inst = i;
      items[c].push_back(t);
    }
    for (int64_t r = 0; r < K[i]; ++r) active[c][r] += int32_t(b->plans[i]->tiles.size());
  }
  std::vector<size_t> item_off(n_shapes, 0);
  std::vector<Tile> all;
  for (size_t c = 0; c < n_shapes; ++c) {
    item_off[c] = all.size();
    all.insert(all.end(), items[c].begin(), items[c].end());
  }
  if (n > 0)
    RSWR_HIP(hipMemcpyAsync(ws + L.inst, inst.data(), n * sizeof(rswr::BatchInst<T>),
                            hipMemcpyHostToDevice, s));
  if (!all.empty())
    RSWR_HIP(hipMemcpyAsync(ws + L.items, all.data(), all.size() * sizeof(Tile),
                            hipMemcpyHostToDevice, s));
  if (!jobs.empty())
    RSWR_HIP(hipMemcpyAsync(ws + L.jobs, jobs.data(), jobs.size() * sizeof(rswr::CopyJob<T>),
                            hipMemcpyHostToDevice, s));

  const auto* inst_d = reinterpret_cast<const rswr::BatchInst<T>*>(ws + L.inst);
  const auto* items_d = reinterpret_cast<const Tile*>(ws + L.items);
  const auto* jobs_d = reinterpret_cast<const rswr::CopyJob<T>*>(ws + L.jobs);
  const int32_t n_jobs = static_cast<int32_t>(jobs.size());
  // Problems of different shapes share nothing: each shape's rounds form
  // their own chain on a stream of their own (fork after the copies, join
  // at the end), so the chains overlap on the device.
  auto enqueue = [&](hipStream_t q) -> rswr_status_t {
    RSWR_HIP(rswr::launch_copy_many<T>(jobs_d, n_jobs, q));
    RSWR_HIP(hipEventRecord(events[0], q));
    for (size_t c = 0; c < n_shapes; ++c) {
      hipStream_t lane = lanes[c];
      RSWR_HIP(hipStreamWaitEvent(lane, events[0], 0));
      for (int64_t r = 0; r < rounds; ++r) {
        if (active[c][r] == 0) break;  // later rounds have fewer problems
        rswr::BatchArgs<T> a{};
        a.items = items_d + item_off[c];
        a.inst = inst_d;
        a.n_items = active[c][r];
        a.round = static_cast<int32_t>(r);
        RSWR_HIP(rswr::launch_fused_batch<T>(a, b->shapes[c].first, b->shapes[c].second,
                                             grid[c], lane));
      }
      RSWR_HIP(hipEventRecord(events[c + 1], lane));
      RSWR_HIP(hipStreamWaitEvent(q, events[c + 1], 0));
    }
    return RSWR_OK;
  };
  GraphKey key{3, reinterpret_cast<int64_t>(ws), n};
  for (int32_t i = 0; i < n; ++i) {
    key.push_back(reinterpret_cast<int64_t>(states[i]));
    key.push_back(reinterpret_cast<int64_t>(f_a[i]));
    key.push_back(reinterpret_cast<int64_t>(f_b[i]));
    key.push_back(n_steps[i]);
  }
  return run_graph_in(b->mu, b->graphs, cap, key, enqueue, s);
}

}  // namespace

extern "C" {

rswr_status_t rswr_batch_plan(const rswr_plan_t* plans, int32_t n, rswr_batch_t* out) {
  if (!out || (n > 0 && !plans) || n < 0) return fail(RSWR_ERR_INVALID_ARG, "bad argument");
  *out = nullptr;
  rswr_batch_s* b = new (std::nothrow) rswr_batch_s;
  if (!b) return fail(RSWR_ERR_NOMEM, "batch allocation");
  for (int32_t i = 0; i < n; ++i) {
    rswr_plan_s* p = plans[i];
    if (!p) {
      delete b;
      return fail(RSWR_ERR_INVALID_ARG, "null plan " + std::to_string(i));
    }
    if (!p->src_node.empty()) {
      delete b;
      return fail(RSWR_ERR_UNSUPPORTED, "batched plans take no interior sources");
    }
    if (i == 0) b->dtype = p->dtype;
    if (p->dtype != b->dtype) {
      delete b;
      return fail(RSWR_ERR_INVALID_ARG, "plans of different dtypes");
    }
    if (!p->fused) {
      delete b;
      return fail(RSWR_ERR_UNSUPPORTED,
                  "plan " + std::to_string(i) + " does not run the fused span");
    }
    const std::pair<int32_t, int32_t> sh{p->threads, p->per_thread};
    auto it = std::find(b->shapes.begin(), b->shapes.end(), sh);
    if (it == b->shapes.end()) {
      b->shapes.push_back(sh);
      it = b->shapes.end() - 1;
    }
    b->shape_of.push_back(static_cast<int32_t>(it - b->shapes.begin()));
    b->plans.push_back(p);
  }
  *out = b;
  return RSWR_OK;
}

rswr_status_t rswr_batch_destroy(rswr_batch_t b) {
  if (!b) return RSWR_OK;
  if (!b->capture.empty()) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : b->capture) {
      (void)hipSetDevice(kv.first);
      (void)hipStreamDestroy(kv.second);
      for (hipStream_t q : b->lanes[kv.first]) (void)hipStreamDestroy(q);
      for (hipEvent_t e : b->events[kv.first]) (void)hipEventDestroy(e);
    }
    for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    (void)hipSetDevice(cur);
  }
  delete b;
  return RSWR_OK;
}

rswr_status_t rswr_batch_workspace_size(rswr_batch_t b, size_t* bytes) {
  if (!b || !bytes) return fail(RSWR_ERR_INVALID_ARG, "null batch or output");
  *bytes = batch_ws_layout(*b).total;
  return RSWR_OK;
}

rswr_status_t rswr_batch_solve(rswr_batch_t b, void* const* states, const void* const* f_a,
                               const void* const* f_b, const int64_t* n_steps,
                               void* workspace, size_t ws_bytes, void* stream) {
  if (!b) return fail(RSWR_ERR_INVALID_ARG, "null batch");
  const int32_t n = static_cast<int32_t>(b->plans.size());
  if (n == 0) return RSWR_OK;
  if (!states || !f_a || !f_b || !n_steps)
    return fail(RSWR_ERR_INVALID_ARG, "null array argument");
  for (int32_t i = 0; i < n; ++i) {
    if (!states[i] || !f_a[i] || !f_b[i])
      return fail(RSWR_ERR_INVALID_ARG, "null pointer for problem " + std::to_string(i));
    if (n_steps[i] < 0) return fail(RSWR_ERR_INVALID_ARG, "negative n_steps");
  }
  const BatchWs L = batch_ws_layout(*b);
  if (!workspace || ws_bytes < L.total)
    return fail(RSWR_ERR_NOMEM, "workspace needs " + std::to_string(L.total) + " bytes");
  char* ws = static_cast<char*>(workspace);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (b->dtype == RSWR_F64)
    return batch_solve<double>(b, states, f_a, f_b, n_steps, ws, L, s);
  return batch_solve<float>(b, states, f_a, f_b, n_steps, ws, L, s);
}

}  // extern "C"
