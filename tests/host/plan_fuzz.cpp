// plan_fuzz.cpp -- drives the host side of the C-ABI (plan construction,
// layout, tiles, sources, the one-launch waits) over many seeded
// descriptors, valid and invalid, for a build of the host code under the
// address and undefined-behaviour sanitizers.  No GPU call is made: a plan
// that never touched a device is destroyed without one.
//
// Checks beside the sanitizers: every call returns a defined status; on
// success the windows satisfy the ordering of Eq. (4) of the method (Wei &
// Zhao, arXiv 2203.10477, Sec. 2.2), the owned ranges tile 0..M-1 (the
// gluing of Eq. (15)), and every owned node is stored by exactly one tile.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/rswr.h"

namespace {

uint64_t g_state = 0x2203104770ull;

uint64_t next_u64() {  // splitmix64
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int64_t uni(int64_t lo, int64_t hi) {  // inclusive
  return lo + static_cast<int64_t>(next_u64() % static_cast<uint64_t>(hi - lo + 1));
}

int g_fail = 0;

void expect(bool ok, const char* what, int64_t c) {
  if (!ok) {
    std::fprintf(stderr, "case %lld: %s\n", static_cast<long long>(c), what);
    ++g_fail;
  }
}

void check_plan(rswr_plan_t p, int64_t c) {
  rswr_plan_info_t info{};
  expect(rswr_plan_info(p, &info) == RSWR_OK, "plan_info", c);
  const int64_t M = info.n_points;
  const int32_t N = info.n_sub;
  std::vector<int64_t> lo(N), hi(N), olo(N), ohi(N);
  expect(rswr_plan_layout(p, lo.data(), hi.data(), olo.data(), ohi.data()) == RSWR_OK,
         "plan_layout", c);
  expect(lo[0] == 0 && hi[N - 1] == M - 1, "windows span the domain", c);
  for (int32_t i = 0; i + 1 < N; ++i)
    expect(lo[i] < lo[i + 1] && lo[i + 1] < hi[i] && hi[i] < hi[i + 1], "Eq. (4) order", c);
  int64_t next = 0;
  for (int32_t i = 0; i < N; ++i) {
    expect(olo[i] == next && ohi[i] >= olo[i], "owned ranges tile the grid", c);
    expect(olo[i] >= lo[i] && ohi[i] <= hi[i], "owned range inside the window", c);
    next = ohi[i] + 1;
  }
  expect(next == M, "owned ranges end at M-1", c);
  expect(info.n_tiles > 0, "tiles", c);
  std::vector<int64_t> t(8 * static_cast<size_t>(info.n_tiles));
  expect(rswr_plan_tiles(p, t.data()) == RSWR_OK, "plan_tiles", c);
  std::vector<uint8_t> cover(static_cast<size_t>(M), 0);
  for (int32_t k = 0; k < info.n_tiles; ++k) {
    const int64_t* x = &t[8 * static_cast<size_t>(k)];
    const int64_t w = x[4];
    expect(w >= 0 && w < N, "tile window", c);
    if (w < 0 || w >= N) continue;
    expect(x[2] >= olo[w] && x[3] <= ohi[w] && x[2] <= x[3] + 1, "stored range owned", c);
    // a tile next to node 0 or node M-1 (end mode 2) also stores that node
    expect(x[2] >= x[0] - (x[5] == 2) && x[3] <= x[1] + (x[6] == 2),
           "stored range inside the region", c);
    expect(x[0] >= 0 || (x[5] == 0 && x[2] >= 0), "region start", c);
    for (int64_t j = x[2]; j <= x[3] && j >= 0 && j < M; ++j) ++cover[static_cast<size_t>(j)];
  }
  bool once = true;
  for (int64_t j = 0; j < M; ++j) once = once && cover[static_cast<size_t>(j)] == 1;
  expect(once, "every node stored by exactly one tile", c);
}

}  // namespace

int main(int argc, char** argv) {
  const int64_t cases = argc > 1 ? std::atoll(argv[1]) : 400;
  int32_t th[64], pt[64], f64[64];
  const int32_t n_shapes = rswr_kernel_shapes(th, pt, f64, 64);
  int64_t made = 0, refused = 0;
  const double courants[] = {0.9, 0.5, 1.0, 0.999, 0.25};
  for (int64_t c = 0; c < cases; ++c) {
    rswr_desc_t d{};
    d.x_a = 0.0;
    d.x_b = 1.0;
    d.n_points = uni(3, 1) ? uni(3, 200000) : uni(3, 64);
    d.a = 0.5 + 0.001 * static_cast<double>(uni(0, 1500));
    d.a_ref = uni(0, 3) == 0 ? d.a * 1.25 : 0.0;
    const int ci = static_cast<int>(uni(0, 4));
    d.courant = courants[ci];
    if (ci == 0 && uni(0, 1)) {
      d.courant_num = 9;
      d.courant_den = 10;
    }
    d.n_sub = static_cast<int32_t>(uni(1, 300));
    d.overlap = static_cast<int32_t>(2 * uni(0, 70));
    d.span = uni(0, 3) == 0 ? static_cast<int32_t>(uni(1, 80)) : 0;
    d.span_mode = uni(0, 4) == 0 ? RSWR_SPAN_QUIET : RSWR_SPAN_FIXED;
    d.dtype = static_cast<int32_t>(uni(0, 1));
    if (uni(0, 2) == 0 && n_shapes > 0) {
      const int64_t s = uni(0, n_shapes - 1);
      d.tile_threads = th[s];
      d.tile_per_thread = pt[s];
    }
    d.no_fuse = uni(0, 5) == 0;
    d.one_launch = static_cast<int32_t>(uni(0, 1));
    // explicit windows: cores cut at random, widened by random half-overlaps
    std::vector<int64_t> slo, shi, nodes;
    if (uni(0, 3) == 0 && d.n_sub >= 2 && d.n_points > 4 * d.n_sub + 8) {
      const int64_t M = d.n_points;
      std::vector<int64_t> cut(static_cast<size_t>(d.n_sub + 1));
      cut[0] = 0;
      cut[static_cast<size_t>(d.n_sub)] = M - 1;
      for (int32_t i = 1; i < d.n_sub; ++i)
        cut[static_cast<size_t>(i)] = (M - 1) * i / d.n_sub + uni(-1, 1);
      slo.resize(static_cast<size_t>(d.n_sub));
      shi.resize(static_cast<size_t>(d.n_sub));
      for (int32_t i = 0; i < d.n_sub; ++i) {
        slo[static_cast<size_t>(i)] = i == 0 ? 0 : cut[static_cast<size_t>(i)] - uni(0, 12);
        shi[static_cast<size_t>(i)] =
            i == d.n_sub - 1 ? M - 1 : cut[static_cast<size_t>(i + 1)] + uni(0, 12);
      }
      d.sub_lo = slo.data();
      d.sub_hi = shi.data();
    }
    // interior sources (the device samples are never read by the plan)
    static float dummy_amp;
    if (uni(0, 3) == 0) {
      d.n_src = static_cast<int32_t>(uni(0, 40));
      for (int32_t q = 0; q < d.n_src; ++q) nodes.push_back(uni(0, d.n_points - 1));
      d.src_node = nodes.data();
      d.src_amp = &dummy_amp;
      d.src_ld = uni(0, 2);
    }
    rswr_plan_t p = nullptr;
    const rswr_status_t st = rswr_plan(&d, &p);
    expect(st >= RSWR_OK && st <= RSWR_ERR_UNSUPPORTED, "status in range", c);
    expect(rswr_status_string(st) != nullptr && rswr_last_error() != nullptr, "strings", c);
    if (st == RSWR_OK) {
      expect(p != nullptr, "plan returned", c);
      check_plan(p, c);
      ++made;
    } else {
      expect(p == nullptr, "no plan on failure", c);
      ++refused;
    }
    expect(rswr_plan_destroy(p) == RSWR_OK, "destroy", c);
  }
  // argument errors
  rswr_plan_t p = nullptr;
  expect(rswr_plan(nullptr, &p) == RSWR_ERR_INVALID_ARG, "null descriptor", -1);
  expect(rswr_plan_info(nullptr, nullptr) == RSWR_ERR_INVALID_ARG, "null plan", -1);
  std::printf("plans %lld refused %lld failures %d\n", static_cast<long long>(made),
              static_cast<long long>(refused), g_fail);
  return g_fail == 0 ? 0 : 1;
}
