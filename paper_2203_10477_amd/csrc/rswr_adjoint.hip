// rswr_adjoint.hip -- gfx950 kernels of the adjoint of the RSWR solve:
// the predict kernels, k_adj_finish and the launchers; the update of the
// two-launch path (the fused update: rswr_adjoint_fused_*.hip).  The
// method and the device code shared by both: rswr_adjoint.h.
#include "rswr_adjoint.h"

namespace rswr {

// the fused update is instantiated in its own translation units
extern template hipError_t launch_adj_update_kind<float, true>(const AdjUpdateArgs<float>&, int,
                                                               int, bool, hipStream_t);
extern template hipError_t launch_adj_update_kind<double, true>(const AdjUpdateArgs<double>&,
                                                                int, int, bool, hipStream_t);

template <typename T>
__global__ __launch_bounds__(64) void k_adj_predict_frame(const AdjPredictArgs<T> p0) {
  const AdjPredictArgs<T> p = batch_problem(p0);
  const int i = blockIdx.x >> 1, side = blockIdx.x & 1;
  const int w = i + side;
  const int64_t o = (side == 0) ? p.lo[i + 1] : p.hi[i];
  const int shat = p.shat;
  const int lane = threadIdx.x;
  T a[2], b[2];
  AdjFrame<T, kAdjFrameSrc> f;
  adj_frame_load(p.w, p.lo, p.hi, p.rec_node, p.n_rec, p.gtr, p.gtr_ld, p.M, p.n_e, o, w,
                 shat, lane, a, b, f);
  T fl = T(0);
  for (int s = 0; s < shat; s += 2) {
    T F = adj_frame_step(a, b, f, p.c2, p.k, p.r, s, lane, s < shat - 1);
    if (s < shat - 1)
      adj_frame_extra(b, f, p.rec_node, p.n_rec, p.gtr, p.gtr_ld, p.M, p.n_e, s, lane);
    fl = (lane == s) ? F : fl;
    if (s + 1 < shat) {
      F = adj_frame_step(b, a, f, p.c2, p.k, p.r, s + 1, lane, s + 1 < shat - 1);
      if (s + 1 < shat - 1)
        adj_frame_extra(a, f, p.rec_node, p.n_rec, p.gtr, p.gtr_ld, p.M, p.n_e, s + 1, lane);
      fl = (lane == s + 1) ? F : fl;
    }
  }
  if (lane < shat) p.flux[static_cast<int64_t>(2 * i + side) * p.ld + lane] = fl;
}

// The same prediction for spans beyond the frame: the light-cone trapezoid
// around o in LDS (window ends inside it keep their exact treatment).
template <typename T>
__global__ __launch_bounds__(64) void k_adj_predict_lds(const AdjPredictArgs<T> p0) {
  const AdjPredictArgs<T> p = batch_problem(p0);
  extern __shared__ unsigned char smem_raw[];
  T* const sm = reinterpret_cast<T*>(smem_raw);
  const int i = blockIdx.x >> 1, side = blockIdx.x & 1;
  const int w = i + side;
  const int64_t o = (side == 0) ? p.lo[i + 1] : p.hi[i];
  const int64_t wlo = p.lo[w], whi = p.hi[w];
  const int shat = p.shat;
  const int64_t A = (o - shat > wlo) ? o - shat : wlo;
  const int64_t B = (o + shat < whi) ? o + shat : whi;
  const int n = static_cast<int>(B - A + 1);
  const int cap = 2 * shat + 1;
  T* w0 = sm;        // W^{L+2}, overwritten with W^L
  T* w1 = sm + cap;  // W^{L+1}
  const int tid = threadIdx.x;
  for (int x = tid; x < n; x += 64) {
    w0[x] = p.w[A + x];
    w1[x] = p.w[p.M + A + x];
  }
  __syncthreads();
  const bool lex = (A == wlo), rex = (B == whi);
  const T zero = T(0);
  T* const row = p.flux + static_cast<int64_t>(2 * i + side) * p.ld;
  const int oi = static_cast<int>(o - A);
  for (int s = 0; s < shat; ++s) {
    if (tid == 0) row[s] = (w1[oi + 1] - w1[oi - 1]) * p.r;
    if (s == shat - 1) break;
    for (int x = tid; x < n; x += 64) {
      const int64_t j = A + x;
      T v;
      if (j == 0 || j == p.M - 1) {
        v = zero;
      } else {
        const T ul = (x == 0) ? (lex ? fma_(-p.q, zero, w1[1]) : zero) : w1[x - 1];
        const T ur = (x == n - 1) ? (rex ? fma_(p.q, zero, w1[n - 2]) : zero) : w1[x + 1];
        v = leap(p.c2, p.k, ul, w1[x], ur, w0[x]);
      }
      w0[x] = v;
    }
    __syncthreads();
    if (tid == 0) {
      const int64_t L = p.n_e - s;  // level just computed
      for (int r = 0; r < p.n_rec; ++r) {
        const int64_t j = p.rec_node[r];
        if (j > 0 && j < p.M - 1 && j >= A && j <= B)
          w0[j - A] = w0[j - A] + p.gtr[static_cast<int64_t>(r) * p.gtr_ld + (L - 1)];
      }
    }
    __syncthreads();
    T* t = w0;
    w0 = w1;
    w1 = t;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_adj_finish(T* grad_fa, T* grad_fb, const T* gtr,
                                                   int64_t gtr_ld, const int64_t* rec_node,
                                                   int32_t n_rec, int64_t M, int64_t n_steps,
                                                   const double* lam_part, int32_t n_part,
                                                   double lam, double* grad_lam) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  // dJ/df: receivers on the Dirichlet nodes add their dJ/dtrace sample, in
  // receiver order (levels spread over the grid; the others are not read)
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t L = 1 + static_cast<int64_t>(blockIdx.x) * 256 + tid; L <= n_steps;
       L += stride) {
    T ga = grad_fa[L], gb = grad_fb[L];
    for (int r = 0; r < n_rec; ++r) {
      const int64_t j = rec_node[r];
      if (j == 0 || j == M - 1) {
        const T g = gtr[static_cast<int64_t>(r) * gtr_ld + (L - 1)];
        if (j == 0) ga = ga + g;
        if (j == M - 1) gb = gb + g;
      }
    }
    grad_fa[L] = ga;
    grad_fb[L] = gb;
  }
  // dJ/dlam: the tiles' partials summed by the first work-group in a fixed
  // order
  if (blockIdx.x != 0) return;
  double t = 0.0;
  for (int i = tid; i < n_part; i += 256) t += lam_part[i];
  red[tid] = t;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) *grad_lam = 2.0 * lam * red[0];
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* __restrict__ dst, T v, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride)
    dst[i] = v;
}

template <typename T>
hipError_t launch_adj_predict(const AdjPredictArgs<T>& a, int shmem_nodes, hipStream_t s) {
  if (a.N < 2) return hipSuccess;
  if (a.shat <= kMaxFusedSpan) {
    hipLaunchKernelGGL(k_adj_predict_frame<T>, dim3(2 * (a.N - 1), ny(a.ys)), dim3(64), 0, s,
                       a);
  } else {
    const size_t shm = static_cast<size_t>(2 * shmem_nodes) * sizeof(T);
    hipLaunchKernelGGL(k_adj_predict_lds<T>, dim3(2 * (a.N - 1), ny(a.ys)), dim3(64), shm, s,
                       a);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_update(const AdjUpdateArgs<T>& a, int threads, int per_thread,
                             bool general, bool fused, hipStream_t s) {
  return fused ? launch_adj_update_kind<T, true>(a, threads, per_thread, general, s)
               : launch_adj_update_kind<T, false>(a, threads, per_thread, general, s);
}

template <typename T>
hipError_t launch_adj_finish(T* grad_fa, T* grad_fb, const T* gtr, int64_t gtr_ld,
                             const int64_t* rec_node, int32_t n_rec, int64_t M,
                             int64_t n_steps, const double* lam_part, int32_t n_part,
                             double lam, double* grad_lam, hipStream_t s) {
  int64_t blocks = (n_steps + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
  hipLaunchKernelGGL(k_adj_finish<T>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                     grad_fa, grad_fb, gtr, gtr_ld, rec_node, n_rec, M, n_steps, lam_part,
                     n_part, lam, grad_lam);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* dst, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill<T>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, dst,
                     v, n);
  return hipGetLastError();
}

template hipError_t launch_adj_predict<float>(const AdjPredictArgs<float>&, int, hipStream_t);
template hipError_t launch_adj_predict<double>(const AdjPredictArgs<double>&, int,
                                               hipStream_t);
template hipError_t launch_adj_update<float>(const AdjUpdateArgs<float>&, int, int, bool,
                                             bool, hipStream_t);
template hipError_t launch_adj_update<double>(const AdjUpdateArgs<double>&, int, int, bool,
                                              bool, hipStream_t);
template hipError_t launch_adj_update_kind<float, false>(const AdjUpdateArgs<float>&, int,
                                                         int, bool, hipStream_t);
template hipError_t launch_adj_update_kind<double, false>(const AdjUpdateArgs<double>&, int,
                                                          int, bool, hipStream_t);
template hipError_t launch_adj_finish<float>(float*, float*, const float*, int64_t,
                                             const int64_t*, int32_t, int64_t, int64_t,
                                             const double*, int32_t, double, double*,
                                             hipStream_t);
template hipError_t launch_adj_finish<double>(double*, double*, const double*, int64_t,
                                              const int64_t*, int32_t, int64_t, int64_t,
                                              const double*, int32_t, double, double*,
                                              hipStream_t);
template hipError_t launch_fill<int32_t>(int32_t*, int32_t, int64_t, hipStream_t);
template hipError_t launch_fill<float>(float*, float, int64_t, hipStream_t);
template hipError_t launch_fill<double>(double*, double, int64_t, hipStream_t);

}  // namespace rswr

