// Deterministic reductions and vector updates for the pseudo-time solver:
// per-variable norms of the Eq. 2 monitor, batched dot products for the
// Gram-Schmidt step of GMRES, and y = a x + b y.
//
// Two stages with a fixed launch shape: each block folds a fixed strided
// subset in a fixed order and writes one partial; one block then folds the
// partials in order.  No atomics, so results are bitwise reproducible.
#include <hip/hip_runtime.h>
#include <cstdint>
#include <mutex>

namespace cfv {

static constexpr int kRBlock = 256;
static constexpr int kRGrid = 1024;  // partials per reduction

template <int B>
__device__ __forceinline__ double block_sum(double x, double* sh) {
  // wavefront reduction then across the block's wavefronts
  for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = x;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < B / 64; ++w) r += sh[w];
  __syncthreads();
  return r;  // valid in thread 0
}

template <int B>
__device__ __forceinline__ double block_max(double x, double* sh) {
  for (int o = 32; o > 0; o >>= 1) x = ::fmax(x, __shfl_down(x, o, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = x;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < B / 64; ++w) r = ::fmax(r, sh[w]);
  __syncthreads();
  return r;  // valid in thread 0
}

// partial[v*kRGrid + block] = max over the block's entries of |a_v| (nvar vectors of length n)
__global__ __launch_bounds__(kRBlock) void absmax_partials(int64_t n, int nvar, const double* __restrict__ a,
                                                          double* __restrict__ part) {
  __shared__ double sh[kRBlock / 64];
  for (int v = 0; v < nvar; ++v) {
    double m = 0.0;
    for (int64_t c = int64_t(blockIdx.x) * kRBlock + threadIdx.x; c < n; c += int64_t(kRGrid) * kRBlock)
      m = ::fmax(m, ::fabs(a[v * n + c]));
    double t = block_max<kRBlock>(m, sh);
    if (threadIdx.x == 0) part[v * kRGrid + blockIdx.x] = t;
  }
}

// partial[block] = max over entries of |x| / (|u| + s_v) over nvar vectors of
// length n, with a per-vector floor s_v (device array); s_v <= 0 drops vector v.
__global__ __launch_bounds__(kRBlock) void ratio_partials(int64_t n, int nvar, const double* __restrict__ x,
                                                         const double* __restrict__ u, const double* __restrict__ sv,
                                                         double* __restrict__ part) {
  __shared__ double sh[kRBlock / 64];
  double m = 0.0;
  for (int v = 0; v < nvar; ++v) {
    const double s = sv[v];
    if (!(s > 0.0)) continue;
    for (int64_t c = int64_t(blockIdx.x) * kRBlock + threadIdx.x; c < n; c += int64_t(kRGrid) * kRBlock)
      m = ::fmax(m, ::fabs(x[v * n + c]) / (::fabs(u[v * n + c]) + s));
  }
  double t = block_max<kRBlock>(m, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// out[v] = max of the partials of vector v (one block per v)
__global__ __launch_bounds__(kRBlock) void fold_max(const double* __restrict__ part, int nvec,
                                                   double* __restrict__ out) {
  __shared__ double sh[kRBlock / 64];
  const int v = blockIdx.x;
  if (v >= nvec) return;
  double m = 0.0;
  for (int b = threadIdx.x; b < kRGrid; b += kRBlock) m = ::fmax(m, part[v * kRGrid + b]);
  double t = block_max<kRBlock>(m, sh);
  if (threadIdx.x == 0) out[v] = t;
}

// partial[v*kRGrid + block] = sum over the block's cells of (a - b)^2 for
// variable v (HasB) or of a^2; four cells' loads in flight per pass, summed in
// cell order
template <bool HasB>
__global__ __launch_bounds__(kRBlock) void sq_partials(int64_t nc, const double* __restrict__ a,
                                                      const double* __restrict__ b, double* __restrict__ part) {
  __shared__ double sh[kRBlock / 64];
  const int64_t S = int64_t(kRGrid) * kRBlock;
  for (int v = 0; v < 9; ++v) {
    const double* av = a + v * nc;
    const double* bv = HasB ? b + v * nc : nullptr;
    double s = 0.0;
    int64_t c = int64_t(blockIdx.x) * kRBlock + threadIdx.x;
    for (; c + 3 * S < nc; c += 4 * S) {
      double x[4], y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        x[u] = av[c + u * S];
        y[u] = HasB ? bv[c + u * S] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double d = x[u] - y[u];
        s += d * d;
      }
    }
    for (; c < nc; c += S) {
      const double d = av[c] - (HasB ? bv[c] : 0.0);
      s += d * d;
    }
    double t = block_sum<kRBlock>(s, sh);
    if (threadIdx.x == 0) part[v * kRGrid + blockIdx.x] = t;
  }
}

// out[v] = (sqrt?) of the sum of partials of variable v (one block per v)
__global__ __launch_bounds__(kRBlock) void fold_partials(const double* __restrict__ part, int nvec,
                                                        double* __restrict__ out, int take_sqrt) {
  __shared__ double sh[kRBlock / 64];
  const int v = blockIdx.x;
  if (v >= nvec) return;
  double s = 0.0;
  for (int b = threadIdx.x; b < kRGrid; b += kRBlock) s += part[v * kRGrid + b];
  double t = block_sum<kRBlock>(s, sh);
  if (threadIdx.x == 0) out[v] = take_sqrt ? ::sqrt(t) : t;
}

// partial[i*kRGrid + block] = sum over the block's entries of V_i . w
__global__ __launch_bounds__(kRBlock) void dot_partials(int64_t n, const double* __restrict__ V, int k,
                                                       const double* __restrict__ w, double* __restrict__ part) {
  __shared__ double sh[kRBlock / 64];
  const int64_t S = int64_t(kRGrid) * kRBlock;
  for (int q = 0; q < k; ++q) {
    const double* x = V + int64_t(q) * n;
    double s = 0.0;
    int64_t c = int64_t(blockIdx.x) * kRBlock + threadIdx.x;
    for (; c + 3 * S < n; c += 4 * S) {  // four entries' loads in flight, summed in entry order
      double xv[4], wv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        xv[u] = x[c + u * S];
        wv[u] = w[c + u * S];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) s += xv[u] * wv[u];
    }
    for (; c < n; c += S) s += x[c] * w[c];
    double t = block_sum<kRBlock>(s, sh);
    if (threadIdx.x == 0) part[q * kRGrid + blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kRBlock) void axpby_kernel(int64_t n, double a, const double* __restrict__ x, double b,
                                                       double* __restrict__ y) {
  for (int64_t c = int64_t(blockIdx.x) * kRBlock + threadIdx.x; c < n; c += int64_t(gridDim.x) * kRBlock)
    y[c] = a * x[c] + b * y[c];
}

// One modified Gram-Schmidt update fused with the next projection:
// w -= (*coef) x, and part[block] = sum over the block's entries of the
// updated w times y (HasY) or times itself (the norm).  The entries of a
// block are those of dot_partials and are summed in the same order; each pass
// of the main loop takes four of them with all loads issued before the first
// store, so a wavefront keeps four times the bytes in flight.
template <bool HasY>
__global__ __launch_bounds__(kRBlock) void axpy_dot_partials(int64_t n, const double* __restrict__ coef,
                                                             const double* __restrict__ x, double* __restrict__ w,
                                                             const double* __restrict__ y, double* __restrict__ part) {
  __shared__ double sh[kRBlock / 64];
  const double a = -coef[0];
  const int64_t S = int64_t(kRGrid) * kRBlock;
  int64_t c = int64_t(blockIdx.x) * kRBlock + threadIdx.x;
  double s = 0.0;
  for (; c + 3 * S < n; c += 4 * S) {
    double wv[4], xv[4], yv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      wv[u] = w[c + u * S];
      xv[u] = x[c + u * S];
      if (HasY) yv[u] = y[c + u * S];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double wn = wv[u] + a * xv[u];
      w[c + u * S] = wn;
      s += (HasY ? yv[u] : wn) * wn;
    }
  }
  for (; c < n; c += S) {
    const double wn = w[c] + a * x[c];
    w[c] = wn;
    s += (HasY ? y[c] : wn) * wn;
  }
  const double t = block_sum<kRBlock>(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// y = x / (*den)
__global__ __launch_bounds__(kRBlock) void div_dev_kernel(int64_t n, const double* __restrict__ den,
                                                          const double* __restrict__ x, double* __restrict__ y) {
  const double d = den[0];
  for (int64_t c = int64_t(blockIdx.x) * kRBlock + threadIdx.x; c < n; c += int64_t(gridDim.x) * kRBlock)
    y[c] = x[c] / d;
}

// w[v*nc + c] += diag[c] * x[v*nc + c]
__global__ __launch_bounds__(kRBlock) void add_diag_kernel(int64_t nc, const double* __restrict__ diag,
                                                           const double* __restrict__ x, double* __restrict__ w) {
  const int64_t n = 9 * nc;
  for (int64_t e = int64_t(blockIdx.x) * kRBlock + threadIdx.x; e < n; e += int64_t(gridDim.x) * kRBlock)
    w[e] += diag[e % nc] * x[e];
}

// y[v*nc + c] = x[v*nc + c] / diag[c] (the Jacobi preconditioner's inverse)
__global__ __launch_bounds__(kRBlock) void div_diag_kernel(int64_t nc, const double* __restrict__ diag,
                                                           const double* __restrict__ x, double* __restrict__ y) {
  const int64_t n = 9 * nc;
  for (int64_t e = int64_t(blockIdx.x) * kRBlock + threadIdx.x; e < n; e += int64_t(gridDim.x) * kRBlock)
    y[e] = x[e] / diag[e % nc];
}

// x = sum_i y[i] V_i over k vectors of length n (coefficients on the device)
__global__ __launch_bounds__(kRBlock) void lincomb_kernel(int64_t n, int k, const double* __restrict__ y,
                                                          const double* __restrict__ V, double* __restrict__ x) {
  for (int64_t c = int64_t(blockIdx.x) * kRBlock + threadIdx.x; c < n; c += int64_t(gridDim.x) * kRBlock) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += y[i] * V[int64_t(i) * n + c];
    x[c] = s;
  }
}

static unsigned stream_blocks(int64_t n) {
  int64_t b = (n + kRBlock - 1) / kRBlock;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return unsigned(b);
}

hipError_t launch_div_dev(int64_t n, const double* den, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(div_dev_kernel, dim3(stream_blocks(n)), dim3(kRBlock), 0, s, n, den, x, y);
  return hipGetLastError();
}

hipError_t launch_add_diag(int64_t nc, const double* diag, const double* x, double* w, hipStream_t s) {
  hipLaunchKernelGGL(add_diag_kernel, dim3(stream_blocks(9 * nc)), dim3(kRBlock), 0, s, nc, diag, x, w);
  return hipGetLastError();
}

hipError_t launch_div_diag(int64_t nc, const double* diag, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(div_diag_kernel, dim3(stream_blocks(9 * nc)), dim3(kRBlock), 0, s, nc, diag, x, y);
  return hipGetLastError();
}

hipError_t launch_lincomb(int64_t n, int k, const double* y, const double* V, double* x, hipStream_t s) {
  hipLaunchKernelGGL(lincomb_kernel, dim3(stream_blocks(n)), dim3(kRBlock), 0, s, n, k, y, V, x);
  return hipGetLastError();
}

int reduce_partials_per_vector() { return kRGrid; }

hipError_t launch_absmax(int64_t n, int nvar, const double* a, double* out, double* part, hipStream_t s) {
  hipLaunchKernelGGL(absmax_partials, dim3(kRGrid), dim3(kRBlock), 0, s, n, nvar, a, part);
  hipLaunchKernelGGL(fold_max, dim3(nvar), dim3(kRBlock), 0, s, part, nvar, out);
  return hipGetLastError();
}

hipError_t launch_ratio_max(int64_t n, int nvar, const double* x, const double* u, const double* sv, double* out,
                            double* part, hipStream_t s) {
  hipLaunchKernelGGL(ratio_partials, dim3(kRGrid), dim3(kRBlock), 0, s, n, nvar, x, u, sv, part);
  hipLaunchKernelGGL(fold_max, dim3(1), dim3(kRBlock), 0, s, part, 1, out);
  return hipGetLastError();
}

hipError_t launch_norms(int64_t nc, const double* a, const double* b, double* out9, double* part, hipStream_t s) {
  if (b)
    hipLaunchKernelGGL(sq_partials<true>, dim3(kRGrid), dim3(kRBlock), 0, s, nc, a, b, part);
  else
    hipLaunchKernelGGL(sq_partials<false>, dim3(kRGrid), dim3(kRBlock), 0, s, nc, a, b, part);
  hipLaunchKernelGGL(fold_partials, dim3(9), dim3(kRBlock), 0, s, part, 9, out9, 1);
  return hipGetLastError();
}

hipError_t launch_dots(int64_t n, const double* V, int k, const double* w, double* out, double* part, hipStream_t s) {
  hipLaunchKernelGGL(dot_partials, dim3(kRGrid), dim3(kRBlock), 0, s, n, V, k, w, part);
  hipLaunchKernelGGL(fold_partials, dim3(k), dim3(kRBlock), 0, s, part, k, out, 0);
  return hipGetLastError();
}

// ------------------------------------------------ dots without allocation
// The partial sums of the allocation-free dot products live in this
// file-scope device array (each device holds its own copy until the process
// ends).  Host code never uses the array's name as an address: its device
// address is taken once per device, with that device current, and the
// kernels get that pointer.  Calls on one device share the array, so calls
// that overlap on one device race; every partial a call reads is written by
// the same call first (nothing needs clearing).
constexpr int kNoAllocMaxVectors = 32;
__device__ __align__(256) double scratch[kNoAllocMaxVectors * kRGrid];

int dots_noalloc_max_vectors() { return kNoAllocMaxVectors; }

static hipError_t scratch_on_current_device(double** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    double* p = nullptr;
    e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

// the kernels of launch_dots with the partials in the device's static array
// (the caller has checked 1 <= k <= kNoAllocMaxVectors)
hipError_t launch_dots_noalloc(int64_t n, const double* V, int k, const double* w, double* out, hipStream_t s) {
  double* part = nullptr;
  const hipError_t e = scratch_on_current_device(&part);
  if (e != hipSuccess) return e;
  return launch_dots(n, V, k, w, out, part, s);
}

hipError_t launch_axpy_dot(int64_t n, const double* coef, const double* x, double* w, const double* y, double* out,
                           double* part, hipStream_t s) {
  if (y)
    hipLaunchKernelGGL(axpy_dot_partials<true>, dim3(kRGrid), dim3(kRBlock), 0, s, n, coef, x, w, y, part);
  else
    hipLaunchKernelGGL(axpy_dot_partials<false>, dim3(kRGrid), dim3(kRBlock), 0, s, n, coef, x, w, y, part);
  hipLaunchKernelGGL(fold_partials, dim3(1), dim3(kRBlock), 0, s, part, 1, out, y ? 0 : 1);
  return hipGetLastError();
}

hipError_t launch_norm2(int64_t n, const double* x, double* out, double* part, hipStream_t s) {
  hipLaunchKernelGGL(dot_partials, dim3(kRGrid), dim3(kRBlock), 0, s, n, x, 1, x, part);
  hipLaunchKernelGGL(fold_partials, dim3(1), dim3(kRBlock), 0, s, part, 1, out, 1);
  return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  int64_t blocks = (n + kRBlock - 1) / kRBlock;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(axpby_kernel, dim3(unsigned(blocks)), dim3(kRBlock), 0, s, n, a, x, b, y);
  return hipGetLastError();
}

}  // namespace cfv
