// The Eq. 2 convergence monitor of the pseudo-time march on the physical
// quantities: per primitive variable (rho, V, B, p, psi), the 2-norm over the
// cells of the change between two states, sqrt(sum_c (a_c^t - a_c^{t+1})^2).
// One streaming pass over both states (144 B per cell), then a fixed-order
// fold of per-block partials (deterministic, no atomics).
#include "cfv_kernels.hpp"

namespace cfv {

static constexpr int kMB = 256;
static constexpr int kMGrid = 1024;

__device__ __forceinline__ double m_block_sum(double x, double* sh) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = x;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kMB / 64; ++w) r += sh[w];
  __syncthreads();
  return r;  // valid in thread 0
}

// part[v * kMGrid + block] = sum over the block's cells of (P_v(a) - P_v(b))^2
__global__ __launch_bounds__(kMB) void prim_delta_partials(int64_t nc, double gamma, const double* __restrict__ a,
                                                           const double* __restrict__ b, double* __restrict__ part) {
  __shared__ double sh[kMB / 64];
  double acc[9];
#pragma unroll
  for (int v = 0; v < 9; ++v) acc[v] = 0.0;
  for (int64_t c = int64_t(blockIdx.x) * kMB + threadIdx.x; c < nc; c += int64_t(kMGrid) * kMB) {
    double ua[9], ub[9], qa[9], qb[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) {
      ua[v] = a[v * nc + c];
      ub[v] = b[v * nc + c];
    }
    cons_to_prim(ua, qa, gamma);
    cons_to_prim(ub, qb, gamma);
#pragma unroll
    for (int v = 0; v < 9; ++v) {
      const double d = qa[v] - qb[v];
      acc[v] += d * d;
    }
  }
#pragma unroll
  for (int v = 0; v < 9; ++v) {
    const double t = m_block_sum(acc[v], sh);
    if (threadIdx.x == 0) part[v * kMGrid + blockIdx.x] = t;
  }
}

// out9[v] = sqrt of the sum of variable v's partials (one block per variable)
__global__ __launch_bounds__(kMB) void prim_delta_fold(const double* __restrict__ part, double* __restrict__ out9) {
  __shared__ double sh[kMB / 64];
  const int v = blockIdx.x;
  double s = 0.0;
  for (int q = threadIdx.x; q < kMGrid; q += kMB) s += part[v * kMGrid + q];
  const double t = m_block_sum(s, sh);
  if (threadIdx.x == 0) out9[v] = ::sqrt(t);
}

int monitor_partials() { return 9 * kMGrid; }

hipError_t launch_prim_delta_norms(int64_t nc, double gamma, const double* a, const double* b, double* out9,
                                   double* part, hipStream_t s, KernelTimer* t) {
  {
    TimedScope ts(t, "monitor", s);
    hipLaunchKernelGGL(prim_delta_partials, dim3(kMGrid), dim3(kMB), 0, s, nc, gamma, a, b, part);
  }
  hipLaunchKernelGGL(prim_delta_fold, dim3(9), dim3(kMB), 0, s, part, out9);
  return hipGetLastError();
}

}  // namespace cfv
