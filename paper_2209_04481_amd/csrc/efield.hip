// The electric field of ideal MHD and the E-free state (Sections 2.2, 3.1).
//
// efield: E = -V x B at every cell centroid, projected on the spherical unit
// vectors there, with per-component maxima and volume-weighted sums of
// squares folded in a fixed order (no atomics: bitwise reproducible).
// efree: the velocity of every cell projected on its field direction, so that
// V x B = 0, with density, field, pressure and psi kept.
//
// Both stream the state once, so they are bound by HBM bandwidth.  The cells
// of one (panel, shell) layer are contiguous; the launch walks tiles of 256
// consecutive cells of one layer, so a block finds its layer with one scalar
// division per tile and every row load is coalesced.
#include "cfv_kernels.hpp"

namespace cfv {

static constexpr int kEB = 256;     // threads per block = cells per tile
static constexpr int kEGrid = 1024;  // blocks, and partials per statistic
static constexpr int kEStats = 9;    // 4 maxima, 4 weighted sums of squares, the volume

__device__ __forceinline__ double e_block_sum(double x, double* sh) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = x;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kEB / 64; ++w) r += sh[w];
  __syncthreads();
  return r;  // valid in thread 0
}

__device__ __forceinline__ double e_block_max(double x, double* sh) {
  for (int o = 32; o > 0; o >>= 1) x = ::fmax(x, __shfl_down(x, o, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = x;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kEB / 64; ++w) r = ::fmax(r, sh[w]);
  __syncthreads();
  return r;  // valid in thread 0
}

// part[q * kEGrid + block], q = 0..3: max |E_r|, |E_theta|, |E_phi|, |E|;
// q = 4..7: sum V E^2 of the same; q = 8: sum V.  E3 (optional): the field.
__global__ __launch_bounds__(kEB) void efield_kernel(DevGrid d, const double* __restrict__ U,
                                                     double* __restrict__ E3, double* __restrict__ part) {
  __shared__ double sh[kEB / 64];
  const int64_t nc = d.g.ncells;
  const int64_t plane = int64_t(d.g.N) * d.g.N;
  const int64_t nchunk = (plane + kEB - 1) / kEB;
  const int64_t ntiles = int64_t(6) * d.g.Nr * nchunk;
  double mx[4] = {0.0, 0.0, 0.0, 0.0}, ss[4] = {0.0, 0.0, 0.0, 0.0}, vs = 0.0;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t layer = t / nchunk;  // uniform over the block
    const int64_t col = (t - layer * nchunk) * kEB + threadIdx.x;
    if (col >= plane) continue;
    const int p = int(layer / d.g.Nr), k = int(layer - int64_t(p) * d.g.Nr);
    const int col32 = int(col);  // a column index of one panel: below N^2
    const int j = col32 / d.g.N, i = col32 - j * d.g.N;
    const int64_t c = layer * plane + col;
    const double rho = U[c];
    const V3 v = mk(U[nc + c] / rho, U[2 * nc + c] / rho, U[3 * nc + c] / rho);
    const V3 B = mk(U[4 * nc + c], U[5 * nc + c], U[6 * nc + c]);
    const V3 E = cross3(B, v);  // -V x B
    V3 rh, th, ph;
    const V3 xc = cell_centre(d.G, d.g, p, k, j, i);
    sph_basis(xc, rh, th, ph);
    const double e[4] = {dot3(E, rh), dot3(E, th), dot3(E, ph), norm3(E)};
    if (E3) {
      E3[c] = e[0];
      E3[nc + c] = e[1];
      E3[2 * nc + c] = e[2];
    }
    const double vol = cell_volume(d.G, d.g, p, k, j, i);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      mx[q] = ::fmax(mx[q], ::fabs(e[q]));
      ss[q] += vol * (e[q] * e[q]);
    }
    vs += vol;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double m = e_block_max(mx[q], sh);
    if (threadIdx.x == 0) part[q * kEGrid + blockIdx.x] = m;
    const double s = e_block_sum(ss[q], sh);
    if (threadIdx.x == 0) part[(4 + q) * kEGrid + blockIdx.x] = s;
  }
  const double s = e_block_sum(vs, sh);
  if (threadIdx.x == 0) part[8 * kEGrid + blockIdx.x] = s;
}

// stats[q] for q = 0..7 (one block each): the maxima, then sqrt(sum V E^2 / sum V)
__global__ __launch_bounds__(kEB) void efield_fold_kernel(const double* __restrict__ part, double* __restrict__ stats) {
  __shared__ double sh[kEB / 64];
  const int q = blockIdx.x;
  if (q < 4) {
    double m = 0.0;
    for (int b = threadIdx.x; b < kEGrid; b += kEB) m = ::fmax(m, part[q * kEGrid + b]);
    const double t = e_block_max(m, sh);
    if (threadIdx.x == 0) stats[q] = t;
    return;
  }
  double s = 0.0, v = 0.0;
  for (int b = threadIdx.x; b < kEGrid; b += kEB) {
    s += part[q * kEGrid + b];
    v += part[8 * kEGrid + b];
  }
  const double ts = e_block_sum(s, sh);
  const double tv = e_block_sum(v, sh);
  if (threadIdx.x == 0) stats[q] = ::sqrt(ts / tv);
}

// Uo = U with V replaced by (V . B / |B|^2) B where B != 0 (else copied); Uo may equal U.
__global__ __launch_bounds__(kEB) void efree_kernel(int64_t nc, double gamma, const double* U, double* Uo) {
  for (int64_t c = int64_t(blockIdx.x) * kEB + threadIdx.x; c < nc; c += int64_t(gridDim.x) * kEB) {
    double u[9], q[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) u[a] = U[a * nc + c];
    cons_to_prim(u, q, gamma);
    const double B2 = q[4] * q[4] + q[5] * q[5] + q[6] * q[6];
    if (B2 > 0.0) {  // else the cell is copied unchanged
      const double par = (q[1] * q[4] + q[2] * q[5] + q[3] * q[6]) / B2;
      q[1] = par * q[4];
      q[2] = par * q[5];
      q[3] = par * q[6];
      prim_to_cons(q, u, gamma);
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) Uo[a * nc + c] = u[a];
  }
}

int efield_partials() { return kEStats * kEGrid; }

hipError_t launch_efield(const DevGrid& d, const double* U, double* E3, double* stats8, double* part, hipStream_t s,
                         KernelTimer* t) {
  {
    TimedScope ts(t, "efield", s);
    hipLaunchKernelGGL(efield_kernel, dim3(kEGrid), dim3(kEB), 0, s, d, U, E3, part);
  }
  hipLaunchKernelGGL(efield_fold_kernel, dim3(8), dim3(kEB), 0, s, part, stats8);
  return hipGetLastError();
}

hipError_t launch_efree(int64_t nc, double gamma, const double* U, double* Uo, hipStream_t s, KernelTimer* t) {
  int64_t blocks = (nc + kEB - 1) / kEB;
  if (blocks > 65535) blocks = 65535;
  if (blocks < 1) blocks = 1;
  TimedScope ts(t, "efree", s);
  hipLaunchKernelGGL(efree_kernel, dim3(unsigned(blocks)), dim3(kEB), 0, s, nc, gamma, U, Uo);
  return hipGetLastError();
}

}  // namespace cfv
