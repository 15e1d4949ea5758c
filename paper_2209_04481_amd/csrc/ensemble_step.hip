// One backward-Euler pseudo-time step (Section 2.1) for every instance of an
// ensemble, in lockstep and entirely on the device: the residual and the JVPs
// are the ensemble march launches; the Krylov vectors, Gram-Schmidt
// coefficients, Givens rotations and the small least-squares solve of each
// instance stay in device memory, so a step needs no host synchronisation and
// can be captured in a graph.
//
// GMRES(m) from x = 0, modified Gram-Schmidt, no restart, as in cfv_solve.
// Vector kernels run on a (blocks, n) grid: blockIdx.y is the instance,
// each block strides over that instance's vector; reductions fold a fixed set
// of per-block partials in a fixed order (deterministic, no atomics).
#include "cfv_kernels.hpp"
#include "cfv_march.hpp"
#include "cfv_step.hpp"

namespace cfv {

hipError_t launch_fused_ensemble(const EnsembleLaunch& e, hipStream_t s, KernelTimer* t);

static constexpr int kSB = 256;  // threads per block

__device__ __forceinline__ double block_sum_step(double x, double* sh) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = x;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < kSB / 64; ++q) r += sh[q];
  __syncthreads();
  return r;  // valid in thread 0
}

// element range of this block within its instance's vector of length len
#define STEP_LOOP(len) for (int64_t e = int64_t(blockIdx.x) * kSB + threadIdx.x; e < (len); e += int64_t(gridDim.x) * kSB)

// Unew = -Unew (the right-hand side -R), and the partial sums of its squares
__global__ __launch_bounds__(kSB) void step_negate_norm_kernel(const StepVec* __restrict__ sv, double* __restrict__ part) {
  __shared__ double sh[kSB / 64];
  const StepVec& v = sv[blockIdx.y];
  const int64_t n9 = 9 * v.nc;
  double s = 0.0;
  STEP_LOOP(n9) {
    const double r = -gld(v.Unew, e);
    gst(v.Unew, e, r);
    s += r * r;
  }
  const double t = block_sum_step(s, sh);
  if (threadIdx.x == 0) part[int64_t(blockIdx.y) * gridDim.x + blockIdx.x] = t;
}

// partial sums of <w, V_i> (i >= 0) or of |w|^2 (i < 0)
__global__ __launch_bounds__(kSB) void step_dot_kernel(const StepVec* __restrict__ sv, int i, double* __restrict__ part) {
  __shared__ double sh[kSB / 64];
  const StepVec& v = sv[blockIdx.y];
  const int64_t n9 = 9 * v.nc;
  const double* a = i >= 0 ? v.V + int64_t(i) * n9 : v.w;
  const int64_t S = int64_t(gridDim.x) * kSB;
  int64_t e = int64_t(blockIdx.x) * kSB + threadIdx.x;
  double s = 0.0;
  for (; e + 3 * S < n9; e += 4 * S) {  // four entries' loads in flight, summed in entry order
    double av[4], wv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av[u] = gld(a, e + u * S);
      wv[u] = gld(v.w, e + u * S);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) s += av[u] * wv[u];
  }
  for (; e < n9; e += S) s += gld(a, e) * gld(v.w, e);
  const double t = block_sum_step(s, sh);
  if (threadIdx.x == 0) part[int64_t(blockIdx.y) * gridDim.x + blockIdx.x] = t;
}

// fold the nb partials of each instance into its scalar at sm[slot] (sqrt if asked)
__global__ __launch_bounds__(kSB) void step_fold_kernel(const StepVec* __restrict__ sv, const double* __restrict__ part,
                                                        int nb, int slot, int take_sqrt) {
  __shared__ double sh[kSB / 64];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += kSB) s += part[int64_t(blockIdx.x) * nb + b];
  const double t = block_sum_step(s, sh);
  if (threadIdx.x == 0) sv[blockIdx.x].sm[slot] = take_sqrt ? ::sqrt(t) : t;
}

// start of the step: g = (beta, 0, ...), H = 0, flags; V_0 = rhs / beta
__global__ void step_init_kernel(const StepVec* __restrict__ sv, int n, int m) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  double* sm = sv[q].sm;
  const StepLayout L(m);
  for (int a = 0; a < L.size; ++a)
    if (a != L.beta) sm[a] = 0.0;
  sm[L.g] = sm[L.beta];
  sm[L.kdone] = 0.0;
  sm[L.stop] = sm[L.beta] > 0.0 ? 0.0 : 1.0;
  // a non-finite residual: no step is taken (the solve stops at once) and
  // the instance's status word says why
  if (!(::fabs(sm[L.beta]) <= 1.7976931348623157e308)) atomicOr(sv[q].flag, 2u);
}

// dst = src / sm[slot] (zero when the scalar is zero); src: Unew (j < 0) or w
__global__ __launch_bounds__(kSB) void step_scale_kernel(const StepVec* __restrict__ sv, int j, int slot) {
  const StepVec& v = sv[blockIdx.y];
  const int64_t n9 = 9 * v.nc;
  const double den = v.sm[slot];
  const double* src = j < 0 ? v.Unew : v.w;
  double* dst = v.V + int64_t(j < 0 ? 0 : j + 1) * n9;
  const int64_t S = int64_t(gridDim.x) * kSB;
  int64_t e = int64_t(blockIdx.x) * kSB + threadIdx.x;
  for (; e + 3 * S < n9; e += 4 * S) {  // four entries per pass, loads before stores
    double xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) xv[u] = gld(src, e + u * S);
#pragma unroll
    for (int u = 0; u < 4; ++u) gst(dst, e + u * S, den != 0.0 ? xv[u] / den : 0.0);
  }
  for (; e < n9; e += S) gst(dst, e, den != 0.0 ? gld(src, e) / den : 0.0);
}

// z = V_j / diag (the Jacobi-preconditioned vector the JVP then reads)
__global__ __launch_bounds__(kSB) void step_precond_kernel(const StepVec* __restrict__ sv, int j) {
  const StepVec& v = sv[blockIdx.y];
  const int64_t n9 = 9 * v.nc;
  const double* x = v.V + int64_t(j) * n9;
  const int64_t S = int64_t(gridDim.x) * kSB;
  for (int64_t e = int64_t(blockIdx.x) * kSB + threadIdx.x; e < n9; e += S)
    gst(v.z, e, gld(x, e) / gld(v.diag, e % v.nc));
}

// w += diag o x with x = V_j, or z (the V/dt part of the operator)
__global__ __launch_bounds__(kSB) void step_add_diag_kernel(const StepVec* __restrict__ sv, int j, int use_z) {
  const StepVec& v = sv[blockIdx.y];
  const int64_t n9 = 9 * v.nc;
  const double* x = use_z ? v.z : v.V + int64_t(j) * n9;
  const int64_t S = int64_t(gridDim.x) * kSB;
  int64_t e = int64_t(blockIdx.x) * kSB + threadIdx.x;
  for (; e + 3 * S < n9; e += 4 * S) {  // four entries per pass, loads before stores
    double wv[4], dv[4], xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      wv[u] = gld(v.w, e + u * S);
      dv[u] = gld(v.diag, (e + u * S) % v.nc);
      xv[u] = gld(x, e + u * S);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) gst(v.w, e + u * S, wv[u] + dv[u] * xv[u]);
  }
  for (; e < n9; e += S) gst(v.w, e, gld(v.w, e) + gld(v.diag, e % v.nc) * gld(x, e));
}

// w -= sm[slot] V_i fused with the next projection: partial sums of the
// updated w times V_next (HasY) or times itself (the norm).  Four entries of
// the block's strided range per pass, loads before stores, summed in entry
// order (the same sums as one entry per pass).
template <bool HasY>
__global__ __launch_bounds__(kSB) void step_axpy_dot_kernel(const StepVec* __restrict__ sv, int i, int slot, int next,
                                                            double* __restrict__ part) {
  __shared__ double sh[kSB / 64];
  const StepVec& v = sv[blockIdx.y];
  const int64_t n9 = 9 * v.nc;
  const double h = v.sm[slot];
  const double* x = v.V + int64_t(i) * n9;
  const double* y = HasY ? v.V + int64_t(next) * n9 : nullptr;
  double* w = v.w;
  const int64_t S = int64_t(gridDim.x) * kSB;
  int64_t e = int64_t(blockIdx.x) * kSB + threadIdx.x;
  double s = 0.0;
  for (; e + 3 * S < n9; e += 4 * S) {
    double wv[4], xv[4], yv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      wv[u] = gld(w, e + u * S);
      xv[u] = gld(x, e + u * S);
      if (HasY) yv[u] = gld(y, e + u * S);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double wn = wv[u] - h * xv[u];
      gst(w, e + u * S, wn);
      s += (HasY ? yv[u] : wn) * wn;
    }
  }
  for (; e < n9; e += S) {
    const double wn = gld(w, e) - h * gld(x, e);
    gst(w, e, wn);
    s += (HasY ? gld(y, e) : wn) * wn;
  }
  const double t = block_sum_step(s, sh);
  if (threadIdx.x == 0) part[int64_t(blockIdx.y) * gridDim.x + blockIdx.x] = t;
}

// column j of H is in sm[hcol + 0..j+1]: rotate it, append the new rotation,
// update g and the relative-residual history (one thread per instance)
__global__ void step_givens_kernel(const StepVec* __restrict__ sv, int n, int m, int j, double* __restrict__ hist) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  double* sm = sv[q].sm;
  const StepLayout L(m);
  if (sm[L.stop] != 0.0) {  // converged exactly or broke down: repeat the last value
    if (hist) hist[int64_t(q) * m + j] = j > 0 ? hist[int64_t(q) * m + j - 1] : 0.0;
    return;
  }
  for (int i = 0; i <= j + 1; ++i) sm[L.H + i * m + j] = sm[L.hcol + i];
  const double hnext = sm[L.hcol + j + 1];
  for (int i = 0; i < j; ++i) {
    const double a = sm[L.H + i * m + j], b = sm[L.H + (i + 1) * m + j];
    const double c = sm[L.cs + i], s = sm[L.sn + i];
    sm[L.H + i * m + j] = c * a + s * b;
    sm[L.H + (i + 1) * m + j] = -s * a + c * b;
  }
  const double a = sm[L.H + j * m + j], b = sm[L.H + (j + 1) * m + j];
  const double den = ::hypot(a, b);
  const double c = a / den, s = b / den;
  sm[L.cs + j] = c;
  sm[L.sn + j] = s;
  sm[L.H + j * m + j] = den;
  sm[L.H + (j + 1) * m + j] = 0.0;
  const double gj = sm[L.g + j];
  sm[L.g + j + 1] = -s * gj;
  sm[L.g + j] = c * gj;
  if (hist) hist[int64_t(q) * m + j] = ::fabs(sm[L.g + j + 1]) / sm[L.beta];
  sm[L.kdone] = double(j + 1);
  if (!(hnext > 0.0)) sm[L.stop] = 1.0;
}

// y = H^-1 g over the kdone completed columns (one thread per instance)
__global__ void step_backsub_kernel(const StepVec* __restrict__ sv, int n, int m) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  double* sm = sv[q].sm;
  const StepLayout L(m);
  const int k = int(sm[L.kdone]);
  for (int i = 0; i < m; ++i) sm[L.y + i] = 0.0;
  for (int i = k - 1; i >= 0; --i) {
    double t = sm[L.g + i];
    for (int a = i + 1; a < k; ++a) t -= sm[L.H + i * m + a] * sm[L.y + a];
    sm[L.y + i] = t / sm[L.H + i * m + i];
  }
}

// Unew = U + sum_i y_i V_i (divided by diag with the Jacobi preconditioner)
__global__ __launch_bounds__(kSB) void step_update_kernel(const StepVec* __restrict__ sv, int m, int precond) {
  const StepVec& v = sv[blockIdx.y];
  const int64_t n9 = 9 * v.nc;
  const StepLayout L(m);
  const int k = int(v.sm[L.kdone]);
  STEP_LOOP(n9) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += gld(v.sm, L.y + i) * gld(v.V, int64_t(i) * n9 + e);
    if (precond) s = s / gld(v.diag, e % v.nc);
    gst(v.Unew, e, gld(v.U, e) + s);
  }
}

#undef STEP_LOOP

hipError_t launch_ensemble_step(const StepLaunch& L, hipStream_t s, KernelTimer* t) {
  const dim3 vgrid(unsigned(L.blocks), unsigned(L.n));
  const unsigned tgrid = unsigned((L.n + 63) / 64);
  const StepLayout Y(L.m);
  // residual of every instance into Unew, then -R, beta, V_0
  {
    TimedScope ts(t, "step_residual", s);
    if (hipError_t e = launch_fused_ensemble(L.res, s, nullptr)) return e;
  }
  for (int q = 0; q < L.n; ++q)
    if (hipError_t e = launch_local_dt(L.dev[q], L.Uh[q], L.cfl, L.diagh[q], L.Wh[q], s, nullptr)) return e;
  hipLaunchKernelGGL(step_negate_norm_kernel, vgrid, dim3(kSB), 0, s, L.sv, L.part);
  hipLaunchKernelGGL(step_fold_kernel, dim3(L.n), dim3(kSB), 0, s, L.sv, L.part, L.blocks, Y.beta, 1);
  hipLaunchKernelGGL(step_init_kernel, dim3(tgrid), dim3(64), 0, s, L.sv, L.n, L.m);
  hipLaunchKernelGGL(step_scale_kernel, vgrid, dim3(kSB), 0, s, L.sv, -1, Y.beta);
  for (int j = 0; j < L.m; ++j) {
    if (L.precond) hipLaunchKernelGGL(step_precond_kernel, vgrid, dim3(kSB), 0, s, L.sv, j);
    {
      TimedScope ts(t, "step_jvp", s);
      if (hipError_t e = launch_march_ensemble(L.jvp[j], true, s, nullptr)) return e;
    }
    TimedScope ts(t, "step_krylov", s);
    hipLaunchKernelGGL(step_add_diag_kernel, vgrid, dim3(kSB), 0, s, L.sv, j, L.precond);
    // modified Gram-Schmidt: h_0 = <w, V_0>, then each update fused with the
    // next projection (for i = j: the norm of w)
    hipLaunchKernelGGL(step_dot_kernel, vgrid, dim3(kSB), 0, s, L.sv, 0, L.part);
    hipLaunchKernelGGL(step_fold_kernel, dim3(L.n), dim3(kSB), 0, s, L.sv, L.part, L.blocks, Y.hcol, 0);
    for (int i = 0; i <= j; ++i) {
      if (i < j)
        hipLaunchKernelGGL(step_axpy_dot_kernel<true>, vgrid, dim3(kSB), 0, s, L.sv, i, Y.hcol + i, i + 1, L.part);
      else
        hipLaunchKernelGGL(step_axpy_dot_kernel<false>, vgrid, dim3(kSB), 0, s, L.sv, i, Y.hcol + i, -1, L.part);
      hipLaunchKernelGGL(step_fold_kernel, dim3(L.n), dim3(kSB), 0, s, L.sv, L.part, L.blocks, Y.hcol + i + 1,
                         i < j ? 0 : 1);
    }
    hipLaunchKernelGGL(step_scale_kernel, vgrid, dim3(kSB), 0, s, L.sv, j, Y.hcol + j + 1);
    hipLaunchKernelGGL(step_givens_kernel, dim3(tgrid), dim3(64), 0, s, L.sv, L.n, L.m, j, L.hist);
  }
  hipLaunchKernelGGL(step_backsub_kernel, dim3(tgrid), dim3(64), 0, s, L.sv, L.n, L.m);
  hipLaunchKernelGGL(step_update_kernel, vgrid, dim3(kSB), 0, s, L.sv, L.m, L.precond);
  return hipGetLastError();
}

}  // namespace cfv
