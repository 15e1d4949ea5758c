// Adjoint (vector-Jacobian product) of the residual: gU = J_U^T w and
// gbr = J_b^T w, as deterministic gather passes without atomics.
//
// The forward residual is R_c = sum_f (+-) F(q_L,f, q_R,f) - V_c S(U_c) with
// face states q = P + G.(x_f - x_cell), G = phi (.) g the limited least-squares
// gradient and P the primitives (ghost states from the boundary laws).
//
//   pass 1  forward gradient/limiter pass (primitives and limited gradients).
//   pass 2  per cell c: for each face, the flux adjoint for c's own side
//           (and the ghost side on boundary faces) with face weight
//           w_L - w_R; then the adjoint of c's reconstruction, limiter and
//           least-squares gradient.  Contributions that land on c itself go
//           to own[c]; those that land on face neighbour n go to out[c][f];
//           those that land on a ghost state are stored for pass 3 (each
//           ghost belongs to exactly one cell).
//   pass 3  per boundary column: the ghost-state adjoints of pass 2 back
//           through the boundary laws onto own[] of the boundary cells and
//           onto the B_r map.
//   pass 4  per cell n: Pb = own[n] + sum over the six neighbours c of
//           out[c][face of c that faces n]; gU = (dP/dU)^T Pb minus the
//           gravity source adjoint.
#include "cfv_vjp.hpp"

namespace cfv {

int64_t vjp_workspace_doubles(const Shape& g) { return vjp_workspace_size(g); }

// the adjoint windows that hold a boundary-layer cell, in order (out: room
// for all of them, or null to count)
int64_t adjoint_boundary_windows(const Shape& g, int64_t* out) {
  int64_t n = 0;
  for (int64_t b = 0; b * kVBlock < g.ncells; ++b)
    if (adjoint_window_has_boundary(g, b * kVBlock)) {
      if (out) out[n] = b;
      ++n;
    }
  return n;
}

// kBoundary false: every window, those holding a boundary-layer cell left
// out; true: the windows listed in bw (their windows, each once or more: a
// window's rows are written, not accumulated, so a repeat writes the same)
template <bool kBoundary>
__global__ __launch_bounds__(kVBlock) void adjoint_kernel(DevGrid, const double* __restrict__ w,
                                                          const double* __restrict__ W, const double* __restrict__ Q,
                                                          double* __restrict__ A, double* __restrict__ Gg,
                                                          const int64_t* __restrict__ bw) {
  __shared__ double lW[63 * kVBlock];  // primitives (9 rows), then the face states (54)
  __shared__ double lw[9 * kVBlock];
  const DevGrid& d = first_kernel_arg<DevGrid>();
  const int64_t nc = d.g.ncells;
  const int64_t c0 = (kBoundary ? gld(bw, int64_t(blockIdx.x)) : int64_t(blockIdx.x)) * kVBlock;
  if (!kBoundary && adjoint_window_has_boundary(d.g, c0)) return;  // the same in every lane
  const int64_t c = c0 + threadIdx.x;
  if (c < nc) {
    // every load of the window issued before the first LDS store (one memory
    // latency for the 72 rows, not one per batch of rows)
    double t[72];
#pragma unroll
    for (int r = 0; r < 9; ++r) t[r] = gld(W, r * nc + c);
#pragma unroll
    for (int r = 0; r < 54; ++r) t[9 + r] = gld(Q, r * nc + c);
#pragma unroll
    for (int r = 0; r < 9; ++r) t[63 + r] = gld(w, r * nc + c);
#pragma unroll
    for (int r = 0; r < 63; ++r) lW[r * kVBlock + threadIdx.x] = t[r];
#pragma unroll
    for (int r = 0; r < 9; ++r) lw[r * kVBlock + threadIdx.x] = t[63 + r];
  }
  __syncthreads();
  if (c < nc) adjoint_cell<kBoundary>(d, w, W, Q, A, Gg, c, lW, lw, c0);
}

// Per boundary column: the ghost states' adjoints through the boundary laws
// (ghost_fold_column in cfv_vjp.hpp).
__global__ __launch_bounds__(kVBlock) void ghost_fold_kernel(DevGrid, const double* __restrict__ W,
                                                             const double* __restrict__ Gg, double* __restrict__ A,
                                                             double* __restrict__ gbr) {
  const DevGrid& d = first_kernel_arg<DevGrid>();
  const int64_t col = int64_t(blockIdx.x) * kVBlock + threadIdx.x;
  if (col >= d.g.nb) return;
  ghost_fold_column(d, W, Gg, A, gbr, col);
}

__global__ __launch_bounds__(kVBlock) void gather_kernel(DevGrid d, const double* __restrict__ U,
                                                         const double* __restrict__ w, const double* __restrict__ A,
                                                         double* __restrict__ gU) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c < d.g.ncells) gather_cell(d, U, w, A, gU, c);
}

hipError_t launch_vjp(const DevGrid& d, const double* U, const double* w, double* gU, double* gbr, double* W,
                      double* A, MarchArgs* slot, int kc, const int64_t* bw, int64_t nbw, hipStream_t s,
                      KernelTimer* t) {
  const int64_t nc = d.g.ncells;
  const dim3 grid(unsigned((nc + kVBlock - 1) / kVBlock));
  // pass 1: the forward gradient march writes the primitives (rows 0..8 of
  // W) and, instead of the limited gradients, the face states they give
  // (the workspace's last 54 rows)
  double* Q = A + int64_t(63) * nc;
  double* Gg = A + int64_t(63 + 54) * nc;
  MarchArgs fa{d, U, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, W, Q};
  hipError_t e = launch_march_grad(fa, slot, kc, s, t);
  if (e != hipSuccess) return e;
  {
    // interior windows, then those with boundary-layer cells (bw[nbw])
    TimedScope ts(t, "adjoint", s);
    hipLaunchKernelGGL(adjoint_kernel<false>, grid, dim3(kVBlock), 0, s, d, w, W, Q, A, Gg, bw);
    if (nbw > 0) hipLaunchKernelGGL(adjoint_kernel<true>, dim3(unsigned(nbw)), dim3(kVBlock), 0, s, d, w, W, Q, A, Gg, bw);
  }
  {
    TimedScope ts(t, "adjoint_ghosts", s);
    hipLaunchKernelGGL(ghost_fold_kernel, dim3(unsigned((d.g.nb + kVBlock - 1) / kVBlock)), dim3(kVBlock), 0, s, d, W,
                       Gg, A, gbr);
  }
  {
    TimedScope ts(t, "adjoint_gather", s);
    hipLaunchKernelGGL(gather_kernel, grid, dim3(kVBlock), 0, s, d, U, w, A, gU);
  }
  return hipGetLastError();
}

}  // namespace cfv
