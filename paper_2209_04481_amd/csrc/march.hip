// Tiled radial-march kernels for the residual and its forward derivative.
//
// A workgroup owns a 16 x 16 tile of columns (i, j) of one panel and a chunk
// of radial layers, and marches upward in k:
//
//  grad pass  per layer: each thread converts its cell to primitives once and
//             publishes them in LDS; the least-squares gradient and the
//             Barth-Jespersen factor then read in-tile neighbours from LDS,
//             radial neighbours from registers (the march keeps layers k-1,
//             k, k+1), and only tile-edge neighbours from global memory.
//             Output: the limited gradient (27 values per cell).
//  flux pass  per layer: each thread reconstructs its six face states; the
//             west and south states go to LDS, so every angular face inside
//             the tile is evaluated once, by its east/north cell; the radial
//             face between k-1 and k is evaluated once from the state carried
//             in registers.  Face fluxes are exchanged through LDS and summed
//             with the sign of the side (canonical owner orientation).
//
// Both passes are written as barrier-separated phase functions over a
// per-thread state, so the same code also runs under a host emulation.
#include "cfv_kernels.hpp"
#include "cfv_march.hpp"

namespace cfv {

// --------------------------------------------------------------- device glue
template <class T>
__global__ __launch_bounds__(kNT) void grad_march_kernel(MarchArgs a) {
  __shared__ double lds[GradWG<T>::kLds];
  TileMap tm;
  if (!tile_of(a.d.g, blockIdx.x, gridDim.x, tm)) return;
  const int t = threadIdx.x;
  GState<T> st;
  GradWG<T>::init(a, tm, st, t, lds);
  for (int k = tm.k0; k < tm.k1; ++k) {
    GradWG<T>::publish(a, tm, st, t, k, lds);
    __syncthreads();
    GradWG<T>::compute(a, tm, st, t, k, lds);
    __syncthreads();
  }
}

template <class T>
__global__ __launch_bounds__(kNT) void flux_march_kernel(MarchArgs a) {
  __shared__ double lds[FluxWG<T>::kLds];
  TileMap tm;
  if (!tile_of(a.d.g, blockIdx.x, gridDim.x, tm)) return;
  const int t = threadIdx.x;
  FState<T> st;
  FluxWG<T>::init(a, tm, st, t);
  for (int k = tm.k0; k < tm.k1; ++k) {
    FluxWG<T>::states(a, tm, st, t, k, lds);
    __syncthreads();
    FluxWG<T>::faces(a, tm, st, t, k, lds);
    __syncthreads();
    FluxWG<T>::accumulate(a, tm, st, t, k, lds);
    __syncthreads();
  }
  FluxWG<T>::finish(a, tm, st, t);
}

hipError_t launch_march(const MarchArgs& a, bool dual, hipStream_t s, KernelTimer* t) {
  const unsigned nb = unsigned(march_blocks(a.d.g));
  if (dual) {
    {
      TimedScope ts(t, "grad_march_jvp", s);
      hipLaunchKernelGGL((grad_march_kernel<Dual>), dim3(nb), dim3(kNT), 0, s, a);
    }
    TimedScope ts(t, "flux_march_jvp", s);
    hipLaunchKernelGGL((flux_march_kernel<Dual>), dim3(nb), dim3(kNT), 0, s, a);
  } else {
    {
      TimedScope ts(t, "grad_march", s);
      hipLaunchKernelGGL((grad_march_kernel<double>), dim3(nb), dim3(kNT), 0, s, a);
    }
    TimedScope ts(t, "flux_march", s);
    hipLaunchKernelGGL((flux_march_kernel<double>), dim3(nb), dim3(kNT), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace cfv
