// Tiled two-pass radial-march kernels: the forward derivative (JVP, T =
// Dual) and the VJP's forward pass (T = double, face states written); the
// residual itself runs as one fused pass (fused.hip).
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
// per-thread state, so the same code also runs under a host emulation.  A
// chunk enters and leaves through warm-up and cool-down iterations of the
// same phases, so the outputs do not depend on the chunk length.
#include "cfv_kernels.hpp"
#include "cfv_march.hpp"

namespace cfv {

// --------------------------------------------------------------- device glue
// One (tile, chunk) of each pass; the single-instance kernels run one per
// workgroup, the ensemble kernels (ensemble.hip) loop over a queue of them.
template <class T, bool Faces = false>
__device__ __forceinline__ void grad_march_tile(const MarchArgs& a0, const TileMap& tm, double* lds) {
  const int t = threadIdx.x;
  GState<T> st;
  GradWG<T>::init(a0, tm, st, t, lds);
  for (int k = GradWG<T>::first_layer(tm); k < tm.k1; ++k) {
    const MarchArgs& a = per_layer(a0);
    // (the second wavefront also fills the plane's ring of out-of-tile
    // neighbours: in the dual pass inside publish)
    GradWG<T>::publish(a, tm, st, t, k, lds);
    if (k < tm.k0) continue;  // warm-up: registers only
    if (t >= kNT / 4 && t < kNT / 2) GradWG<T>::ring_late(a, tm, st, t - kNT / 4, k, lds);
    __syncthreads();
    GradWG<T>::template compute<Faces>(a, tm, st, t, k, lds);
    // the plane is written again by the next layer (a second plane to drop
    // this barrier made both gradient passes slower: more LDS per workgroup)
    __syncthreads();
    // the dual pass's staged tile-edge states, written again only after the
    // next layer's first barrier
    GradWG<T>::flush_edges(a, tm, t, k, lds);
  }
}

template <class T>
__device__ __forceinline__ void flux_march_tile(const MarchArgs& a0, const TileMap& tm, double* lds) {
  const int t = threadIdx.x;
  FState<T> st;
  FluxWG<T>::init(a0, tm, st, t);
  const int kl = FluxWG<T>::last_layer(a0.d.g, tm);
  for (int k = FluxWG<T>::first_layer(tm); k <= kl; ++k) {
    const MarchArgs& a = per_layer(a0);
    // (the second wavefront also loads the ring of out-of-tile neighbour
    // states)
    FluxWG<T>::states(a, tm, st, t, k, lds);
    if (k < tm.k0 || k >= tm.k1) continue;  // warm-up or cool-down: registers only
    __syncthreads();
    FluxWG<T>::faces(a, tm, st, t, k, lds);
    __syncthreads();
    // no barrier after it: the next layer's states and ring slots overwrite
    // buffers that only the face phase (before the barrier above) reads
    FluxWG<T>::accumulate(a, tm, st, t, k, lds);
  }
  FluxWG<T>::finish(a0, tm, st, t);
}

// ----------------------------------------------------------------- ensemble
__global__ void reset_counters_kernel(unsigned* c) {
  if (threadIdx.x < 2) c[threadIdx.x] = 0u;
}

// copies its by-value descriptor into device memory (the single-instance
// launch is the one-instance ensemble, whose descriptor lives in a slot)
__global__ void put_args_kernel(MarchArgs, MarchArgs* __restrict__ dst) {
  static_assert(sizeof(MarchArgs) % 8 == 0, "descriptor copied in 8-byte words");
  constexpr int kW = int(sizeof(MarchArgs) / 8);
  const uint64_t* src = (const uint64_t*)&first_kernel_arg<MarchArgs>();
  uint64_t* d = reinterpret_cast<uint64_t*>(dst);
  for (int q = threadIdx.x; q < kW; q += blockDim.x) d[q] = src[q];
}

// next item of this workgroup: static (XCD-aware strided) or from the queue
__device__ __forceinline__ int64_t next_item(const EnsembleLaunch& e, int64_t step, unsigned* counter, int* slot) {
  if (e.queue) {
    __syncthreads();  // every thread has read the previous slot
    if (threadIdx.x == 0) *slot = int(atomicAdd(counter, 1u));
    __syncthreads();
    return *slot;
  }
  // workgroup b sits on XCD b % 8 as the (b / 8)-th of Q = blocks / 8; the
  // XCD's workgroups share a contiguous eighth of the queue
  const int64_t Q = e.blocks / 8, per = (e.total + 7) / 8;
  const int64_t x = blockIdx.x % 8, r = blockIdx.x / 8;
  const int64_t w = r + step * Q, idx = x * per + w;
  return w < per && idx < e.total ? idx : e.total;
}

// the item index is the same in every lane: say so, so that descriptor and
// table reads become scalar loads
__device__ __forceinline__ int64_t uniform(int64_t v) {
  const uint64_t u = uint64_t(v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(u));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(u >> 32));
  return int64_t((uint64_t(hi) << 32) | lo);
}

__device__ __forceinline__ int find_instance(const int64_t* __restrict__ off, int n, int64_t w) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= w) lo = mid; else hi = mid;
  }
  return lo;
}

// Wavefronts per SIMD each pass is compiled for (register budget 512 / n per
// lane; the LDS of n workgroups must fit in 160 KB).  Measured on the 13.3M-
// cell shell: the residual passes run faster at 2 than at 1 despite a few
// hundred bytes of spills (the flux pass 3.56 against 3.92 ms), and slower
// at 3 or 4; the JVP gradient pass is slower at 2 (4.33 against 3.58 ms) and
// the JVP flux pass needs 158 KB of LDS, so both JVP passes stay at 1.
template <class T, bool Flux>
struct MarchOccupancy {
  static constexpr int value = sizeof(T) == sizeof(double) ? 2 : 1;
};

template <class T, bool Flux, bool Faces = false>
__global__ __launch_bounds__(kNT, (MarchOccupancy<T, Flux>::value)) void march_ensemble_kernel(EnsembleLaunch e) {
  constexpr int kL = Flux ? FluxWG<T>::kLds : GradWG<T>::kLds;
  __shared__ double lds[kL];
  __shared__ int slot;
  unsigned* counter = e.counters + (Flux ? 1 : 0);
  for (int64_t step = 0;; ++step) {
    const int64_t q = uniform(next_item(e, step, counter, &slot));
    if (q >= e.total) break;
    const int64_t w = e.perm ? uniform(e.perm[q]) : q;
    const int inst = e.n > 1 ? int(uniform(find_instance(e.item_off, e.n, w))) : 0;
    const MarchArgs& a = constant_args(e.args + inst);
    TileMap tm;
    tile_of_logical(a.d.g, e.n > 1 ? w - e.item_off[inst] : w, tm, e.kc);
    __syncthreads();  // the previous item's LDS reads are done
    if (Flux)
      flux_march_tile<T>(a, tm, lds);
    else
      grad_march_tile<T, Faces>(a, tm, lds);
  }
}

hipError_t launch_fused_ensemble(const EnsembleLaunch& e, hipStream_t s, KernelTimer* t);
hipError_t launch_fused(const MarchArgs& a, MarchArgs* slot, int kc, hipStream_t s, KernelTimer* t);

// dual: the JVP's two passes; otherwise the fused residual march, and e must
// then describe its items (fused_items per instance, chunks of e.kc layers)
hipError_t launch_march_ensemble(const EnsembleLaunch& e, bool dual, hipStream_t s, KernelTimer* t) {
  if (e.total <= 0) return hipSuccess;
  if (!dual) return launch_fused_ensemble(e, s, t);
  if (e.queue) hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, s, e.counters);
  {
    TimedScope ts(t, "grad_march_ens_jvp", s);
    hipLaunchKernelGGL((march_ensemble_kernel<Dual, false>), dim3(e.blocks), dim3(kNT), 0, s, e);
  }
  TimedScope ts(t, "flux_march_ens_jvp", s);
  hipLaunchKernelGGL((march_ensemble_kernel<Dual, true>), dim3(e.blocks), dim3(kNT), 0, s, e);
  return hipGetLastError();
}

// One instance: the descriptor goes to the context's slot, then the same
// persistent kernels run with one workgroup per item (no queue, no table).
hipError_t launch_march(const MarchArgs& a, MarchArgs* slot, bool dual, int kc, hipStream_t s, KernelTimer* t) {
  if (!dual) return launch_fused(a, slot, kc, s, t);  // the residual: one fused pass (fused.hip)
  if (!a.E) return hipErrorInvalidValue;  // the flux pass's ring reads the tile-edge states
  hipLaunchKernelGGL(put_args_kernel, dim3(1), dim3(64), 0, s, a, slot);
  const int64_t total = march_logical_blocks(a.d.g, kc);
  EnsembleLaunch e{slot, nullptr, nullptr, nullptr, 1, total, 0, unsigned(march_blocks(a.d.g, kc)), kc};
  {
    TimedScope ts(t, "grad_march_jvp", s);
    hipLaunchKernelGGL((march_ensemble_kernel<Dual, false>), dim3(e.blocks), dim3(kNT), 0, s, e);
  }
  TimedScope ts(t, "flux_march_jvp", s);
  hipLaunchKernelGGL((march_ensemble_kernel<Dual, true>), dim3(e.blocks), dim3(kNT), 0, s, e);
  return hipGetLastError();
}

hipError_t launch_march_grad(const MarchArgs& a, MarchArgs* slot, int kc, hipStream_t s, KernelTimer* t) {
  hipLaunchKernelGGL(put_args_kernel, dim3(1), dim3(64), 0, s, a, slot);
  const int64_t total = march_logical_blocks(a.d.g, kc);
  EnsembleLaunch e{slot, nullptr, nullptr, nullptr, 1, total, 0, unsigned(march_blocks(a.d.g, kc)), kc};
  TimedScope ts(t, "grad_march_fwd", s);
  if (a.Q)
    hipLaunchKernelGGL((march_ensemble_kernel<double, false, true>), dim3(e.blocks), dim3(kNT), 0, s, e);
  else
    hipLaunchKernelGGL((march_ensemble_kernel<double, false>), dim3(e.blocks), dim3(kNT), 0, s, e);
  return hipGetLastError();
}

}  // namespace cfv
