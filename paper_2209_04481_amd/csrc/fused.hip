// Fused radial march of the residual (phase functions in cfv_fused.hpp): one
// pass per layer over a 16 x 16 block of columns, the 14 x 14 tile inside it
// and its ring, computes the limited gradients, the face states, every face
// flux of the tile once and the residual.  HBM sees U read (plus the ring and
// chunk-boundary layers, mostly from L2) and R written.
//
// Per layer, two barriers: after the primitives are published, and after the
// gradients and the exchanged face states; the face fluxes a layer exchanges
// are summed after the next layer's first barrier.  A
// chunk of layers [k0, k1) also evaluates the gradient of the layer below it
// (for the state on its bottom face) and of the layer above it (for its top
// face); those layers take no fluxes.  One workgroup per CU: the block keeps
// three layers of primitives and the exchange buffers in LDS (148 KB).
#include "cfv_fused.hpp"

namespace cfv {

template <class T>
__device__ __forceinline__ void fused_march_tile(const MarchArgs& a0, const FTile& tm, double* lds) {
  const MarchArgs& a = a0;
  const int t = threadIdx.x;
  const Shape& g = a.d.g;
  const int kb = tm.k0 > 0 ? tm.k0 - 1 : 0;
  const int ke = tm.k1 < g.Nr ? tm.k1 : tm.k1 - 1;
  FuState<T> st;
  FusedWG<T>::init(a, tm, st, t, kb, lds);
  for (int k = FusedWG<T>::first_publish(kb); k < kb; ++k) FusedWG<T>::publish_block(a, st, t, k, lds);
  for (int k = kb; k <= ke; ++k) {
    const MarchArgs& a = per_layer(a0);
    const int mode = k < tm.k0 ? 1 : k >= tm.k1 ? 2 : 0;
    FusedWG<T>::publish(a, tm, st, t, k, lds);
    __syncthreads();
    // the previous layer's fluxes from the west and south neighbours: the
    // barrier above also orders them, so the flux phase needs none of its own
    if (k - 1 >= tm.k0 && k - 1 < tm.k1) FusedWG<T>::accumulate(a, tm, st, t, k - 1, lds);
    FusedWG<T>::gradient(a, tm, st, t, k, mode, lds);
    __syncthreads();
    if (mode == 0) FusedWG<T>::flux(a, tm, st, t, k, lds);
  }
  if (ke < tm.k1) {  // the chunk's last layer is the shell's outermost: no layer follows
    __syncthreads();
    FusedWG<T>::accumulate(a, tm, st, t, ke, lds);
  }
  record_nonphysical(a.d, st.role == 1 && st.bad);
}

// the item index is the same in every lane: scalar registers for the
// descriptor and table reads
__device__ __forceinline__ int64_t fused_uniform(int64_t v) {
  const uint64_t u = uint64_t(v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(u));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(u >> 32));
  return int64_t((uint64_t(hi) << 32) | lo);
}

__device__ __forceinline__ int fused_find_instance(const int64_t* __restrict__ off, int n, int64_t w) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= w) lo = mid; else hi = mid;
  }
  return lo;
}

// Items (instance, tile, chunk) taken statically (each XCD a contiguous
// eighth of the list) or from a device counter.
template <class T>
__global__ __launch_bounds__(kFL, 1) void fused_march_kernel(EnsembleLaunch e) {
  __shared__ double lds[FusedWG<T>::kLds];
  __shared__ int slot;
  for (int64_t step = 0;; ++step) {
    int64_t q;
    if (e.queue) {
      __syncthreads();
      if (threadIdx.x == 0) slot = int(atomicAdd(e.counters, 1u));
      __syncthreads();
      q = slot;
    } else {
      const int64_t Q = e.blocks / 8, per = (e.total + 7) / 8;
      const int64_t x = blockIdx.x % 8, r = blockIdx.x / 8;
      const int64_t w = r + step * Q, idx = x * per + w;
      q = w < per && idx < e.total ? idx : e.total;
    }
    q = fused_uniform(q);
    if (q >= e.total) break;
    const int64_t w = e.perm ? fused_uniform(e.perm[q]) : q;
    const int inst = e.n > 1 ? int(fused_uniform(fused_find_instance(e.item_off, e.n, w))) : 0;
    const MarchArgs& a = constant_args(e.args + inst);
    FTile tm;
    fused_tile_of(a.d.g, e.kc, e.n > 1 ? w - e.item_off[inst] : w, tm);
    __syncthreads();  // the previous item's LDS reads are done
    fused_march_tile<T>(a, tm, lds);
  }
}

__global__ void fused_reset_counter_kernel(unsigned* c) {
  if (threadIdx.x == 0) c[0] = 0u;
}

__global__ void fused_put_args_kernel(MarchArgs, MarchArgs* __restrict__ dst) {
  static_assert(sizeof(MarchArgs) % 8 == 0, "descriptor copied in 8-byte words");
  constexpr int kW = int(sizeof(MarchArgs) / 8);
  const uint64_t* src = (const uint64_t*)&first_kernel_arg<MarchArgs>();
  uint64_t* d = reinterpret_cast<uint64_t*>(dst);
  for (int q = threadIdx.x; q < kW; q += blockDim.x) d[q] = src[q];
}

hipError_t launch_fused_ensemble(const EnsembleLaunch& e, hipStream_t s, KernelTimer* t) {
  if (e.total <= 0) return hipSuccess;
  if (e.queue) hipLaunchKernelGGL(fused_reset_counter_kernel, dim3(1), dim3(64), 0, s, e.counters);
  TimedScope ts(t, e.n > 1 ? "fused_march_ens" : "fused_march", s);
  hipLaunchKernelGGL(fused_march_kernel<double>, dim3(e.blocks), dim3(kFL), 0, s, e);
  return hipGetLastError();
}

// One instance: the descriptor to the context's slot, one workgroup per item
// (a multiple of 8 workgroups so that the XCD split is a bijection).
hipError_t launch_fused(const MarchArgs& a, MarchArgs* slot, int kc, hipStream_t s, KernelTimer* t) {
  hipLaunchKernelGGL(fused_put_args_kernel, dim3(1), dim3(64), 0, s, a, slot);
  const int64_t total = fused_items(a.d.g, kc);
  EnsembleLaunch e{slot, nullptr, nullptr, nullptr, 1, total, 0, unsigned((total + 7) / 8 * 8), kc};
  return launch_fused_ensemble(e, s, t);
}

}  // namespace cfv
