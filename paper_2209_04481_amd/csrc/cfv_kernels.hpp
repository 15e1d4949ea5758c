// Shared declarations of the device-side launch context and I/O helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "cfv_math.hpp"
#include "cfv_topo.hpp"

namespace cfv {

// Everything a kernel needs to know about one problem instance.
struct DevGrid {
  Shape g;
  GeomRef G;
  Params pr;
  const double* br;  // inner-boundary B_r map, 6N^2, order (p, j, i)
};

// load/store a scalar of type T from a value array and (for Dual) a tangent array
__host__ __device__ __forceinline__ void ldT(const double* a, const double*, int64_t i, double& x) { x = a[i]; }
__host__ __device__ __forceinline__ void ldT(const double* a, const double* b, int64_t i, Dual& x) {
  x = Dual(a[i], b ? b[i] : 0.0);
}
__host__ __device__ __forceinline__ void stT(double* a, double*, int64_t i, double x) { a[i] = x; }
__host__ __device__ __forceinline__ void stT(double* a, double* b, int64_t i, Dual x) {
  a[i] = x.v;
  b[i] = x.d;
}

// Ghost primitives of boundary cell (p,k,j,i) across local face lf (0 inner,
// 1 outer), given its own primitives qI and centre xI.
template <class T>
__host__ __device__ __forceinline__ void ghost_prims(const DevGrid& d, int p, int k, int j, int i, int lf, const T qI[9],
                                            V3 xI, T br, T qG[9], V3& xG) {
  V3 S, xf;
  face_geom(d.G, d.g, p, k, j, i, lf, S, xf);
  xG = ghost_centre(xI, S, xf);
  if (lf == 0)
    inner_ghost(qI, xf, br, qG, d.pr);
  else
    outer_ghost(qI, xI, xG, xf, qG, d.pr);
}

// Optional per-launch timer: brackets each kernel launch with events on the
// launch stream (see capi.cpp).  Null means no timing.
struct KernelTimer {
  virtual void begin(const char* name, hipStream_t s) = 0;
  virtual void end(hipStream_t s) = 0;
  virtual ~KernelTimer() = default;
};

struct TimedScope {
  KernelTimer* t;
  hipStream_t s;
  TimedScope(KernelTimer* t_, const char* name, hipStream_t s_) : t(t_), s(s_) {
    if (t) t->begin(name, s);
  }
  ~TimedScope() {
    if (t) t->end(s);
  }
};

// launchers (residual.hip)
hipError_t launch_residual(const DevGrid& d, const double* U, double* R, double* W, hipStream_t s,
                           KernelTimer* t = nullptr);
hipError_t launch_jvp(const DevGrid& d, const double* U, const double* v, const double* dbr, double* Jv, double* R,
                      double* W, double* Wd, hipStream_t s, KernelTimer* t = nullptr);
hipError_t launch_geometry(const DevGrid& d, double* xc, double* vol, double* xf, double* S, hipStream_t s);
hipError_t launch_local_dt(const DevGrid& d, const double* U, double cfl, double* diag, double* W, hipStream_t s,
                           KernelTimer* t = nullptr);
hipError_t launch_grad_limit_forward(const DevGrid& d, const double* U, double* W, hipStream_t s,
                                     KernelTimer* t = nullptr);

}  // namespace cfv
