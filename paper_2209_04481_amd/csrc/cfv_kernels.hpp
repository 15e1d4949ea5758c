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
  const double* bth = nullptr;  // inner-boundary B_theta map (large-E law), same order
  unsigned* flag = nullptr;     // non-physical state word (bit 0), nullable
  const int32_t* ftab = nullptr;  // per-tile stencil tables of the fused march (cfv_fused.hpp)
};

// A face state is physical when its density and pressure are positive (a NaN
// fails too); the kernels record any other in the instance's flag word with
// an integer OR (order-free, so results stay deterministic).
template <class T>
__host__ __device__ __forceinline__ bool physical(const T q[9]) {
  return val(q[0]) > 0.0 && val(q[7]) > 0.0;
}
__host__ __device__ __forceinline__ void record_nonphysical(const DevGrid& d, bool bad) {
  if (!bad || !d.flag) return;
#if defined(__HIP_DEVICE_COMPILE__)
  atomicOr(d.flag, 1u);
#else
  *d.flag |= 1u;
#endif
}

// The first kernel argument read in place from the kernel-argument segment:
// large descriptors (grid, parameters) are then loaded where they are used
// instead of being preloaded whole into scalar registers, which spill.
#if defined(__HIP__)
template <class A>
__device__ __forceinline__ const A& first_kernel_arg() {
  return *(const A*)__builtin_amdgcn_kernarg_segment_ptr();
}
#endif

// load/store a scalar of type T from a value array and (for Dual) a tangent array
__host__ __device__ __forceinline__ void ldT(const double* a, const double*, int64_t i, double& x) { x = gld(a, i); }
__host__ __device__ __forceinline__ void ldT(const double* a, const double* b, int64_t i, Dual& x) {
  x = Dual(gld(a, i), b ? gld(b, i) : 0.0);
}
__host__ __device__ __forceinline__ void stT(double* a, double*, int64_t i, double x) { gst(a, i, x); }
__host__ __device__ __forceinline__ void stT(double* a, double* b, int64_t i, Dual x) {
  gst(a, i, x.v);
  gst(b, i, x.d);
}

// Ghost primitives of boundary cell (p,k,j,i) across local face lf (0 inner,
// 1 outer), given its own primitives qI and centre xI.
template <class T>
__host__ __device__ __forceinline__ void ghost_prims(const DevGrid& d, int p, int k, int j, int i, int lf, const T qI[9],
                                            V3 xI, T br, T qG[9], V3& xG) {
  V3 S, xf;
  face_geom(d.G, d.g, p, k, j, i, lf, S, xf);
  xG = ghost_centre(xI, S, xf);
  if (lf == 0) {
    if (d.pr.inner_mode == 1)
      inner_ghost_large_e(qI, xf, br, gld(d.bth, column_of(d.g, p, j, i)), qG, d.pr);
    else
      inner_ghost(qI, xf, br, qG, d.pr);
  } else {
    outer_ghost(qI, xI, xG, xf, qG, d.pr);
  }
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

// Unweighted least-squares gradient over the six face neighbours,
//   g = M^-1 sum_n dx_n (q_n - q_c),  M = sum_n dx_n dx_n^T,
// written as g = sum_n W_n (q_n - q_c) with the weights W_n = M^-1 dx_n (M is
// inverted by cofactors), followed by the Barth-Jespersen factor.  Extremes
// over the cell and its neighbours keep the earlier candidate on ties (the
// cell first, then neighbours in local face order).
struct LsqWeights {
  V3 W[6];
  __host__ __device__ explicit LsqWeights(const V3 dx[6]) {
    double m00 = 0, m01 = 0, m02 = 0, m11 = 0, m12 = 0, m22 = 0;
#pragma unroll
    for (int n = 0; n < 6; ++n) {
      m00 += dx[n].x * dx[n].x; m01 += dx[n].x * dx[n].y; m02 += dx[n].x * dx[n].z;
      m11 += dx[n].y * dx[n].y; m12 += dx[n].y * dx[n].z; m22 += dx[n].z * dx[n].z;
    }
    const double c00 = m11 * m22 - m12 * m12, c01 = m02 * m12 - m01 * m22, c02 = m01 * m12 - m02 * m11;
    const double c11 = m00 * m22 - m02 * m02, c12 = m01 * m02 - m00 * m12, c22 = m00 * m11 - m01 * m01;
    const double idet = recip_refined(m00 * c00 + m01 * c01 + m02 * c02);
    const double i00 = c00 * idet, i01 = c01 * idet, i02 = c02 * idet;
    const double i11 = c11 * idet, i12 = c12 * idet, i22 = c22 * idet;
#pragma unroll
    for (int n = 0; n < 6; ++n)
      W[n] = mk(i00 * dx[n].x + i01 * dx[n].y + i02 * dx[n].z, i01 * dx[n].x + i11 * dx[n].y + i12 * dx[n].z,
                i02 * dx[n].x + i12 * dx[n].y + i22 * dx[n].z);
  }
};

// limited gradient of one variable from its cell value and six neighbours
template <class T>
__host__ __device__ __forceinline__ void limited_grad(const LsqWeights& L, const V3 dxf[6], int limiter, T qc,
                                             const T qn[6], T& gx, T& gy, T& gz) {
  gx = T(0.0); gy = T(0.0); gz = T(0.0);
  T qmax = qc, qmin = qc;
#pragma unroll
  for (int n = 0; n < 6; ++n) {
    const T dq = qn[n] - qc;
    gx += L.W[n].x * dq; gy += L.W[n].y * dq; gz += L.W[n].z * dq;
    qmax = pick_max(qmax, qn[n]);
    qmin = pick_min(qmin, qn[n]);
  }
  if (!limiter) return;
  // Barth-Jespersen: the smallest ratio (q_ext - q_c) / (g . (x_f - x_c))
  // below 1, ties keeping the earlier candidate (1 first, then faces in
  // local order).  The numerator is qmax - qc where the projection d2 is
  // positive and qmin - qc where it is negative, so the candidates are the
  // face with the largest d2 and the face with the smallest (the first of
  // equal ones); their magnitudes are compared cross-multiplied, and an
  // exact tie between the two goes to the earlier face.  One reciprocal.
  T dhi = T(0.0), dlo = T(0.0);
  int fhi = 6, flo = 6;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const T d2 = gx * dxf[f].x + gy * dxf[f].y + gz * dxf[f].z;
    if (val(d2) > val(dhi)) { dhi = d2; fhi = f; }
    if (val(d2) < val(dlo)) { dlo = d2; flo = f; }
  }
  const double up = val(qmax) - val(qc), down = val(qc) - val(qmin), adhi = val(dhi), adlo = -val(dlo);
  double bn = 1.0, bd = 1.0;
  int pick = 0;
  if (up * bd < bn * adhi) {
    bn = up;
    bd = adhi;
    pick = 1;
  }
  const double lhs = down * bd, rhs = bn * adlo;
  if (lhs < rhs || (lhs == rhs && pick == 1 && flo < fhi)) pick = 2;
  if (pick == 0) return;
  const T phi = pick == 1 ? ratio_refined(qmax - qc, dhi) : ratio_refined(qmin - qc, dlo);
  gx = phi * gx; gy = phi * gy; gz = phi * gz;
}

// The same for plain values, with fewer selects: no derivative follows the
// choice, so the extremes are taken by max/min, the candidates are the
// largest and the smallest projection (max/min), and which of two equal
// ratios is kept does not matter (the numerator has the sign of the
// denominator, so num / den = |num| / |den|); with no ratio below 1 the
// factor is 1.
template <>
__host__ __device__ __forceinline__ void limited_grad<double>(const LsqWeights& L, const V3 dxf[6], int limiter,
                                                              double qc, const double qn[6], double& gx,
                                                              double& gy, double& gz) {
  gx = 0.0; gy = 0.0; gz = 0.0;
  double qmax = qc, qmin = qc;
#pragma unroll
  for (int n = 0; n < 6; ++n) {
    const double dq = qn[n] - qc;
    gx += L.W[n].x * dq; gy += L.W[n].y * dq; gz += L.W[n].z * dq;
    qmax = ::fmax(qmax, qn[n]);
    qmin = ::fmin(qmin, qn[n]);
  }
  if (!limiter) return;
  double dmax = 0.0, dmin = 0.0;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const double d2 = gx * dxf[f].x + gy * dxf[f].y + gz * dxf[f].z;
    dmax = ::fmax(dmax, d2);
    dmin = ::fmin(dmin, d2);
  }
  const double up = qmax - qc, down = qc - qmin, ad = -dmin;
  double bn = 1.0, bd = 1.0;
  if (up * bd < bn * dmax) {
    bn = up;
    bd = dmax;
  }
  if (down * bd < bn * ad) {
    bn = down;
    bd = ad;
  }
  const double phi = ratio_refined(bn, bd);
  gx = phi * gx; gy = phi * gy; gz = phi * gz;
}

// launchers (residual.hip)
hipError_t launch_geometry(const DevGrid& d, double* xc, double* vol, double* xf, double* S, hipStream_t s);
hipError_t launch_local_dt(const DevGrid& d, const double* U, double cfl, double* diag, double* W, hipStream_t s,
                           KernelTimer* t = nullptr);
hipError_t launch_grad_limit_forward(const DevGrid& d, const double* U, double* W, hipStream_t s,
                                     KernelTimer* t = nullptr);

}  // namespace cfv
