// Device-side physics of the coronal finite-volume MHD residual.
//
// Everything state-dependent is templated on the scalar type T: T = double
// gives the residual, T = Dual (value + one tangent) gives the exact forward
// derivative (JVP) from the same source.  Geometry is always plain double.
// Branches (min/max picks, |v_n|, the clamp under the square root) are taken
// on primal values, so the tangent follows the active branch.
//
// Physics (paper Section 2.1, Eqs. 14-17; boundary laws Sections 3.2, 4.1):
//   conservative U = (rho, rho v, B, E, psi), E = p/(gamma-1) + rho|v|^2/2 + |B|^2/2
//   primitive    P = (rho, v, B, p, psi)
//   normal flux  (rho v_n, rho v v_n + p_T n - B B_n, v_n B - B_n v + psi n,
//                 (E + p_T) v_n - B_n (v.B), c_h^2 B_n),  p_T = p + |B|^2/2
//   Rusanov      F = ((F_L + F_R)/2 - s/2 (U_R - U_L)) |S|,
//                s = max(|v_n,L| + c_f,L, |v_n,R| + c_f,R, c_h)
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace cfv {

// ---------------------------------------------------------------- dual number
struct Dual {
  double v, d;
  __host__ __device__ Dual() : v(0.0), d(0.0) {}
  __host__ __device__ Dual(double a) : v(a), d(0.0) {}
  __host__ __device__ Dual(double a, double b) : v(a), d(b) {}
};
__host__ __device__ __forceinline__ Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__host__ __device__ __forceinline__ Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__host__ __device__ __forceinline__ Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__host__ __device__ __forceinline__ Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
// 1/b: on the GPU the hardware reciprocal refined by two Newton steps
// (e = 1 - b r, r += r e; each squares the relative error), within an ulp or
// so of the IEEE quotient for normal b, at about half a division's
// instructions.  For tangents, and for reciprocals that every pass takes
// through recip() below, so that the passes agree with each other bit for
// bit.  recip_refined(-b) = -recip_refined(b) exactly.  On the host, 1 / b.
__host__ __device__ __forceinline__ double recip_refined(double b) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(b);
  double e = __builtin_fma(-b, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-b, r, 1.0);
  return __builtin_fma(r, e, r);
#else
  return 1.0 / b;
#endif
}
__host__ __device__ __forceinline__ double tangent_recip(double b) { return recip_refined(b); }
__host__ __device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) * tangent_recip(b.v));
}
__host__ __device__ __forceinline__ Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
__host__ __device__ __forceinline__ Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
__host__ __device__ __forceinline__ Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
__host__ __device__ __forceinline__ Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
__host__ __device__ __forceinline__ Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
__host__ __device__ __forceinline__ Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
__host__ __device__ __forceinline__ Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d * tangent_recip(b)); }
__host__ __device__ __forceinline__ Dual operator/(double a, Dual b) {
  double q = a / b.v;
  return Dual(q, -q * b.d * tangent_recip(b.v));
}
__host__ __device__ __forceinline__ Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
__host__ __device__ __forceinline__ Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
// Square root on the GPU: the hardware reciprocal square root refined by
// Goldschmidt's iteration (one coupled step for sqrt(x) and 1/(2 sqrt(x)),
// then two Newton corrections of the root), the sequence the compiler
// expands sqrt into, without its rescaling of inputs below 2^-767 and its
// special-value fix-ups: the same bits for every other finite positive x.
// Here x = 0 gives 0 and negative or non-finite x NaN (no state of the
// method takes the roots of such tiny values).  On the host, sqrt.
// With half_rcp, also 1/(2 sqrt(x)) for a tangent: Goldschmidt's estimate
// with one more Newton step against the final root (x = 0: not finite, as
// the IEEE quotient's).
__host__ __device__ __forceinline__ double sqrt_nonneg(double x, double* half_rcp = nullptr) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = __builtin_fma(-h, g, 0.5);
  g = __builtin_fma(g, r, g);
  h = __builtin_fma(h, r, h);
  double d = __builtin_fma(-g, g, x);
  g = __builtin_fma(d, h, g);
  d = __builtin_fma(-g, g, x);
  g = __builtin_fma(d, h, g);
  if (half_rcp) {
    const double e = __builtin_fma(-2.0 * g, h, 1.0);
    *half_rcp = __builtin_fma(h, e, h);
  }
  return x == 0.0 ? 0.0 : g;
#else
  const double s = ::sqrt(x);
  if (half_rcp) *half_rcp = 1.0 / (2.0 * s);
  return s;
#endif
}

__host__ __device__ __forceinline__ Dual sqrt(Dual a) {
  double h;
  const double s = sqrt_nonneg(a.v, &h);
  return Dual(s, a.d * h);
}

// 1/b with the value of recip_refined for plain values and Dual values alike
__host__ __device__ __forceinline__ double recip(double b) { return recip_refined(b); }
__host__ __device__ __forceinline__ Dual recip(Dual b) {
  const double r = recip_refined(b.v);
  return Dual(r, -(b.d * r) * r);
}

// n / d for |n| <= |d| (a limiter ratio) by the refined reciprocal.  A
// subnormal d's reciprocal overflows, so d below 2^-1000 is first scaled,
// with n, by 2^64 (exact); for every other d the bits are n * recip(d).
__host__ __device__ __forceinline__ double ratio_refined(double n, double d) {
  const double s = ::fabs(d) < 0x1p-1000 ? 0x1p+64 : 1.0;
  return (n * s) * recip_refined(d * s);
}
__host__ __device__ __forceinline__ Dual ratio_refined(Dual n, Dual d) {
  const double s = ::fabs(d.v) < 0x1p-1000 ? 0x1p+64 : 1.0;
  return (n * s) * recip(d * s);
}

__host__ __device__ __forceinline__ double val(double a) { return a; }
__host__ __device__ __forceinline__ double val(Dual a) { return a.v; }
__host__ __device__ __forceinline__ double dsqrt(double a) { return sqrt_nonneg(a); }
__host__ __device__ __forceinline__ Dual dsqrt(Dual a) { return sqrt(a); }
template <class T> __host__ __device__ __forceinline__ T tabs(T a) { return val(a) < 0.0 ? -a : a; }
// min/max that keep the first argument on ties; the pick follows the values
template <class T> __host__ __device__ __forceinline__ T pick_min(T a, T b) { return val(a) <= val(b) ? a : b; }
template <class T> __host__ __device__ __forceinline__ T pick_max(T a, T b) { return val(a) >= val(b) ? a : b; }
// plain values carry nothing that depends on which argument wins: the
// hardware's abs modifier and min/max instructions (the same values; only a
// NaN argument, which makes the flux NaN anyway, is passed over)
__host__ __device__ __forceinline__ double tabs(double a) { return ::fabs(a); }
__host__ __device__ __forceinline__ double pick_min(double a, double b) { return ::fmin(a, b); }
__host__ __device__ __forceinline__ double pick_max(double a, double b) { return ::fmax(a, b); }
__host__ __device__ __forceinline__ Dual powd(Dual a, double e) {
  double p = ::pow(a.v, e);
  return Dual(p, e == 0.0 ? 0.0 : e * ::pow(a.v, e - 1.0) * a.d);
}
__host__ __device__ __forceinline__ double powd(double a, double e) { return ::pow(a, e); }

// ------------------------------------------------------- global memory access
// Loads and stores through pointers to device (global) memory that the
// compiler cannot prove global, because they come from descriptor tables or
// structures: without this it emits flat instructions, which also count
// against the LDS wait counter, so LDS waits would also wait for them.  Only
// for pointers into device memory allocations (never LDS or stack).
template <class T>
__host__ __device__ __forceinline__ T gld(const T* p, int64_t i) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ((const __attribute__((address_space(1))) T*)p)[i];
#else
  return p[i];
#endif
}
template <class T>
__host__ __device__ __forceinline__ void gst(T* p, int64_t i, T v) {
#if defined(__HIP_DEVICE_COMPILE__)
  ((__attribute__((address_space(1))) T*)p)[i] = v;
#else
  p[i] = v;
#endif
}

// ------------------------------------------------------------------- vectors
struct V3 {
  double x, y, z;
};
__host__ __device__ __forceinline__ V3 mk(double x, double y, double z) { return V3{x, y, z}; }
__host__ __device__ __forceinline__ V3 operator+(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__host__ __device__ __forceinline__ V3 operator-(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__host__ __device__ __forceinline__ V3 operator*(double s, V3 a) { return V3{s * a.x, s * a.y, s * a.z}; }
__host__ __device__ __forceinline__ double dot3(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__host__ __device__ __forceinline__ V3 cross3(V3 a, V3 b) {
  return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__host__ __device__ __forceinline__ double norm3(V3 a) { return sqrt_nonneg(dot3(a, a)); }

// --------------------------------------------------------------- parameters
struct Params {
  double gamma, c_h, G, vr_star, rho_b, T_b;
  int limiter;
  int inner_mode;
  double outer_exp[8];  // rho, B_r, B_theta, B_phi, V_r, V_theta, V_phi, p
  int outer_vr_mass;
  int outer_psi_zero;
};

// ------------------------------------------------------------ state algebra
// prim[] = (rho, vx, vy, vz, Bx, By, Bz, p, psi)
template <class T>
__host__ __device__ __forceinline__ void cons_to_prim(const T u[9], T q[9], double gamma) {
  T rho = u[0];
  T irho = recip(rho);
  T vx = u[1] * irho, vy = u[2] * irho, vz = u[3] * irho;
  T v2 = vx * vx + vy * vy + vz * vz;
  T B2 = u[4] * u[4] + u[5] * u[5] + u[6] * u[6];
  q[0] = rho; q[1] = vx; q[2] = vy; q[3] = vz;
  q[4] = u[4]; q[5] = u[5]; q[6] = u[6];
  q[7] = (gamma - 1.0) * (u[7] - 0.5 * rho * v2 - 0.5 * B2);
  q[8] = u[8];
}

template <class T>
__host__ __device__ __forceinline__ void prim_to_cons(const T q[9], T u[9], double gamma) {
  T v2 = q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  T B2 = q[4] * q[4] + q[5] * q[5] + q[6] * q[6];
  u[0] = q[0];
  u[1] = q[0] * q[1]; u[2] = q[0] * q[2]; u[3] = q[0] * q[3];
  u[4] = q[4]; u[5] = q[5]; u[6] = q[6];
  u[7] = q[7] * (1.0 / (gamma - 1.0)) + 0.5 * q[0] * v2 + 0.5 * B2;
  u[8] = q[8];
}

// |v_n| + c_f of one side (c_f the fast magnetosonic speed along n)
template <class T>
__host__ __device__ __forceinline__ T side_speed(const T q[9], V3 n, double gamma) {
  T rho = q[0], bx = q[4], by = q[5], bz = q[6], p = q[7];
  T vn = q[1] * n.x + q[2] * n.y + q[3] * n.z;
  T bn = bx * n.x + by * n.y + bz * n.z;
  T B2 = bx * bx + by * by + bz * bz;
  T irho = recip(rho);
  T a2 = gamma * p * irho;
  T b2 = B2 * irho;
  T bn2 = bn * bn * irho;
  T s = a2 + b2;
  T disc = s * s - 4.0 * a2 * bn2;
  T sd = val(disc) > 0.0 ? dsqrt(disc) : T(0.0);
  T cf = dsqrt(0.5 * (s + sd));
  return tabs(vn) + cf;
}

// F += wf * (F(q).n) + wu * U(q): one side's share of the Rusanov flux
// (igm1 = 1 / (gamma - 1))
template <class T>
__host__ __device__ __forceinline__ void side_accumulate(const T q[9], V3 n, double wf, T wu, T F[9],
                                                         double igm1, double c_h) {
  T rho = q[0], vx = q[1], vy = q[2], vz = q[3], bx = q[4], by = q[5], bz = q[6], p = q[7], psi = q[8];
  T vn = vx * n.x + vy * n.y + vz * n.z;
  T bn = bx * n.x + by * n.y + bz * n.z;
  T B2 = bx * bx + by * by + bz * bz;
  T v2 = vx * vx + vy * vy + vz * vz;
  T pT = p + 0.5 * B2;
  T E = p * igm1 + 0.5 * rho * v2 + 0.5 * B2;
  T rvn = rho * vn;
  T vb = vx * bx + vy * by + vz * bz;
  F[0] += wf * rvn + wu * rho;
  F[1] += wf * (rvn * vx + pT * n.x - bx * bn) + wu * (rho * vx);
  F[2] += wf * (rvn * vy + pT * n.y - by * bn) + wu * (rho * vy);
  F[3] += wf * (rvn * vz + pT * n.z - bz * bn) + wu * (rho * vz);
  F[4] += wf * (vn * bx - bn * vx + psi * n.x) + wu * bx;
  F[5] += wf * (vn * by - bn * vy + psi * n.y) + wu * by;
  F[6] += wf * (vn * bz - bn * vz + psi * n.z) + wu * bz;
  F[7] += wf * ((E + pT) * vn - bn * vb) + wu * E;
  F[8] += wf * ((c_h * c_h) * bn) + wu * psi;
}

// normal physical flux for unit n; also returns |v_n| + c_f
template <class T>
__host__ __device__ __forceinline__ T phys_flux(const T q[9], V3 n, T F[9], double gamma, double c_h) {
  for (int v = 0; v < 9; ++v) F[v] = T(0.0);
  side_accumulate(q, n, 1.0, T(0.0), F, 1.0 / (gamma - 1.0), c_h);
  return side_speed(q, n, gamma);
}

// Rusanov flux through the face of vector area S (L -> R); returns s.
//   F = (F_L + F_R)/2 |S| - s/2 (U_R - U_L) |S|,  s = max(lam_L, lam_R, c_h)
// |S| and 1/|S| from one square-root sequence
__host__ __device__ __forceinline__ double area_and_inverse(V3 S, double& ia) {
  double h;
  const double area = sqrt_nonneg(dot3(S, S), &h);
  ia = 2.0 * h;
  return area;
}

template <class T>
__host__ __device__ __forceinline__ T rusanov(const T qL[9], const T qR[9], V3 S, T F[9], const Params& pr) {
  double ia;
  const double area = area_and_inverse(S, ia);
  const V3 n = mk(S.x * ia, S.y * ia, S.z * ia);
  T s = pick_max(side_speed(qL, n, pr.gamma), side_speed(qR, n, pr.gamma));
  s = pick_max(s, T(pr.c_h));
  const T hs = 0.5 * s;
  for (int v = 0; v < 9; ++v) F[v] = T(0.0);
  const double igm1 = 1.0 / (pr.gamma - 1.0);  // invariant: hoisted out of the marches' loops
  side_accumulate(qL, n, 0.5, hs, F, igm1, pr.c_h);
  side_accumulate(qR, n, 0.5, -hs, F, igm1, pr.c_h);
  for (int v = 0; v < 9; ++v) F[v] = F[v] * area;
  return s;
}

// spherical unit vectors at x (Eqs. 20-21); within a relative distance 1e-12
// of the polar axis, where theta and phi would be set by rounding, the limit
// along the meridian phi = 0.
__host__ __device__ __forceinline__ void sph_basis(V3 x, V3& rh, V3& th, V3& ph) {
  double r = norm3(x);
  double rc = ::sqrt(x.x * x.x + x.y * x.y);
  double ir = 1.0 / r;
  rh = mk(x.x * ir, x.y * ir, x.z * ir);
  if (rc <= 1e-12 * r) {
    th = mk(x.z >= 0.0 ? 1.0 : -1.0, 0.0, 0.0);
    ph = mk(0.0, 1.0, 0.0);
    return;
  }
  double irc = 1.0 / rc;
  th = mk(x.x * x.z * irc * ir, x.y * x.z * irc * ir, -rc * ir);
  ph = mk(-x.y * irc, x.x * irc, 0.0);
}

// Inner low-E ghost (Section 3.2, Eq. 25).  Dirichlet values are face averages,
// so G = 2b - I.  The boundary field keeps the interior tangential part and
// takes the map's radial part; the boundary velocity is V_r* B_r B_b / |B_b|^2.
template <class T>
__host__ __device__ __forceinline__ void inner_ghost(const T qI[9], V3 xf, T br, T qG[9], const Params& pr) {
  double ir = 1.0 / norm3(xf);
  V3 rh = mk(xf.x * ir, xf.y * ir, xf.z * ir);
  T bIr = qI[4] * rh.x + qI[5] * rh.y + qI[6] * rh.z;
  T dB = br - bIr;
  T bbx = qI[4] + dB * rh.x, bby = qI[5] + dB * rh.y, bbz = qI[6] + dB * rh.z;
  T bb2 = bbx * bbx + bby * bby + bbz * bbz;
  if (val(bb2) <= 1e-30) bb2 = T(1e-30);
  T fac = pr.vr_star * br / bb2;
  qG[0] = 2.0 * pr.rho_b - qI[0];
  qG[1] = 2.0 * (fac * bbx) - qI[1];
  qG[2] = 2.0 * (fac * bby) - qI[2];
  qG[3] = 2.0 * (fac * bbz) - qI[3];
  qG[4] = 2.0 * bbx - qI[4];
  qG[5] = 2.0 * bby - qI[5];
  qG[6] = 2.0 * bbz - qI[6];
  qG[7] = 2.0 * (pr.rho_b * pr.T_b) - qI[7];
  qG[8] = -qI[8];
}

// Inner large-E ghost (Section 3.2, Eqs. 20-24): B_r and B_theta imposed
// (Dirichlet), B_phi Neumann; the velocity V_par (B_r, B_theta, 0) with
// V_par = V_r* B_r / (B_r^2 + B_theta^2); rho, p, psi as the low-E law.
template <class T>
__host__ __device__ __forceinline__ void inner_ghost_large_e(const T qI[9], V3 xf, T br, double bth, T qG[9],
                                                             const Params& pr) {
  V3 rh, th, ph;
  sph_basis(xf, rh, th, ph);
  const T bph = qI[4] * ph.x + qI[5] * ph.y + qI[6] * ph.z;
  const T bbx = br * rh.x + bth * th.x + bph * ph.x;
  const T bby = br * rh.y + bth * th.y + bph * ph.y;
  const T bbz = br * rh.z + bth * th.z + bph * ph.z;
  T pol2 = br * br + bth * bth;
  if (val(pol2) <= 1e-30) pol2 = T(1e-30);
  const T vpar = pr.vr_star * br / pol2;
  const T vr = vpar * br, vt = vpar * bth;
  qG[0] = 2.0 * pr.rho_b - qI[0];
  qG[1] = 2.0 * (vr * rh.x + vt * th.x) - qI[1];
  qG[2] = 2.0 * (vr * rh.y + vt * th.y) - qI[2];
  qG[3] = 2.0 * (vr * rh.z + vt * th.z) - qI[3];
  qG[4] = 2.0 * bbx - qI[4];
  qG[5] = 2.0 * bby - qI[5];
  qG[6] = 2.0 * bbz - qI[6];
  qG[7] = 2.0 * (pr.rho_b * pr.T_b) - qI[7];
  qG[8] = -qI[8];
}

// Outer ghost: Table 2 laws G = I (r_I/r_G)^e in spherical components at the
// face centroid, V_r by V_r r^2 rho = const when selected, psi_b = 0 or G = I.
template <class T>
__host__ __device__ __forceinline__ void outer_ghost(const T qI[9], V3 xI, V3 xG, V3 xf, T qG[9], const Params& pr) {
  V3 rh, th, ph;
  sph_basis(xf, rh, th, ph);
  double rI = norm3(xI), rG = norm3(xG);
  double q = rI / rG;
  const double* e = pr.outer_exp;
  T rho = qI[0] * ::pow(q, e[0]);
  T br = (qI[4] * rh.x + qI[5] * rh.y + qI[6] * rh.z) * ::pow(q, e[1]);
  T bt = (qI[4] * th.x + qI[5] * th.y + qI[6] * th.z) * ::pow(q, e[2]);
  T bp = (qI[4] * ph.x + qI[5] * ph.y) * ::pow(q, e[3]);
  T vr = qI[1] * rh.x + qI[2] * rh.y + qI[3] * rh.z;
  if (pr.outer_vr_mass)
    vr = vr * ((rI * rI) * qI[0]) / ((rG * rG) * rho);
  else
    vr = vr * ::pow(q, e[4]);
  T vt = (qI[1] * th.x + qI[2] * th.y + qI[3] * th.z) * ::pow(q, e[5]);
  T vp = (qI[1] * ph.x + qI[2] * ph.y) * ::pow(q, e[6]);
  qG[0] = rho;
  qG[1] = vr * rh.x + vt * th.x + vp * ph.x;
  qG[2] = vr * rh.y + vt * th.y + vp * ph.y;
  qG[3] = vr * rh.z + vt * th.z;
  qG[4] = br * rh.x + bt * th.x + bp * ph.x;
  qG[5] = br * rh.y + bt * th.y + bp * ph.y;
  qG[6] = br * rh.z + bt * th.z;
  qG[7] = qI[7] * ::pow(q, e[7]);
  qG[8] = pr.outer_psi_zero ? -qI[8] : qI[8];
}

// gravity source times volume: V (0, rho g, 0, g . m, 0), g = -G x/|x|^3
template <class T>
__host__ __device__ __forceinline__ void gravity_source(const T u[9], V3 x, double vol, double G, T S[9]) {
  double r = norm3(x);
  double f = -G / (r * r * r) * vol;
  V3 gv = mk(f * x.x, f * x.y, f * x.z);
  S[0] = T(0.0);
  S[1] = u[0] * gv.x; S[2] = u[0] * gv.y; S[3] = u[0] * gv.z;
  S[4] = T(0.0); S[5] = T(0.0); S[6] = T(0.0);
  S[7] = u[1] * gv.x + u[2] * gv.y + u[3] * gv.z;
  S[8] = T(0.0);
}

}  // namespace cfv
