// Cell-centric kernels: the forward pass the adjoint replays, the local time
// step, and the geometry export.
//
// grad_limit: per cell, primitives of the cell and its six face neighbours
// (ghost states on boundary faces), the unweighted least-squares gradient,
// and the Barth-Jespersen factor; writes the primitives and the limited
// gradient (9 + 27 values) to a workspace.
// flux (diagonal form): per cell, for each of its six faces, reconstructs
// both sides at the face centroid and takes the Rusanov speed times the face
// area: the backward-Euler diagonal.  (The same routine with the flux
// accumulation is the cell-centric residual, templated on the scalar; the
// residual and JVP themselves run in the radial-march kernels.)
#include "cfv_kernels.hpp"

namespace cfv {

static constexpr int kBlock = 256;

// outputs: value array optional; tangent array written for Dual when given
__host__ __device__ __forceinline__ void store_out(double* R, double*, int64_t i, double x) {
  if (R) R[i] = x;
}
__host__ __device__ __forceinline__ void store_out(double* R, double* Rd, int64_t i, Dual x) {
  if (R) R[i] = x.v;
  if (Rd) Rd[i] = x.d;
}

template <class T>
__host__ __device__ inline void grad_limit_cell(const DevGrid& d, const double* __restrict__ U,
                                                const double* __restrict__ Ud, const double* __restrict__ dbr,
                                                double* __restrict__ W, double* __restrict__ Wd, int64_t c) {
  const int64_t nc = d.g.ncells;
  int p, k, j, i;
  decode(d.g, c, p, k, j, i);
  T u[9], qc[9];
#pragma unroll
  for (int v = 0; v < 9; ++v) ldT(U, Ud, v * nc + c, u[v]);
  cons_to_prim(u, qc, d.pr.gamma);
  const V3 xc = cell_centre(d.G, d.g, p, k, j, i);

  T qn[6][9];
  V3 dx[6], dxf[6];
#pragma unroll
  for (int lf = 0; lf < 6; ++lf) {
    Nbr nb = neighbour(d.g, p, k, j, i, lf);
    V3 S, xf;
    bool own;
    canon_face(d.G, d.g, p, k, j, i, lf, nb, c, S, xf, own);
    dxf[lf] = xf - xc;
    V3 xn;
    if (nb.id >= nc) {
      const int64_t col = (int64_t(p) * d.g.N + j) * d.g.N + i;
      T br;
      if (lf == 0) ldT(d.br, dbr, col, br); else br = T(0.0);
      ghost_prims(d, p, k, j, i, lf, qc, xc, br, qn[lf], xn);
    } else {
      T un[9];
      for (int v = 0; v < 9; ++v) ldT(U, Ud, v * nc + nb.id, un[v]);
      cons_to_prim(un, qn[lf], d.pr.gamma);
      xn = cell_centre(d.G, d.g, nb.p, nb.k, nb.j, nb.i);
    }
    dx[lf] = xn - xc;
  }
  const LsqWeights L(dx);
#pragma unroll
  for (int v = 0; v < 9; ++v) {
    T q6[6] = {qn[0][v], qn[1][v], qn[2][v], qn[3][v], qn[4][v], qn[5][v]};
    T gx, gy, gz;
    limited_grad(L, dxf, d.pr.limiter, qc[v], q6, gx, gy, gz);
    stT(W, Wd, v * nc + c, qc[v]);
    stT(W, Wd, (9 + 3 * v) * nc + c, gx);
    stT(W, Wd, (10 + 3 * v) * nc + c, gy);
    stT(W, Wd, (11 + 3 * v) * nc + c, gz);
  }
}

template <class T, bool kDiag>
__host__ __device__ inline void flux_cell(const DevGrid& d, const double* __restrict__ U,
                                          const double* __restrict__ Ud, const double* __restrict__ dbr,
                                          const double* __restrict__ W, const double* __restrict__ Wd,
                                          double* __restrict__ R, double* __restrict__ Rd, double* __restrict__ diag,
                                          double cfl, int64_t c) {
  const int64_t nc = d.g.ncells;
  int p, k, j, i;
  decode(d.g, c, p, k, j, i);
  const V3 xc = cell_centre(d.G, d.g, p, k, j, i);
  T Pc[9], Gc[27];
#pragma unroll
  for (int v = 0; v < 9; ++v) ldT(W, Wd, v * nc + c, Pc[v]);
#pragma unroll
  for (int v = 0; v < 27; ++v) ldT(W, Wd, (9 + v) * nc + c, Gc[v]);
  T acc[9];
#pragma unroll
  for (int v = 0; v < 9; ++v) acc[v] = T(0.0);
  double speed_area = 0.0;

  for (int lf = 0; lf < 6; ++lf) {
    Nbr nb = neighbour(d.g, p, k, j, i, lf);
    V3 S, xf;
    bool own;
    canon_face(d.G, d.g, p, k, j, i, lf, nb, c, S, xf, own);
    T qs[9], qo[9];
    const V3 ds = xf - xc;
#pragma unroll
    for (int v = 0; v < 9; ++v) qs[v] = Pc[v] + (Gc[3 * v] * ds.x + Gc[3 * v + 1] * ds.y + Gc[3 * v + 2] * ds.z);
    if (nb.id >= nc) {
      const int64_t col = (int64_t(p) * d.g.N + j) * d.g.N + i;
      T br;
      if (lf == 0) ldT(d.br, dbr, col, br); else br = T(0.0);
      V3 xG;
      ghost_prims(d, p, k, j, i, lf, Pc, xc, br, qo, xG);
    } else {
      const V3 xn = cell_centre(d.G, d.g, nb.p, nb.k, nb.j, nb.i);
      const V3 dn = xf - xn;
#pragma unroll
      for (int v = 0; v < 9; ++v) {
        T P, gx, gy, gz;
        ldT(W, Wd, v * nc + nb.id, P);
        ldT(W, Wd, (9 + 3 * v) * nc + nb.id, gx);
        ldT(W, Wd, (10 + 3 * v) * nc + nb.id, gy);
        ldT(W, Wd, (11 + 3 * v) * nc + nb.id, gz);
        qo[v] = P + (gx * dn.x + gy * dn.y + gz * dn.z);
      }
    }
    // orientation by value, so that lanes owning and not owning their face
    // (at panel edges) share one code path
    T F[9];
    const T* L = own ? qs : qo;
    const T* R = own ? qo : qs;
    T s = rusanov(L, R, S, F, d.pr);
#pragma unroll
    for (int v = 0; v < 9; ++v) acc[v] += own ? F[v] : -F[v];
    if (kDiag) speed_area += val(s) * norm3(S);
  }
  T u[9], src[9];
#pragma unroll
  for (int v = 0; v < 9; ++v) ldT(U, Ud, v * nc + c, u[v]);
  gravity_source(u, xc, cell_volume(d.G, d.g, p, k, j, i), d.pr.G, src);
#pragma unroll
  for (int v = 0; v < 9; ++v) {
    store_out(R, Rd, v * nc + c, acc[v] - src[v]);
  }
  if (kDiag) diag[c] = speed_area / cfl;
}

template <class T>
__global__ __launch_bounds__(kBlock) void grad_limit_kernel(DevGrid d, const double* __restrict__ U,
                                                            const double* __restrict__ Ud,
                                                            const double* __restrict__ dbr, double* __restrict__ W,
                                                            double* __restrict__ Wd) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c < d.g.ncells) grad_limit_cell<T>(d, U, Ud, dbr, W, Wd, c);
}

template <class T, bool kDiag>
__global__ __launch_bounds__(kBlock) void flux_kernel(DevGrid d, const double* __restrict__ U,
                                                      const double* __restrict__ Ud, const double* __restrict__ dbr,
                                                      const double* __restrict__ W, const double* __restrict__ Wd,
                                                      double* __restrict__ R, double* __restrict__ Rd,
                                                      double* __restrict__ diag, double cfl) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c < d.g.ncells) flux_cell<T, kDiag>(d, U, Ud, dbr, W, Wd, R, Rd, diag, cfl, c);
}

__global__ __launch_bounds__(kBlock) void geometry_kernel(DevGrid d, double* xc, double* vol, double* xf, double* S) {
  const int64_t nc = d.g.ncells;
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  int p, k, j, i;
  decode(d.g, c, p, k, j, i);
  V3 x = cell_centre(d.G, d.g, p, k, j, i);
  xc[3 * c] = x.x; xc[3 * c + 1] = x.y; xc[3 * c + 2] = x.z;
  vol[c] = cell_volume(d.G, d.g, p, k, j, i);
  for (int lf = 0; lf < 6; ++lf) {
    Nbr nb = neighbour(d.g, p, k, j, i, lf);
    V3 s, f;
    bool own;
    canon_face(d.G, d.g, p, k, j, i, lf, nb, c, s, f, own);
    const double sg = own ? 1.0 : -1.0;
    const int64_t o = (c * 6 + lf) * 3;
    S[o] = sg * s.x; S[o + 1] = sg * s.y; S[o + 2] = sg * s.z;
    xf[o] = f.x; xf[o + 1] = f.y; xf[o + 2] = f.z;
  }
}

static inline dim3 grid_for(int64_t n) { return dim3(unsigned((n + kBlock - 1) / kBlock)); }

hipError_t launch_grad_limit_forward(const DevGrid& d, const double* U, double* W, hipStream_t s, KernelTimer* t) {
  TimedScope ts(t, "grad_limit", s);
  hipLaunchKernelGGL((grad_limit_kernel<double>), grid_for(d.g.ncells), dim3(kBlock), 0, s, d, U, nullptr, nullptr,
                     W, nullptr);
  return hipGetLastError();
}

hipError_t launch_local_dt(const DevGrid& d, const double* U, double cfl, double* diag, double* W, hipStream_t s,
                           KernelTimer*) {
  const int64_t nc = d.g.ncells;
  hipLaunchKernelGGL((grad_limit_kernel<double>), grid_for(nc), dim3(kBlock), 0, s, d, U, nullptr, nullptr, W,
                     nullptr);
  hipLaunchKernelGGL((flux_kernel<double, true>), grid_for(nc), dim3(kBlock), 0, s, d, U, nullptr, nullptr, W,
                     nullptr, nullptr, nullptr, diag, cfl);
  return hipGetLastError();
}

hipError_t launch_geometry(const DevGrid& d, double* xc, double* vol, double* xf, double* S, hipStream_t s) {
  hipLaunchKernelGGL(geometry_kernel, grid_for(d.g.ncells), dim3(kBlock), 0, s, d, xc, vol, xf, S);
  return hipGetLastError();
}

}  // namespace cfv
