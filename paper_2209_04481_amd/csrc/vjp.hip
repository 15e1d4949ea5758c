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
//           ghost contributions are folded back through the boundary law into
//           c and the B_r map (each ghost belongs to exactly one cell).
//   pass 3  per cell n: Pb = own[n] + sum over the six neighbours c of
//           out[c][face of c that faces n]; gU = (dP/dU)^T Pb minus the
//           gravity source adjoint.
#include "cfv_adjoint.hpp"
#include "cfv_kernels.hpp"

namespace cfv {

static constexpr int kVBlock = 256;

int64_t vjp_workspace_doubles(const Shape& g) { return int64_t(63) * g.ncells; }

// Adjoint of the ghost law for the ghost of boundary cell (p,k,j,i) across
// face lf: accumulates (dqG/dqI)^T qGb into qIb and returns (dqG/dbr)^T qGb.
__host__ __device__ inline double ghost_adjoint(const DevGrid& d, int p, int k, int j, int i, int lf,
                                                const double qI[9], V3 xI, double br, const double qGb[9],
                                                double qIb[9]) {
  double brb = 0.0;
  const int nin = lf == 0 ? 10 : 9;
  for (int a = 0; a < nin; ++a) {
    Dual q[9], qG[9];
    for (int v = 0; v < 9; ++v) q[v] = Dual(qI[v], v == a ? 1.0 : 0.0);
    Dual b(br, a == 9 ? 1.0 : 0.0);
    V3 xG;
    ghost_prims(d, p, k, j, i, lf, q, xI, b, qG, xG);
    double t = 0.0;
    for (int v = 0; v < 9; ++v) t += qG[v].d * qGb[v];
    if (a < 9) qIb[a] += t; else brb = t;
  }
  return brb;
}

__host__ __device__ inline void adjoint_cell(const DevGrid& d, const double* __restrict__ w,
                                             const double* __restrict__ W, double* __restrict__ A,
                                             double* __restrict__ gbr, int64_t c) {
  const int64_t nc = d.g.ncells;
  int p, k, j, i;
  decode(d.g, c, p, k, j, i);
  const V3 xc = cell_centre(d.G, d.g, p, k, j, i);
  double Pc[9], Gc[27], wc[9];
  for (int v = 0; v < 9; ++v) Pc[v] = W[v * nc + c];
  for (int v = 0; v < 27; ++v) Gc[v] = W[(9 + v) * nc + c];
  for (int v = 0; v < 9; ++v) wc[v] = w[v * nc + c];
  const int64_t col = (int64_t(p) * d.g.N + j) * d.g.N + i;
  const double brc = d.br[col];

  // ---- recompute c's own stencil: offsets, weights, extremes, unlimited gradient
  V3 dx[6], dxf[6];
  double qGin[9], qGout[9];
  for (int lf = 0; lf < 6; ++lf) {
    Nbr nb = neighbour(d.g, p, k, j, i, lf);
    V3 S, xf;
    bool own;
    canon_face(d.G, d.g, p, k, j, i, lf, nb, c, S, xf, own);
    dxf[lf] = xf - xc;
    V3 xn;
    if (nb.id >= nc) {
      ghost_prims(d, p, k, j, i, lf, Pc, xc, lf == 0 ? brc : 0.0, lf == 0 ? qGin : qGout, xn);
    } else {
      xn = cell_centre(d.G, d.g, nb.p, nb.k, nb.j, nb.i);
    }
    dx[lf] = xn - xc;
  }
  const LsqWeights Lw(dx);
  double gxs[9], gys[9], gzs[9], qmax[9], qmin[9];
  int amax[9], amin[9];
  for (int v = 0; v < 9; ++v) {
    gxs[v] = gys[v] = gzs[v] = 0.0;
    qmax[v] = qmin[v] = Pc[v];
    amax[v] = amin[v] = -1;
  }
  for (int lf = 0; lf < 6; ++lf) {
    Nbr nb = neighbour(d.g, p, k, j, i, lf);
    for (int v = 0; v < 9; ++v) {
      const double qn = nb.id >= nc ? (lf == 0 ? qGin : qGout)[v] : W[v * nc + nb.id];
      const double dq = qn - Pc[v];
      gxs[v] += Lw.W[lf].x * dq; gys[v] += Lw.W[lf].y * dq; gzs[v] += Lw.W[lf].z * dq;
      if (!(qmax[v] >= qn)) { qmax[v] = qn; amax[v] = lf; }
      if (!(qmin[v] <= qn)) { qmin[v] = qn; amin[v] = lf; }
    }
  }

  // ---- flux adjoints: own side (and ghost side) of each face
  double Pb[9], Gb[27], PbGin[9], PbGout[9];
  for (int v = 0; v < 9; ++v) Pb[v] = PbGin[v] = PbGout[v] = 0.0;
  for (int v = 0; v < 27; ++v) Gb[v] = 0.0;
  for (int lf = 0; lf < 6; ++lf) {
    Nbr nb = neighbour(d.g, p, k, j, i, lf);
    V3 S, xf;
    bool own;
    canon_face(d.G, d.g, p, k, j, i, lf, nb, c, S, xf, own);
    double qs[9], qo[9], wb[9];
    const V3 ds = dxf[lf];
    for (int v = 0; v < 9; ++v) qs[v] = Pc[v] + (Gc[3 * v] * ds.x + Gc[3 * v + 1] * ds.y + Gc[3 * v + 2] * ds.z);
    const bool ghost = nb.id >= nc;
    if (ghost) {
      for (int v = 0; v < 9; ++v) {
        qo[v] = (lf == 0 ? qGin : qGout)[v];
        wb[v] = wc[v];  // the ghost carries no residual
      }
    } else {
      const V3 dn = xf - cell_centre(d.G, d.g, nb.p, nb.k, nb.j, nb.i);
      for (int v = 0; v < 9; ++v) {
        const int64_t o = nb.id;
        qo[v] = W[v * nc + o] + (W[(9 + 3 * v) * nc + o] * dn.x + W[(10 + 3 * v) * nc + o] * dn.y +
                                 W[(11 + 3 * v) * nc + o] * dn.z);
        const double wn = w[v * nc + o];
        wb[v] = own ? wc[v] - wn : wn - wc[v];  // w_L - w_R
      }
    }
    double qLb[9], qRb[9];
    for (int v = 0; v < 9; ++v) qLb[v] = qRb[v] = 0.0;
    if (own)
      rusanov_adjoint(qs, qo, S, wb, qLb, qRb, d.pr);
    else
      rusanov_adjoint(qo, qs, S, wb, qLb, qRb, d.pr);
    const double* qsb = own ? qLb : qRb;
    for (int v = 0; v < 9; ++v) {
      Pb[v] += qsb[v];
      Gb[3 * v] += qsb[v] * ds.x;
      Gb[3 * v + 1] += qsb[v] * ds.y;
      Gb[3 * v + 2] += qsb[v] * ds.z;
    }
    if (ghost) {
      double* pg = lf == 0 ? PbGin : PbGout;
      for (int v = 0; v < 9; ++v) pg[v] += qRb[v];
    }
  }

  // ---- limiter and gradient adjoint, per variable
  double out[6][9];
  for (int lf = 0; lf < 6; ++lf)
    for (int v = 0; v < 9; ++v) out[lf][v] = 0.0;
  for (int v = 0; v < 9; ++v) {
    const double gx = gxs[v], gy = gys[v], gz = gzs[v];
    double gbx = Gb[3 * v], gby = Gb[3 * v + 1], gbz = Gb[3 * v + 2];
    if (d.pr.limiter) {
      // the same choice as the forward limiter (limited_grad)
      double phi = 1.0, num = 0.0, den = 1.0, bn = 1.0, bd = 1.0;
      int act = -1;
      V3 dact = mk(0.0, 0.0, 0.0);
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        const double d2 = gx * dxf[f].x + gy * dxf[f].y + gz * dxf[f].z;
        if (d2 != 0.0) {
          const double nm = d2 > 0.0 ? qmax[v] - Pc[v] : qmin[v] - Pc[v];
          const double an = ::fabs(nm), ad = ::fabs(d2);
          if (an * bd < bn * ad) {
            bn = an;
            bd = ad;
            num = nm;
            den = d2;
            act = f;
            dact = dxf[f];
          }
        }
      }
      if (act >= 0) phi = num / den;
      const double phib = gbx * gx + gby * gy + gbz * gz;
      gbx *= phi; gby *= phi; gbz *= phi;
      if (act >= 0) {
        const double numb = phib / den;
        const double denb = -phib * phi / den;
        gbx += denb * dact.x; gby += denb * dact.y; gbz += denb * dact.z;
        const int ext = den > 0.0 ? amax[v] : amin[v];
        Pb[v] -= numb;
        if (ext < 0) {
          Pb[v] += numb;
        } else {
          Nbr nb = neighbour(d.g, p, k, j, i, ext);
          if (nb.id >= nc) (ext == 0 ? PbGin : PbGout)[v] += numb;
          else out[ext][v] += numb;
        }
      }
    }
    // g = sum_n W_n (q_n - q_c): q_n gets W_n . gb, the cell minus their sum
    for (int lf = 0; lf < 6; ++lf) {
      const double t = Lw.W[lf].x * gbx + Lw.W[lf].y * gby + Lw.W[lf].z * gbz;
      Pb[v] -= t;
      const bool ghost = (lf == 0 && k == 0) || (lf == 1 && k == d.g.Nr - 1);
      if (ghost) (lf == 0 ? PbGin : PbGout)[v] += t;
      else out[lf][v] += t;
    }
  }

  // ---- ghost laws back onto the cell and the B_r map
  if (k == 0) {
    const double brb = ghost_adjoint(d, p, k, j, i, 0, Pc, xc, brc, PbGin, Pb);
    if (gbr) gbr[col] = brb;
  }
  if (k == d.g.Nr - 1) (void)ghost_adjoint(d, p, k, j, i, 1, Pc, xc, 0.0, PbGout, Pb);

  for (int v = 0; v < 9; ++v) A[v * nc + c] = Pb[v];
  for (int lf = 0; lf < 6; ++lf)
    for (int v = 0; v < 9; ++v) A[(9 + 9 * lf + v) * nc + c] = out[lf][v];
}

__host__ __device__ inline void gather_cell(const DevGrid& d, const double* __restrict__ U,
                                            const double* __restrict__ w, const double* __restrict__ A,
                                            double* __restrict__ gU, int64_t c) {
  const int64_t nc = d.g.ncells;
  int p, k, j, i;
  decode(d.g, c, p, k, j, i);
  double Pb[9];
  for (int v = 0; v < 9; ++v) Pb[v] = A[v * nc + c];
  for (int lf = 0; lf < 6; ++lf) {
    Nbr nb = neighbour(d.g, p, k, j, i, lf);
    if (nb.id >= nc) continue;
    for (int v = 0; v < 9; ++v) Pb[v] += A[(9 + 9 * nb.back + v) * nc + nb.id];
  }
  double u[9], Ub[9];
  for (int v = 0; v < 9; ++v) u[v] = U[v * nc + c];
  prim_adjoint(u, Pb, Ub, d.pr.gamma);
  // source: R -= V (0, rho g, 0, g . m, 0)
  const V3 xc = cell_centre(d.G, d.g, p, k, j, i);
  const double vol = cell_volume(d.G, d.g, p, k, j, i);
  const double r = norm3(xc);
  const double f = -d.pr.G / (r * r * r) * vol;
  const V3 gv = mk(f * xc.x, f * xc.y, f * xc.z);
  const double wE = w[7 * nc + c];
  Ub[0] -= gv.x * w[1 * nc + c] + gv.y * w[2 * nc + c] + gv.z * w[3 * nc + c];
  Ub[1] -= gv.x * wE;
  Ub[2] -= gv.y * wE;
  Ub[3] -= gv.z * wE;
  for (int v = 0; v < 9; ++v) gU[v * nc + c] = Ub[v];
}

__global__ __launch_bounds__(kVBlock) void adjoint_kernel(DevGrid d, const double* __restrict__ w,
                                                          const double* __restrict__ W, double* __restrict__ A,
                                                          double* __restrict__ gbr) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c < d.g.ncells) adjoint_cell(d, w, W, A, gbr, c);
}

__global__ __launch_bounds__(kVBlock) void gather_kernel(DevGrid d, const double* __restrict__ U,
                                                         const double* __restrict__ w, const double* __restrict__ A,
                                                         double* __restrict__ gU) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c < d.g.ncells) gather_cell(d, U, w, A, gU, c);
}

hipError_t launch_vjp(const DevGrid& d, const double* U, const double* w, double* gU, double* gbr, double* W,
                      double* A, hipStream_t s, KernelTimer* t) {
  const int64_t nc = d.g.ncells;
  const dim3 grid(unsigned((nc + kVBlock - 1) / kVBlock));
  hipError_t e = launch_grad_limit_forward(d, U, W, s, t);
  if (e != hipSuccess) return e;
  {
    TimedScope ts(t, "adjoint", s);
    hipLaunchKernelGGL(adjoint_kernel, grid, dim3(kVBlock), 0, s, d, w, W, A, gbr);
  }
  {
    TimedScope ts(t, "adjoint_gather", s);
    hipLaunchKernelGGL(gather_kernel, grid, dim3(kVBlock), 0, s, d, U, w, A, gU);
  }
  return hipGetLastError();
}

}  // namespace cfv
