// Per-cell pieces of the adjoint (vector-Jacobian product) of the residual,
// used by the kernels of vjp.hip and by the host emulation of the kernels.
// The passes and their data flow are described in vjp.hip.
#pragma once
#include "cfv_adjoint.hpp"
#include "cfv_kernels.hpp"
#include "cfv_march.hpp"

namespace cfv {

// 63 adjoint rows, the 54 face-state rows of the forward pass, then the
// adjoints of the inner and outer ghost states (2 x 9 rows of 6N^2)
inline int64_t vjp_workspace_size(const Shape& g) { return int64_t(63 + 54) * g.ncells + 18 * g.nb; }

constexpr int kVBlock = 256;

// Whether the adjoint's window of cells [c0, c0 + kVBlock) holds a cell of
// a boundary layer (k = 0 or Nr - 1): cells run through a panel's layers in
// order, so only the window's first and last cells need looking at.
__host__ __device__ inline bool adjoint_window_has_boundary(const Shape& g, int64_t c0) {
  const int64_t c1 = (c0 + kVBlock < g.ncells ? c0 + kVBlock : g.ncells) - 1;
  const int64_t NN = int64_t(g.N) * g.N, per = NN * g.Nr;
  const int64_t p0 = c0 / per, p1 = c1 / per;
  const int k0 = int((c0 - p0 * per) / NN), k1 = int((c1 - p1 * per) / NN);
  return p0 != p1 || k0 == 0 || k1 == g.Nr - 1;
}


// Adjoint of the ghost law for the ghost of boundary cell (p,k,j,i) across
// face lf: accumulates (dqG/dqI)^T qGb into qIb and returns (dqG/dbr)^T qGb,
// one forward-derivative pass of the ghost law per input.
__host__ __device__ __forceinline__ double ghost_adjoint(const DevGrid& d, int p, int k, int j, int i, int lf,
                                                         const double qI[9], V3 xI, double br, const double qGb[9],
                                                         double qIb[9]) {
  double brb = 0.0;
  const int nin = lf == 0 ? 10 : 9;
#pragma unroll 1
  for (int a = 0; a < nin; ++a) {
    Dual q[9], qG[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) q[v] = Dual(qI[v], v == a ? 1.0 : 0.0);
    const Dual b(br, a == 9 ? 1.0 : 0.0);
    V3 xG;
    ghost_prims(d, p, k, j, i, lf, q, xI, b, qG, xG);
    double t = 0.0;
#pragma unroll
    for (int v = 0; v < 9; ++v) t += qG[v].d * qGb[v];
#pragma unroll
    for (int v = 0; v < 9; ++v) qIb[v] += v == a ? t : 0.0;
    brb = a == 9 ? t : brb;
  }
  return brb;
}

// Pass 2 for cell c.  No local array is indexed by a run-time value (such
// arrays would live in scratch memory): face loops either unroll or branch on
// the face id before touching per-face arrays.  The workgroup's 256
// consecutive cells [c0, c0 + 256) have their workspace rows and weights in
// LDS (lW: primitives and the six reconstructed face states the forward pass
// left in Q; lw: weights); neighbours inside that window are read from there
// (nearly all of the i +- 1 and most of the j +- 1 neighbours), the others
// from global memory.  A neighbour's state on a shared face is its stored
// face state: 9 values instead of its 36 primitives and gradients.  Most of
// this pass's time is neighbour loads at one wavefront per SIMD.
// kBoundary false: the cell is in neither boundary layer (the caller knows),
// so the ghost states and their code are left out.
template <bool kBoundary>
__host__ __device__ inline void adjoint_cell(const DevGrid& d, const double* __restrict__ w,
                                             const double* __restrict__ W, const double* __restrict__ Q,
                                             double* __restrict__ A, double* __restrict__ Gg, int64_t c,
                                             const double* lW, const double* lw, int64_t c0) {
  const int64_t nc = d.g.ncells;
  int p, k, j, i;
  decode(d.g, c, p, k, j, i);
  const bool bin = kBoundary && k == 0, bout = kBoundary && k == d.g.Nr - 1;
  const V3 xc = cell_centre(d.G, d.g, p, k, j, i);
  // rows of cells in the workgroup's window [c0, c0 + kVBlock) come from LDS
  // (one flat load serves either memory: the select stays a single load)
  auto wr = [&](int row, int64_t id) -> double {
    const int64_t l = id - c0;
    return (l >= 0 && l < kVBlock) ? lw[row * kVBlock + l] : w[row * nc + id];
  };
  // state of cell id on its local face lf, as the forward pass reconstructed it
  auto Qr = [&](int lf, int v, int64_t id) -> double {
    const int64_t l = id - c0;
    return (l >= 0 && l < kVBlock) ? lW[(9 + 9 * lf + v) * kVBlock + l] : Q[(9 * lf + v) * nc + id];
  };
  // the LDS window holds copies of global rows, so any row may also be read
  // from global memory: the cell itself always from LDS, radial neighbours
  // (never in the window once a layer has 256 cells) always from global
  // memory, angular ones from wherever they are in the face loop and from
  // global memory in the variable loop (below)
  const int lc = int(c - c0);
  double Pc[9], wc[9];
#pragma unroll
  for (int v = 0; v < 9; ++v) {
    Pc[v] = lW[v * kVBlock + lc];
    wc[v] = lw[v * kVBlock + lc];
  }
  const int64_t col = column_of(d.g, p, j, i);
  const double brc = gld(d.br, col);

  // ---- ghost states, then per face: geometry once and the flux adjoint for
  // this cell's side (and the ghost side); the face loop is unrolled so that
  // per-face arrays are indexed statically and faces can overlap
  double qGin[9], qGout[9];
  if (!kBoundary)  // no ghost in an interior window: the ghost paths below are never taken
#pragma unroll
    for (int v = 0; v < 9; ++v) qGin[v] = qGout[v] = 0.0;
  if (bin) {
    V3 xG;
    ghost_prims(d, p, k, j, i, 0, Pc, xc, brc, qGin, xG);
  }
  if (bout) {
    V3 xG;
    ghost_prims(d, p, k, j, i, 1, Pc, xc, 0.0, qGout, xG);
  }
  V3 dx[6], dxf[6];
  int64_t nid[6];
  double Pb[9], Gb[27], PbGin[9], PbGout[9];
#pragma unroll
  for (int v = 0; v < 9; ++v) Pb[v] = PbGin[v] = PbGout[v] = 0.0;
#pragma unroll
  for (int v = 0; v < 27; ++v) Gb[v] = 0.0;
#pragma unroll
  for (int lf = 0; lf < 6; ++lf) {
    const Nbr nb = neighbour(d.g, p, k, j, i, lf);
    V3 S, xf;
    bool own;
    canon_face(d.G, d.g, p, k, j, i, lf, nb, c, S, xf, own);
    const V3 ds = xf - xc;
    dxf[lf] = ds;
    nid[lf] = nb.id;
    const bool ghost = nb.id >= nc;
    V3 xn;
    if (ghost)
      xn = ghost_centre(xc, S, xf);
    else
      xn = cell_centre(d.G, d.g, nb.p, nb.k, nb.j, nb.i);
    dx[lf] = xn - xc;
    double qs[9], qo[9], wb[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) qs[v] = lW[(9 + 9 * lf + v) * kVBlock + lc];
    if (ghost) {
#pragma unroll
      for (int v = 0; v < 9; ++v) {
        qo[v] = lf == 0 ? qGin[v] : qGout[v];
        wb[v] = wc[v];  // the ghost carries no residual
      }
    } else {
      const int64_t o = nb.id;
      // w_L - w_R: (wc - wn) signed by the orientation (a product, the same
      // bits as the other difference, instead of two differences and a select)
      const double sg = own ? 1.0 : -1.0;
      // the neighbour's state on this face, as the forward pass reconstructed it
#pragma unroll
      for (int v = 0; v < 9; ++v) {
        qo[v] = lf < 2 ? gld(Q, (9 * nb.back + v) * nc + o) : Qr(nb.back, v, o);
        const double wn = lf < 2 ? gld(w, v * nc + o) : wr(v, o);
        wb[v] = (wc[v] - wn) * sg;
      }
    }
    double qLb[9], qRb[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) qLb[v] = qRb[v] = 0.0;
    // this cell's side (into qLb whatever its orientation: the owner is not
    // the same on every lane's face at panel edges, and one code path keeps
    // such wavefronts from running both), and the ghost side on a boundary
    // face, which this cell always owns
    if (ghost)
      rusanov_adjoint(qs, qo, S, wb, qLb, qRb, d.pr, true, true);
    else
      rusanov_adjoint_side(qs, qo, S, wb, qLb, d.pr, own);
#pragma unroll
    for (int v = 0; v < 9; ++v) {
      const double qsb = qLb[v];
      Pb[v] += qsb;
      Gb[3 * v] += qsb * ds.x;
      Gb[3 * v + 1] += qsb * ds.y;
      Gb[3 * v + 2] += qsb * ds.z;
      if (ghost) {
        if (lf == 0) PbGin[v] += qRb[v];
        else PbGout[v] += qRb[v];
      }
    }
  }
  const LsqWeights Lw(dx);

  // ---- per variable: recompute the gradient and limiter choice, then their
  // adjoint; contributions to the six neighbours are stored at once.  The
  // neighbours' values of variable v + 2 are loaded before variable v's
  // arithmetic, so the loads of later variables are in flight while earlier
  // ones compute (one wait per variable had left them exposed).  They are
  // global loads even inside the window (cache hits there): a value from a
  // flat load can only be waited for together with every memory access in
  // flight, the prefetched ones included.
  auto neighbour_values = [&](int v, double q[6]) {
#pragma unroll
    for (int lf = 0; lf < 6; ++lf) {
      if (lf == 0 && bin) q[lf] = qGin[v];
      else if (lf == 1 && bout) q[lf] = qGout[v];
      else q[lf] = gld(W, v * nc + nid[lf]);
    }
  };
  double qn1[6], qn2[6];  // variables v + 1 and v + 2
  neighbour_values(0, qn1);
  neighbour_values(1, qn2);
#pragma unroll
  for (int v = 0; v < 9; ++v) {
    double qn[6];
#pragma unroll
    for (int lf = 0; lf < 6; ++lf) {
      qn[lf] = qn1[lf];
      qn1[lf] = qn2[lf];
    }
    if (v + 2 < 9) neighbour_values(v + 2, qn2);
    const double qc = Pc[v];
    double gx = 0.0, gy = 0.0, gz = 0.0, qmax = qc, qmin = qc;
    int amax = -1, amin = -1;
#pragma unroll
    for (int lf = 0; lf < 6; ++lf) {
      const double dq = qn[lf] - qc;
      gx += Lw.W[lf].x * dq; gy += Lw.W[lf].y * dq; gz += Lw.W[lf].z * dq;
      if (!(qmax >= qn[lf])) { qmax = qn[lf]; amax = lf; }
      if (!(qmin <= qn[lf])) { qmin = qn[lf]; amin = lf; }
    }
    double gbx = Gb[3 * v], gby = Gb[3 * v + 1], gbz = Gb[3 * v + 2];
    double o[6];
#pragma unroll
    for (int lf = 0; lf < 6; ++lf) o[lf] = 0.0;
    double pb = Pb[v];
    if (d.pr.limiter) {
      // the choice of the dual limiter (limited_grad): the face with the
      // largest positive projection or the one with the most negative (the
      // first of equal ones), an exact tie between them to the earlier face
      double dhi = 0.0, dlo = 0.0;
      int fhi = 6, flo = 6;
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        const double d2 = gx * dxf[f].x + gy * dxf[f].y + gz * dxf[f].z;
        if (d2 > dhi) { dhi = d2; fhi = f; }
        if (d2 < dlo) { dlo = d2; flo = f; }
      }
      const double up = qmax - qc, down = qc - qmin;
      double bn = 1.0, bd = 1.0;
      int pick = 0;
      if (up * bd < bn * dhi) {
        bn = up;
        bd = dhi;
        pick = 1;
      }
      const double lhs = down * bd, rhs = bn * -dlo;
      if (lhs < rhs || (lhs == rhs && pick == 1 && flo < fhi)) pick = 2;
      const int act = pick == 1 ? fhi : pick == 2 ? flo : -1;
      const double num = pick == 1 ? qmax - qc : qmin - qc;
      const double den = pick == 1 ? dhi : pick == 2 ? dlo : 1.0;
      // phi as limited_grad takes it (num and den share their sign)
      const double rd = recip(den);
      const double phi = act >= 0 ? ratio_refined(num, den) : 1.0;
      const double phib = gbx * gx + gby * gy + gbz * gz;
      gbx *= phi; gby *= phi; gbz *= phi;
      if (act >= 0) {
        const double numb = phib * rd;
        const double denb = -phib * phi * rd;
        // den = g . dxf[act] (a masked sum, not dxf[act]: a run-time index
        // would put the array in scratch)
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          const double wf = f == act ? denb : 0.0;
          gbx += wf * dxf[f].x; gby += wf * dxf[f].y; gbz += wf * dxf[f].z;
        }
        const int ext = den > 0.0 ? amax : amin;
        pb -= numb;
        if (ext < 0) pb += numb;
#pragma unroll
        for (int lf = 0; lf < 6; ++lf)
          if (ext == lf) o[lf] += numb;
      }
    }
    // g = sum_n W_n (q_n - q_c): q_n gets W_n . gb, the cell minus their sum
#pragma unroll
    for (int lf = 0; lf < 6; ++lf) {
      const double t = Lw.W[lf].x * gbx + Lw.W[lf].y * gby + Lw.W[lf].z * gbz;
      pb -= t;
      o[lf] += t;
    }
    Pb[v] = pb;
    // ghost positions fold back below; cell positions go to the gather pass
#pragma unroll
    for (int v2 = 0; v2 < 9; ++v2) {
      if (v2 != v) continue;
      if (bin) PbGin[v2] += o[0];
      if (bout) PbGout[v2] += o[1];
    }
    gst(A, (9 + v) * nc + c, bin ? 0.0 : o[0]);
    gst(A, (18 + v) * nc + c, bout ? 0.0 : o[1]);
#pragma unroll
    for (int lf = 2; lf < 6; ++lf) gst(A, (9 + 9 * lf + v) * nc + c, o[lf]);
  }

  // ---- ghost laws back onto the cell and the B_r map
  // the ghost states' adjoints go back through the boundary laws in a pass
  // of their own (ghost_fold_kernel), which keeps that code out of this one
  if (bin)
#pragma unroll
    for (int v = 0; v < 9; ++v) gst(Gg, v * d.g.nb + col, PbGin[v]);
  if (bout)
#pragma unroll
    for (int v = 0; v < 9; ++v) gst(Gg, (9 + v) * d.g.nb + col, PbGout[v]);
#pragma unroll
  for (int v = 0; v < 9; ++v) gst(A, v * nc + c, Pb[v]);
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

// Per boundary column: the adjoints of the inner and outer ghost states
// through the boundary laws, onto the boundary cell (its own adjoint row) and
// the B_r map.  Both sides in order (a one-layer shell has one cell for both).
__host__ __device__ inline void ghost_fold_column(const DevGrid& d, const double* __restrict__ W,
                                                  const double* __restrict__ Gg, double* __restrict__ A,
                                                  double* __restrict__ gbr, int64_t col) {
  const int64_t nc = d.g.ncells;
  const int p = int(col / (int64_t(d.g.N) * d.g.N));
  const int rest = int(col - int64_t(p) * d.g.N * d.g.N);
  const int j = rest / d.g.N, i = rest - j * d.g.N;
#pragma unroll 1
  for (int side = 0; side < 2; ++side) {
    const int k = side == 0 ? 0 : d.g.Nr - 1;
    const int64_t c = cell_index(d.g, p, k, j, i);
    double Pc[9], qGb[9], dPb[9];
    for (int v = 0; v < 9; ++v) {
      Pc[v] = W[v * nc + c];
      qGb[v] = Gg[(9 * side + v) * d.g.nb + col];
      dPb[v] = 0.0;
    }
    const V3 xc = cell_centre(d.G, d.g, p, k, j, i);
    const double brb = ghost_adjoint(d, p, k, j, i, side, Pc, xc, side == 0 ? gld(d.br, col) : 0.0, qGb, dPb);
    for (int v = 0; v < 9; ++v) A[v * nc + c] += dPb[v];
    if (side == 0 && gbr) gbr[col] = brb;
  }
}

}  // namespace cfv
