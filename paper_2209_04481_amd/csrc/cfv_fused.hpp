// Phase functions of the fused radial march (fused.hip): per layer, the
// limited gradients, face states, face fluxes and the residual of a tile in
// one pass, so that HBM sees U read and R written and nothing between.
//
// A workgroup's 16 x 16 lanes are a block of columns: the inner 14 x 14 are
// the tile (its residual is computed) and the lanes around them hold the ring
// of out-of-tile face neighbours, whose limited gradients give their states
// on the tile's edge faces.  Every lane computes one gradient per layer
// (inner and ring lanes alike, so the wavefronts stay balanced).  Across
// panel edges and cube corners the ring cells lie in other panels with their
// own orientation; which cell each ring lane holds, where its angular
// neighbours are (block lanes or a further layer of 64 outer slots) and which
// of its faces it shares with the tile come from a per-tile table built on
// the host (cfv_grid).
//
// The primitives of three layers (k - 1, k, k + 1) of the block live in LDS,
// so nothing per cell is carried in registers across layers except the
// state on the cell's top face and its partial residual.  The next layer's
// conservative state is loaded one layer ahead (prefetch into registers).
//
// Everything here is __host__ __device__; the device glue is in fused.hip.
#pragma once
#include "cfv_march.hpp"

namespace cfv {

constexpr int kFB = 16;               // block width (lanes per row)
constexpr int kFT = kFB - 2;          // inner tile width
constexpr int kFL = kFB * kFB;        // lanes per workgroup
constexpr int kOuterSlots = 64;       // further neighbours of ring cells

// ---------------------------------------------------------- stencil table
// Per tile (p, tile j, tile i), kFTab int32:
//   bcol[256]    column of the cell lane (bi, bj) holds (-1: none)
//   bnb[256][4]  ring lanes: positions of the cell's four angular neighbours
//                in its own local face order (W, E, S, N of its panel):
//                0..255 a block lane, 256 + e an outer slot
//   bback[256]   ring lanes: the cell's local face (2..5) shared with the tile
//   ocol[64]     column of outer slot e (-1: unused)
constexpr int kFTabCol = 0, kFTabNb = kFL, kFTabBack = kFTabNb + 4 * kFL, kFTabOcol = kFTabBack + kFL;
constexpr int kFTab = kFTabOcol + kOuterSlots;

__host__ __device__ __forceinline__ int fused_tiles_1d(int N) { return (N + kFT - 1) / kFT; }
__host__ __device__ __forceinline__ int64_t fused_tile_count(const Shape& g) {
  return 6 * int64_t(fused_tiles_1d(g.N)) * fused_tiles_1d(g.N);
}
__host__ __device__ __forceinline__ int fused_chunks(const Shape& g, int kc) { return (g.Nr + kc - 1) / kc; }
__host__ __device__ __forceinline__ int64_t fused_items(const Shape& g, int kc) {
  return fused_tile_count(g) * fused_chunks(g, kc);
}

struct FTile {
  int p, j0, i0, k0, k1, wi, wj;  // panel, inner origin, chunk [k0, k1), inner widths
  int64_t id;                     // tile index into the table
};

// item l (chunk fastest, then tile i, tile j, panel)
__host__ __device__ __forceinline__ void fused_tile_of(const Shape& g, int kc, int64_t l, FTile& tm) {
  const int nt = fused_tiles_1d(g.N), nch = fused_chunks(g, kc);
  const int ch = int(l % nch);
  const int64_t tile = l / nch;
  const int ti = int(tile % nt), tj = int((tile / nt) % nt);
  tm.p = int(tile / (int64_t(nt) * nt));
  tm.id = tile;
  tm.i0 = ti * kFT;
  tm.j0 = tj * kFT;
  tm.wi = g.N - tm.i0 < kFT ? g.N - tm.i0 : kFT;
  tm.wj = g.N - tm.j0 < kFT ? g.N - tm.j0 : kFT;
  tm.k0 = ch * kc;
  tm.k1 = tm.k0 + kc < g.Nr ? tm.k0 + kc : g.Nr;
}

// lane roles: 1 inner (a tile cell), 2 ring (a face neighbour of the tile across
// one of its edges), 0 none (block corners and lanes beyond a partial tile)
__host__ __device__ __forceinline__ int fused_role(int bi, int bj, int wi, int wj) {
  const bool ii = bi >= 1 && bi <= wi, jj = bj >= 1 && bj <= wj;
  if (ii && jj) return 1;
  if ((ii && (bj == 0 || bj == wj + 1)) || (jj && (bi == 0 || bi == wi + 1))) return 2;
  return 0;
}

// ---------------------------------------------------------- per-lane state
template <class T>
struct FuState {
  int bi, bj, role;
  int p, j, i;       // the lane's cell (a ring cell in its own panel's coordinates)
  int64_t col;
  int nb[4];         // positions of the angular neighbours (local face order)
  int32_t ncol[4];   // columns of the angular neighbours
  V3 cc;             // the column's centroid sum: a layer's centroid is rs_k cc
  V3 dn[4], fe[4];   // per unit rs_k: angular neighbours' centroid and face-centroid offsets
  V3 fw;             // per unit rs_k: the centroid offset of an inner lane's west face, a ring lane's shared face
  V3 fa, na;         // area vectors per unit (r_k+1^2 - r_k^2) / 2 of the flux phase's first and second faces
  bool fown, nown;   // and whether their table orientation points away from the evaluating cell
  V3 sr, xr;         // radial faces per unit radius: area vector r^2 sr, centroid r xr
  double om;         // the column's solid-angle factor: volume (r_k+1^3 - r_k^3) om / 3
  int32_t fcol;      // west / south ring lanes: the column of the inner cell across the shared face
  int back;          // ring: the local face shared with the tile
  int64_t obase;     // the outer slot this lane loads (lanes 0..63): its cell at layer 0, -1: none
  bool bad;          // met a non-physical face state
  T Un[9];           // conservative state of the next layer (prefetched)
  T On[9];           // the outer slot's conservative state of the next layer
  T qtop[9];         // state of layer k-1 on its top face (inner lanes)
  T acc[9];          // residual of layer k-1 without its top face, then of layer k
  T qE[9], qN[9];    // states on the east and north faces of layer k (inner lanes)
};

// Geometry of a cell's gradient stencil at layer k: centroid, offsets of the
// six neighbours' centroids (mirrored ghost centres on the boundary) and of
// the six face centroids.  The shell is separable: a layer's centroid is
// rs_k cc (rs_k = (r_k + r_k+1) / 8, cc the column's centroid sum) and an
// angular face's centroid 2 rs_k b_q, so the angular offsets are rs_k times
// per-column constants (dn, fe) that the work item loads once.
__host__ __device__ __forceinline__ void stencil_geometry(const GeomRef& G, const Shape& g, int k, V3 cc, V3 sr,
                                                          V3 xr, const V3 dn[4], const V3 fe[4], V3& xc, V3 dx[6],
                                                          V3 dxf[6]) {
  const double r0 = radius_uniform(G, k), r1 = radius_uniform(G, k + 1);
  const double rs = 0.125 * (r0 + r1);
  xc = rs * cc;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    dx[2 + q] = rs * dn[q];
    dxf[2 + q] = rs * fe[q];
  }
  const V3 xf0 = r0 * xr, xf1 = r1 * xr;
  dxf[0] = xf0 - xc;
  dxf[1] = xf1 - xc;
  if (k > 0) {
    dx[0] = (0.125 * (radius_uniform(G, k - 1) + r0) - rs) * cc;
  } else {
    dx[0] = ghost_centre(xc, (r0 * r0) * sr, xf0) - xc;
  }
  if (k + 1 < g.Nr) {
    dx[1] = (0.125 * (r1 + radius_uniform(G, k + 2)) - rs) * cc;
  } else {
    dx[1] = ghost_centre(xc, (r1 * r1) * sr, xf1) - xc;
  }
}

template <class T>
__host__ __device__ __forceinline__ void load_cons(const MarchArgs& a, int64_t c, T u[9]) {
  for (int v = 0; v < 9; ++v) ldT(a.U, a.Ud, v * a.d.g.ncells + c, u[v]);
}

template <class T>
struct FusedWG {
  // LDS in units of T: block primitives of three layers (rotating by k mod 3,
  // 3 x 9 x 256), outer slots of layer k (9 rows of 64 at the planes' row
  // stride of 256, so that a neighbour's nine values sit at one base plus
  // fixed offsets whether it is a block lane or an outer slot), the exchanged face states
  // (west: inner lanes' west state, ring lanes' state on the shared face;
  // south: inner lanes' south state; 9 x 256 each), and the face fluxes
  // signed from lane t toward its east (t + 1) and north (t + 16) neighbour
  // (9 x 256 each)
  static constexpr int kPL = 0, kPO = kPL + 3 * 9 * kFL, kSW = kPO + 9 * kFL, kSS = kSW + 9 * kFL,
                       kFE = kSS + 9 * kFL, kFN = kFE + 9 * kFL, kTot = kFN + 9 * kFL;
  static constexpr int kLds = kTot * int(sizeof(T) / sizeof(double));

  __host__ __device__ static const int32_t* table(const MarchArgs& a, const FTile& tm) {
    return a.d.ftab + tm.id * kFTab;
  }
  __host__ __device__ static int plane(int k) { return kPL + (k % 3) * 9 * kFL; }

  // ---------------------------------------------------------------- init
  __host__ __device__ static void init(const MarchArgs& a, const FTile& tm, FuState<T>& st, int t, int kb,
                                       double* lds) {
    const Shape& g = a.d.g;
    const GeomRef& G = a.d.G;
    const int32_t* tab = table(a, tm);
    st.bi = t % kFB;
    st.bj = t / kFB;
    st.role = fused_role(st.bi, st.bj, tm.wi, tm.wj);
    st.bad = false;
    const int32_t col = gld(tab + kFTabCol, t);
    // a lane without a cell works on the tile's first cell (results unused)
    st.col = col >= 0 ? col : column_of(g, tm.p, tm.j0, tm.i0);
    column_pji(g, st.col, st.p, st.j, st.i);
    if (st.role == 2) {
      for (int q = 0; q < 4; ++q) st.nb[q] = gld(tab + kFTabNb, 4 * t + q);
      st.back = gld(tab + kFTabBack, t);
    } else {
      const int tt = st.role == 1 ? t : (kFB + 1);  // inner lanes' neighbours in the block
      st.nb[0] = tt - 1;
      st.nb[1] = tt + 1;
      st.nb[2] = tt - kFB;
      st.nb[3] = tt + kFB;
      st.back = 2;
    }
    const int64_t ocol = t < kOuterSlots ? int64_t(gld(tab + kFTabOcol, t)) : -1;
    st.obase = -1;
    if (ocol >= 0) {
      int op, oj, oi;
      column_pji(g, ocol, op, oj, oi);
      st.obase = cell_index(g, op, 0, oj, oi);
    }
    // per-item constants the layers reuse (loaded once, not per layer)
    for (int q = 0; q < 4; ++q) st.ncol[q] = gld(G.cn, q * G.ncol + st.col);
    st.cc = cg3(G, CG_CSUM, st.col);
    {
      const int bq = (st.role == 1 ? 2 : st.back) - 2;  // the face, 0..3 (a lane without a cell: west)
      st.fw = 2.0 * cg3(G, CG_ANG + 6 * (bq >= 0 && bq < 4 ? bq : 0) + 3, st.col) - st.cc;
    }
    st.sr = cg3(G, CG_SR, st.col);
    st.xr = cg3(G, CG_XR, st.col);
    st.om = gld(G.cg, CG_OMEGA * G.ncol + st.col);
    for (int q = 0; q < 4; ++q) {
      st.dn[q] = cg3(G, CG_CSUM, st.ncol[q]) - st.cc;
      st.fe[q] = 2.0 * cg3(G, CG_ANG + 6 * q + 3, st.col) - st.cc;
    }
    st.fcol = st.role == 2 && (st.bi == 0 || st.bj == 0) ? gld(tab + kFTabCol, st.bi == 0 ? t + 1 : t + kFB) : 0;
    {
      // the flux phase's faces: an inner lane's east (q = 1) and north (3)
      // faces, an edge ring lane's inner neighbour's west (0) or south (2)
      const bool inner = st.role == 1;
      const int64_t fc = inner ? st.col : int64_t(st.fcol);
      const int fq = inner ? 1 : st.bi == 0 ? 0 : 2;
      st.fa = cg3(G, CG_ANG + 6 * fq, fc);
      st.fown = (gld(G.cn, (4 + fq) * G.ncol + fc) >> 8) != 0;
      st.na = cg3(G, CG_ANG + 6 * 3, st.col);
      st.nown = (gld(G.cn, (4 + 3) * G.ncol + st.col) >> 8) != 0;
    }
    // the first layer the block publishes (the planes of layers kb - 1 and
    // kb fill through publish_block steps before layer kb, the same code as
    // every later layer's, so that every plane holds the same bits whatever
    // the chunk length); its state loaded ahead
    (void)lds;
    load_cons(a, cell_index(g, st.p, kb > 0 ? kb - 1 : 0, st.j, st.i), st.Un);
    if (st.obase >= 0) load_cons(a, st.obase + int64_t(kb) * g.N * g.N, st.On);
  }

  // the publish steps before layer kb: k = first_publish(kb) .. kb - 1
  __host__ __device__ static int first_publish(int kb) { return (kb > 0 ? kb - 1 : 0) - 1; }

  // ------------------------------------------------------------- publish
  // Step k: the prefetched layer k + 1 of the block to LDS (as primitives),
  // then the load of layer k + 2; and (publish) layer k of the outer slots,
  // then the load of their layer k + 1.
  __host__ __device__ static void publish_block(const MarchArgs& a, FuState<T>& st, int t, int k, double* lds) {
    const Shape& g = a.d.g;
    T* L = lds_as<T>(lds);
    if (k + 1 < g.Nr) {
      T q[9];
      cons_to_prim(st.Un, q, a.d.pr.gamma);
      for (int v = 0; v < 9; ++v) L[plane(k + 1) + v * kFL + t] = q[v];
      if (k + 2 < g.Nr) load_cons(a, cell_index(g, st.p, k + 2, st.j, st.i), st.Un);
    }
  }

  __host__ __device__ static void publish(const MarchArgs& a, const FTile& tm, FuState<T>& st, int t, int k,
                                          double* lds) {
    const Shape& g = a.d.g;
    T* L = lds_as<T>(lds);
    publish_block(a, st, t, k, lds);
    if (st.obase >= 0) {
      T q[9];
      cons_to_prim(st.On, q, a.d.pr.gamma);
      for (int v = 0; v < 9; ++v) L[kPO + v * kFL + t] = q[v];
      if (k + 1 < g.Nr) load_cons(a, st.obase + int64_t(k + 1) * g.N * g.N, st.On);
    }
    (void)tm;
  }

  // value of variable v of layer k at block position pos (or outer slot)
  __host__ __device__ static T at(const T* L, int pos, int v, int k) {
    return L[(pos < kFL ? plane(k) + pos : kPO + (pos - kFL)) + v * kFL];
  }

  // -------------------------------------------------------------- gradient
  // The lane's cell at layer k: its limited gradient and face states.
  // mode 0 (main layer): inner lanes keep the bottom, top, east and north
  // states, put the west and south states in LDS, take the bottom face's flux
  // (closing layer k - 1), the boundary faces and gravity; ring lanes put
  // their state on the face they share with the tile in LDS.  mode 1
  // (warm-up, the layer below the chunk): inner lanes keep the top state.
  // mode 2 (cool-down, the layer above the chunk): inner lanes close the
  // chunk's last layer with the bottom face's flux.
  __host__ __device__ static void gradient(const MarchArgs& a, const FTile& tm, FuState<T>& st, int t, int k,
                                           int mode, double* lds) {
    const Shape& g = a.d.g;
    const GeomRef& G = a.d.G;
    T* L = lds_as<T>(lds);
    V3 xc, dx[6], dxf[6];
    stencil_geometry(G, g, k, st.cc, st.sr, st.xr, st.dn, st.fe, xc, dx, dxf);
    const LsqWeights W(dx);
    T P0[9];
    for (int v = 0; v < 9; ++v) P0[v] = L[plane(k) + v * kFL + t];
    T gin[9], gout[9];
    if (k == 0) {
      V3 xG;
      ghost_prims(a.d, st.p, k, st.j, st.i, 0, P0, xc, map_br<T>(a, st.col), gin, xG);
    }
    if (k + 1 == g.Nr) {
      V3 xG;
      ghost_prims(a.d, st.p, k, st.j, st.i, 1, P0, xc, T(0.0), gout, xG);
    }
    const bool inner = st.role == 1;
    // the west face of an inner lane, the shared face of a ring lane: its
    // centroid offset, rs_k times the item's constant (indexing dxf by a
    // run-time face would put the array in scratch memory)
    const V3 dw = (0.125 * (radius_uniform(G, k) + radius_uniform(G, k + 1))) * st.fw;
    T qB[9], qT[9];
#pragma unroll
    for (int v = 0; v < 9; ++v) {
      T qn[6];
      qn[0] = k > 0 ? L[plane(k - 1) + v * kFL + t] : gin[v];
      qn[1] = k + 1 < g.Nr ? L[plane(k + 1) + v * kFL + t] : gout[v];
#pragma unroll
      for (int q = 0; q < 4; ++q) qn[2 + q] = at(L, st.nb[q], v, k);
      T gx, gy, gz;
      limited_grad(W, dxf, a.d.pr.limiter, P0[v], qn, gx, gy, gz);
      const T p0 = P0[v];
      // every mode computes and publishes the same states (the warm-up and
      // cool-down layers' are overwritten before any flux phase reads them):
      // no branch on the mode here, so one code path, and one rounding,
      // serves every layer whatever the chunk length
      qB[v] = p0 + (gx * dxf[0].x + gy * dxf[0].y + gz * dxf[0].z);
      qT[v] = p0 + (gx * dxf[1].x + gy * dxf[1].y + gz * dxf[1].z);
      st.qE[v] = p0 + (gx * dxf[3].x + gy * dxf[3].y + gz * dxf[3].z);
      st.qN[v] = p0 + (gx * dxf[5].x + gy * dxf[5].y + gz * dxf[5].z);
      const T qW = p0 + (gx * dw.x + gy * dw.y + gz * dw.z);  // a ring lane's: on the shared face
      const T qS = p0 + (gx * dxf[4].x + gy * dxf[4].y + gz * dxf[4].z);
      L[kSW + v * kFL + t] = qW;
      L[kSS + v * kFL + t] = qS;
    }
    if (!inner) return;
    if (mode == 1) {  // warm-up: the top state only
      for (int v = 0; v < 9; ++v) st.qtop[v] = qT[v];
      return;
    }
    if (k == 0) st.bad = st.bad || !physical(gin);
    st.bad = st.bad || !physical(qB);
    // the bottom face closes layer k - 1 (stored when the chunk owns it)
    {
      const double r0 = radius_uniform(G, k);
      V3 S = (r0 * r0) * st.sr;
      if (k == 0) S = mk(-S.x, -S.y, -S.z);  // the inner boundary face, outward
      T F[9];
      if (k == 0) {
        rusanov(qB, gin, S, F, a.d.pr);
        for (int v = 0; v < 9; ++v) st.acc[v] = F[v];
      } else {
        rusanov(st.qtop, qB, S, F, a.d.pr);
        if (k - 1 >= tm.k0) {
          for (int v = 0; v < 9; ++v) st.acc[v] += F[v];
          store_res(a, cell_index(g, st.p, k - 1, st.j, st.i), st.acc);
        }
        for (int v = 0; v < 9; ++v) st.acc[v] = -F[v];
      }
    }
    if (mode == 2) return;
    st.bad = st.bad || !physical(qT) || !physical(st.qE) || !physical(st.qN);
    {
      T w[9], s[9];
      for (int v = 0; v < 9; ++v) {
        w[v] = L[kSW + v * kFL + t];
        s[v] = L[kSS + v * kFL + t];
      }
      st.bad = st.bad || !physical(w) || !physical(s);
    }
    // gravity: R -= V S(U) at the centroid, from the cell's primitives
    {
      T u[9], src[9];
      u[0] = P0[0];
      for (int d = 1; d < 4; ++d) u[d] = P0[0] * P0[d];
      for (int v = 4; v < 9; ++v) u[v] = T(0.0);
      const double r0 = radius_uniform(G, k), r1 = radius_uniform(G, k + 1);
      gravity_source(u, xc, (r1 * r1 * r1 - r0 * r0 * r0) * st.om * (1.0 / 3.0), a.d.pr.G, src);
      for (int v = 0; v < 9; ++v) st.acc[v] -= src[v];
    }
    for (int v = 0; v < 9; ++v) st.qtop[v] = qT[v];
    if (k == g.Nr - 1) {  // the outer boundary face
      st.bad = st.bad || !physical(gout);
      V3 S, xf;
      bool own;
      canon_face<true>(G, g, st.p, k, st.j, st.i, 1, Nbr{}, 0, S, xf, own);
      T F[9];
      rusanov(qT, gout, S, F, a.d.pr);
      for (int v = 0; v < 9; ++v) st.acc[v] += F[v];
    }
  }

  // ---------------------------------------------------------------- flux
  // Inner lanes: the east and north faces (the neighbour's state from LDS:
  // an inner cell's west or south state, or a ring cell's shared-face state).
  // West and south ring lanes: the tile's west and south edge faces.  Each
  // flux is stored signed from this lane toward its east or north neighbour.
  __host__ __device__ static void flux(const MarchArgs& a, const FTile& tm, FuState<T>& st, int t, int k,
                                       double* lds) {
    const GeomRef& G = a.d.G;
    T* L = lds_as<T>(lds);
    const int bi = st.bi, bj = st.bj;
    const bool inner = st.role == 1;
    // First face, one evaluation for both kinds of lane (a wavefront holds
    // both): an inner lane's east face, or the face between a west (south)
    // ring lane and the inner cell east (north) of it, in that inner cell's
    // frame.  Stored signed from the lane toward its east or north neighbour.
    if (inner || (st.role == 2 && (bi == 0 || bj == 0))) {
      const bool west = bi == 0;
      const int tn = inner ? t + 1 : west ? t + 1 : t + kFB;  // the other side's lane
      const double r0 = radius_uniform(G, k), r1 = radius_uniform(G, k + 1);
      const V3 S = (0.5 * (r1 * r1 - r0 * r0)) * st.fa;
      const bool own = st.fown;
      T qs[9], qo[9], F[9];
      for (int v = 0; v < 9; ++v) {
        qs[v] = inner ? st.qE[v] : L[(west ? kSW : kSS) + v * kFL + tn];
        qo[v] = L[kSW + v * kFL + (inner ? tn : t)];
      }
      face_flux(own, qs, qo, S, F, a.d.pr);
      // an inner lane's flux leaves it eastward; a ring lane's leaves the
      // inner cell through its west / south face, toward the ring lane
      const bool neg = inner ? !own : own;
      const double sg = neg ? -1.0 : 1.0;  // a product by +-1: the same bits as the negation
      for (int v = 0; v < 9; ++v) {
        const T f = F[v] * sg;
        if (inner) st.acc[v] += f;
        L[(inner || west ? kFE : kFN) + v * kFL + t] = f;
      }
    }
    // second face: an inner lane's north face
    if (inner) {
      const double r0 = radius_uniform(G, k), r1 = radius_uniform(G, k + 1);
      const V3 S = (0.5 * (r1 * r1 - r0 * r0)) * st.na;
      const bool own = st.nown;
      const bool ring_n = bj == tm.wj;  // the north neighbour is a ring cell: its shared-face state
      T qo[9], F[9];
      for (int v = 0; v < 9; ++v) qo[v] = L[(ring_n ? kSW : kSS) + v * kFL + t + kFB];
      face_flux(own, st.qN, qo, S, F, a.d.pr);
      const double sg = own ? 1.0 : -1.0;
      for (int v = 0; v < 9; ++v) {
        const T f = F[v] * sg;
        st.acc[v] += f;
        L[kFN + v * kFL + t] = f;
      }
    }
  }

  // ---------------------------------------------------------- accumulate
  // Inner lanes: the fluxes from the west and south neighbours; the layer's
  // residual then waits for its top face (next layer), except the outermost.
  // Runs after the next layer's first barrier (the flux buffers are written
  // again only after its second), or after a barrier of its own when no layer
  // follows.
  __host__ __device__ static void accumulate(const MarchArgs& a, const FTile& tm, FuState<T>& st, int t, int k,
                                             double* lds) {
    if (st.role != 1) return;
    const T* L = lds_as<T>(lds);
    for (int v = 0; v < 9; ++v) st.acc[v] -= L[kFE + v * kFL + t - 1] + L[kFN + v * kFL + t - kFB];
    if (k == a.d.g.Nr - 1) store_res(a, cell_index(a.d.g, st.p, k, st.j, st.i), st.acc);
    (void)tm;
  }
};

}  // namespace cfv
