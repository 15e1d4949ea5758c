// Phase functions of the tiled radial-march kernels (see march.hip).
// Everything here is __host__ __device__ so that the same code runs on the
// GPU and under a host emulation of a workgroup.
#pragma once
#include "cfv_kernels.hpp"

namespace cfv {

constexpr int kTI = 16, kTJ = 16, kNT = kTI * kTJ;  // tile of columns
constexpr int kKC = 16;                             // radial layers per chunk (default)

struct MarchArgs {
  DevGrid d;
  const double* U;
  const double* Ud;   // tangent of U (Dual only; null means zero)
  const double* dbr;  // tangent of the B_r map (Dual only; nullable)
  double* G;          // limited gradients [27][ncells]
  double* Gd;         // their tangents (Dual only)
  double* R;          // residual (nullable for Dual)
  double* Rd;         // tangent of the residual (Dual only)
  double* P = nullptr;  // primitives [9][ncells] written by the gradient pass (nullable)
  double* Q = nullptr;  // face states [6 x 9][ncells] (row 9 lf + v) written by the face-state gradient pass
  double* E = nullptr;  // dual march: tile-edge face states (edge_buffer_doubles), written by the gradient
                        // pass, read by the flux pass's ring
};

struct TileMap {
  int p, j0, i0, k0, k1;
};

// Tile-edge face states of the dual march: for every tile, layer and edge
// slot (64 slots: 16 east faces of the last column by row, 16 north faces of
// the last row by column, 16 west faces of the first column by row, 16 south
// faces of the first row by column), the edge cell's state on that face (9
// values, then their 9 tangents), at [tile][layer][18][64].  The gradient
// pass writes them (its edge cells have their limited gradients at hand);
// the flux pass's ring reads a neighbour tile's 18 contiguous rows instead of
// that cell's primitives and gradients (72 values, strided by N along the
// tile's east and west edges).
constexpr int kEdgeSlots = 64, kEdgeLayer = 18 * kEdgeSlots;
__host__ __device__ __forceinline__ int march_tiles_1d(int N) { return (N + 15) / 16; }
__host__ __device__ __forceinline__ int64_t edge_buffer_doubles(const Shape& g) {
  const int64_t nt = march_tiles_1d(g.N);
  return 6 * nt * nt * int64_t(g.Nr) * kEdgeLayer;
}
__host__ __device__ __forceinline__ int64_t march_tile_index(const Shape& g, int p, int j0, int i0) {
  const int64_t nt = march_tiles_1d(g.N);
  return (int64_t(p) * nt + j0 / 16) * nt + i0 / 16;
}

// work items (tile, chunk of kc layers) of one instance
__host__ __device__ __forceinline__ int64_t march_logical_blocks(const Shape& g, int kc) {
  const int64_t nti = (g.N + kTI - 1) / kTI, ntj = (g.N + kTJ - 1) / kTJ, nch = (g.Nr + kc - 1) / kc;
  return 6 * ntj * nti * nch;
}

// Chunk length for a march over `tiles` column tiles of Nr layers with
// `slots` workgroups resident at once: of the chunk counts n, the one that
// minimises the rounds of work items times the layers an item marches (its
// own, plus one warm-up and one cool-down layer); kc = ceil(Nr / n).
inline int balanced_chunk(int64_t tiles, int Nr, int64_t slots) {
  int best = Nr;
  int64_t best_cost = -1;
  for (int n = 1; n <= Nr; ++n) {
    const int kc = (Nr + n - 1) / n;
    if ((Nr + kc - 1) / kc != n) continue;  // the same chunks as a smaller n
    const int64_t rounds = (tiles * n + slots - 1) / slots;
    const int64_t cost = rounds * (kc + 2);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = kc;
    }
  }
  return best;
}

// launch size: a multiple of 8 so that the XCD split is a bijection
__host__ __device__ __forceinline__ int64_t march_blocks(const Shape& g, int kc) {
  return (march_logical_blocks(g, kc) + 7) / 8 * 8;
}

// logical block l (chunk fastest, then tile i, tile j, panel) -> tile and chunk
__host__ __device__ __forceinline__ void tile_of_logical(const Shape& g, int64_t l, TileMap& tm, int kc) {
  const int64_t nti = (g.N + kTI - 1) / kTI, ntj = (g.N + kTJ - 1) / kTJ, nch = (g.Nr + kc - 1) / kc;
  int64_t r = l;
  const int ch = int(r % nch);
  r /= nch;
  const int ti = int(r % nti);
  r /= nti;
  const int tj = int(r % ntj);
  tm.p = int(r / ntj);
  tm.j0 = tj * kTJ;
  tm.i0 = ti * kTI;
  tm.k0 = ch * kc;
  tm.k1 = tm.k0 + kc < g.Nr ? tm.k0 + kc : g.Nr;
}

// ------------------------------------------------------------- small helpers
template <class T>
__host__ __device__ __forceinline__ T* lds_as(double* lds) {
  return reinterpret_cast<T*>(lds);
}

// A launch's descriptor (no kernel writes it while one runs) read through
// the constant address space: at a uniform address its fields become scalar
// loads, which the vector memory counter does not track, so reading one does
// not wait for the loads and stores in flight (a vector load of the field
// would: the compiler cannot prove that the kernel's own stores leave the
// descriptor alone).
__host__ __device__ __forceinline__ const MarchArgs& constant_args(const MarchArgs* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return *(const MarchArgs*)reinterpret_cast<const __attribute__((address_space(4))) MarchArgs*>(uniform_address(p));
#else
  return *p;
#endif
}

#if defined(__HIPCC__)
// the same descriptor, but a value the compiler cannot follow: reads through
// it are not hoisted out of the layer loop (the descriptor's fields would
// otherwise stay in scalar registers across the whole item and spill)
__device__ __forceinline__ const MarchArgs& per_layer(const MarchArgs& a) {
  const MarchArgs* p = &a;
  asm volatile("" : "+s"(p));
  return constant_args(p);
}
#endif

template <class T>
__host__ __device__ __forceinline__ void load_prims(const MarchArgs& a, int64_t c, T P[9]) {
  const int64_t nc = a.d.g.ncells;
  T u[9];
  for (int v = 0; v < 9; ++v) ldT(a.U, a.Ud, v * nc + c, u[v]);
  cons_to_prim(u, P, a.d.pr.gamma);
}

template <class T>
__host__ __device__ __forceinline__ void load_grad(const MarchArgs& a, int64_t c, T Gr[27]) {
  const int64_t nc = a.d.g.ncells;
  for (int v = 0; v < 27; ++v) ldT(a.G, a.Gd, v * nc + c, Gr[v]);
}

template <class T>
__host__ __device__ __forceinline__ void recon(const T P[9], const T Gr[27], V3 d, T q[9]) {
  for (int v = 0; v < 9; ++v) q[v] = P[v] + (Gr[3 * v] * d.x + Gr[3 * v + 1] * d.y + Gr[3 * v + 2] * d.z);
}

// column -> (panel, j, i); columns are below 2^31 (32-bit division)
__host__ __device__ __forceinline__ void column_pji(const Shape& g, int64_t col, int& p, int& j, int& i) {
  const uint32_t n = uint32_t(g.N);
  uint32_t t = uint32_t(col);
  i = int(t % n);
  t /= n;
  j = int(t % n);
  p = int(t / n);
}

template <class T>
__host__ __device__ __forceinline__ T map_br(const MarchArgs& a, int64_t col) {
  T b;
  ldT(a.d.br, a.dbr, col, b);
  return b;
}

// canonical flux across a face: owner on the left
template <class T>
__host__ __device__ __forceinline__ void face_flux(bool own, const T qs[9], const T qo[9], V3 S, T F[9], const Params& pr) {
  const T* L = own ? qs : qo;
  const T* R = own ? qo : qs;
  rusanov(L, R, S, F, pr);
}

// ======================================================== gradient pass
// LDS plane of (kTI + 2) x (kTJ + 2) positions: the tile at offset (1, 1)
// and a ring.  Every in-plane neighbour of an active cell has a position:
// an active in-tile cell publishes itself; for a neighbour that is not (tile
// edge, panel edge, or beyond a partial tile) the one active cell next to it
// stores its centroid sums once per item, and the second wavefront loads its
// primitives for every layer (ring()).
constexpr int kPW = kTI + 2, kPH = kTJ + 2, kPlane = kPW * kPH;
__host__ __device__ __forceinline__ int plane_pos(int ti, int tj) { return (tj + 1) * kPW + (ti + 1); }
__host__ __device__ __forceinline__ void dir_offset(int q, int& dx, int& dy) {
  dx = q == 0 ? -1 : q == 1 ? 1 : 0;
  dy = q == 2 ? -1 : q == 3 ? 1 : 0;
}

template <class T>
struct GState {
  int p, j, i;
  int64_t col;
  bool act;
  T Pm[9], P0[9], Pp[9];
  int64_t rc0;  // ring threads: the ring slot's cell at layer 0 (-1: no slot)
  unsigned emask;  // dual pass: the tile edges the cell lies on (bit = edge slot kind 0..3)
  int es0, es1;    // dual pass: the edge slots of the first two of them (-1: none)
  unsigned erest;  // and the others (one-cell-wide tiles only)
  V3 fe0, fe1;     // their face-centroid offsets per unit rs_k
  // the column's geometry per item (centroid sum, radial face centroid per
  // unit radius, angular face-centroid offsets per unit rs_k)
  V3 cc, xr, fe[4];
};

// Ring slot r (0..63) of a tile: the out-of-tile neighbour across one edge
// face of the tile (kind 0: east of row idx's last cell, 1: north of column
// idx's last cell, 2: west of row idx's first cell, 3: south of column idx's
// first cell).  Returns false for a slot beyond a partial tile; otherwise the
// tile cell (ti, tj), the face direction q (0..3: W, E, S, N) and the
// neighbour's column.
__host__ __device__ __forceinline__ bool ring_slot(const MarchArgs& a, const TileMap& tm, int r, int& ti, int& tj,
                                                   int& q, int64_t& ncol) {
  const Shape& g = a.d.g;
  const int kind = r >> 4, idx = r & 15;
  const int tiL = (g.N - tm.i0 < kTI ? g.N - tm.i0 : kTI) - 1;
  const int tjL = (g.N - tm.j0 < kTJ ? g.N - tm.j0 : kTJ) - 1;
  ti = kind == 0 ? tiL : kind == 2 ? 0 : idx;
  tj = kind == 1 ? tjL : kind == 3 ? 0 : idx;
  q = kind == 0 ? 1 : kind == 1 ? 3 : kind == 2 ? 0 : 2;
  if (ti > tiL || tj > tjL) return false;
  ncol = gld(a.d.G.cn, q * a.d.G.ncol + column_of(g, tm.p, tm.j0 + tj, tm.i0 + ti));
  return true;
}

template <class T>
struct GradWG {
  static constexpr int kTw = int(sizeof(T) / sizeof(double));
  // primitives plane (9 T per position), then the column centroid sums (3)
  static constexpr int kCs = 9 * kPlane * kTw;
  // dual pass: a layer's tile-edge face states, staged for one coalesced
  // write ([18][64] doubles, the edge buffer's layout)
  static constexpr int kEs = kCs + 3 * kPlane;
  static constexpr int kLds = kEs + (sizeof(T) > sizeof(double) ? kEdgeLayer : 0);

  __host__ __device__ static bool in_tile_active(const Shape& g, const TileMap& tm, int ti, int tj) {
    return ti >= 0 && ti < kTI && tj >= 0 && tj < kTJ && tm.i0 + ti < g.N && tm.j0 + tj < g.N;
  }

  __host__ __device__ static void init(const MarchArgs& a, const TileMap& tm, GState<T>& st, int t, double* lds) {
    const Shape& g = a.d.g;
    const GeomRef& G = a.d.G;
    const int ti = t % kTI, tj = t / kTI;
    st.p = tm.p;
    st.j = tm.j0 + tj;
    st.i = tm.i0 + ti;
    st.act = st.j < g.N && st.i < g.N;
    st.rc0 = -1;
    {
      // east (kind 0), north (1), west (2), south (3) tile edges of the cell
      const int tiL = (g.N - tm.i0 < kTI ? g.N - tm.i0 : kTI) - 1;
      const int tjL = (g.N - tm.j0 < kTJ ? g.N - tm.j0 : kTJ) - 1;
      st.emask = unsigned(ti == tiL) | unsigned(tj == tjL) << 1 | unsigned(ti == 0) << 2 | unsigned(tj == 0) << 3;
      st.es0 = st.es1 = -1;
      st.erest = 0;
    }
    if (t >= kNT / 4 && t < kNT / 2) {  // the ring slot's neighbour cell, decoded once per item
      int ti2, tj2, q;
      int64_t ncol;
      if (ring_slot(a, tm, t - kNT / 4, ti2, tj2, q, ncol)) {
        int np, nj, ni;
        column_pji(g, ncol, np, nj, ni);
        st.rc0 = cell_index(g, np, 0, nj, ni);
      }
    }
    if (!st.act) return;
    st.col = column_of(g, st.p, st.j, st.i);
    double* cs = lds + kCs;
    const V3 c0 = cg3(G, CG_CSUM, st.col);
    const int me = plane_pos(ti, tj);
    cs[me] = c0.x; cs[kPlane + me] = c0.y; cs[2 * kPlane + me] = c0.z;
    for (int q = 0; q < 4; ++q) {
      int dx, dy;
      dir_offset(q, dx, dy);
      if (in_tile_active(g, tm, ti + dx, tj + dy)) continue;
      const V3 cn = cg3(G, CG_CSUM, gld(G.cn, q * G.ncol + st.col));
      const int pos = plane_pos(ti + dx, tj + dy);
      cs[pos] = cn.x; cs[kPlane + pos] = cn.y; cs[2 * kPlane + pos] = cn.z;
    }
    for (int v = 0; v < 9; ++v) st.Pm[v] = st.P0[v] = st.Pp[v] = T(0.0);
    st.cc = c0;
    st.xr = cg3(G, CG_XR, st.col);
    for (int q = 0; q < 4; ++q) st.fe[q] = 2.0 * cg3(G, CG_ANG + 6 * q + 3, st.col) - c0;
    // the first two tile edges of the cell as slots and face offsets (kind
    // 0..3: east, north, west, south faces, q = 1, 3, 0, 2)
    st.fe0 = st.fe1 = mk(0.0, 0.0, 0.0);
    for (int kind = 0; kind < 4; ++kind) {
      if (!((st.emask >> kind) & 1u)) continue;
      const int q = kind == 0 ? 1 : kind == 1 ? 3 : kind == 2 ? 0 : 2;
      const int slot = kind * 16 + ((kind & 1) ? ti : tj);
      const V3 f = q == 0 ? st.fe[0] : q == 1 ? st.fe[1] : q == 2 ? st.fe[2] : st.fe[3];
      if (st.es0 < 0) { st.es0 = slot; st.fe0 = f; }
      else if (st.es1 < 0) { st.es1 = slot; st.fe1 = f; }
      else st.erest |= 1u << kind;
    }
  }

  // First layer of the march of a chunk [k0, k1): the layers k0 - 1 and k0
  // enter the registers through the warm-up iterations k < k0, which run this
  // phase alone, so every layer's primitives come from the same code whatever
  // the chunk length (and the outputs with them, bit for bit).
  __host__ __device__ static int first_layer(const TileMap& tm) { return tm.k0 >= 1 ? tm.k0 - 2 : -1; }

  // layer k: load the primitives of layer k + 1; publish layer k's in LDS
  // (a warm-up iteration only shifts the registers instead).  In the dual
  // pass (one wavefront per SIMD) a ring lane (second wavefront) also fills
  // its ring position of layer k here, its loads issued before the cell's
  // own so that both wait for memory once; the plain pass (two wavefronts
  // per SIMD, the other hides the wait) fills it after publishing
  // (ring_late), which spills less.
  static constexpr bool kEarlyRing = sizeof(T) > sizeof(double);
  __host__ __device__ static void publish(const MarchArgs& a, const TileMap& tm, GState<T>& st, int t, int k,
                                          double* lds) {
    const Shape& g = a.d.g;
    const int64_t nc = g.ncells;
    const bool rl = kEarlyRing && k >= tm.k0 && st.rc0 >= 0;  // rc0 >= 0: a ring lane with a neighbour
    T ur[9];
    if (rl)
      for (int v = 0; v < 9; ++v) ldT(a.U, a.Ud, v * nc + st.rc0 + int64_t(k) * g.N * g.N, ur[v]);
    if (st.act) {
      const int ti = t % kTI, tj = t / kTI;
      if (k + 1 >= 0 && k + 1 < g.Nr) load_prims(a, cell_index(g, st.p, k + 1, st.j, st.i), st.Pp);
      if (k < tm.k0) {
        for (int v = 0; v < 9; ++v) {
          st.Pm[v] = st.P0[v];
          st.P0[v] = st.Pp[v];
        }
      } else {
        T* L = lds_as<T>(lds);
        const int me = plane_pos(ti, tj);
        for (int v = 0; v < 9; ++v) L[v * kPlane + me] = st.P0[v];
        if (a.P) {
          const int64_t c = cell_index(g, st.p, k, st.j, st.i);
          for (int v = 0; v < 9; ++v) gst(a.P, v * g.ncells + c, val(st.P0[v]));
        }
      }
    }
    if (rl) ring(a, tm, t - kNT / 4, ur, lds);
  }

  // the plain pass's ring position r of layer k (the lanes r + kNT / 4)
  __host__ __device__ static void ring_late(const MarchArgs& a, const TileMap& tm, const GState<T>& st, int r,
                                            int k, double* lds) {
    if (kEarlyRing || st.rc0 < 0) return;
    const Shape& g = a.d.g;
    T u[9];
    for (int v = 0; v < 9; ++v) ldT(a.U, a.Ud, v * g.ncells + st.rc0 + int64_t(k) * g.N * g.N, u[v]);
    ring(a, tm, r, u, lds);
  }

  // Ring position r of layer k from the neighbour's state u (the plane's
  // out-of-tile neighbours, filled by one wavefront in one pass instead of a
  // divergent pass per direction in every wavefront): kind 0 east of row idx's last cell, 1 north of
  // column idx's last cell, 2 west of row idx's first cell, 3 south of
  // column idx's first cell.
  __host__ __device__ static void ring(const MarchArgs& a, const TileMap& tm, int r, const T u[9], double* lds) {
    const Shape& g = a.d.g;
    const int kind = r >> 4, idx = r & 15;
    const int tiL = (g.N - tm.i0 < kTI ? g.N - tm.i0 : kTI) - 1;
    const int tjL = (g.N - tm.j0 < kTJ ? g.N - tm.j0 : kTJ) - 1;
    const int ti = kind == 0 ? tiL : kind == 2 ? 0 : idx;
    const int tj = kind == 1 ? tjL : kind == 3 ? 0 : idx;
    const int q = kind == 0 ? 1 : kind == 1 ? 3 : kind == 2 ? 0 : 2;
    int dx, dy;
    dir_offset(q, dx, dy);
    T qn[9];
    cons_to_prim(u, qn, a.d.pr.gamma);
    T* L = lds_as<T>(lds);
    const int pos = plane_pos(ti + dx, tj + dy);
    for (int v = 0; v < 9; ++v) L[v * kPlane + pos] = qn[v];
  }

  // Faces: write the reconstructed face states to a.Q instead of the
  // gradients to a.G (the VJP's forward pass; a separate instantiation so
  // that the residual's pass does not carry the stores' registers)
  template <bool Faces = false>
  __host__ __device__ static void compute(const MarchArgs& a, const TileMap& tm, GState<T>& st, int t, int k,
                                          double* lds) {
    if (!st.act) return;
    const Shape& g = a.d.g;
    const GeomRef& G = a.d.G;
    const T* L = lds_as<T>(lds);
    const double* cs = lds + kCs;
    const int ti = t % kTI, tj = t / kTI;
    const double r0 = radius_uniform(G, k), r1 = radius_uniform(G, k + 1);
    const double rs = 0.125 * (r0 + r1);
    const V3 xc = rs * st.cc;
    // geometry: neighbour offsets and face-centroid offsets
    V3 dx[6], dxf[6];
    int pos[4];
    {
      // a layer's centroid is rs_k cc, an angular face's centroid 2 rs_k b_q,
      // a radial face's r xr: offsets from the item's constants
      const V3 xf0 = r0 * st.xr, xf1 = r1 * st.xr;
      dxf[0] = xf0 - xc;
      dxf[1] = xf1 - xc;
      if (k > 0) {
        dx[0] = (0.125 * (radius_uniform(G, k - 1) + r0) - rs) * st.cc;
      } else {
        const V3 S = (r0 * r0) * cg3(G, CG_SR, st.col);
        dx[0] = ghost_centre(xc, S, xf0) - xc;
      }
      if (k + 1 < g.Nr) {
        dx[1] = (0.125 * (r1 + radius_uniform(G, k + 2)) - rs) * st.cc;
      } else {
        const V3 S = (r1 * r1) * cg3(G, CG_SR, st.col);
        dx[1] = ghost_centre(xc, S, xf1) - xc;
      }
#pragma unroll
      for (int lf = 2; lf < 6; ++lf) {
        int ddx, ddy;
        dir_offset(lf - 2, ddx, ddy);
        pos[lf - 2] = plane_pos(ti + ddx, tj + ddy);
        const int q = pos[lf - 2];
        dxf[lf] = rs * st.fe[lf - 2];
        dx[lf] = rs * (mk(cs[q], cs[kPlane + q], cs[2 * kPlane + q]) - st.cc);
      }
    }
    const LsqWeights W(dx);
    // ghost states on the boundary layers
    T gin[9], gout[9];
    if (k == 0) {
      V3 xG;
      ghost_prims(a.d, st.p, k, st.j, st.i, 0, st.P0, xc, map_br<T>(a, st.col), gin, xG);
    }
    if (k + 1 == g.Nr) {
      V3 xG;
      ghost_prims(a.d, st.p, k, st.j, st.i, 1, st.P0, xc, T(0.0), gout, xG);
    }
    const int64_t c = cell_index(g, st.p, k, st.j, st.i);
    bool bad = false;
    if constexpr (Faces) {
      if (k == 0) bad = bad || !physical(gin);
      if (k + 1 == g.Nr) bad = bad || !physical(gout);
    }
#pragma unroll
    for (int v = 0; v < 9; ++v) {
      T qn[6];
      qn[0] = k > 0 ? st.Pm[v] : gin[v];
      qn[1] = k + 1 < g.Nr ? st.Pp[v] : gout[v];
#pragma unroll
      for (int q = 0; q < 4; ++q) qn[2 + q] = L[v * kPlane + pos[q]];
      T gx, gy, gz;
      limited_grad(W, dxf, a.d.pr.limiter, st.P0[v], qn, gx, gy, gz);
      if constexpr (!Faces) {
        stT(a.G, a.Gd, (3 * v) * g.ncells + c, gx);
        stT(a.G, a.Gd, (3 * v + 1) * g.ncells + c, gy);
        stT(a.G, a.Gd, (3 * v + 2) * g.ncells + c, gz);
        if constexpr (sizeof(T) > sizeof(double)) {
          // the states on the cell's tile-edge faces (the same expression as
          // the flux pass's reconstruction) for the neighbour tiles' rings,
          // staged in LDS (flush_edges writes the layer's block)
          double* Es = lds + kEs;
          if (st.es0 >= 0) {  // rs_k fe is dxf of that face: the same products
            const V3 d0 = rs * st.fe0;
            const T qf = st.P0[v] + (gx * d0.x + gy * d0.y + gz * d0.z);
            Es[v * kEdgeSlots + st.es0] = qf.v;
            Es[(9 + v) * kEdgeSlots + st.es0] = qf.d;
          }
          if (st.es1 >= 0) {
            const V3 d1 = rs * st.fe1;
            const T qf = st.P0[v] + (gx * d1.x + gy * d1.y + gz * d1.z);
            Es[v * kEdgeSlots + st.es1] = qf.v;
            Es[(9 + v) * kEdgeSlots + st.es1] = qf.d;
          }
          if (st.erest) {
#pragma unroll
            for (int kind = 0; kind < 4; ++kind) {
              if (!((st.erest >> kind) & 1u)) continue;
              const int lf = kind == 0 ? 3 : kind == 1 ? 5 : kind == 2 ? 2 : 4;  // E, N, W, S
              const T qf = st.P0[v] + (gx * dxf[lf].x + gy * dxf[lf].y + gz * dxf[lf].z);
              const int slot = kind * 16 + ((kind & 1) ? ti : tj);
              Es[v * kEdgeSlots + slot] = qf.v;
              Es[(9 + v) * kEdgeSlots + slot] = qf.d;
            }
          }
        }
      } else {  // instead of the gradient, the reconstructed state at each face centroid
#pragma unroll
        for (int lf = 0; lf < 6; ++lf) {
          const double qf = val(st.P0[v] + (gx * dxf[lf].x + gy * dxf[lf].y + gz * dxf[lf].z));
          gst(a.Q, (9 * lf + v) * g.ncells + c, qf);
          if (v == 0 || v == 7) bad = bad || !(qf > 0.0);
        }
      }
    }
    if constexpr (Faces) record_nonphysical(a.d, bad);
    for (int v = 0; v < 9; ++v) {
      st.Pm[v] = st.P0[v];
      st.P0[v] = st.Pp[v];
    }
    (void)tm;
  }

  // dual pass, after the barrier that ends layer k's compute step: lanes
  // 128..191 write the layer's staged tile-edge states (slots of edge cells
  // beyond a partial tile hold stale values that no ring reads)
  __host__ __device__ static void flush_edges(const MarchArgs& a, const TileMap& tm, int t, int k,
                                              const double* lds) {
    if constexpr (sizeof(T) > sizeof(double)) {
      if (!a.E || t < 2 * kEdgeSlots || t >= 3 * kEdgeSlots) return;
      const Shape& g = a.d.g;
      const int r = t - 2 * kEdgeSlots;
      const int64_t eb = (march_tile_index(g, tm.p, tm.j0, tm.i0) * g.Nr + k) * kEdgeLayer + r;
      const double* Es = lds + kEs;
#pragma unroll
      for (int row = 0; row < 18; ++row) gst(a.E, eb + row * kEdgeSlots, Es[row * kEdgeSlots + r]);
    } else {
      (void)a; (void)tm; (void)t; (void)k; (void)lds;
    }
  }
};

// ============================================================ flux pass
template <class T>
struct FState {
  int p, j, i;
  int64_t col;
  bool act;
  T qtop[9];  // top-face state of layer k-1
  T accp[9];  // residual of layer k-1 without its top face
  T acc[9];   // residual of layer k so far
  T q3[9], q5[9];
  bool bad;   // a face state of this column met a non-positive density or pressure
  int64_t ebase;  // ring threads: the slot's state in the edge buffer at layer 0 (-1: no slot)
  int own_ws;  // bit 0 (1): the cell owns its west (south) face
};

template <class T>
__host__ __device__ __forceinline__ void store_res(const MarchArgs& a, int64_t c, const T r[9]);
template <>
__host__ __device__ __forceinline__ void store_res<double>(const MarchArgs& a, int64_t c, const double r[9]) {
  for (int v = 0; v < 9; ++v) gst(a.R, v * a.d.g.ncells + c, r[v]);
}
template <>
__host__ __device__ __forceinline__ void store_res<Dual>(const MarchArgs& a, int64_t c, const Dual r[9]) {
  for (int v = 0; v < 9; ++v) {
    if (a.R) gst(a.R, v * a.d.g.ncells + c, r[v].v);
    gst(a.Rd, v * a.d.g.ncells + c, r[v].d);
  }
}

template <class T>
struct FluxWG {
  // LDS, in units of T: the west and south face states of the tile's cells
  // (18 rows of kNT), their east and north face fluxes (18 rows), the states
  // of the out-of-tile neighbours across the tile's four edges on the shared
  // faces (9 rows of kRing: east edge by row, north by column, west by row,
  // south by column) and the signed fluxes of the tile's west and south edge
  // faces (9 rows of kEdge: south by column, then west by row)
  static constexpr int kRing = 4 * 16, kEdge = 2 * 16;
  static_assert(kTI == 16 && kTJ == 16, "ring and edge slots are laid out for 16 x 16 tiles");
  static constexpr int kRingOff = 36 * kNT, kEdgeOff = kRingOff + 9 * kRing;
  static constexpr int kLds = (kEdgeOff + 9 * kEdge) * int(sizeof(T) / sizeof(double));

  // last active column and row of the tile (partial tiles at the panel edge)
  __host__ __device__ static int last_ti(const Shape& g, const TileMap& tm) {
    return (g.N - tm.i0 < kTI ? g.N - tm.i0 : kTI) - 1;
  }
  __host__ __device__ static int last_tj(const Shape& g, const TileMap& tm) {
    return (g.N - tm.j0 < kTJ ? g.N - tm.j0 : kTJ) - 1;
  }

  // ring slot r of layer k: the state of the out-of-tile neighbour across
  // one edge face of the tile, on that face, as the neighbour tile's
  // gradient pass left it in the edge buffer (one wavefront loads all 64,
  // in the states phase)
  __host__ __device__ static void ring_load(const MarchArgs& a, const FState<T>& st, int k, T q[9]) {
    const int64_t e = st.ebase + int64_t(k) * kEdgeLayer;
    for (int v = 0; v < 9; ++v) ldT(a.E, a.E + 9 * kEdgeSlots, e + v * kEdgeSlots, q[v]);
  }
  __host__ __device__ static void ring_store(int r, const T q[9], double* lds) {
    T* Rg = lds_as<T>(lds) + kRingOff;
    for (int v = 0; v < 9; ++v) Rg[v * kRing + r] = q[v];
  }

  __host__ __device__ static void init(const MarchArgs& a, const TileMap& tm, FState<T>& st, int t) {
    const Shape& g = a.d.g;
    st.p = tm.p;
    st.j = tm.j0 + t / kTI;
    st.i = tm.i0 + t % kTI;
    st.act = st.j < g.N && st.i < g.N;
    st.bad = false;
    for (int v = 0; v < 9; ++v) st.qtop[v] = T(0.0);
    st.ebase = -1;
    st.own_ws = 0;
    if (st.act) {  // the west and south faces' orientations, once per item
      const int64_t col = column_of(g, st.p, st.j, st.i);
      st.own_ws = int((gld(a.d.G.cn, 4 * a.d.G.ncol + col) >> 8) != 0) |
                  int((gld(a.d.G.cn, 6 * a.d.G.ncol + col) >> 8) != 0) << 1;
    }
    if (t >= kNT / 4 && t < kNT / 4 + kRing) {  // the ring slot's source in the edge buffer, once per item
      int ti, tj, q;
      int64_t ncol;
      if (ring_slot(a, tm, t - kNT / 4, ti, tj, q, ncol)) {
        // the neighbour cell, its tile and the edge slot of its face back
        // toward this tile (local faces 2..5: W, E, S, N)
        int np, nj, ni;
        column_pji(g, ncol, np, nj, ni);
        const int back = (gld(a.d.G.cn, (4 + q) * a.d.G.ncol + column_of(g, tm.p, tm.j0 + tj, tm.i0 + ti)) & 0xff) - 2;
        const int kind = back == 1 ? 0 : back == 3 ? 1 : back == 0 ? 2 : 3;
        const int slot = kind * 16 + ((kind & 1) ? ni % 16 : nj % 16);
        const int64_t tile = march_tile_index(g, np, nj - nj % 16, ni - ni % 16);
        st.ebase = tile * g.Nr * kEdgeLayer + slot;
      }
    }
  }

  // Layers of the march of a chunk [k0, k1): a warm-up iteration k0 - 1
  // gives the top-face state of the layer below the chunk, a cool-down
  // iteration k1 the flux through the chunk's top face, both from the same
  // code as every other layer's (so the outputs do not depend on the chunk
  // length, bit for bit).
  __host__ __device__ static int first_layer(const TileMap& tm) { return tm.k0 > 0 ? tm.k0 - 1 : 0; }
  __host__ __device__ static int last_layer(const Shape& g, const TileMap& tm) {
    return tm.k1 < g.Nr ? tm.k1 : tm.k1 - 1;
  }

  // layer k's face states and its bottom face's flux, which completes the
  // residual of layer k - 1.  A warm-up layer (k < k0) runs this phase alone
  // for its top-face state, a cool-down layer (k = k1) for the flux through
  // the chunk's top face; what else they compute is overwritten or unused.
  // A ring lane (second wavefront) of a marched layer also fills its ring
  // slot, the loads issued with the cell's own (one wait for both).
  __host__ __device__ static void states(const MarchArgs& a, const TileMap& tm, FState<T>& st, int t, int k,
                                         double* lds) {
    const bool rl = k >= tm.k0 && k < tm.k1 && st.ebase >= 0;  // ebase >= 0: a ring lane with a slot
    T rq[9];
    if (rl) ring_load(a, st, k, rq);
    if (!st.act) {
      if (rl) ring_store(t - kNT / 4, rq, lds);
      return;
    }
    const Shape& g = a.d.g;
    const GeomRef& G = a.d.G;
    st.col = column_of(g, st.p, st.j, st.i);
    const int64_t c = cell_index(g, st.p, k, st.j, st.i);
    T u[9], P[9], Gr[27];
    for (int v = 0; v < 9; ++v) ldT(a.U, a.Ud, v * g.ncells + c, u[v]);
    cons_to_prim(u, P, a.d.pr.gamma);
    if (rl) ring_store(t - kNT / 4, rq, lds);
    load_grad(a, c, Gr);
    const V3 xc = cell_centre<true>(G, g, st.p, k, st.j, st.i);

    // radial face below: k - 1/2 (owner k-1), or the inner boundary face
    {
      V3 S, xf;
      bool own;
      canon_face<true>(G, g, st.p, k, st.j, st.i, 0, Nbr{}, 0, S, xf, own);
      T qb[9], F[9];
      recon(P, Gr, xf - xc, qb);
      st.bad = st.bad || !physical(qb);
      if (k == 0) {
        T qG[9];
        V3 xG;
        ghost_prims(a.d, st.p, k, st.j, st.i, 0, P, xc, map_br<T>(a, st.col), qG, xG);
        st.bad = st.bad || !physical(qG);
        rusanov(qb, qG, S, F, a.d.pr);
        for (int v = 0; v < 9; ++v) st.acc[v] = F[v];
      } else {
        rusanov(st.qtop, qb, S, F, a.d.pr);
        if (k - 1 >= tm.k0) {
          for (int v = 0; v < 9; ++v) st.accp[v] += F[v];
          store_res(a, c - int64_t(g.N) * g.N, st.accp);
        }
        for (int v = 0; v < 9; ++v) st.acc[v] = -F[v];
      }
    }
    // gravity source
    {
      T src[9];
      gravity_source(u, xc, cell_volume<true>(G, g, st.p, k, st.j, st.i), a.d.pr.G, src);
      for (int v = 0; v < 9; ++v) st.acc[v] -= src[v];
    }
    // top face state (and the outer boundary face)
    {
      V3 S, xf;
      bool own;
      canon_face<true>(G, g, st.p, k, st.j, st.i, 1, Nbr{}, 0, S, xf, own);
      recon(P, Gr, xf - xc, st.qtop);
      st.bad = st.bad || !physical(st.qtop);
      if (k == g.Nr - 1) {
        T qG[9], F[9];
        V3 xG;
        ghost_prims(a.d, st.p, k, st.j, st.i, 1, P, xc, T(0.0), qG, xG);
        st.bad = st.bad || !physical(qG);
        rusanov(st.qtop, qG, S, F, a.d.pr);
        for (int v = 0; v < 9; ++v) st.acc[v] += F[v];
      }
    }
    // angular face states: west and south to LDS, east and north kept
    T* Sb = lds_as<T>(lds);
    for (int q = 0; q < 4; ++q) {
      V3 S, xf;
      bool own;
      canon_face<true>(G, g, st.p, k, st.j, st.i, 2 + q, Nbr{}, 0, S, xf, own);
      T s[9];
      recon(P, Gr, xf - xc, s);
      st.bad = st.bad || !physical(s);
      if (q == 0)
        for (int v = 0; v < 9; ++v) Sb[v * kNT + t] = s[v];
      else if (q == 2)
        for (int v = 0; v < 9; ++v) Sb[(9 + v) * kNT + t] = s[v];
      else if (q == 1)
        for (int v = 0; v < 9; ++v) st.q3[v] = s[v];
      else
        for (int v = 0; v < 9; ++v) st.q5[v] = s[v];
    }
  }

  // east and north faces of every cell (neighbour states from LDS: in-tile
  // or ring); the west and south faces on the tile's edges by the first kEdge
  // threads, for the edge cells, with their signed fluxes left in LDS
  __host__ __device__ static void faces(const MarchArgs& a, const TileMap& tm, FState<T>& st, int t, int k,
                                        double* lds) {
    const Shape& g = a.d.g;
    const GeomRef& G = a.d.G;
    const T* Sb = lds_as<T>(lds);
    T* Fb = lds_as<T>(lds) + 18 * kNT;
    const T* Rg = lds_as<T>(lds) + kRingOff;
    T* Eb = lds_as<T>(lds) + kEdgeOff;
    const int ti = t % kTI, tj = t / kTI;
    const int tiL = last_ti(g, tm), tjL = last_tj(g, tm);
    if (st.act) {
      for (int h = 0; h < 2; ++h) {
        const int q = h == 0 ? 1 : 3;
        V3 S, xf;
        bool own;
        canon_face<true>(G, g, st.p, k, st.j, st.i, 2 + q, Nbr{}, 0, S, xf, own);
        T qs[9], qo[9], F[9];
        if (h == 0) {
          for (int v = 0; v < 9; ++v) qs[v] = st.q3[v];
          // the neighbour's state from the tile or the ring, one code path
          // for both (lanes of one wavefront take either)
          const bool in = ti < tiL;
          const T* src = in ? Sb + t + 1 : Rg + tj;
          const int stride = in ? kNT : kRing;
          for (int v = 0; v < 9; ++v) qo[v] = src[v * stride];
        } else {
          for (int v = 0; v < 9; ++v) qs[v] = st.q5[v];
          const bool in = tj < tjL;
          const T* src = in ? Sb + 9 * kNT + t + kTI : Rg + 16 + ti;
          const int stride = in ? kNT : kRing;
          for (int v = 0; v < 9; ++v) qo[v] = src[v * stride];
        }
        face_flux(own, qs, qo, S, F, a.d.pr);
        const double sg = own ? 1.0 : -1.0;  // a product by +-1: the same bits as the select
        for (int v = 0; v < 9; ++v) st.acc[v] += F[v] * sg;
        for (int v = 0; v < 9; ++v) Fb[(9 * h + v) * kNT + t] = F[v];
      }
    }
    if (t < kEdge) {
      const bool south = t < 16;
      const int eti = south ? t : 0, etj = south ? 0 : t - 16;
      if (eti <= tiL && etj <= tjL) {
        const int q = south ? 2 : 0;
        const int tc = etj * kTI + eti;
        V3 S, xf;
        bool own;
        canon_face<true>(G, g, tm.p, k, tm.j0 + etj, tm.i0 + eti, 2 + q, Nbr{}, 0, S, xf, own);
        T qs[9], qo[9], F[9];
        for (int v = 0; v < 9; ++v) {
          qs[v] = Sb[((south ? 9 : 0) + v) * kNT + tc];
          qo[v] = Rg[v * kRing + (south ? 48 + eti : 32 + etj)];
        }
        face_flux(own, qs, qo, S, F, a.d.pr);
        for (int v = 0; v < 9; ++v) Eb[v * kEdge + t] = own ? F[v] : -F[v];
      }
    }
  }

  __host__ __device__ static void accumulate(const MarchArgs& a, const TileMap& tm, FState<T>& st, int t, int k,
                                             double* lds) {
    if (!st.act) return;
    const Shape& g = a.d.g;
    const T* Fb = lds_as<T>(lds) + 18 * kNT;
    const T* Eb = lds_as<T>(lds) + kEdgeOff;
    const int ti = t % kTI, tj = t / kTI;
    if (ti > 0) {
      const double sg = (st.own_ws & 1) ? 1.0 : -1.0;  // the west face's orientation
      for (int v = 0; v < 9; ++v) st.acc[v] += Fb[v * kNT + t - 1] * sg;
    } else {
      for (int v = 0; v < 9; ++v) st.acc[v] += Eb[v * kEdge + 16 + tj];
    }
    if (tj > 0) {
      const double sg = (st.own_ws & 2) ? 1.0 : -1.0;  // the south face's
      for (int v = 0; v < 9; ++v) st.acc[v] += Fb[(9 + v) * kNT + t - kTI] * sg;
    } else {
      for (int v = 0; v < 9; ++v) st.acc[v] += Eb[v * kEdge + ti];
    }
    for (int v = 0; v < 9; ++v) st.accp[v] = st.acc[v];
    if (k == g.Nr - 1) store_res(a, cell_index(g, st.p, k, st.j, st.i), st.acc);
    (void)tm;
  }

  __host__ __device__ static void finish(const MarchArgs& a, const TileMap&, FState<T>& st, int) {
    record_nonphysical(a.d, st.act && st.bad);
  }
};

// One instance; slot: device memory for one descriptor, owned by the caller
// (calls sharing a slot must be ordered on one stream).
// kc: layers per work item (chunk)
hipError_t launch_march(const MarchArgs& a, MarchArgs* slot, bool dual, int kc, hipStream_t s, KernelTimer* t);
// The gradient pass alone (double): limited gradients into a.G and, when
// a.P is set, the primitives into a.P.
hipError_t launch_march_grad(const MarchArgs& a, MarchArgs* slot, int kc, hipStream_t s, KernelTimer* t);

// Ensemble launch: n instances described by args[n] (device), with
// item_off[n + 1] (device) the prefix sums of march_logical_blocks per
// instance (unused when n = 1).  Items (instance, tile, chunk) are taken in
// the order perm[total] (device; null = identity) either statically (each of
// the 8 XCDs takes a contiguous eighth of the list, strided over its
// workgroups) or from a device counter (queue != 0; counters[2] are reset by
// the launch itself).
struct EnsembleLaunch {
  const MarchArgs* args;
  const int64_t* item_off;
  const int64_t* perm;
  unsigned* counters;
  int n;
  int64_t total;
  int queue;
  unsigned blocks;
  int kc = kKC;  // layers per chunk (the items' depth), for both marches
};
hipError_t launch_march_ensemble(const EnsembleLaunch& e, bool dual, hipStream_t s, KernelTimer* t);

}  // namespace cfv
