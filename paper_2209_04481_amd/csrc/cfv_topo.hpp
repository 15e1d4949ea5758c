// Cubed-sphere shell topology and geometry, shared by host and device code.
//
// Grid (the unstructured shell of the paper's Section 2.1, here a gnomonic
// equiangular cubed sphere extruded radially): panel p maps (a, b) =
// (tan xi, tan eta) to the directions
//   P0 (1, a, b)  P1 (-a, 1, b)  P2 (-1, -a, b)  P3 (a, -1, b)  P4 (-b, a, 1)  P5 (b, a, -1).
// Cell (p, k, j, i) spans radii r_k..r_{k+1} and corners (i..i+1, j..j+1);
// c = ((p*Nr + k)*N + j)*N + i.  Local faces: 0 r-, 1 r+, 2 xi- (W),
// 3 xi+ (E), 4 eta- (S), 5 eta+ (N).  Ghost ids: ncells + (p*N+j)*N+i for the
// inner boundary, ncells + 6N^2 + (p*N+j)*N+i for the outer boundary.
//
// Adjacency across panel edges comes from a closed-form edge table (below);
// the geometry of a face is always evaluated from its owner cell (the lower
// index, or the interior cell for a boundary face), so both sides see the
// same numbers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "cfv_math.hpp"

namespace cfv {

// Edge e of panel p (0 W: i = -1, 1 E: i = N, 2 S: j = -1, 3 N: j = N) touches
// panel q at (i', j') with each coordinate coded 0 -> 0, 1 -> N-1, 2 -> s,
// 3 -> N-1-s, where s is the position along the edge (j on W/E, i on S/N);
// back is the edge of q that leads back to p.
struct EdgeLink {
  int8_t q, ci, cj, back;
};
enum : int8_t { EW = 0, EE = 1, ES = 2, EN = 3 };

__host__ __device__ inline EdgeLink edge_link(int p, int e) {
  // clang-format off
  const EdgeLink T[6][4] = {
    {{3, 1, 2, EE}, {1, 0, 2, EW}, {5, 2, 1, EN}, {4, 2, 0, ES}},
    {{0, 1, 2, EE}, {2, 0, 2, EW}, {5, 1, 3, EE}, {4, 1, 2, EE}},
    {{1, 1, 2, EE}, {3, 0, 2, EW}, {5, 3, 0, ES}, {4, 3, 1, EN}},
    {{2, 1, 2, EE}, {0, 0, 2, EW}, {5, 0, 2, EW}, {4, 0, 3, EW}},
    {{3, 3, 1, EN}, {1, 2, 1, EN}, {0, 2, 1, EN}, {2, 3, 1, EN}},
    {{3, 2, 0, ES}, {1, 3, 0, ES}, {2, 3, 0, ES}, {0, 2, 0, ES}},
  };
  // clang-format on
  return T[p][e];
}

__host__ __device__ inline int edge_coord(int code, int s, int M) {
  return code == 0 ? 0 : code == 1 ? M : code == 2 ? s : M - s;
}

struct Shape {
  int N, Nr;
  int64_t ncells, nb;
};

__host__ __device__ inline int64_t cell_index(const Shape& g, int p, int k, int j, int i) {
  return ((int64_t(p) * g.Nr + k) * g.N + j) * g.N + i;
}

__host__ __device__ inline void decode(const Shape& g, int64_t c, int& p, int& k, int& j, int& i) {
  i = int(c % g.N);
  int64_t t = c / g.N;
  j = int(t % g.N);
  t /= g.N;
  k = int(t % g.Nr);
  p = int(t / g.Nr);
}

struct Nbr {
  int64_t id;  // cell index, or ghost id (>= ncells)
  int p, k, j, i;
  int back;  // local face of the neighbour that faces back (cells only)
};

__host__ __device__ inline Nbr neighbour(const Shape& g, int p, int k, int j, int i, int lf) {
  Nbr n{0, p, k, j, i, lf ^ 1};
  const int N = g.N, M = g.N - 1;
  int e = -1, s = 0;
  switch (lf) {
    case 0:
      if (k == 0) { n.id = g.ncells + (int64_t(p) * N + j) * N + i; n.back = -1; return n; }
      n.k = k - 1; break;
    case 1:
      if (k == g.Nr - 1) { n.id = g.ncells + g.nb + (int64_t(p) * N + j) * N + i; n.back = -1; return n; }
      n.k = k + 1; break;
    case 2: if (i == 0) { e = EW; s = j; } else n.i = i - 1; break;
    case 3: if (i == M) { e = EE; s = j; } else n.i = i + 1; break;
    case 4: if (j == 0) { e = ES; s = i; } else n.j = j - 1; break;
    default: if (j == M) { e = EN; s = i; } else n.j = j + 1; break;
  }
  if (e >= 0) {
    EdgeLink L = edge_link(p, e);
    n.p = L.q;
    n.i = edge_coord(L.ci, s, M);
    n.j = edge_coord(L.cj, s, M);
    n.back = 2 + L.back;
  }
  n.id = cell_index(g, n.p, n.k, n.j, n.i);
  return n;
}

// ------------------------------------------------------------------ geometry
// D: unit corner directions [p][j'][i'][3], j', i' in 0..N; r: Nr+1 radii.
struct GeomRef {
  const double* D;
  const double* r;
};

__host__ __device__ inline V3 corner(const GeomRef& G, const Shape& g, int p, int jj, int ii) {
  const double* d = G.D + ((int64_t(p) * (g.N + 1) + jj) * (g.N + 1) + ii) * 3;
  return mk(d[0], d[1], d[2]);
}

// vertex offsets (dk, dj, di) per local face, ordered so that
// S = 1/2 (v2 - v0) x (v3 - v1) points out of the cell.
__host__ __device__ inline void face_vertex_offsets(int lf, int off[4][3]) {
  // clang-format off
  const int T[6][4][3] = {
    {{0,0,0},{0,1,0},{0,1,1},{0,0,1}},
    {{1,0,0},{1,0,1},{1,1,1},{1,1,0}},
    {{0,0,0},{1,0,0},{1,1,0},{0,1,0}},
    {{0,0,1},{0,1,1},{1,1,1},{1,0,1}},
    {{0,0,0},{0,0,1},{1,0,1},{1,0,0}},
    {{0,1,0},{1,1,0},{1,1,1},{0,1,1}},
  };
  // clang-format on
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 3; ++b) off[a][b] = T[lf][a][b];
}

// vector area (outward from cell (p,k,j,i)) and centroid of local face lf
__host__ __device__ inline void face_geom(const GeomRef& G, const Shape& g, int p, int k, int j, int i, int lf,
                                          V3& S, V3& xf) {
  int off[4][3];
  face_vertex_offsets(lf, off);
  V3 v[4];
  for (int a = 0; a < 4; ++a) {
    double r = G.r[k + off[a][0]];
    v[a] = r * corner(G, g, p, j + off[a][1], i + off[a][2]);
  }
  V3 c = cross3(v[2] - v[0], v[3] - v[1]);
  S = 0.5 * c;
  xf = 0.25 * (((v[0] + v[1]) + v[2]) + v[3]);
}

__host__ __device__ inline V3 cell_centre(const GeomRef& G, const Shape& g, int p, int k, int j, int i) {
  V3 s = ((corner(G, g, p, j, i) + corner(G, g, p, j, i + 1)) + corner(G, g, p, j + 1, i)) + corner(G, g, p, j + 1, i + 1);
  return (0.125 * (G.r[k] + G.r[k + 1])) * s;
}

// V = 1/3 sum_f x_f . S_f; only the two radial faces contribute (the angular
// faces lie in planes through the origin), giving (r1^3 - r0^3)/3 * omega.
__host__ __device__ inline double cell_volume(const GeomRef& G, const Shape& g, int p, int k, int j, int i) {
  V3 d0 = corner(G, g, p, j, i), d1 = corner(G, g, p, j, i + 1);
  V3 d2 = corner(G, g, p, j + 1, i + 1), d3 = corner(G, g, p, j + 1, i);
  V3 c = cross3(d2 - d0, d3 - d1);
  double omega = dot3(0.25 * (((d0 + d1) + d2) + d3), 0.5 * c);
  double r0 = G.r[k], r1 = G.r[k + 1];
  return (r1 * r1 * r1 - r0 * r0 * r0) * omega / 3.0;
}

// canonical geometry of the face across local face lf of cell (p,k,j,i): the
// owner's vector area (pointing from the owner to the other side) and the
// owner's centroid; owner tells whether (p,k,j,i) is the owner.
__host__ __device__ inline void canon_face(const GeomRef& G, const Shape& g, int p, int k, int j, int i, int lf,
                                           const Nbr& nb, int64_t self, V3& S, V3& xf, bool& owner) {
  owner = (nb.id >= g.ncells) || (nb.id > self);
  if (owner) {
    face_geom(G, g, p, k, j, i, lf, S, xf);
  } else {
    face_geom(G, g, nb.p, nb.k, nb.j, nb.i, nb.back, S, xf);
  }
}

// mirror of the boundary cell centre across its boundary face
__host__ __device__ inline V3 ghost_centre(V3 xI, V3 S, V3 xf) {
  double ia = 1.0 / norm3(S);
  V3 n = mk(S.x * ia, S.y * ia, S.z * ia);
  double d = dot3(xf - xI, n);
  return xI + (2.0 * d) * n;
}

}  // namespace cfv
