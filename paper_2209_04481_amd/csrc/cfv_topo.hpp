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

__host__ __device__ __forceinline__ EdgeLink edge_link(int p, int e) {
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

__host__ __device__ __forceinline__ int edge_coord(int code, int s, int M) {
  return code == 0 ? 0 : code == 1 ? M : code == 2 ? s : M - s;
}

struct Shape {
  int N, Nr;
  int64_t ncells, nb;
};

__host__ __device__ __forceinline__ int64_t cell_index(const Shape& g, int p, int k, int j, int i) {
  return ((int64_t(p) * g.Nr + k) * g.N + j) * g.N + i;
}

// (cell indices are below 2^31, which cfv_grid_create enforces: 32-bit
// unsigned division, far cheaper on the GPU than 64-bit)
__host__ __device__ __forceinline__ void decode(const Shape& g, int64_t c, int& p, int& k, int& j, int& i) {
  const uint32_t n = uint32_t(g.N), nr = uint32_t(g.Nr);
  uint32_t t = uint32_t(c);
  i = int(t % n);
  t /= n;
  j = int(t % n);
  t /= n;
  k = int(t % nr);
  p = int(t / nr);
}

struct Nbr {
  int64_t id;  // cell index, or ghost id (>= ncells)
  int p, k, j, i;
  int back;  // local face of the neighbour that faces back (cells only)
};

__host__ __device__ __forceinline__ Nbr neighbour(const Shape& g, int p, int k, int j, int i, int lf) {
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

// vertex offsets (dk, dj, di) per local face, ordered so that
// S = 1/2 (v2 - v0) x (v3 - v1) points out of the cell.
__host__ __device__ __forceinline__ void face_vertex_offsets(int lf, int off[4][3]) {
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

// ------------------------------------------------------------------ geometry
// All cell and face geometry is separable in the radius: a cell (column col,
// layer k) has centroid (r_k + r_{k+1})/8 * csum, volume (r_{k+1}^3 - r_k^3)/3 *
// omega, radial faces at radius r with vector area r^2 sr and centroid r xr,
// and angular faces with vector area (r_{k+1}^2 - r_k^2)/2 * a and centroid
// (r_k + r_{k+1})/4 * b.  The per-column numbers are built on the host from
// the cell vertices (the vertex formulas at unit radii), and for every angular
// face they are the OWNER's numbers, so both sides of a face use the same
// values.  Column tables, each of length ncol = 6N^2, component-major:
enum : int {
  CG_CSUM = 0, CG_OMEGA = 3, CG_SR = 4, CG_XR = 7, CG_ANG = 10,  // + 6*q: a (3), b (3), q = lf - 2
  CG_NCOMP = 34
};
// integer tables (component-major, 4 angular faces q = lf - 2):
//   cn[q*ncol + col]      neighbour column across face q
//   cn[(4+q)*ncol + col]  back local face of the neighbour | owner flag << 8
struct GeomRef {
  const double* cg;
  const int32_t* cn;
  const double* r;
  int64_t ncol;
};

// a 64-bit address from its halves as readfirstlane returns them (signed
// 32-bit ints): each half taken as unsigned, or the low half's bit 31 would
// spread over the high half and give an address outside any allocation
__host__ __device__ __forceinline__ uint64_t join_address(int hi, int lo) {
  return (uint64_t(uint32_t(hi)) << 32) | uint64_t(uint32_t(lo));
}
#if defined(__HIP_DEVICE_COMPILE__)
// an address that is the same in every lane, as the compiler's uniform value
__device__ __forceinline__ uint64_t uniform_address(const void* p) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  return join_address(__builtin_amdgcn_readfirstlane(int(uint32_t(a >> 32))),
                      __builtin_amdgcn_readfirstlane(int(uint32_t(a))));
}
#endif

// r_k for a layer k that is the same in every lane of the wavefront (the
// layer of a radial march): a scalar load.  A vector load would be waited for
// with the vector memory counter, which also counts the loads and stores in
// flight (a march's prefetch of the next layer, its residual stores), so
// using the radius would wait for all of them.
__host__ __device__ __forceinline__ double radius_uniform(const GeomRef& G, int k) {
#if defined(__HIP_DEVICE_COMPILE__)
  return *reinterpret_cast<const __attribute__((address_space(4))) double*>(uniform_address(G.r + k));
#else
  return G.r[k];
#endif
}

__host__ __device__ __forceinline__ int64_t column_of(const Shape& g, int p, int j, int i) {
  return (int64_t(p) * g.N + j) * g.N + i;
}

__host__ __device__ __forceinline__ V3 cg3(const GeomRef& G, int comp, int64_t col) {
  return mk(gld(G.cg, comp * G.ncol + col), gld(G.cg, (comp + 1) * G.ncol + col), gld(G.cg, (comp + 2) * G.ncol + col));
}

// r_k; kUniformK: k is the same in every lane (radius_uniform)
template <bool kUniformK = false>
__host__ __device__ __forceinline__ double radius(const GeomRef& G, int k) {
  return kUniformK ? radius_uniform(G, k) : gld(G.r, k);
}

template <bool kUniformK = false>
__host__ __device__ __forceinline__ V3 cell_centre(const GeomRef& G, const Shape& g, int p, int k, int j, int i) {
  return (0.125 * (radius<kUniformK>(G, k) + radius<kUniformK>(G, k + 1))) * cg3(G, CG_CSUM, column_of(g, p, j, i));
}

template <bool kUniformK = false>
__host__ __device__ __forceinline__ double cell_volume(const GeomRef& G, const Shape& g, int p, int k, int j, int i) {
  const double r0 = radius<kUniformK>(G, k), r1 = radius<kUniformK>(G, k + 1);
  return (r1 * r1 * r1 - r0 * r0 * r0) * gld(G.cg, CG_OMEGA * G.ncol + column_of(g, p, j, i)) * (1.0 / 3.0);
}

// canonical geometry of the face across local face lf of cell (p,k,j,i): the
// owner's vector area (pointing from the owner to the other side), the
// owner's centroid, and whether (p,k,j,i) is the owner.  The owner of a face
// is the cell with the lower index, or the interior cell on the boundary.
template <bool kUniformK = false>
__host__ __device__ __forceinline__ void canon_face_col(const GeomRef& G, int64_t col, int k, int lf, V3& S, V3& xf,
                                                        bool& owner) {
  if (lf < 2) {
    const double r = radius<kUniformK>(G, k + lf);
    const V3 sr = cg3(G, CG_SR, col);
    S = (r * r) * sr;
    xf = r * cg3(G, CG_XR, col);
    owner = lf == 1 || k == 0;
    if (lf == 0 && k == 0) S = mk(-S.x, -S.y, -S.z);  // boundary face: outward
    return;
  }
  const int q = lf - 2;
  const double r0 = radius<kUniformK>(G, k), r1 = radius<kUniformK>(G, k + 1);
  S = (0.5 * (r1 * r1 - r0 * r0)) * cg3(G, CG_ANG + 6 * q, col);
  xf = (0.25 * (r0 + r1)) * cg3(G, CG_ANG + 6 * q + 3, col);
  owner = (gld(G.cn, (4 + q) * G.ncol + col) >> 8) != 0;
}

template <bool kUniformK = false>
__host__ __device__ __forceinline__ void canon_face(const GeomRef& G, const Shape& g, int p, int k, int j, int i, int lf,
                                           const Nbr&, int64_t, V3& S, V3& xf, bool& owner) {
  canon_face_col<kUniformK>(G, column_of(g, p, j, i), k, lf, S, xf, owner);
}

// vector area pointing out of cell (p,k,j,i) and centroid of its face lf
__host__ __device__ __forceinline__ void face_geom(const GeomRef& G, const Shape& g, int p, int k, int j, int i, int lf,
                                          V3& S, V3& xf) {
  bool own;
  canon_face(G, g, p, k, j, i, lf, Nbr{}, 0, S, xf, own);
  if (!own) S = mk(-S.x, -S.y, -S.z);
}

// mirror of the boundary cell centre across its boundary face
__host__ __device__ __forceinline__ V3 ghost_centre(V3 xI, V3 S, V3 xf) {
  double ia = 1.0 / norm3(S);
  V3 n = mk(S.x * ia, S.y * ia, S.z * ia);
  double d = dot3(xf - xI, n);
  return xI + (2.0 * d) * n;
}

}  // namespace cfv
