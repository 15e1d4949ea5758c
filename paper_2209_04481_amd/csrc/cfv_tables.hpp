// Host construction of a shell's grid tables: the unit corner directions of
// the cubed-sphere panels, the per-column geometry and neighbour tables the
// kernels rebuild every cell's geometry from, and the per-tile stencil tables
// of the fused march.  Shared by the library (cfv_grid_create) and the host
// emulation of the kernels, so both see the same numbers.
#pragma once
#include <algorithm>
#include <cmath>
#include <vector>

#include "cfv_fused.hpp"

namespace cfv {

struct GridTables {
  Shape g;
  std::vector<double> r;      // Nr + 1
  std::vector<double> D;      // 6 (N+1)^2 3 unit corner directions
  std::vector<double> cg;     // CG_NCOMP x 6N^2 column geometry
  std::vector<int32_t> cn;    // 8 x 6N^2 angular neighbours and face ownership
  std::vector<int32_t> ftab;  // per-tile stencil tables of the fused march (cfv_fused.hpp)
  GeomRef host_ref() const {
    GeomRef G;
    G.cg = cg.data();
    G.cn = cn.data();
    G.r = r.data();
    G.ncol = g.nb;
    return G;
  }
};

// Unit corner directions of the equiangular gnomonic panels: node (p, jj, ii)
// points along the panel's direction at (tan xi_ii, tan eta_jj).
inline void build_corner_directions(GridTables& G) {
  const double kPiTables = 3.14159265358979323846;
  const int N = G.g.N;
  const int n1 = N + 1;
  G.D.resize(size_t(6) * n1 * n1 * 3);
  std::vector<double> t(n1);
  for (int q = 0; q <= N; ++q) t[q] = std::tan(-kPiTables / 4 + q * (kPiTables / 2) / N);
  for (int p = 0; p < 6; ++p)
    for (int jj = 0; jj <= N; ++jj)
      for (int ii = 0; ii <= N; ++ii) {
        const double a = t[ii], b = t[jj];
        double x, y, z;
        switch (p) {
          case 0: x = 1; y = a; z = b; break;
          case 1: x = -a; y = 1; z = b; break;
          case 2: x = -1; y = -a; z = b; break;
          case 3: x = a; y = -1; z = b; break;
          case 4: x = -b; y = a; z = 1; break;
          default: x = b; y = a; z = -1; break;
        }
        const double nrm = std::sqrt(x * x + y * y + z * z);
        double* d = &G.D[((size_t(p) * n1 + jj) * n1 + ii) * 3];
        d[0] = x / nrm;
        d[1] = y / nrm;
        d[2] = z / nrm;
      }
}

// Per-column geometry from the cell vertices at unit radii (see cfv_topo.hpp).
inline void build_column_tables(GridTables& G) {
  const Shape& s = G.g;
  const int N = s.N, n1 = N + 1;
  const int64_t ncol = s.nb;
  G.cg.assign(size_t(CG_NCOMP) * ncol, 0.0);
  G.cn.assign(size_t(8) * ncol, 0);
  auto D = [&](int p, int jj, int ii) {
    const double* d = &G.D[((size_t(p) * n1 + jj) * n1 + ii) * 3];
    return mk(d[0], d[1], d[2]);
  };
  auto put = [&](int comp, int64_t col, V3 v) {
    G.cg[comp * ncol + col] = v.x;
    G.cg[(comp + 1) * ncol + col] = v.y;
    G.cg[(comp + 2) * ncol + col] = v.z;
  };
  // vertex-formula area and centroid of local face lf of column (p,j,i) with
  // radii (ra, rb) for the layers dk = 0, 1
  auto face_at = [&](int p, int j, int i, int lf, double ra, double rb, V3& S, V3& xf) {
    int off[4][3];
    face_vertex_offsets(lf, off);
    V3 v[4];
    for (int a = 0; a < 4; ++a) v[a] = (off[a][0] ? rb : ra) * D(p, j + off[a][1], i + off[a][2]);
    S = 0.5 * cross3(v[2] - v[0], v[3] - v[1]);
    xf = 0.25 * (((v[0] + v[1]) + v[2]) + v[3]);
  };
  for (int p = 0; p < 6; ++p)
    for (int j = 0; j < N; ++j)
      for (int i = 0; i < N; ++i) {
        const int64_t col = column_of(s, p, j, i);
        put(CG_CSUM, col, ((D(p, j, i) + D(p, j, i + 1)) + D(p, j + 1, i)) + D(p, j + 1, i + 1));
        V3 sr, xr;
        face_at(p, j, i, 1, 1.0, 1.0, sr, xr);
        put(CG_SR, col, sr);
        put(CG_XR, col, xr);
        G.cg[CG_OMEGA * ncol + col] = dot3(xr, sr);
        for (int q = 0; q < 4; ++q) {
          const int lf = 2 + q;
          Nbr nb = neighbour(s, p, 0, j, i, lf);
          const int64_t ncolv = column_of(s, nb.p, nb.j, nb.i);
          const bool own = ncolv > col;
          V3 a, b, dummy;
          if (own) {
            face_at(p, j, i, lf, 0.0, 1.0, a, dummy);
            face_at(p, j, i, lf, 1.0, 1.0, dummy, b);
          } else {
            face_at(nb.p, nb.j, nb.i, nb.back, 0.0, 1.0, a, dummy);
            face_at(nb.p, nb.j, nb.i, nb.back, 1.0, 1.0, dummy, b);
          }
          put(CG_ANG + 6 * q, col, 2.0 * a);
          put(CG_ANG + 6 * q + 3, col, 2.0 * b);
          G.cn[q * ncol + col] = int32_t(ncolv);
          G.cn[(4 + q) * ncol + col] = nb.back | (own ? 256 : 0);
        }
      }
}

// Per-tile stencil tables of the fused march (layout in cfv_fused.hpp): for
// each 14 x 14 tile, the cell each lane of its 16 x 16 block holds (the tile
// inside, the ring of face neighbours across its edges around it), and for
// each ring cell the positions of its four angular neighbours among the
// block's lanes and the further outer slots, and the face it shares with the
// tile.  Returns false if a tile needs more outer slots than the layout holds.
inline bool build_tile_tables(GridTables& G) {
  const Shape& s = G.g;
  const int N = s.N, nt = fused_tiles_1d(N);
  G.ftab.assign(size_t(fused_tile_count(s)) * kFTab, -1);
  for (int p = 0; p < 6; ++p)
    for (int tjb = 0; tjb < nt; ++tjb)
      for (int tib = 0; tib < nt; ++tib) {
        const int i0 = tib * kFT, j0 = tjb * kFT;
        const int wi = std::min(kFT, N - i0), wj = std::min(kFT, N - j0);
        int32_t* T = &G.ftab[size_t((int64_t(p) * nt + tjb) * nt + tib) * kFTab];
        for (int bj = 0; bj < kFB; ++bj)
          for (int bi = 0; bi < kFB; ++bi) {
            const int t = bj * kFB + bi, role = fused_role(bi, bj, wi, wj);
            if (role == 1) {
              T[kFTabCol + t] = int32_t(column_of(s, p, j0 + bj - 1, i0 + bi - 1));
            } else if (role == 2) {
              // the tile cell next to this ring lane and its face toward it
              int ci = bi - 1, cj = bj - 1, lf;
              if (bi == 0) { ci = 0; lf = 2; }
              else if (bi == wi + 1) { ci = wi - 1; lf = 3; }
              else if (bj == 0) { cj = 0; lf = 4; }
              else { cj = wj - 1; lf = 5; }
              const Nbr nb = neighbour(s, p, 0, j0 + cj, i0 + ci, lf);
              T[kFTabCol + t] = int32_t(column_of(s, nb.p, nb.j, nb.i));
              T[kFTabBack + t] = nb.back;
            }
          }
        std::vector<int64_t> outer;
        for (int t = 0; t < kFL; ++t) {
          if (fused_role(t % kFB, t / kFB, wi, wj) != 2) continue;
          int rp, rj, ri;
          column_pji(s, T[kFTabCol + t], rp, rj, ri);
          for (int q = 0; q < 4; ++q) {
            const Nbr n2 = neighbour(s, rp, 0, rj, ri, 2 + q);
            const int64_t nc = column_of(s, n2.p, n2.j, n2.i);
            int pos = -1;
            for (int u = 0; u < kFL && pos < 0; ++u)
              if (T[kFTabCol + u] == nc && fused_role(u % kFB, u / kFB, wi, wj) != 0) pos = u;
            if (pos < 0) {
              size_t e = 0;
              while (e < outer.size() && outer[e] != nc) ++e;
              if (e == outer.size()) outer.push_back(nc);
              pos = kFL + int(e);
            }
            T[kFTabNb + 4 * t + q] = pos;
          }
        }
        if (outer.size() > size_t(kOuterSlots)) return false;
        for (size_t e = 0; e < outer.size(); ++e) T[kFTabOcol + e] = int32_t(outer[e]);
      }
  return true;
}

// All tables of the shell with 6 N x N panels and the Nr + 1 radii r (the
// caller has checked the arguments); false if a tile of the fused march needs
// more outer stencil slots than its layout holds.
inline bool build_grid_tables(int N, int Nr, const double* r, GridTables& G) {
  G.g.N = N;
  G.g.Nr = Nr;
  G.g.nb = 6LL * N * N;
  G.g.ncells = G.g.nb * Nr;
  G.r.assign(r, r + Nr + 1);
  build_corner_directions(G);
  build_column_tables(G);
  return build_tile_tables(G);
}

}  // namespace cfv
