// Host emulation of the library's kernels (test infrastructure).
//
// The kernels are written as barrier-separated phase functions over a
// per-lane state (cfv_fused.hpp, cfv_march.hpp, cfv_vjp.hpp), all
// __host__ __device__.  This file runs them on the CPU: a workgroup is 256
// lane states and an LDS array, a barrier is the end of a loop over the lanes,
// so every phase function sees exactly the data the GPU kernel's would.  Built
// with AddressSanitizer and UndefinedBehaviorSanitizer, an index outside any
// array (LDS, the grid tables, U, the outputs, the workspaces) stops the run;
// LDS starts each work item filled with NaN, so a read of an LDS value the
// item never wrote reaches the outputs, which the tests compare with the
// oracle.
//
// C entry points (host arrays, layouts as in cfv.h): the residual by the
// fused march, the JVP by the two-pass dual march, the VJP by the gradient
// march with face states, the adjoint, the ghost fold and the gather.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include "cfv.h"
#include "cfv_fused.hpp"
#include "cfv_tables.hpp"
#include "cfv_vjp.hpp"

using namespace cfv;

namespace {

const double kPoison = std::numeric_limits<double>::quiet_NaN();

struct HostShell {
  GridTables t;
  DevGrid d;
  std::vector<double> br, bth;
  unsigned flag = 0;
  bool ok = false;
  HostShell(int N, int Nr, const double* r, const cfv_params* p, const double* br_in, const double* bth_in) {
    if (!build_grid_tables(N, Nr, r, t)) return;
    br.assign(br_in, br_in + t.g.nb);
    bth.assign(size_t(t.g.nb), 0.0);
    if (bth_in) bth.assign(bth_in, bth_in + t.g.nb);
    d.g = t.g;
    d.G = t.host_ref();
    d.pr.gamma = p->gamma;
    d.pr.c_h = p->c_h;
    d.pr.G = p->G;
    d.pr.vr_star = p->vr_star;
    d.pr.rho_b = p->rho_b;
    d.pr.T_b = p->T_b;
    d.pr.limiter = p->limiter;
    d.pr.inner_mode = p->inner_mode;
    for (int q = 0; q < 8; ++q) d.pr.outer_exp[q] = p->outer_exp[q];
    d.pr.outer_vr_mass = p->outer_vr_mass;
    d.pr.outer_psi_zero = p->outer_psi_zero;
    d.br = br.data();
    d.bth = bth.data();
    d.flag = &flag;
    d.ftab = t.ftab.data();
    ok = true;
  }
};

// the fused residual march, one work item (tile, chunk) after the other
void fused_residual(const MarchArgs& a, int kc) {
  using WG = FusedWG<double>;
  const Shape& g = a.d.g;
  std::vector<double> lds(size_t(WG::kLds));
  std::vector<FuState<double>> st(kFL);
  const int64_t items = fused_items(g, kc);
  for (int64_t l = 0; l < items; ++l) {
    FTile tm;
    fused_tile_of(g, kc, l, tm);
    std::fill(lds.begin(), lds.end(), kPoison);
    const int kb = tm.k0 > 0 ? tm.k0 - 1 : 0;
    const int ke = tm.k1 < g.Nr ? tm.k1 : tm.k1 - 1;
    for (int t = 0; t < kFL; ++t) WG::init(a, tm, st[t], t, kb, lds.data());
    for (int k = WG::first_publish(kb); k < kb; ++k)
      for (int t = 0; t < kFL; ++t) WG::publish_block(a, st[t], t, k, lds.data());
    for (int k = kb; k <= ke; ++k) {
      const int mode = k < tm.k0 ? 1 : k >= tm.k1 ? 2 : 0;
      for (int t = 0; t < kFL; ++t) WG::publish(a, tm, st[t], t, k, lds.data());
      for (int t = 0; t < kFL; ++t) WG::gradient(a, tm, st[t], t, k, mode, lds.data());
      if (mode == 0) {
        for (int t = 0; t < kFL; ++t) WG::flux(a, tm, st[t], t, k, lds.data());
        for (int t = 0; t < kFL; ++t) WG::accumulate(a, tm, st[t], t, k, lds.data());
      }
    }
    for (int t = 0; t < kFL; ++t) record_nonphysical(a.d, st[t].role == 1 && st[t].bad);
  }
}

// the two-pass march (gradient pass, then flux pass), as march.hip runs it
template <class T, bool Faces = false>
void grad_march(const MarchArgs& a, int kc) {
  const Shape& g = a.d.g;
  std::vector<double> lds(size_t(GradWG<T>::kLds));
  std::vector<GState<T>> st(kNT);
  for (int64_t l = 0; l < march_logical_blocks(g, kc); ++l) {
    TileMap tm;
    tile_of_logical(g, l, tm, kc);
    std::fill(lds.begin(), lds.end(), kPoison);
    for (int t = 0; t < kNT; ++t) GradWG<T>::init(a, tm, st[t], t, lds.data());
    for (int k = GradWG<T>::first_layer(tm); k < tm.k1; ++k) {
      if (k < tm.k0) {
        for (int t = 0; t < kNT; ++t) GradWG<T>::publish(a, tm, st[t], t, k, lds.data());
        continue;
      }
      for (int t = 0; t < kNT; ++t) {
        GradWG<T>::publish(a, tm, st[t], t, k, lds.data());
        if (t >= kNT / 4 && t < kNT / 2) GradWG<T>::ring(a, tm, st[t], t - kNT / 4, k, lds.data());
      }
      for (int t = 0; t < kNT; ++t) GradWG<T>::template compute<Faces>(a, tm, st[t], t, k, lds.data());
    }
  }
}

template <class T>
void flux_march(const MarchArgs& a, int kc) {
  const Shape& g = a.d.g;
  std::vector<double> lds(size_t(FluxWG<T>::kLds));
  std::vector<FState<T>> st(kNT);
  for (int64_t l = 0; l < march_logical_blocks(g, kc); ++l) {
    TileMap tm;
    tile_of_logical(g, l, tm, kc);
    std::fill(lds.begin(), lds.end(), kPoison);
    for (int t = 0; t < kNT; ++t) FluxWG<T>::init(a, tm, st[t], t);
    for (int k = FluxWG<T>::first_layer(tm); k <= FluxWG<T>::last_layer(g, tm); ++k) {
      if (k < tm.k0 || k >= tm.k1) {
        for (int t = 0; t < kNT; ++t) FluxWG<T>::states(a, tm, st[t], t, k, lds.data());
        continue;
      }
      for (int t = 0; t < kNT; ++t) {
        FluxWG<T>::states(a, tm, st[t], t, k, lds.data());
        if (t >= kNT / 4 && t < kNT / 4 + FluxWG<T>::kRing) FluxWG<T>::ring(a, tm, st[t], t - kNT / 4, k, lds.data());
      }
      for (int t = 0; t < kNT; ++t) FluxWG<T>::faces(a, tm, st[t], t, k, lds.data());
      for (int t = 0; t < kNT; ++t) FluxWG<T>::accumulate(a, tm, st[t], t, k, lds.data());
    }
    for (int t = 0; t < kNT; ++t) FluxWG<T>::finish(a, tm, st[t], t);
  }
}

}  // namespace

extern "C" {

// R = R(U, B_r) by the fused march with chunks of kc layers; flag (nullable)
// receives the non-physical state word.  Returns 0, or 1 on bad arguments.
int host_residual(int N, int Nr, const double* r, const cfv_params* p, const double* U, const double* br,
                  const double* bth, int kc, double* R, unsigned* flag) {
  if (kc < 1) return 1;
  HostShell s(N, Nr, r, p, br, bth);
  if (!s.ok) return 1;
  MarchArgs a{s.d, U, nullptr, nullptr, nullptr, nullptr, R, nullptr};
  fused_residual(a, kc);
  if (flag) *flag = s.flag;
  return 0;
}

// Jv = J_U v + J_b dbr (dbr nullable) by the dual two-pass march with chunks
// of kc layers; R (nullable) receives the residual it evaluates along.
int host_jvp(int N, int Nr, const double* r, const cfv_params* p, const double* U, const double* br,
             const double* bth, int kc, const double* v, const double* dbr, double* Jv, double* R) {
  if (kc < 1) return 1;
  HostShell s(N, Nr, r, p, br, bth);
  if (!s.ok) return 1;
  const int64_t nc = s.t.g.ncells;
  std::vector<double> G(size_t(27) * nc, kPoison), Gd(size_t(27) * nc, kPoison);
  MarchArgs a{s.d, U, v, dbr, G.data(), Gd.data(), R, Jv};
  grad_march<Dual>(a, kc);
  flux_march<Dual>(a, kc);
  return 0;
}

// gU = J_U^T w and gbr = J_b^T w (gbr nullable) by the adjoint passes, the
// forward gradient march in chunks of kc layers.
int host_vjp(int N, int Nr, const double* r, const cfv_params* p, const double* U, const double* br,
             const double* bth, int kc, const double* w, double* gU, double* gbr) {
  if (kc < 1) return 1;
  HostShell s(N, Nr, r, p, br, bth);
  if (!s.ok) return 1;
  const Shape& g = s.t.g;
  const int64_t nc = g.ncells;
  std::vector<double> W(size_t(36) * nc, kPoison);
  std::vector<double> A(size_t(vjp_workspace_size(g)), kPoison);
  double* Q = A.data() + int64_t(63) * nc;
  double* Gg = A.data() + int64_t(63 + 54) * nc;
  // pass 1: primitives and face states
  MarchArgs fa{s.d, U, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, W.data(), Q};
  grad_march<double, true>(fa, kc);
  // pass 2: the adjoint of each cell, with the block window of 256 cells
  std::vector<double> lW(size_t(63) * kVBlock), lw(size_t(9) * kVBlock);
  for (int64_t c0 = 0; c0 < nc; c0 += kVBlock) {
    std::fill(lW.begin(), lW.end(), kPoison);
    std::fill(lw.begin(), lw.end(), kPoison);
    for (int t = 0; t < kVBlock && c0 + t < nc; ++t) {
      for (int q = 0; q < 9; ++q) lW[q * kVBlock + t] = W[q * nc + c0 + t];
      for (int q = 0; q < 54; ++q) lW[(9 + q) * kVBlock + t] = Q[q * nc + c0 + t];
      for (int q = 0; q < 9; ++q) lw[q * kVBlock + t] = w[q * nc + c0 + t];
    }
    for (int t = 0; t < kVBlock && c0 + t < nc; ++t)
      adjoint_cell(s.d, w, W.data(), Q, A.data(), Gg, c0 + t, lW.data(), lw.data(), c0);
  }
  // pass 3: the ghost states' adjoints through the boundary laws
  for (int64_t col = 0; col < g.nb; ++col) ghost_fold_column(s.d, W.data(), Gg, A.data(), gbr, col);
  // pass 4: gather
  for (int64_t c = 0; c < nc; ++c) gather_cell(s.d, U, w, A.data(), gU, c);
  return 0;
}

}  // extern "C"
