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

// Lanes of one workgroup between two barriers: the device runs them in any
// interleaving, the emulation one lane after the other, first to last or (the
// tests run both) last to first.  A phase that reads what another lane writes
// before the next barrier gives different results in the two orders.
bool g_reverse = false;

template <class F>
void lanes(int n, F&& f) {
  for (int q = 0; q < n; ++q) f(g_reverse ? n - 1 - q : q);
}

// the fused residual march, one work item (tile, chunk) after the other, with
// the kernel's barriers (fused.hip) between the lane loops
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
    lanes(kFL, [&](int t) {
      WG::init(a, tm, st[t], t, kb, lds.data());
      for (int k = WG::first_publish(kb); k < kb; ++k) WG::publish_block(a, st[t], t, k, lds.data());
      WG::publish(a, tm, st[t], t, kb, lds.data());
    });
    for (int k = kb; k <= ke; ++k) {
      const int mode = k < tm.k0 ? 1 : k >= tm.k1 ? 2 : 0;
      lanes(kFL, [&](int t) {
        if (k - 1 >= tm.k0 && k - 1 < tm.k1) WG::accumulate(a, tm, st[t], t, k - 1, lds.data());
        WG::gradient(a, tm, st[t], t, k, mode, lds.data());
      });
      lanes(kFL, [&](int t) {
        if (mode == 0) WG::flux(a, tm, st[t], t, k, lds.data());
        if (k + 1 <= ke) WG::publish(a, tm, st[t], t, k + 1, lds.data());
      });
    }
    if (ke < tm.k1) lanes(kFL, [&](int t) { WG::accumulate(a, tm, st[t], t, ke, lds.data()); });
    for (int t = 0; t < kFL; ++t) record_nonphysical(a.d, st[t].role == 1 && st[t].bad);
  }
}

// the two-pass march (gradient pass, then flux pass), with march.hip's barriers
template <class T, bool Faces = false>
void grad_march(const MarchArgs& a, int kc) {
  const Shape& g = a.d.g;
  std::vector<double> lds(size_t(GradWG<T>::kLds));
  std::vector<GState<T>> st(kNT);
  for (int64_t l = 0; l < march_logical_blocks(g, kc); ++l) {
    TileMap tm;
    tile_of_logical(g, l, tm, kc);
    std::fill(lds.begin(), lds.end(), kPoison);
    // two barriers per layer (after the publish and ring steps, after the
    // compute): a segment is the previous layer's edge flush, the warm-up
    // and this layer's publish and ring, or its compute
    for (int k = tm.k0; k <= tm.k1; ++k) {
      lanes(kNT, [&](int t) {
        if (k == tm.k0) {  // the item's start and its warm-up layers
          GradWG<T>::init(a, tm, st[t], t, lds.data());
          for (int kw = GradWG<T>::first_layer(tm); kw < tm.k0; ++kw)
            GradWG<T>::publish(a, tm, st[t], t, kw, lds.data());
        }
        if (k > tm.k0) GradWG<T>::flush_edges(a, tm, t, k - 1, lds.data());
        if (k < tm.k1) {
          GradWG<T>::publish(a, tm, st[t], t, k, lds.data());  // and the dual pass's ring
          if (t >= kNT / 4 && t < kNT / 2) GradWG<T>::ring_late(a, tm, st[t], t - kNT / 4, k, lds.data());
        }
      });
      if (k < tm.k1) lanes(kNT, [&](int t) { GradWG<T>::template compute<Faces>(a, tm, st[t], t, k, lds.data()); });
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
    const int kf = FluxWG<T>::first_layer(tm), kl = FluxWG<T>::last_layer(g, tm);
    // two barriers per layer (after the states and ring slots, after the
    // faces): a segment is the faces, or the previous layer's accumulation,
    // the warm-up or cool-down states and this layer's states and ring slots
    for (int k = tm.k0; k <= tm.k1; ++k) {
      lanes(kNT, [&](int t) {
        if (k == tm.k0) {  // the item's start and its warm-up layer
          FluxWG<T>::init(a, tm, st[t], t);
          for (int kw = kf; kw < tm.k0; ++kw) FluxWG<T>::states(a, tm, st[t], t, kw, lds.data());
        }
        if (k > tm.k0) FluxWG<T>::accumulate(a, tm, st[t], t, k - 1, lds.data());
        if (k <= kl) FluxWG<T>::states(a, tm, st[t], t, k, lds.data());  // and the ring slots
        if (k == tm.k1) FluxWG<T>::finish(a, tm, st[t], t);
      });
      if (k < tm.k1) lanes(kNT, [&](int t) { FluxWG<T>::faces(a, tm, st[t], t, k, lds.data()); });
    }
  }
}

}  // namespace

extern "C" {

// Lane order of the emulated workgroups from now on: 0 first to last, 1 last
// to first.
void host_set_lane_order(int reverse) { g_reverse = reverse != 0; }

// The join of the two address halves behind the kernels' uniform (scalar)
// loads, as readfirstlane returns them.
uint64_t host_join_address(int hi, int lo) { return join_address(hi, lo); }

// The dual Barth-Jespersen limited gradient of one variable (limited_grad
// with T = Dual) for given least-squares weights W (6 x 3, so that the
// unlimited gradient is sum_n W_n (q_n - q_c)), face offsets dxf (6 x 3),
// the cell's and neighbours' values and tangents; out: gx, gy, gz values,
// then their tangents.
void host_limited_grad_dual(const double* W, const double* dxf, double qc_v, double qc_d, const double* qn_v,
                            const double* qn_d, int limiter, double* out) {
  V3 dx[6], df[6];
  for (int n = 0; n < 6; ++n) {
    dx[n] = mk(1.0, 0.0, 0.0);
    df[n] = mk(dxf[3 * n], dxf[3 * n + 1], dxf[3 * n + 2]);
  }
  LsqWeights L(dx);
  for (int n = 0; n < 6; ++n) L.W[n] = mk(W[3 * n], W[3 * n + 1], W[3 * n + 2]);
  Dual qn[6];
  for (int n = 0; n < 6; ++n) qn[n] = Dual(qn_v[n], qn_d[n]);
  Dual gx, gy, gz;
  limited_grad(L, df, limiter, Dual(qc_v, qc_d), qn, gx, gy, gz);
  out[0] = gx.v; out[1] = gy.v; out[2] = gz.v;
  out[3] = gx.d; out[4] = gy.d; out[5] = gz.d;
}

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
  std::vector<double> E(size_t(edge_buffer_doubles(s.t.g)), kPoison);
  MarchArgs a{s.d, U, v, dbr, G.data(), Gd.data(), R, Jv};
  a.E = E.data();
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
    // the variant the device runs for this window (interior windows leave
    // the ghost code out)
    const bool bnd = adjoint_window_has_boundary(g, c0);
    for (int t = 0; t < kVBlock && c0 + t < nc; ++t) {
      if (bnd)
        adjoint_cell<true>(s.d, w, W.data(), Q, A.data(), Gg, c0 + t, lW.data(), lw.data(), c0);
      else
        adjoint_cell<false>(s.d, w, W.data(), Q, A.data(), Gg, c0 + t, lW.data(), lw.data(), c0);
    }
  }
  // pass 3: the ghost states' adjoints through the boundary laws
  for (int64_t col = 0; col < g.nb; ++col) ghost_fold_column(s.d, W.data(), Gg, A.data(), gbr, col);
  // pass 4: gather
  for (int64_t c = 0; c < nc; ++c) gather_cell(s.d, U, w, A.data(), gU, c);
  return 0;
}

}  // extern "C"
