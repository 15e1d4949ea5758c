// C ABI of the coronal finite-volume MHD library: grid construction on the
// host, device contexts, and the stream-ordered entry points declared in
// include/cfv.h.
#include "../../include/cfv.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cfv_fused.hpp"
#include "cfv_kernels.hpp"
#include "cfv_march.hpp"
#include "cfv_step.hpp"
#include "cfv_tables.hpp"

namespace cfv {
int reduce_partials_per_vector();
hipError_t launch_efield(const DevGrid& d, const double* U, double* E3, double* stats8, double* part, hipStream_t s,
                         KernelTimer* t);
hipError_t launch_efree(int64_t nc, double gamma, const double* U, double* Uo, hipStream_t s, KernelTimer* t);
int efield_partials();
hipError_t launch_prim_delta_norms(int64_t nc, double gamma, const double* a, const double* b, double* out9,
                                   double* part, hipStream_t s, KernelTimer* t);
int monitor_partials();
hipError_t launch_norms(int64_t nc, const double* a, const double* b, double* out9, double* part, hipStream_t s);
hipError_t launch_dots(int64_t n, const double* V, int k, const double* w, double* out, double* part, hipStream_t s);
hipError_t launch_dots_noalloc(int64_t n, const double* V, int k, const double* w, double* out, hipStream_t s);
int dots_noalloc_max_vectors();
hipError_t launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);
hipError_t launch_fused_ensemble(const EnsembleLaunch& e, hipStream_t s, KernelTimer* t);
hipError_t launch_vjp(const DevGrid& d, const double* U, const double* w, double* gU, double* gbr, double* W,
                      double* A, MarchArgs* slot, int kc, const int64_t* bw, int64_t nbw, hipStream_t s,
                      KernelTimer* t);
int64_t vjp_workspace_doubles(const Shape& g);
int64_t adjoint_boundary_windows(const Shape& g, int64_t* out);
hipError_t launch_div_dev(int64_t n, const double* den, const double* x, double* y, hipStream_t s);
hipError_t launch_add_diag(int64_t nc, const double* diag, const double* x, double* w, hipStream_t s);
hipError_t launch_div_diag(int64_t nc, const double* diag, const double* x, double* y, hipStream_t s);
hipError_t launch_lincomb(int64_t n, int k, const double* y, const double* V, double* x, hipStream_t s);
hipError_t launch_norm2(int64_t n, const double* x, double* out, double* part, hipStream_t s);
hipError_t launch_axpy_dot(int64_t n, const double* coef, const double* x, double* w, const double* y, double* out,
                           double* part, hipStream_t s);
hipError_t launch_absmax(int64_t n, int nvar, const double* a, double* out, double* part, hipStream_t s);
hipError_t launch_ratio_max(int64_t n, int nvar, const double* x, const double* u, const double* sv, double* out,
                            double* part, hipStream_t s);
}  // namespace cfv

struct cfv_grid : cfv::GridTables {};

// Records an event pair around every kernel launch while enabled.
struct EventTimer : cfv::KernelTimer {
  struct Rec {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void begin(const char* name, hipStream_t s) override {
    Rec r{name, take(), take()};
    if (r.a) (void)hipEventRecord(r.a, s);
    recs.push_back(r);
  }
  void end(hipStream_t s) override {
    if (!recs.empty() && recs.back().b) (void)hipEventRecord(recs.back().b, s);
  }
  void recycle() {
    for (auto& r : recs) {
      if (r.a) pool.push_back(r.a);
      if (r.b) pool.push_back(r.b);
    }
    recs.clear();
  }
  ~EventTimer() override {
    recycle();
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

struct cfv_ctx {
  const cfv_grid* grid = nullptr;
  EventTimer timer;
  bool timing = false;
  cfv::KernelTimer* tm() { return timing ? &timer : nullptr; }
  int device = 0;
  cfv::Params pr{};
  double* dcg = nullptr;
  int32_t* dcn = nullptr;
  double* dr = nullptr;
  double* dbr = nullptr;
  double* dbth = nullptr;  // inner B_theta map (large-E law), zero until set
  double* W = nullptr;     // 36 ncells: primitives + limited gradients
  double* Wd = nullptr;    // 36 ncells: their tangents
  double* E = nullptr;     // dual march: tile-edge face states (edge_buffer_doubles)
  double* A = nullptr;     // adjoint workspace
  int64_t* dbwin = nullptr;  // the adjoint windows holding boundary-layer cells
  int64_t nbwin = 0;
  double* part = nullptr;  // reduction partials
  int part_vectors = 0;
  cfv::MarchArgs* slot = nullptr;  // descriptor of the current march launch
  // Krylov workspace (allocated on first use, grown as needed)
  int kry_m = 0;
  double* kry_V = nullptr;    // (m + 1) vectors of 9 ncells
  double* kry_w = nullptr;    // 9 ncells
  double* kry_r = nullptr;    // 9 ncells: residual / rhs scratch
  double* kry_d = nullptr;    // ncells: diagonal scratch
  double* kry_x = nullptr;    // 9 ncells: solution of the implicit step
  double* kry_s = nullptr;    // device scalars: H column (m + 2) and y (m)
  // second-derivative workspace (allocated on first use)
  double* dir_u = nullptr;    // 9 ncells: shifted state
  double* dir_g = nullptr;    // 9 ncells: second evaluation
  double* dir_b = nullptr;    // 3 x 6N^2: shifted maps and the second B_r gradient
  double* dir_s = nullptr;    // 32 device scalars
  // steady-march workspace (allocated on first use)
  double* st_u = nullptr;     // 9 ncells: the other state of the march
  double* st_m = nullptr;     // 9 device scalars: the monitor
  unsigned* dflag = nullptr;  // non-physical state word set by the kernels
  int32_t* dftab = nullptr;   // per-tile stencil tables of the fused march
  int precond = 0;            // GMRES preconditioner: 0 none, 1 Jacobi (right, by the diagonal)
  int chunk = 0;              // layers per work item of the marches (0: balanced_chunk per march)
  int fused_chunk = cfv::kKC;  // the balanced choices for this grid and device
  int dual_chunk = cfv::kKC;
  int march_chunk(bool dual) const { return chunk ? chunk : dual ? dual_chunk : fused_chunk; }
  cfv::DevGrid dev() const {
    cfv::DevGrid d;
    d.g = grid->g;
    d.G.cg = dcg;
    d.G.cn = dcn;
    d.G.r = dr;
    d.G.ncol = grid->g.nb;
    d.pr = pr;
    d.br = dbr;
    d.bth = dbth;
    d.flag = dflag;
    d.ftab = dftab;
    return d;
  }
};

namespace {
thread_local std::string g_err;

cfv_status fail(cfv_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

cfv_status hip_fail(hipError_t e, const char* where) {
  return fail(CFV_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define CFV_HIP(call)                                        \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return hip_fail(e_, #call);        \
  } while (0)

constexpr int kMaxChunk = 4096;  // largest chunk length (layers per work item)

cfv_status check_ctx(const cfv_ctx* c) {
  if (!c || !c->grid) return fail(CFV_ERR_ARG, "null context");
  return CFV_OK;
}

template <class T>
cfv_status dmalloc(T** p, size_t n) {
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T));
  if (e != hipSuccess) return fail(CFV_ERR_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e));
  return CFV_OK;
}
}  // namespace

extern "C" {

const char* cfv_last_error(void) { return g_err.c_str(); }

cfv_status cfv_grid_create(int32_t N, int32_t Nr, const double* r_nodes, cfv_grid** out) {
  g_err.clear();
  if (!out || !r_nodes) return fail(CFV_ERR_ARG, "null argument");
  if (N < 2 || Nr < 1) return fail(CFV_ERR_ARG, "need N >= 2 and Nr >= 1");
  if (N > 16384) return fail(CFV_ERR_ARG, "need N <= 16384 (per-panel column indices are 32-bit)");
  if (6LL * N * N * Nr > 2147483647LL)
    return fail(CFV_ERR_ARG, "need 6 N^2 Nr < 2^31 cells (one-thread-per-cell launches use 32-bit grids)");
  for (int k = 0; k < Nr; ++k)
    if (!(r_nodes[k + 1] > r_nodes[k]) || !(r_nodes[k] > 0.0))
      return fail(CFV_ERR_ARG, "r_nodes must be positive and strictly increasing");
  cfv_grid* g = new (std::nothrow) cfv_grid;
  if (!g) return fail(CFV_ERR_ALLOC, "host allocation");
  if (!cfv::build_grid_tables(N, Nr, r_nodes, *g)) {
    delete g;
    return fail(CFV_ERR_ARG, "a tile needs more outer stencil slots than the fused march holds");
  }
  *out = g;
  return CFV_OK;
}

void cfv_grid_destroy(cfv_grid* g) { delete g; }

cfv_status cfv_grid_sizes(const cfv_grid* g, int64_t* ncells, int64_t* nfaces, int64_t* nbnd) {
  if (!g) return fail(CFV_ERR_ARG, "null grid");
  const int64_t n2 = int64_t(g->g.N) * g->g.N;
  if (ncells) *ncells = g->g.ncells;
  if (nfaces) *nfaces = 6 * n2 * (g->g.Nr + 1) + 12 * n2 * g->g.Nr;
  if (nbnd) *nbnd = g->g.nb;
  return CFV_OK;
}

cfv_status cfv_grid_faces_to_host(const cfv_grid* g, int64_t* L, int64_t* R, int8_t* kind) {
  if (!g || !L || !R || !kind) return fail(CFV_ERR_ARG, "null argument");
  const cfv::Shape& s = g->g;
  int64_t f = 0;
  for (int64_t c = 0; c < s.ncells; ++c) {
    int p, k, j, i;
    cfv::decode(s, c, p, k, j, i);
    for (int lf = 0; lf < 6; ++lf) {
      cfv::Nbr nb = cfv::neighbour(s, p, k, j, i, lf);
      if (nb.id >= s.ncells || nb.id > c) {
        L[f] = c;
        R[f] = nb.id;
        kind[f] = nb.id >= s.ncells + s.nb ? 2 : (nb.id >= s.ncells ? 1 : 0);
        ++f;
      }
    }
  }
  return CFV_OK;
}

cfv_status cfv_grid_geometry_to_host(const cfv_grid* g, double* S_f, double* x_f, double* V_c, double* x_c) {
  if (!g || !S_f || !x_f || !V_c || !x_c) return fail(CFV_ERR_ARG, "null argument");
  const cfv::Shape& s = g->g;
  const cfv::GeomRef G = g->host_ref();
  int64_t f = 0;
  for (int64_t c = 0; c < s.ncells; ++c) {
    int p, k, j, i;
    cfv::decode(s, c, p, k, j, i);
    const cfv::V3 xc = cfv::cell_centre(G, s, p, k, j, i);
    x_c[3 * c] = xc.x;
    x_c[3 * c + 1] = xc.y;
    x_c[3 * c + 2] = xc.z;
    V_c[c] = cfv::cell_volume(G, s, p, k, j, i);
    for (int lf = 0; lf < 6; ++lf) {
      const cfv::Nbr nb = cfv::neighbour(s, p, k, j, i, lf);
      if (!(nb.id >= s.ncells || nb.id > c)) continue;
      cfv::V3 S, xf;
      bool own;
      cfv::canon_face(G, s, p, k, j, i, lf, nb, c, S, xf, own);
      S_f[3 * f] = S.x;
      S_f[3 * f + 1] = S.y;
      S_f[3 * f + 2] = S.z;
      x_f[3 * f] = xf.x;
      x_f[3 * f + 1] = xf.y;
      x_f[3 * f + 2] = xf.z;
      ++f;
    }
  }
  return CFV_OK;
}

cfv_status cfv_ctx_create(const cfv_grid* g, const cfv_params* prm, cfv_ctx** out) {
  g_err.clear();
  if (!g || !prm || !out) return fail(CFV_ERR_ARG, "null argument");
  if (!(prm->gamma > 1.0) || !(prm->c_h > 0.0) || prm->G < 0.0 || !(prm->rho_b > 0.0) || !(prm->T_b > 0.0))
    return fail(CFV_ERR_ARG, "need gamma > 1, c_h > 0, G >= 0, rho_b > 0, T_b > 0");
  if (prm->limiter != 0 && prm->limiter != 1) return fail(CFV_ERR_ARG, "limiter must be 0 or 1");
  if (prm->inner_mode != 0 && prm->inner_mode != 1)
    return fail(CFV_ERR_ARG, "inner_mode must be 0 (low-E) or 1 (large-E)");
  cfv_ctx* c = new (std::nothrow) cfv_ctx;
  if (!c) return fail(CFV_ERR_ALLOC, "host allocation");
  c->grid = g;
  CFV_HIP(hipGetDevice(&c->device));
  {
    int cus = 0;
    CFV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
    if (cus < 1) cus = 1;
    // one workgroup of either march per compute unit (LDS and registers)
    const cfv::Shape& sh = g->g;
    const int64_t dual_tiles = 6LL * ((sh.N + cfv::kTI - 1) / cfv::kTI) * ((sh.N + cfv::kTJ - 1) / cfv::kTJ);
    c->fused_chunk = cfv::balanced_chunk(cfv::fused_tile_count(sh), sh.Nr, cus);
    c->dual_chunk = cfv::balanced_chunk(dual_tiles, sh.Nr, cus);
  }
  c->pr.gamma = prm->gamma;
  c->pr.c_h = prm->c_h;
  c->pr.G = prm->G;
  c->pr.vr_star = prm->vr_star;
  c->pr.rho_b = prm->rho_b;
  c->pr.T_b = prm->T_b;
  c->pr.limiter = prm->limiter;
  c->pr.inner_mode = prm->inner_mode;
  for (int q = 0; q < 8; ++q) c->pr.outer_exp[q] = prm->outer_exp[q];
  c->pr.outer_vr_mass = prm->outer_vr_mass;
  c->pr.outer_psi_zero = prm->outer_psi_zero;
  const int64_t nc = g->g.ncells;
  cfv_status st;
  c->part_vectors = 32;
  if ((st = dmalloc(&c->dcg, g->cg.size())) || (st = dmalloc(&c->dcn, g->cn.size())) ||
      (st = dmalloc(&c->dr, g->r.size())) ||
      (st = dmalloc(&c->dbr, size_t(g->g.nb))) || (st = dmalloc(&c->dbth, size_t(g->g.nb))) ||
      (st = dmalloc(&c->W, size_t(36) * nc)) ||
      (st = dmalloc(&c->Wd, size_t(36) * nc)) || (st = dmalloc(&c->E, size_t(cfv::edge_buffer_doubles(g->g)))) ||
      (st = dmalloc(&c->A, size_t(cfv::vjp_workspace_doubles(g->g)))) ||
      (st = dmalloc(&c->part, size_t(c->part_vectors) * cfv::reduce_partials_per_vector())) ||
      (st = dmalloc(&c->slot, 1)) || (st = dmalloc(&c->dflag, 1)) || (st = dmalloc(&c->dftab, g->ftab.size()))) {
    cfv_ctx_destroy(c);
    return st;
  }
  std::vector<int64_t> bwin(size_t(cfv::adjoint_boundary_windows(g->g, nullptr)));
  c->nbwin = cfv::adjoint_boundary_windows(g->g, bwin.data());
  if ((st = dmalloc(&c->dbwin, bwin.size() > 0 ? bwin.size() : 1))) {
    cfv_ctx_destroy(c);
    return st;
  }
  hipError_t e = hipMemcpy(c->dcg, g->cg.data(), g->cg.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->dcn, g->cn.data(), g->cn.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->dr, g->r.data(), g->r.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(c->dbr, 0, size_t(g->g.nb) * sizeof(double));
  if (e == hipSuccess) e = hipMemset(c->dbth, 0, size_t(g->g.nb) * sizeof(double));
  if (e == hipSuccess) e = hipMemset(c->dflag, 0, sizeof(unsigned));
  if (e == hipSuccess)
    e = hipMemcpy(c->dftab, g->ftab.data(), g->ftab.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && !bwin.empty())
    e = hipMemcpy(c->dbwin, bwin.data(), bwin.size() * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    cfv_ctx_destroy(c);
    return hip_fail(e, "uploading grid tables");
  }
  *out = c;
  return CFV_OK;
}

void cfv_ctx_destroy(cfv_ctx* c) {
  if (!c) return;
  double* bufs[] = {c->dcg, c->dr, c->dbr, c->dbth, c->W, c->Wd, c->E, c->A, c->part};
  for (double* b : bufs)
    if (b) (void)hipFree(b);
  if (c->dcn) (void)hipFree(c->dcn);
  if (c->slot) (void)hipFree(c->slot);
  if (c->dflag) (void)hipFree(c->dflag);
  if (c->dftab) (void)hipFree(c->dftab);
  if (c->dbwin) (void)hipFree(c->dbwin);
  double* kb[] = {c->kry_V, c->kry_w, c->kry_r, c->kry_d, c->kry_s, c->kry_x,
                  c->dir_u, c->dir_g, c->dir_b, c->dir_s, c->st_u, c->st_m};
  for (double* b : kb)
    if (b) (void)hipFree(b);
  delete c;
}

cfv_status cfv_set_inner_br(cfv_ctx* c, const double* br, int64_t n, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!br) return fail(CFV_ERR_ARG, "null B_r map");
  if (n != c->grid->g.nb) return fail(CFV_ERR_SIZE, "B_r map length must be 6 N^2");
  CFV_HIP(hipMemcpyAsync(c->dbr, br, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
  return CFV_OK;
}

cfv_status cfv_set_inner_btheta(cfv_ctx* c, const double* bth, int64_t n, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!bth) return fail(CFV_ERR_ARG, "null B_theta map");
  if (n != c->grid->g.nb) return fail(CFV_ERR_SIZE, "B_theta map length must be 6 N^2");
  CFV_HIP(hipMemcpyAsync(c->dbth, bth, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
  return CFV_OK;
}

cfv_status cfv_geometry(cfv_ctx* c, double* xc, double* vol, double* xf, double* S, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!xc || !vol || !xf || !S) return fail(CFV_ERR_ARG, "null output");
  CFV_HIP(cfv::launch_geometry(c->dev(), xc, vol, xf, S, s));
  return CFV_OK;
}

cfv_status cfv_residual(cfv_ctx* c, const double* U, double* R, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!U || !R) return fail(CFV_ERR_ARG, "null state or output");
  cfv::MarchArgs a{c->dev(), U, nullptr, nullptr, c->W, nullptr, R, nullptr};
  CFV_HIP(cfv::launch_march(a, c->slot, false, c->march_chunk(false), s, c->tm()));
  return CFV_OK;
}

cfv_status cfv_jvp(cfv_ctx* c, const double* U, const double* v, const double* dbr, double* Jv, double* R,
                   hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!U || !v || !Jv) return fail(CFV_ERR_ARG, "null state, direction or output");
  cfv::MarchArgs a{c->dev(), U, v, dbr, c->W, c->Wd, R, Jv};
  a.E = c->E;
  CFV_HIP(cfv::launch_march(a, c->slot, true, c->march_chunk(true), s, c->tm()));
  return CFV_OK;
}

cfv_status cfv_vjp(cfv_ctx* c, const double* U, const double* w, double* gU, double* gbr, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!U || !w || !gU) return fail(CFV_ERR_ARG, "null state, weights or output");
  CFV_HIP(cfv::launch_vjp(c->dev(), U, w, gU, gbr, c->W, c->A, c->slot, c->march_chunk(true), c->dbwin, c->nbwin, s,
                          c->tm()));
  return CFV_OK;
}

cfv_status cfv_local_dt(cfv_ctx* c, const double* U, double cfl, double* diag, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!U || !diag) return fail(CFV_ERR_ARG, "null state or output");
  if (!(cfl > 0.0)) return fail(CFV_ERR_ARG, "cfl must be positive");
  CFV_HIP(cfv::launch_local_dt(c->dev(), U, cfl, diag, c->W, s, c->tm()));
  return CFV_OK;
}

// read and clear a device flag word (synchronises s)
static cfv_status take_flags(unsigned* dflag, unsigned* out, hipStream_t s) {
  unsigned h = 0;
  CFV_HIP(hipMemcpyAsync(&h, dflag, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  CFV_HIP(hipStreamSynchronize(s));
  if (h) CFV_HIP(hipMemsetAsync(dflag, 0, sizeof(unsigned), s));
  *out = h;
  return CFV_OK;
}

cfv_status cfv_status_flags(cfv_ctx* c, int32_t* flags, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  unsigned h = 0;
  if (cfv_status st = take_flags(c->dflag, &h, s)) return st;
  if (flags) *flags = int32_t(h);
  if (h & 1u) return fail(CFV_ERR_NONPHYSICAL, "a face state with non-positive or NaN density or pressure was met");
  return CFV_OK;
}

cfv_status cfv_efield(cfv_ctx* c, const double* U, double* E3, double* stats8, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!U || !stats8) return fail(CFV_ERR_ARG, "null state or statistics output");
  if (cfv::efield_partials() > c->part_vectors * cfv::reduce_partials_per_vector())
    return fail(CFV_ERR_ALLOC, "reduction workspace too small");
  CFV_HIP(cfv::launch_efield(c->dev(), U, E3, stats8, c->part, s, c->tm()));
  return CFV_OK;
}

cfv_status cfv_efree_state(cfv_ctx* c, const double* U, double* U_out, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!U || !U_out) return fail(CFV_ERR_ARG, "null state or output");
  const int64_t n = 9 * c->grid->g.ncells;
  if (U != U_out && U_out < U + n && U < U_out + n) return fail(CFV_ERR_ARG, "U_out partially overlaps U");
  CFV_HIP(cfv::launch_efree(c->grid->g.ncells, c->pr.gamma, U, U_out, s, c->tm()));
  return CFV_OK;
}

cfv_status cfv_norms(cfv_ctx* c, const double* a, const double* b, double* out9, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!a || !out9) return fail(CFV_ERR_ARG, "null input or output");
  CFV_HIP(cfv::launch_norms(c->grid->g.ncells, a, b, out9, c->part, s));
  return CFV_OK;
}

cfv_status cfv_dots(cfv_ctx* c, const double* V, int32_t k, const double* w, double* out, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!V || !w || !out) return fail(CFV_ERR_ARG, "null input or output");
  if (k < 1 || k > c->part_vectors) return fail(CFV_ERR_ARG, "k must be in 1..32");
  CFV_HIP(cfv::launch_dots(9 * c->grid->g.ncells, V, k, w, out, c->part, s));
  return CFV_OK;
}

cfv_status cfv_dots_noalloc(int64_t n, const double* V, int32_t k, const double* w, double* out, hipStream_t s) {
  if (!V || !w || !out) return fail(CFV_ERR_ARG, "null input or output");
  if (n < 0) return fail(CFV_ERR_ARG, "n must be non-negative");
  if (k < 1 || k > cfv::dots_noalloc_max_vectors())
    return fail(CFV_ERR_ARG, "k must be in 1.." + std::to_string(cfv::dots_noalloc_max_vectors()) +
                                 " (the static partial-sum array holds that many vectors)");
  CFV_HIP(cfv::launch_dots_noalloc(n, V, k, w, out, s));
  return CFV_OK;
}

cfv_status cfv_axpby(cfv_ctx* c, int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!x || !y || n < 0) return fail(CFV_ERR_ARG, "bad vector arguments");
  CFV_HIP(cfv::launch_axpby(n, a, x, b, y, s));
  return CFV_OK;
}

// ------------------------------------------------------------------ solver
static cfv_status ensure_krylov(cfv_ctx* c, int m) {
  if (c->kry_m >= m) return CFV_OK;
  double* kb[] = {c->kry_V, c->kry_w, c->kry_r, c->kry_d, c->kry_s, c->kry_x};
  for (double* b : kb)
    if (b) (void)hipFree(b);
  c->kry_V = c->kry_w = c->kry_r = c->kry_d = c->kry_s = c->kry_x = nullptr;
  c->kry_m = 0;
  const size_t n = size_t(9) * c->grid->g.ncells;
  cfv_status st;
  if ((st = dmalloc(&c->kry_V, size_t(m + 1) * n)) || (st = dmalloc(&c->kry_w, n)) || (st = dmalloc(&c->kry_r, n)) ||
      (st = dmalloc(&c->kry_d, size_t(c->grid->g.ncells))) || (st = dmalloc(&c->kry_s, size_t(2 * m + 4))) ||
      (st = dmalloc(&c->kry_x, n)))
    return st;
  c->kry_m = m;
  return CFV_OK;
}

// w = (diag + J) x  or  (diag + J^T) x
static cfv_status apply_operator(cfv_ctx* c, const double* U, const double* diag, int transpose, const double* x,
                                 double* w, hipStream_t s) {
  if (transpose) {
    CFV_HIP(cfv::launch_vjp(c->dev(), U, x, w, nullptr, c->W, c->A, c->slot, c->march_chunk(true), c->dbwin, c->nbwin,
                            s, c->tm()));
  } else {
    cfv::MarchArgs a{c->dev(), U, x, nullptr, c->W, c->Wd, nullptr, w};
    a.E = c->E;
    CFV_HIP(cfv::launch_march(a, c->slot, true, c->march_chunk(true), s, c->tm()));
  }
  CFV_HIP(cfv::launch_add_diag(c->grid->g.ncells, diag, x, w, s));
  return CFV_OK;
}

cfv_status cfv_solve(cfv_ctx* c, const double* U, const double* diag, const double* rhs, int32_t transpose,
                     int32_t m, int32_t max_restarts, double rtol, double* x, double* hist, int32_t hist_len,
                     int32_t* iters, double* final_rel, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!U || !diag || !rhs || !x) return fail(CFV_ERR_ARG, "null argument");
  if (m < 1 || m > 200 || max_restarts < 0) return fail(CFV_ERR_ARG, "need 1 <= m <= 200 and max_restarts >= 0");
  if (cfv_status st = ensure_krylov(c, m)) return st;
  const int64_t n = 9 * c->grid->g.ncells;
  double* V = c->kry_V;
  double* w = c->kry_w;
  double* r = c->kry_r;
  double* hd = c->kry_s;           // H column on the device (m + 2)
  double* yd = c->kry_s + m + 2;   // least-squares solution (m)
  std::vector<double> H(size_t(m + 1) * m), cs(m), sn(m), g(m + 1), col(m + 2), y(m);
  auto Hc = [&](int i, int j) -> double& { return H[size_t(i) * m + j]; };
  CFV_HIP(hipMemsetAsync(x, 0, size_t(n) * sizeof(double), s));
  // |rhs| for the relative residual
  double bnorm = 0.0;
  CFV_HIP(cfv::launch_norm2(n, rhs, hd, c->part, s));
  CFV_HIP(hipMemcpyAsync(&bnorm, hd, sizeof(double), hipMemcpyDeviceToHost, s));
  CFV_HIP(hipStreamSynchronize(s));
  if (!std::isfinite(bnorm)) return fail(CFV_ERR_NONPHYSICAL, "the right-hand side is not finite");
  int total = 0;
  double rel = bnorm > 0.0 ? 1.0 : 0.0;
  if (bnorm == 0.0) {
    if (iters) *iters = 0;
    if (final_rel) *final_rel = 0.0;
    return CFV_OK;
  }
  for (int cycle = 0; cycle <= max_restarts; ++cycle) {
    // r = rhs - A x
    if (cycle == 0) {
      CFV_HIP(hipMemcpyAsync(r, rhs, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
      if (cfv_status st = apply_operator(c, U, diag, transpose, x, w, s)) return st;
      CFV_HIP(cfv::launch_axpby(n, 1.0, rhs, 0.0, r, s));
      CFV_HIP(cfv::launch_axpby(n, -1.0, w, 1.0, r, s));
    }
    double beta = 0.0;
    CFV_HIP(cfv::launch_norm2(n, r, hd, c->part, s));
    CFV_HIP(hipMemcpyAsync(&beta, hd, sizeof(double), hipMemcpyDeviceToHost, s));
    CFV_HIP(cfv::launch_div_dev(n, hd, r, V, s));
    CFV_HIP(hipStreamSynchronize(s));
    if (!std::isfinite(beta)) return fail(CFV_ERR_NONPHYSICAL, "the Krylov residual is not finite");
    if (!(beta > 0.0)) break;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int kdone = 0;
    bool stop = false;
    for (int j = 0; j < m; ++j) {
      double* vj = V + size_t(j) * n;
      if (c->precond == 1) {  // right preconditioning: w = A D^-1 v_j (r is free inside the cycle)
        CFV_HIP(cfv::launch_div_diag(c->grid->g.ncells, diag, vj, r, s));
        vj = r;
      }
      if (cfv_status st = apply_operator(c, U, diag, transpose, vj, w, s)) return st;
      // modified Gram-Schmidt, coefficients on the device: h_0 = <w, V_0>, then
      // each update w -= h_i V_i is fused with the next projection
      // h_{i+1} = <w, V_{i+1}> (for i = j: the norm of w)
      CFV_HIP(cfv::launch_dots(n, V, 1, w, hd, c->part, s));
      for (int i = 0; i <= j; ++i)
        CFV_HIP(cfv::launch_axpy_dot(n, hd + i, V + size_t(i) * n, w, i < j ? V + size_t(i + 1) * n : nullptr,
                                     hd + i + 1, c->part, s));
      CFV_HIP(hipMemcpyAsync(col.data(), hd, size_t(j + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
      CFV_HIP(hipStreamSynchronize(s));
      for (int i = 0; i <= j + 1; ++i) {
        if (!std::isfinite(col[i])) return fail(CFV_ERR_NONPHYSICAL, "a Krylov projection is not finite");
        Hc(i, j) = col[i];
      }
      const double hnext = col[j + 1];
      if (hnext > 0.0) CFV_HIP(cfv::launch_div_dev(n, hd + j + 1, w, V + size_t(j + 1) * n, s));
      // Givens rotations on the new column
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * Hc(i, j) + sn[i] * Hc(i + 1, j);
        Hc(i + 1, j) = -sn[i] * Hc(i, j) + cs[i] * Hc(i + 1, j);
        Hc(i, j) = t;
      }
      const double den = std::hypot(Hc(j, j), Hc(j + 1, j));
      cs[j] = Hc(j, j) / den;
      sn[j] = Hc(j + 1, j) / den;
      Hc(j, j) = den;
      Hc(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      rel = std::fabs(g[j + 1]) / bnorm;
      if (hist && total < hist_len) hist[total] = rel;
      ++total;
      kdone = j + 1;
      if (rel <= rtol || !(hnext > 0.0)) {
        stop = true;
        break;
      }
    }
    // back substitution and x += V y
    for (int i = kdone - 1; i >= 0; --i) {
      double t = g[i];
      for (int q = i + 1; q < kdone; ++q) t -= Hc(i, q) * y[q];
      y[i] = t / Hc(i, i);
    }
    CFV_HIP(hipMemcpyAsync(yd, y.data(), size_t(kdone) * sizeof(double), hipMemcpyHostToDevice, s));
    CFV_HIP(cfv::launch_lincomb(n, kdone, yd, V, w, s));
    if (c->precond == 1) {  // x += D^-1 V y
      CFV_HIP(cfv::launch_div_diag(c->grid->g.ncells, diag, w, r, s));
      CFV_HIP(cfv::launch_axpby(n, 1.0, r, 1.0, x, s));
    } else {
      CFV_HIP(cfv::launch_axpby(n, 1.0, w, 1.0, x, s));
    }
    CFV_HIP(hipStreamSynchronize(s));
    if (stop) break;
  }
  if (iters) *iters = total;
  if (final_rel) *final_rel = rel;
  return CFV_OK;
}

cfv_status cfv_be_step(cfv_ctx* c, const double* U, double cfl, int32_t m, int32_t max_restarts, double rtol,
                       double* U_new, double* hist, int32_t hist_len, int32_t* iters, double* final_rel,
                       hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!U || !U_new || U_new == U) return fail(CFV_ERR_ARG, "null state, or U_new aliases U");
  if (!(cfl > 0.0)) return fail(CFV_ERR_ARG, "cfl must be positive");
  if (m < 1 || m > 200) return fail(CFV_ERR_ARG, "need 1 <= m <= 200");
  if (cfv_status st = ensure_krylov(c, m)) return st;
  const int64_t n = 9 * c->grid->g.ncells;
  // U_new holds the right-hand side -R(U) during the solve
  cfv::MarchArgs a{c->dev(), U, nullptr, nullptr, c->W, nullptr, U_new, nullptr};
  CFV_HIP(cfv::launch_march(a, c->slot, false, c->march_chunk(false), s, c->tm()));
  CFV_HIP(cfv::launch_axpby(n, 0.0, U_new, -1.0, U_new, s));
  CFV_HIP(cfv::launch_local_dt(c->dev(), U, cfl, c->kry_d, c->W, s, c->tm()));
  if (cfv_status st = cfv_solve(c, U, c->kry_d, U_new, 0, m, max_restarts, rtol, c->kry_x, hist, hist_len, iters,
                                final_rel, s))
    return st;
  CFV_HIP(hipMemcpyAsync(U_new, U, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
  CFV_HIP(cfv::launch_axpby(n, 1.0, c->kry_x, 1.0, U_new, s));
  return CFV_OK;
}

// ------------------------------------------------------ steady march
cfv_status cfv_monitor(cfv_ctx* c, const double* a, const double* b, double* out9, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!a || !b || !out9) return fail(CFV_ERR_ARG, "null state or output");
  if (cfv::monitor_partials() > c->part_vectors * cfv::reduce_partials_per_vector())
    return fail(CFV_ERR_ALLOC, "reduction workspace too small");
  CFV_HIP(cfv::launch_prim_delta_norms(c->grid->g.ncells, c->pr.gamma, a, b, out9, c->part, s, c->tm()));
  return CFV_OK;
}

cfv_status cfv_steady(cfv_ctx* c, double* U, const cfv_steady_cfg* cfg, double* hist, double* cfl_hist,
                      int32_t* iters, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!U || !cfg) return fail(CFV_ERR_ARG, "null state or configuration");
  if (!(cfg->cfl0 > 0.0) || !(cfg->cfl_max >= cfg->cfl0)) return fail(CFV_ERR_ARG, "need 0 < cfl0 <= cfl_max");
  if (cfg->every < 1 || cfg->max_iters < 0) return fail(CFV_ERR_ARG, "need every >= 1 and max_iters >= 0");
  if (cfg->monitor < 0 || cfg->monitor > 8) return fail(CFV_ERR_ARG, "monitor must be a variable 0..8");
  if (cfg->m < 1 || cfg->m > 200 || cfg->max_restarts < 0) return fail(CFV_ERR_ARG, "need 1 <= m <= 200");
  if (iters) *iters = 0;
  const int64_t n = 9 * c->grid->g.ncells;
  if (!c->st_u) {
    cfv_status st;
    if ((st = dmalloc(&c->st_u, size_t(n))) || (st = dmalloc(&c->st_m, 9))) {
      if (c->st_u) (void)hipFree(c->st_u);
      c->st_u = c->st_m = nullptr;
      return st;
    }
  }
  double* cur = U;
  double* nxt = c->st_u;
  cfv_status out = CFV_OK;
  int32_t done = 0;
  while (done < cfg->max_iters) {
    const double cfl = std::min(std::ldexp(cfg->cfl0, done / cfg->every), cfg->cfl_max);
    out = cfv_be_step(c, cur, cfl, cfg->m, cfg->max_restarts, cfg->rtol, nxt, nullptr, 0, nullptr, nullptr, s);
    if (out == CFV_ERR_NONPHYSICAL) {  // the step is counted, its monitors are NaN, U keeps the state before it
      if (hist)
        for (int v = 0; v < 9; ++v) hist[int64_t(done) * 9 + v] = std::nan("");
      if (cfl_hist) cfl_hist[done] = cfl;
      ++done;
      break;
    }
    if (out == CFV_OK) out = cfv_monitor(c, cur, nxt, c->st_m, s);
    double mon[9];
    if (out == CFV_OK) {
      hipError_t e = hipMemcpyAsync(mon, c->st_m, sizeof(mon), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) out = hip_fail(e, "monitor read-back");
    }
    if (out != CFV_OK) break;
    bool finite = true;
    for (int v = 0; v < 9; ++v) {
      mon[v] = std::log10(mon[v]);
      if (std::isnan(mon[v]) || (std::isinf(mon[v]) && mon[v] > 0.0)) finite = false;
      if (hist) hist[int64_t(done) * 9 + v] = mon[v];
    }
    if (cfl_hist) cfl_hist[done] = cfl;
    ++done;
    if (!finite) {
      out = fail(CFV_ERR_NONPHYSICAL, "the march produced a non-finite state");
      break;
    }
    std::swap(cur, nxt);
    if (mon[cfg->monitor] < cfg->target) break;
  }
  if (iters) *iters = done;
  // the last accepted state back into U (also after an error)
  if (cur != U) {
    const hipError_t e = hipMemcpyAsync(U, cur, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess && out == CFV_OK) out = hip_fail(e, "state copy-back");
  }
  return out;
}

// ------------------------------------------------- second derivatives
static cfv_status ensure_dir(cfv_ctx* c) {
  if (c->dir_u) return CFV_OK;
  const size_t n = size_t(9) * c->grid->g.ncells;
  cfv_status st;
  if ((st = dmalloc(&c->dir_u, n)) || (st = dmalloc(&c->dir_g, n)) ||
      (st = dmalloc(&c->dir_b, size_t(3) * c->grid->g.nb)) || (st = dmalloc(&c->dir_s, 32))) {
    double* kb[] = {c->dir_u, c->dir_g, c->dir_b, c->dir_s};
    for (double* b : kb)
      if (b) (void)hipFree(b);
    c->dir_u = c->dir_g = c->dir_b = c->dir_s = nullptr;
    return st;
  }
  return CFV_OK;
}

// max over entries of |x| / (|u| + 1e-3 max|u_v|) for nvar vectors of length
// n (vectors with u identically zero are left out); synchronises the stream.
static cfv_status step_ratio(cfv_ctx* c, int64_t n, int nvar, const double* x, const double* u, double* ratio,
                             hipStream_t s) {
  double* amax = c->dir_s;       // nvar <= 9
  double* sv = c->dir_s + 12;    // floors
  double* out = c->dir_s + 24;
  CFV_HIP(cfv::launch_absmax(n, nvar, u, amax, c->part, s));
  double h[9];
  CFV_HIP(hipMemcpyAsync(h, amax, size_t(nvar) * sizeof(double), hipMemcpyDeviceToHost, s));
  CFV_HIP(hipStreamSynchronize(s));
  for (int v = 0; v < nvar; ++v) h[v] = h[v] > 0.0 ? 1e-3 * h[v] : 0.0;
  CFV_HIP(hipMemcpyAsync(sv, h, size_t(nvar) * sizeof(double), hipMemcpyHostToDevice, s));
  CFV_HIP(cfv::launch_ratio_max(n, nvar, x, u, sv, out, c->part, s));
  CFV_HIP(hipMemcpyAsync(ratio, out, sizeof(double), hipMemcpyDeviceToHost, s));
  CFV_HIP(hipStreamSynchronize(s));
  return CFV_OK;
}

cfv_status cfv_vjp_dir(cfv_ctx* c, const double* U, const double* w, const double* x, double eps, double* gU2,
                       double* gbr2, double* h_used, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!U || !w || !x || !gU2) return fail(CFV_ERR_ARG, "null state, weights, direction or output");
  if (!(eps > 0.0) || !(eps < 1.0)) return fail(CFV_ERR_ARG, "eps must lie in (0, 1)");
  if (cfv_status st = ensure_dir(c)) return st;
  const int64_t nc = c->grid->g.ncells, n = 9 * nc, nb = c->grid->g.nb;
  double ratio = 0.0;
  if (cfv_status st = step_ratio(c, nc, 9, x, U, &ratio, s)) return st;
  const double h = ratio > 0.0 ? eps / ratio : eps;
  if (h_used) *h_used = h;
  double* gbm = c->dir_b;
  // + side into the outputs, - side into the workspace
  CFV_HIP(hipMemcpyAsync(c->dir_u, U, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
  CFV_HIP(cfv::launch_axpby(n, h, x, 1.0, c->dir_u, s));
  CFV_HIP(cfv::launch_vjp(c->dev(), c->dir_u, w, gU2, gbr2, c->W, c->A, c->slot, c->march_chunk(true), c->dbwin,
                          c->nbwin, s, c->tm()));
  CFV_HIP(hipMemcpyAsync(c->dir_u, U, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
  CFV_HIP(cfv::launch_axpby(n, -h, x, 1.0, c->dir_u, s));
  CFV_HIP(cfv::launch_vjp(c->dev(), c->dir_u, w, c->dir_g, gbr2 ? gbm : nullptr, c->W, c->A, c->slot,
                          c->march_chunk(true), c->dbwin, c->nbwin, s, c->tm()));
  const double ih = 0.5 / h;
  CFV_HIP(cfv::launch_axpby(n, -ih, c->dir_g, ih, gU2, s));
  if (gbr2) CFV_HIP(cfv::launch_axpby(nb, -ih, gbm, ih, gbr2, s));
  return CFV_OK;
}

cfv_status cfv_jvp_dir(cfv_ctx* c, const double* U, const double* v, const double* dU, const double* dbr, double eps,
                       double* Jv2, double* h_used, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!U || !v || !dU || !Jv2) return fail(CFV_ERR_ARG, "null state, vectors or output");
  if (!(eps > 0.0) || !(eps < 1.0)) return fail(CFV_ERR_ARG, "eps must lie in (0, 1)");
  if (cfv_status st = ensure_dir(c)) return st;
  const int64_t nc = c->grid->g.ncells, n = 9 * nc, nb = c->grid->g.nb;
  double ratio = 0.0, rb = 0.0;
  if (cfv_status st = step_ratio(c, nc, 9, dU, U, &ratio, s)) return st;
  if (dbr)
    if (cfv_status st = step_ratio(c, nb, 1, dbr, c->dbr, &rb, s)) return st;
  const double rmax = ratio > rb ? ratio : rb;
  const double h = rmax > 0.0 ? eps / rmax : eps;
  if (h_used) *h_used = h;
  double* brp = c->dir_b;
  double* brm = c->dir_b + nb;
  cfv::DevGrid dp = c->dev(), dm = c->dev();
  if (dbr) {
    CFV_HIP(hipMemcpyAsync(brp, c->dbr, size_t(nb) * sizeof(double), hipMemcpyDeviceToDevice, s));
    CFV_HIP(cfv::launch_axpby(nb, h, dbr, 1.0, brp, s));
    CFV_HIP(hipMemcpyAsync(brm, c->dbr, size_t(nb) * sizeof(double), hipMemcpyDeviceToDevice, s));
    CFV_HIP(cfv::launch_axpby(nb, -h, dbr, 1.0, brm, s));
    dp.br = brp;
    dm.br = brm;
  }
  CFV_HIP(hipMemcpyAsync(c->dir_u, U, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
  CFV_HIP(cfv::launch_axpby(n, h, dU, 1.0, c->dir_u, s));
  {
    cfv::MarchArgs a{dp, c->dir_u, v, nullptr, c->W, c->Wd, nullptr, Jv2};
    a.E = c->E;
    CFV_HIP(cfv::launch_march(a, c->slot, true, c->march_chunk(true), s, c->tm()));
  }
  CFV_HIP(hipMemcpyAsync(c->dir_u, U, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
  CFV_HIP(cfv::launch_axpby(n, -h, dU, 1.0, c->dir_u, s));
  {
    cfv::MarchArgs a{dm, c->dir_u, v, nullptr, c->W, c->Wd, nullptr, c->dir_g};
    a.E = c->E;
    CFV_HIP(cfv::launch_march(a, c->slot, true, c->march_chunk(true), s, c->tm()));
  }
  const double ih = 0.5 / h;
  CFV_HIP(cfv::launch_axpby(n, -ih, c->dir_g, ih, Jv2, s));
  return CFV_OK;
}

}  // extern "C"

namespace {
// per kernel name: total milliseconds and launches of the recorded events; clears the record
cfv_status timing_read(EventTimer& timer, int32_t max, char* names, double* total_ms, int64_t* count, int32_t* n) {
  if (!names || !total_ms || !count || !n || max < 1) return fail(CFV_ERR_ARG, "bad timing buffers");
  std::vector<std::string> keys;
  std::vector<double> ms;
  std::vector<int64_t> cnt;
  for (auto& r : timer.recs) {
    float t = 0.f;
    if (!r.a || !r.b) continue;
    CFV_HIP(hipEventSynchronize(r.b));
    CFV_HIP(hipEventElapsedTime(&t, r.a, r.b));
    size_t q = 0;
    while (q < keys.size() && keys[q] != r.name) ++q;
    if (q == keys.size()) {
      keys.emplace_back(r.name);
      ms.push_back(0.0);
      cnt.push_back(0);
    }
    ms[q] += t;
    cnt[q] += 1;
  }
  timer.recycle();
  const int m = int(keys.size()) < max ? int(keys.size()) : max;
  for (int q = 0; q < m; ++q) {
    std::strncpy(names + 32 * q, keys[q].c_str(), 31);
    names[32 * q + 31] = 0;
    total_ms[q] = ms[q];
    count[q] = cnt[q];
  }
  *n = m;
  return CFV_OK;
}

}  // namespace

// ----------------------------------------------------------------- ensemble
struct cfv_ensemble {
  std::vector<cfv_ctx*> ctx;
  cfv_tuning tune{};
  int device = 0;
  int num_cu = 0;
  std::vector<int64_t> off;             // n + 1 prefix sums of items
  int64_t total = 0;
  cfv::MarchArgs* dargs = nullptr;      // n descriptors
  int64_t* doff = nullptr;              // n + 1
  int64_t* dperm = nullptr;             // total
  unsigned* dcnt = nullptr;             // 2 queue counters
  bool bound = false;
  bool dual = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  EventTimer timer;
  bool timing = false;
  // backward-Euler step mode (cfv_ensemble_bind_be_step)
  int mode = 0;                          // 0: residual / JVP, 1: backward-Euler step
  cfv::MarchArgs* step_args = nullptr;   // (m + 1) x n: residual table, then one JVP table per Krylov vector
  size_t step_args_n = 0;
  cfv::StepVec* step_sv = nullptr;       // n
  double* step_arena = nullptr;          // Krylov vectors, work vectors, diagonals, scalars
  size_t step_arena_n = 0;
  double* step_part = nullptr;           // n x kStepBlocks partial sums
  cfv::StepLaunch step;
  double* mon = nullptr;                 // 9 n device scalars: monitors of the batched march
  unsigned* dflags = nullptr;            // n non-physical state words, one per instance
  int precond = 0;                       // the step's GMRES preconditioner (at the next step binding)
  // the fused residual march's items (its own tiles, chunks of kc layers)
  int kc = cfv::kKC;                     // layers per item of both marches
  std::vector<int64_t> foff;             // n + 1 prefix sums of fused items
  int64_t ftotal = 0;
  int64_t* dfoff = nullptr;
  int64_t* dfperm = nullptr;
};

namespace {
void drop_graph(cfv_ensemble* e) {
  if (e->exec) (void)hipGraphExecDestroy(e->exec);
  if (e->graph) (void)hipGraphDestroy(e->graph);
  e->exec = nullptr;
  e->graph = nullptr;
}

cfv_status check_tuning(const cfv_tuning* t) {
  if (!t) return fail(CFV_ERR_ARG, "null tuning");
  if ((t->queue != 0 && t->queue != 1) || t->blocks_per_cu < 1 || t->blocks_per_cu > 16 ||
      (t->order != 0 && t->order != 1) || t->chunk_layers < 0 || t->chunk_layers > kMaxChunk)
    return fail(CFV_ERR_ARG, "tuning: queue 0|1, blocks_per_cu 1..16, order 0|1, chunk_layers 0..4096");
  return CFV_OK;
}

// processing order of the items: instance order, or the items of the largest
// tiles first (cost ~ active columns x layers of the item), stable; the
// same for the fused march's items
cfv_status upload_fused_perm(cfv_ensemble* e) {
  std::vector<int64_t> perm(size_t(e->ftotal));
  for (int64_t w = 0; w < e->ftotal; ++w) perm[size_t(w)] = w;
  if (e->tune.order == 1) {
    std::vector<int32_t> cost(size_t(e->ftotal));
    for (size_t q = 0; q < e->ctx.size(); ++q) {
      const cfv::Shape& g = e->ctx[q]->grid->g;
      for (int64_t l = 0; l < e->foff[q + 1] - e->foff[q]; ++l) {
        cfv::FTile tm;
        cfv::fused_tile_of(g, e->kc, l, tm);
        cost[size_t(e->foff[q] + l)] = (tm.wi + 2) * (tm.wj + 2) * (tm.k1 - tm.k0 + 2);
      }
    }
    std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) { return cost[size_t(a)] > cost[size_t(b)]; });
  }
  CFV_HIP(hipMemcpy(e->dfperm, perm.data(), perm.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  return CFV_OK;
}

cfv_status upload_perm(cfv_ensemble* e) {
  if (cfv_status st = upload_fused_perm(e)) return st;
  std::vector<int64_t> perm(size_t(e->total));
  for (int64_t w = 0; w < e->total; ++w) perm[size_t(w)] = w;
  if (e->tune.order == 1) {
    std::vector<int32_t> cost(size_t(e->total));
    for (size_t q = 0; q < e->ctx.size(); ++q) {
      const cfv::Shape& g = e->ctx[q]->grid->g;
      for (int64_t l = 0; l < e->off[q + 1] - e->off[q]; ++l) {
        cfv::TileMap tm;
        cfv::tile_of_logical(g, l, tm, e->kc);
        const int wi = std::min(cfv::kTI, g.N - tm.i0), wj = std::min(cfv::kTJ, g.N - tm.j0);
        cost[size_t(e->off[q] + l)] = wi * wj * (tm.k1 - tm.k0);
      }
    }
    std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) { return cost[size_t(a)] > cost[size_t(b)]; });
  }
  CFV_HIP(hipMemcpy(e->dperm, perm.data(), perm.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  return CFV_OK;
}

// the item lists of both marches for chunks of e->kc layers: prefix sums per
// instance, device copies (reallocated when they grow) and the processing order
cfv_status build_items(cfv_ensemble* e) {
  const size_t n = e->ctx.size();
  const int64_t old_total = e->dperm ? e->total : 0, old_ftotal = e->dfperm ? e->ftotal : 0;
  e->off.assign(n + 1, 0);
  e->foff.assign(n + 1, 0);
  for (size_t q = 0; q < n; ++q) {
    const cfv::Shape& g = e->ctx[q]->grid->g;
    e->off[q + 1] = e->off[q] + cfv::march_logical_blocks(g, e->kc);
    e->foff[q + 1] = e->foff[q] + cfv::fused_items(g, e->kc);
  }
  e->total = e->off[n];
  e->ftotal = e->foff[n];
  cfv_status st;
  if (e->total > old_total) {
    if (e->dperm) (void)hipFree(e->dperm);
    e->dperm = nullptr;
    if ((st = dmalloc(&e->dperm, size_t(e->total)))) return st;
  }
  if (e->ftotal > old_ftotal) {
    if (e->dfperm) (void)hipFree(e->dfperm);
    e->dfperm = nullptr;
    if ((st = dmalloc(&e->dfperm, size_t(e->ftotal)))) return st;
  }
  CFV_HIP(hipMemcpy(e->doff, e->off.data(), e->off.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  CFV_HIP(hipMemcpy(e->dfoff, e->foff.data(), e->foff.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  return upload_perm(e);
}

unsigned ensemble_blocks(const cfv_ensemble* e, int64_t total) {
  int64_t b = int64_t(e->tune.blocks_per_cu) * e->num_cu;
  const int64_t cap = (total + 7) / 8 * 8;
  if (b > cap) b = cap;
  b = b / 8 * 8;
  if (b < 8) b = 8;
  return unsigned(b);
}

constexpr int kStepBlocks = 128;  // vector blocks per instance in the step's reductions

cfv_status ensemble_launch(cfv_ensemble* e, hipStream_t s, bool timed) {
  cfv::KernelTimer* t = timed && e->timing ? &e->timer : nullptr;
  const int n = int(e->ctx.size());
  if (e->mode == 1) {
    cfv::StepLaunch& L = e->step;
    L.res = cfv::EnsembleLaunch{e->step_args, e->dfoff, e->dfperm, e->dcnt, n, e->ftotal, e->tune.queue,
                                ensemble_blocks(e, e->ftotal), e->kc};
    for (int j = 0; j < L.m; ++j) {
      L.jvp[size_t(j)] = cfv::EnsembleLaunch{e->step_args + size_t(1 + j) * n, e->doff, e->dperm, e->dcnt, n, e->total,
                                             e->tune.queue, ensemble_blocks(e, e->total), e->kc};
    }
    CFV_HIP(cfv::launch_ensemble_step(L, s, t));
    return CFV_OK;
  }
  if (!e->dual) {  // the residual: the fused march over its own item list
    const cfv::EnsembleLaunch Lf{e->dargs, e->dfoff, e->dfperm, e->dcnt, n, e->ftotal, e->tune.queue,
                                 ensemble_blocks(e, e->ftotal), e->kc};
    CFV_HIP(cfv::launch_fused_ensemble(Lf, s, t));
    return CFV_OK;
  }
  cfv::EnsembleLaunch L{e->dargs, e->doff, e->dperm, e->dcnt, n, e->total, e->tune.queue, ensemble_blocks(e, e->total),
                        e->kc};
  CFV_HIP(cfv::launch_march_ensemble(L, e->dual, s, t));
  return CFV_OK;
}
}  // namespace
extern "C" {

cfv_status cfv_ensemble_create(cfv_ctx* const* ctxs, int32_t n, const cfv_tuning* t, cfv_ensemble** out) {
  g_err.clear();
  if (!ctxs || !out || n < 1) return fail(CFV_ERR_ARG, "need n >= 1 contexts and an output");
  if (cfv_status st = check_tuning(t)) return st;
  int dev = 0;
  CFV_HIP(hipGetDevice(&dev));
  for (int q = 0; q < n; ++q) {
    if (cfv_status st = check_ctx(ctxs[q])) return st;
    if (ctxs[q]->device != dev) return fail(CFV_ERR_ARG, "all contexts must live on the current device");
  }
  cfv_ensemble* e = new (std::nothrow) cfv_ensemble;
  if (!e) return fail(CFV_ERR_ALLOC, "host allocation");
  e->ctx.assign(ctxs, ctxs + n);
  e->tune = *t;
  e->device = dev;
  hipError_t he = hipDeviceGetAttribute(&e->num_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (he != hipSuccess || e->num_cu < 1) {
    delete e;
    return fail(CFV_ERR_HIP, "cannot query the compute unit count");
  }
  e->kc = t->chunk_layers ? t->chunk_layers : cfv::kKC;
  cfv_status st;
  if ((st = dmalloc(&e->dargs, size_t(n))) || (st = dmalloc(&e->doff, size_t(n) + 1)) ||
      (st = dmalloc(&e->dcnt, 2)) || (st = dmalloc(&e->dflags, size_t(n))) ||
      (st = dmalloc(&e->dfoff, size_t(n) + 1))) {
    cfv_ensemble_destroy(e);
    return st;
  }
  he = hipMemset(e->dflags, 0, size_t(n) * sizeof(unsigned));
  if (he != hipSuccess) {
    cfv_ensemble_destroy(e);
    return fail(CFV_ERR_HIP, hipGetErrorString(he));
  }
  if ((st = build_items(e))) {
    cfv_ensemble_destroy(e);
    return st;
  }
  *out = e;
  return CFV_OK;
}

void cfv_ensemble_destroy(cfv_ensemble* e) {
  if (!e) return;
  drop_graph(e);
  void* bufs[] = {e->dargs, e->doff, e->dperm, e->dcnt, e->step_args, e->step_sv, e->step_arena, e->step_part,
                  e->mon, e->dflags, e->dfoff, e->dfperm};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete e;
}

cfv_status cfv_ensemble_set_tuning(cfv_ensemble* e, const cfv_tuning* t) {
  if (!e) return fail(CFV_ERR_ARG, "null ensemble");
  if (cfv_status st = check_tuning(t)) return st;
  e->tune = *t;
  drop_graph(e);
  const int kc = t->chunk_layers ? t->chunk_layers : cfv::kKC;
  if (kc == e->kc) return upload_perm(e);
  e->kc = kc;
  return build_items(e);
}

cfv_status cfv_ensemble_set_preconditioner(cfv_ensemble* e, int32_t kind) {
  if (!e) return fail(CFV_ERR_ARG, "null ensemble");
  if (kind != 0 && kind != 1) return fail(CFV_ERR_ARG, "preconditioner: 0 (none) or 1 (Jacobi)");
  e->precond = kind;
  if (e->mode == 1) {  // a bound step keeps its tables: bind it again
    drop_graph(e);
    e->bound = false;
  }
  return CFV_OK;
}

cfv_status cfv_ensemble_items(const cfv_ensemble* e, int64_t* total, int32_t* blocks) {
  if (!e) return fail(CFV_ERR_ARG, "null ensemble");
  if (total) *total = e->total;
  if (blocks) *blocks = int32_t(ensemble_blocks(e, e->total));
  return CFV_OK;
}

cfv_status cfv_ensemble_bind(cfv_ensemble* e, const double* const* U, const double* const* v,
                             const double* const* dbr, double* const* R, double* const* Jv) {
  if (!e) return fail(CFV_ERR_ARG, "null ensemble");
  if (!U) return fail(CFV_ERR_ARG, "null state array");
  const bool dual = v != nullptr;
  if (dual && !Jv) return fail(CFV_ERR_ARG, "a JVP needs Jv outputs");
  if (!dual && (!R || Jv || dbr)) return fail(CFV_ERR_ARG, "a residual-only ensemble needs R and no Jv or dbr");
  const size_t n = e->ctx.size();
  std::vector<cfv::MarchArgs> h(n);
  for (size_t q = 0; q < n; ++q) {
    cfv_ctx* c = e->ctx[q];
    if (!U[q] || (dual && (!v[q] || !Jv[q])) || (!dual && !R[q]))
      return fail(CFV_ERR_ARG, "null pointer for instance " + std::to_string(q));
    h[q] = cfv::MarchArgs{c->dev(), U[q], dual ? v[q] : nullptr, dbr ? dbr[q] : nullptr, c->W,
                          dual ? c->Wd : nullptr, R ? R[q] : nullptr, dual ? Jv[q] : nullptr};
    h[q].E = dual ? c->E : nullptr;
    h[q].d.flag = e->dflags + q;
  }
  CFV_HIP(hipMemcpy(e->dargs, h.data(), n * sizeof(cfv::MarchArgs), hipMemcpyHostToDevice));
  e->dual = dual;
  e->bound = true;
  e->mode = 0;
  drop_graph(e);
  return CFV_OK;
}

cfv_status cfv_ensemble_bind_be_step(cfv_ensemble* e, const double* const* U, double* const* U_new, double cfl,
                                     int32_t m, double* hist) {
  if (!e) return fail(CFV_ERR_ARG, "null ensemble");
  if (!U || !U_new) return fail(CFV_ERR_ARG, "null state arrays");
  if (!(cfl > 0.0)) return fail(CFV_ERR_ARG, "cfl must be positive");
  if (m < 1 || m > 200) return fail(CFV_ERR_ARG, "need 1 <= m <= 200");
  const size_t n = e->ctx.size();
  for (size_t q = 0; q < n; ++q) {
    if (!U[q] || !U_new[q]) return fail(CFV_ERR_ARG, "null pointer for instance " + std::to_string(q));
    if (U[q] == U_new[q]) return fail(CFV_ERR_ARG, "U_new aliases U for instance " + std::to_string(q));
  }
  const cfv::StepLayout Y(m);
  size_t need = 0;
  for (size_t q = 0; q < n; ++q) {
    const size_t nc = size_t(e->ctx[q]->grid->g.ncells);
    need += size_t(m + 3) * 9 * nc + nc + size_t(Y.size);
  }
  drop_graph(e);
  cfv_status st;
  if (need > e->step_arena_n) {
    if (e->step_arena) (void)hipFree(e->step_arena);
    e->step_arena = nullptr;
    e->step_arena_n = 0;
    if ((st = dmalloc(&e->step_arena, need))) return st;
    e->step_arena_n = need;
  }
  const size_t nargs = size_t(m + 1) * n;
  if (nargs > e->step_args_n) {
    if (e->step_args) (void)hipFree(e->step_args);
    e->step_args = nullptr;
    e->step_args_n = 0;
    if ((st = dmalloc(&e->step_args, nargs))) return st;
    e->step_args_n = nargs;
  }
  if (!e->step_sv && (st = dmalloc(&e->step_sv, n))) return st;
  if (!e->step_part && (st = dmalloc(&e->step_part, n * kStepBlocks))) return st;
  std::vector<cfv::StepVec> sv(n);
  std::vector<cfv::MarchArgs> args(nargs);
  cfv::StepLaunch& L = e->step;
  L.n = int(n);
  L.m = m;
  L.blocks = kStepBlocks;
  L.cfl = cfl;
  L.precond = e->precond;
  L.sv = e->step_sv;
  L.part = e->step_part;
  L.hist = hist;
  L.jvp.assign(size_t(m), cfv::EnsembleLaunch{});
  L.dev.clear();
  L.Uh.clear();
  L.diagh.clear();
  L.Wh.clear();
  double* p = e->step_arena;
  for (size_t q = 0; q < n; ++q) {
    cfv_ctx* c = e->ctx[q];
    const int64_t nc = c->grid->g.ncells, n9 = 9 * nc;
    cfv::StepVec& v = sv[q];
    v.U = U[q];
    v.Unew = U_new[q];
    v.V = p;
    p += size_t(m + 1) * n9;
    v.w = p;
    p += n9;
    v.z = p;
    p += n9;
    double* diag = p;
    p += nc;
    v.diag = diag;
    v.sm = p;
    p += Y.size;
    v.nc = nc;
    v.flag = e->dflags + q;
    cfv::DevGrid d = c->dev();
    d.flag = e->dflags + q;
    args[q] = cfv::MarchArgs{d, U[q], nullptr, nullptr, c->W, nullptr, U_new[q], nullptr};
    for (int j = 0; j < m; ++j) {
      args[size_t(1 + j) * n + q] =
          cfv::MarchArgs{d, U[q], e->precond ? v.z : v.V + size_t(j) * n9, nullptr, c->W, c->Wd, nullptr, v.w};
      args[size_t(1 + j) * n + q].E = c->E;
    }
    L.dev.push_back(d);
    L.Uh.push_back(U[q]);
    L.diagh.push_back(diag);
    L.Wh.push_back(c->W);
  }
  CFV_HIP(hipMemcpy(e->step_sv, sv.data(), n * sizeof(cfv::StepVec), hipMemcpyHostToDevice));
  CFV_HIP(hipMemcpy(e->step_args, args.data(), nargs * sizeof(cfv::MarchArgs), hipMemcpyHostToDevice));
  e->mode = 1;
  e->bound = true;
  return CFV_OK;
}

cfv_status cfv_ensemble_run(cfv_ensemble* e, hipStream_t s) {
  if (!e) return fail(CFV_ERR_ARG, "null ensemble");
  if (!e->bound) return fail(CFV_ERR_ARG, "bind the instance buffers first");
  return ensemble_launch(e, s, true);
}

cfv_status cfv_ensemble_residual_jvp(cfv_ensemble* e, const double* const* U, const double* const* v,
                                     double* const* R, double* const* Jv, hipStream_t s) {
  if (cfv_status st = cfv_ensemble_bind(e, U, v, nullptr, R, Jv)) return st;
  return cfv_ensemble_run(e, s);
}

cfv_status cfv_ensemble_graph_capture(cfv_ensemble* e, hipStream_t s) {
  if (!e) return fail(CFV_ERR_ARG, "null ensemble");
  if (!e->bound) return fail(CFV_ERR_ARG, "bind the instance buffers first");
  if (!s) return fail(CFV_ERR_ARG, "capture needs a created (non-null) stream");
  drop_graph(e);
  CFV_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  cfv_status st = ensemble_launch(e, s, false);
  hipGraph_t g = nullptr;
  const hipError_t he = hipStreamEndCapture(s, &g);
  if (st) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (he != hipSuccess) return fail(CFV_ERR_HIP, hipGetErrorString(he));
  e->graph = g;
  CFV_HIP(hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0));
  return CFV_OK;
}

cfv_status cfv_ensemble_graph_launch(cfv_ensemble* e, hipStream_t s) {
  if (!e) return fail(CFV_ERR_ARG, "null ensemble");
  if (!e->exec) return fail(CFV_ERR_ARG, "no captured graph (capture after the last bind or tuning change)");
  CFV_HIP(hipGraphLaunch(e->exec, s));
  return CFV_OK;
}

cfv_status cfv_ensemble_status_flags(cfv_ensemble* e, int32_t* flags, hipStream_t s) {
  if (!e) return fail(CFV_ERR_ARG, "null ensemble");
  const size_t n = e->ctx.size();
  std::vector<unsigned> h(n);
  CFV_HIP(hipMemcpyAsync(h.data(), e->dflags, n * sizeof(unsigned), hipMemcpyDeviceToHost, s));
  CFV_HIP(hipStreamSynchronize(s));
  CFV_HIP(hipMemsetAsync(e->dflags, 0, n * sizeof(unsigned), s));
  int first = -1;
  for (size_t q = 0; q < n; ++q) {
    if (flags) flags[q] = int32_t(h[q]);
    if (h[q] && first < 0) first = int(q);
  }
  if (first >= 0)
    return fail(CFV_ERR_NONPHYSICAL, "instance " + std::to_string(first) +
                                         " met a non-positive or NaN face state or a non-finite step");
  return CFV_OK;
}

cfv_status cfv_ensemble_steady(cfv_ensemble* e, double* const* U, double* const* U_work, const cfv_steady_cfg* cfg,
                               double* hist, int32_t* steps, int32_t* iters, hipStream_t s) {
  if (!e) return fail(CFV_ERR_ARG, "null ensemble");
  if (!U || !U_work || !cfg) return fail(CFV_ERR_ARG, "null state arrays or configuration");
  if (!(cfg->cfl0 > 0.0) || !(cfg->cfl_max >= cfg->cfl0)) return fail(CFV_ERR_ARG, "need 0 < cfl0 <= cfl_max");
  if (cfg->every < 1 || cfg->max_iters < 0) return fail(CFV_ERR_ARG, "need every >= 1 and max_iters >= 0");
  if (cfg->monitor < 0 || cfg->monitor > 8) return fail(CFV_ERR_ARG, "monitor must be a variable 0..8");
  if (cfg->m < 1 || cfg->m > 200) return fail(CFV_ERR_ARG, "need 1 <= m <= 200");
  const size_t n = e->ctx.size();
  for (size_t q = 0; q < n; ++q) {
    if (!U[q] || !U_work[q]) return fail(CFV_ERR_ARG, "null pointer for instance " + std::to_string(q));
    if (U[q] == U_work[q]) return fail(CFV_ERR_ARG, "U_work aliases U for instance " + std::to_string(q));
  }
  if (!e->mon)
    if (cfv_status st = dmalloc(&e->mon, 9 * n)) return st;
  std::vector<char> active(n, 1);
  std::vector<int32_t> taken(n, 0);
  std::vector<double> mon(9 * n);
  std::vector<unsigned> flg(n);
  CFV_HIP(hipMemsetAsync(e->dflags, 0, n * sizeof(unsigned), s));
  if (hist)
    for (size_t a = 0; a < n * size_t(cfg->max_iters) * 9; ++a) hist[a] = std::nan("");
  cfv_status out = CFV_OK;
  int nonphys = -1;  // first instance that produced a non-finite state
  double bound_cfl = -1.0;
  int32_t done = 0;
  size_t live = n;
  while (done < cfg->max_iters && live > 0) {
    const double cfl = std::min(std::ldexp(cfg->cfl0, done / cfg->every), cfg->cfl_max);
    if (cfl != bound_cfl) {  // the step's diagonal depends on the CFL: bind (and capture) again
      if ((out = cfv_ensemble_bind_be_step(e, U, U_work, cfl, cfg->m, nullptr))) break;
      if (s && (out = cfv_ensemble_graph_capture(e, s))) break;
      bound_cfl = cfl;
    }
    out = s ? cfv_ensemble_graph_launch(e, s) : cfv_ensemble_run(e, s);
    for (size_t q = 0; q < n && out == CFV_OK; ++q)
      if (active[q]) out = cfv_monitor(e->ctx[q], U[q], U_work[q], e->mon + 9 * q, s);
    if (out == CFV_OK) {
      hipError_t he = hipMemcpyAsync(mon.data(), e->mon, 9 * n * sizeof(double), hipMemcpyDeviceToHost, s);
      if (he == hipSuccess) he = hipMemcpyAsync(flg.data(), e->dflags, n * sizeof(unsigned), hipMemcpyDeviceToHost, s);
      if (he == hipSuccess) he = hipStreamSynchronize(s);
      if (he != hipSuccess) out = hip_fail(he, "monitor read-back");
    }
    if (out != CFV_OK) break;
    for (size_t q = 0; q < n; ++q) {
      if (!active[q]) continue;
      bool finite = !(flg[q] & 2u);  // the step's residual norm was not finite
      for (int v = 0; v < 9; ++v) {
        const double x = std::log10(mon[9 * q + v]);
        if (std::isnan(x) || (std::isinf(x) && x > 0.0)) finite = false;
        if (hist) hist[(q * size_t(cfg->max_iters) + size_t(done)) * 9 + v] = x;
      }
      ++taken[q];
      if (!finite) {  // keep the state before this step and stop the instance
        if (nonphys < 0) nonphys = int(q);
        active[q] = 0;
        --live;
        continue;
      }
      const size_t bytes = size_t(9) * size_t(e->ctx[q]->grid->g.ncells) * sizeof(double);
      const hipError_t he = hipMemcpyAsync(U[q], U_work[q], bytes, hipMemcpyDeviceToDevice, s);
      if (he != hipSuccess) return hip_fail(he, "state update");
      if (std::log10(mon[9 * q + cfg->monitor]) < cfg->target) {
        active[q] = 0;
        --live;
      }
    }
    ++done;
  }
  if (steps)
    for (size_t q = 0; q < n; ++q) steps[q] = taken[q];
  if (iters) *iters = done;
  if (out == CFV_OK && nonphys >= 0)
    out = fail(CFV_ERR_NONPHYSICAL, "instance " + std::to_string(nonphys) + " produced a non-finite state");
  return out;
}

cfv_status cfv_ensemble_timing_enable(cfv_ensemble* e, int32_t on) {
  if (!e) return fail(CFV_ERR_ARG, "null ensemble");
  e->timing = on != 0;
  return CFV_OK;
}

cfv_status cfv_ensemble_timing_read(cfv_ensemble* e, int32_t max, char* names, double* total_ms, int64_t* count,
                                    int32_t* n) {
  if (!e) return fail(CFV_ERR_ARG, "null ensemble");
  return timing_read(e->timer, max, names, total_ms, count, n);
}

cfv_status cfv_timing_enable(cfv_ctx* c, int32_t on) {
  if (cfv_status st = check_ctx(c)) return st;
  c->timing = on != 0;
  return CFV_OK;
}

cfv_status cfv_timing_read(cfv_ctx* c, int32_t max, char* names, double* total_ms, int64_t* count, int32_t* n) {
  if (cfv_status st = check_ctx(c)) return st;
  return timing_read(c->timer, max, names, total_ms, count, n);
}

cfv_status cfv_set_preconditioner(cfv_ctx* c, int32_t kind) {
  if (cfv_status st = check_ctx(c)) return st;
  if (kind != 0 && kind != 1) return fail(CFV_ERR_ARG, "preconditioner: 0 (none) or 1 (Jacobi)");
  c->precond = kind;
  return CFV_OK;
}

cfv_status cfv_set_chunk_layers(cfv_ctx* c, int32_t kc) {
  if (cfv_status st = check_ctx(c)) return st;
  if (kc < 0 || kc > kMaxChunk) return fail(CFV_ERR_ARG, "chunk layers: 0 (balanced) or 1..4096");
  c->chunk = kc;
  return CFV_OK;
}

}  // extern "C"
