// C ABI of the coronal finite-volume MHD library: grid construction on the
// host, device contexts, and the stream-ordered entry points declared in
// include/cfv.h.
#include "../../include/cfv.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cfv_kernels.hpp"
#include "cfv_march.hpp"

namespace cfv {
int reduce_partials_per_vector();
hipError_t launch_norms(int64_t nc, const double* a, const double* b, double* out9, double* part, hipStream_t s);
hipError_t launch_dots(int64_t n, const double* V, int k, const double* w, double* out, double* part, hipStream_t s);
hipError_t launch_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);
hipError_t launch_vjp(const DevGrid& d, const double* U, const double* w, double* gU, double* gbr, double* W,
                      double* A, hipStream_t s, KernelTimer* t);
int64_t vjp_workspace_doubles(const Shape& g);
}  // namespace cfv

struct cfv_grid {
  cfv::Shape g;
  std::vector<double> r;   // Nr + 1
  std::vector<double> D;   // 6 (N+1)^2 3 unit corner directions
  std::vector<double> cg;  // CG_NCOMP x 6N^2 column geometry
  std::vector<int32_t> cn; // 8 x 6N^2 angular neighbours and face ownership
  cfv::GeomRef host_ref() const {
    cfv::GeomRef G;
    G.cg = cg.data();
    G.cn = cn.data();
    G.r = r.data();
    G.ncol = g.nb;
    return G;
  }
};

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
  double* W = nullptr;     // 36 ncells: primitives + limited gradients
  double* Wd = nullptr;    // 36 ncells: their tangents
  double* A = nullptr;     // adjoint workspace
  double* part = nullptr;  // reduction partials
  int part_vectors = 0;
  cfv::DevGrid dev() const {
    cfv::DevGrid d;
    d.g = grid->g;
    d.G.cg = dcg;
    d.G.cn = dcn;
    d.G.r = dr;
    d.G.ncol = grid->g.nb;
    d.pr = pr;
    d.br = dbr;
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

const double kPi = 3.14159265358979323846;

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

// Per-column geometry from the cell vertices at unit radii (see cfv_topo.hpp).
static void build_column_tables(cfv_grid& G) {
  using cfv::V3;
  const cfv::Shape& s = G.g;
  const int N = s.N, n1 = N + 1;
  const int64_t ncol = s.nb;
  G.cg.assign(size_t(cfv::CG_NCOMP) * ncol, 0.0);
  G.cn.assign(size_t(8) * ncol, 0);
  auto D = [&](int p, int jj, int ii) {
    const double* d = &G.D[((size_t(p) * n1 + jj) * n1 + ii) * 3];
    return cfv::mk(d[0], d[1], d[2]);
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
    cfv::face_vertex_offsets(lf, off);
    V3 v[4];
    for (int a = 0; a < 4; ++a) v[a] = (off[a][0] ? rb : ra) * D(p, j + off[a][1], i + off[a][2]);
    S = 0.5 * cfv::cross3(v[2] - v[0], v[3] - v[1]);
    xf = 0.25 * (((v[0] + v[1]) + v[2]) + v[3]);
  };
  for (int p = 0; p < 6; ++p)
    for (int j = 0; j < N; ++j)
      for (int i = 0; i < N; ++i) {
        const int64_t col = cfv::column_of(s, p, j, i);
        put(cfv::CG_CSUM, col, ((D(p, j, i) + D(p, j, i + 1)) + D(p, j + 1, i)) + D(p, j + 1, i + 1));
        V3 sr, xr;
        face_at(p, j, i, 1, 1.0, 1.0, sr, xr);
        put(cfv::CG_SR, col, sr);
        put(cfv::CG_XR, col, xr);
        G.cg[cfv::CG_OMEGA * ncol + col] = cfv::dot3(xr, sr);
        for (int q = 0; q < 4; ++q) {
          const int lf = 2 + q;
          cfv::Nbr nb = cfv::neighbour(s, p, 0, j, i, lf);
          const int64_t ncolv = cfv::column_of(s, nb.p, nb.j, nb.i);
          const bool own = ncolv > col;
          V3 a, b, dummy;
          if (own) {
            face_at(p, j, i, lf, 0.0, 1.0, a, dummy);
            face_at(p, j, i, lf, 1.0, 1.0, dummy, b);
          } else {
            face_at(nb.p, nb.j, nb.i, nb.back, 0.0, 1.0, a, dummy);
            face_at(nb.p, nb.j, nb.i, nb.back, 1.0, 1.0, dummy, b);
          }
          put(cfv::CG_ANG + 6 * q, col, 2.0 * a);
          put(cfv::CG_ANG + 6 * q + 3, col, 2.0 * b);
          G.cn[q * ncol + col] = int32_t(ncolv);
          G.cn[(4 + q) * ncol + col] = nb.back | (own ? 256 : 0);
        }
      }
}

extern "C" {

const char* cfv_last_error(void) { return g_err.c_str(); }

cfv_status cfv_grid_create(int32_t N, int32_t Nr, const double* r_nodes, cfv_grid** out) {
  g_err.clear();
  if (!out || !r_nodes) return fail(CFV_ERR_ARG, "null argument");
  if (N < 2 || Nr < 1) return fail(CFV_ERR_ARG, "need N >= 2 and Nr >= 1");
  for (int k = 0; k < Nr; ++k)
    if (!(r_nodes[k + 1] > r_nodes[k]) || !(r_nodes[k] > 0.0))
      return fail(CFV_ERR_ARG, "r_nodes must be positive and strictly increasing");
  cfv_grid* g = new (std::nothrow) cfv_grid;
  if (!g) return fail(CFV_ERR_ALLOC, "host allocation");
  g->g.N = N;
  g->g.Nr = Nr;
  g->g.nb = 6LL * N * N;
  g->g.ncells = g->g.nb * Nr;
  g->r.assign(r_nodes, r_nodes + Nr + 1);
  const int n1 = N + 1;
  g->D.resize(size_t(6) * n1 * n1 * 3);
  std::vector<double> t(n1);
  for (int q = 0; q <= N; ++q) t[q] = std::tan(-kPi / 4 + q * (kPi / 2) / N);
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
        double* d = &g->D[((size_t(p) * n1 + jj) * n1 + ii) * 3];
        d[0] = x / nrm;
        d[1] = y / nrm;
        d[2] = z / nrm;
      }
  build_column_tables(*g);
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

cfv_status cfv_ctx_create(const cfv_grid* g, const cfv_params* prm, cfv_ctx** out) {
  g_err.clear();
  if (!g || !prm || !out) return fail(CFV_ERR_ARG, "null argument");
  if (!(prm->gamma > 1.0) || !(prm->c_h > 0.0) || prm->G < 0.0 || !(prm->rho_b > 0.0) || !(prm->T_b > 0.0))
    return fail(CFV_ERR_ARG, "need gamma > 1, c_h > 0, G >= 0, rho_b > 0, T_b > 0");
  if (prm->limiter != 0 && prm->limiter != 1) return fail(CFV_ERR_ARG, "limiter must be 0 or 1");
  if (prm->inner_mode != 0) return fail(CFV_ERR_ARG, "inner_mode: only the low-E boundary (0) is provided");
  cfv_ctx* c = new (std::nothrow) cfv_ctx;
  if (!c) return fail(CFV_ERR_ALLOC, "host allocation");
  c->grid = g;
  CFV_HIP(hipGetDevice(&c->device));
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
      (st = dmalloc(&c->dbr, size_t(g->g.nb))) || (st = dmalloc(&c->W, size_t(36) * nc)) ||
      (st = dmalloc(&c->Wd, size_t(36) * nc)) ||
      (st = dmalloc(&c->A, size_t(cfv::vjp_workspace_doubles(g->g)))) ||
      (st = dmalloc(&c->part, size_t(c->part_vectors) * cfv::reduce_partials_per_vector()))) {
    cfv_ctx_destroy(c);
    return st;
  }
  hipError_t e = hipMemcpy(c->dcg, g->cg.data(), g->cg.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->dcn, g->cn.data(), g->cn.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->dr, g->r.data(), g->r.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(c->dbr, 0, size_t(g->g.nb) * sizeof(double));
  if (e != hipSuccess) {
    cfv_ctx_destroy(c);
    return hip_fail(e, "uploading grid tables");
  }
  *out = c;
  return CFV_OK;
}

void cfv_ctx_destroy(cfv_ctx* c) {
  if (!c) return;
  double* bufs[] = {c->dcg, c->dr, c->dbr, c->W, c->Wd, c->A, c->part};
  for (double* b : bufs)
    if (b) (void)hipFree(b);
  if (c->dcn) (void)hipFree(c->dcn);
  delete c;
}

cfv_status cfv_set_inner_br(cfv_ctx* c, const double* br, int64_t n, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!br) return fail(CFV_ERR_ARG, "null B_r map");
  if (n != c->grid->g.nb) return fail(CFV_ERR_SIZE, "B_r map length must be 6 N^2");
  CFV_HIP(hipMemcpyAsync(c->dbr, br, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
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
  CFV_HIP(cfv::launch_march(a, false, s, c->tm()));
  return CFV_OK;
}

cfv_status cfv_jvp(cfv_ctx* c, const double* U, const double* v, const double* dbr, double* Jv, double* R,
                   hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!U || !v || !Jv) return fail(CFV_ERR_ARG, "null state, direction or output");
  cfv::MarchArgs a{c->dev(), U, v, dbr, c->W, c->Wd, R, Jv};
  CFV_HIP(cfv::launch_march(a, true, s, c->tm()));
  return CFV_OK;
}

cfv_status cfv_vjp(cfv_ctx* c, const double* U, const double* w, double* gU, double* gbr, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!U || !w || !gU) return fail(CFV_ERR_ARG, "null state, weights or output");
  CFV_HIP(cfv::launch_vjp(c->dev(), U, w, gU, gbr, c->W, c->A, s, c->tm()));
  return CFV_OK;
}

cfv_status cfv_local_dt(cfv_ctx* c, const double* U, double cfl, double* diag, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!U || !diag) return fail(CFV_ERR_ARG, "null state or output");
  if (!(cfl > 0.0)) return fail(CFV_ERR_ARG, "cfl must be positive");
  CFV_HIP(cfv::launch_local_dt(c->dev(), U, cfl, diag, c->W, s, c->tm()));
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

cfv_status cfv_axpby(cfv_ctx* c, int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!x || !y || n < 0) return fail(CFV_ERR_ARG, "bad vector arguments");
  CFV_HIP(cfv::launch_axpby(n, a, x, b, y, s));
  return CFV_OK;
}

cfv_status cfv_timing_enable(cfv_ctx* c, int32_t on) {
  if (cfv_status st = check_ctx(c)) return st;
  c->timing = on != 0;
  return CFV_OK;
}

cfv_status cfv_timing_read(cfv_ctx* c, int32_t max, char* names, double* total_ms, int64_t* count, int32_t* n) {
  if (cfv_status st = check_ctx(c)) return st;
  if (!names || !total_ms || !count || !n || max < 1) return fail(CFV_ERR_ARG, "bad timing buffers");
  std::vector<std::string> keys;
  std::vector<double> ms;
  std::vector<int64_t> cnt;
  for (auto& r : c->timer.recs) {
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
  c->timer.recycle();
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

}  // extern "C"
