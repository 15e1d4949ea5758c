/*
 * cfv.h -- C ABI of the MI355X coronal finite-volume MHD library.
 *
 * The library evaluates, on one GPU and in FP64, the finite-volume residual
 * of ideal MHD with hyperbolic divergence cleaning on a spherical shell (the
 * discretisation of Brchnelova et al., "To E or not to E", Section 2.1 and
 * Eqs. 14-17), with the paper's low-E and large-E inner boundaries (Section
 * 3.2, Eqs. 20-25) and the Table 2 outer ghost laws (Section 4.1), its exact
 * Jacobian-vector product and its adjoint (vector-Jacobian product), the
 * implicit backward-Euler pseudo-time step and the march to a steady state
 * (Sections 2.1, 4.1), batched over ensembles of shells, and the E-field
 * diagnostic and E-free state (Sections 2.2, 3.1).
 *
 * Conventions
 *  - Every function returns cfv_status (0 = CFV_OK).  On failure
 *    cfv_last_error() returns a thread-local message.  No C++ exception
 *    crosses this boundary.
 *  - Device buffers are owned by the caller and passed as plain pointers to
 *    FP64 data on the current device.  The library owns its grid tables, the
 *    B_r map copy and its workspaces (allocated at cfv_ctx_create).
 *  - All device work is enqueued asynchronously on the hipStream_t given.
 *    The *_to_host functions, the solver entry points (cfv_solve,
 *    cfv_be_step, cfv_vjp_dir, cfv_jvp_dir, cfv_steady, cfv_ensemble_steady)
 *    and cfv_timing_read synchronise that stream, as each one states.
 *  - A context's workspaces are shared by all calls on it: calls on one
 *    context (or on an ensemble and its contexts) must be ordered, by one
 *    stream or by synchronisation between streams.
 *  - State layout (SoA): U[v*ncells + c] with v = 0..8 the conservative
 *    variables (rho, rho vx, rho vy, rho vz, Bx, By, Bz, E, psi), nondimensional
 *    (rho_ref, B_ref of Eq. 1, V_ref = B_ref/sqrt(mu0 rho_ref), lengths in R_sun).
 *  - Cell order c = ((p*Nr + k)*N + j)*N + i over 6 cubed-sphere panels p,
 *    radial layers k and angular indices j, i.  The B_r map has 6N^2 values in
 *    the order (p*N + j)*N + i (one per inner boundary face).
 *  - Residual R is the integrated form: R_c = sum over faces of the outward
 *    numerical flux times the face area minus V_c S(U_c), so dU/dt = -R/V.
 */
#ifndef CFV_H
#define CFV_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cfv_status;
enum {
  CFV_OK = 0,
  CFV_ERR_ARG = 1,          /* null pointer, bad size or bad parameter */
  CFV_ERR_SIZE = 2,         /* a length does not match the grid */
  CFV_ERR_HIP = 3,          /* a HIP runtime call failed */
  CFV_ERR_NONPHYSICAL = 4,  /* non-positive density or pressure met */
  CFV_ERR_NOT_CONVERGED = 5,
  CFV_ERR_ALLOC = 6         /* device or host allocation failed */
};

typedef struct cfv_grid cfv_grid;
typedef struct cfv_ctx cfv_ctx;
typedef struct cfv_ensemble cfv_ensemble;

/* Physical and numerical parameters (nondimensional). */
typedef struct {
  double gamma;      /* polytropic index */
  double c_h;        /* divergence-cleaning speed (Section 3.3: 1) */
  double G;          /* GM_sun/(R_sun V_ref^2): gravity g = -G x/|x|^3 */
  double vr_star;    /* inner radial outflow, Eq. 22: 1935.07 m/s / V_ref */
  double rho_b;      /* inner boundary density */
  double T_b;        /* inner boundary temperature as p/rho */
  int32_t limiter;   /* 0: none, 1: Barth-Jespersen */
  int32_t inner_mode;/* 0: low-E inner boundary (Section 3.2, Eq. 25);
                        1: large-E (Wind-Predict) boundary (Section 3.2,
                        Eqs. 20-24), with the B_theta map of
                        cfv_set_inner_btheta */
  double outer_exp[8]; /* outer ghost powers e in G = I (r_I/r_G)^e for
                          rho, B_r, B_theta, B_phi, V_r, V_theta, V_phi, p (Table 2) */
  int32_t outer_vr_mass;  /* 1: V_r r^2 rho = const instead of outer_exp[4] */
  int32_t outer_psi_zero; /* 1: psi_b = 0 (G = -I); 0: zero gradient (G = I) */
} cfv_params;

/* Thread-local message of the last failure (empty string if none). */
const char* cfv_last_error(void);

/* ----------------------------------------------------------------- grid --
 * Cubed-sphere shell with 6 N x N panels (2 <= N <= 16384) and Nr >= 1 radial layers between the
 * Nr+1 strictly increasing radii r_nodes (host array, copied), at most 2^31 - 1 cells in all
 * (CFV_ERR_ARG otherwise, checked before anything is allocated).  Host only:
 * builds topology (closed-form panel-edge table) and the corner directions. */
cfv_status cfv_grid_create(int32_t N, int32_t Nr, const double* r_nodes, cfv_grid** out);
void cfv_grid_destroy(cfv_grid* g);
/* ncells = 6N^2 Nr; nfaces = 6N^2(Nr+1) + 12N^2 Nr; nbnd = 6N^2 per boundary. */
cfv_status cfv_grid_sizes(const cfv_grid* g, int64_t* ncells, int64_t* nfaces, int64_t* nbnd);
/* Canonical face list (host arrays of length nfaces): cells in increasing
 * order, local faces (r-, r+, xi-, xi+, eta-, eta+); a face is listed by the
 * cell whose neighbour is a ghost or has a larger index.  R of a boundary
 * face is a ghost id: ncells + col (inner) or ncells + 6N^2 + col (outer).
 * kind: 0 interior, 1 inner boundary, 2 outer boundary. */
cfv_status cfv_grid_faces_to_host(const cfv_grid* g, int64_t* L, int64_t* R, int8_t* kind);
/* Geometry of the finite-volume discretisation (Section 2.1) as the kernels
 * rebuild it from the per-column tables, on the host (no device needed):
 * S_f and x_f (host, 3 nfaces, face order of cfv_grid_faces_to_host) the
 * vector area pointing from L to R (out of the domain on boundary faces) and
 * the centroid of each face; V_c (ncells) and x_c (3 ncells) the volume and
 * centroid of each cell.  Vector areas come from the face's four vertices,
 * S = (v2 - v0) x (v3 - v1) / 2, so the six areas of a cell sum to zero;
 * V_c = sum_f x_f . S_f / 3.  Caller-owned outputs; CFV_ERR_ARG on a null
 * pointer. */
cfv_status cfv_grid_geometry_to_host(const cfv_grid* g, double* S_f, double* x_f, double* V_c, double* x_c);

/* ------------------------------------------------------------- context --
 * Binds a grid and parameters to the current HIP device: uploads the grid
 * tables and allocates the workspaces.  The grid must outlive the context. */
cfv_status cfv_ctx_create(const cfv_grid* g, const cfv_params* prm, cfv_ctx** out);
void cfv_ctx_destroy(cfv_ctx* ctx);
/* Copy the inner-boundary B_r map (device array of n = 6N^2 values, order
 * (p*N + j)*N + i, one per inner face, nondimensional): the magnetogram-
 * imposed radial field of the inner ghost cells (Section 3.2: B_r Dirichlet
 * from the map; with the low-E law the boundary velocity is parallel to the
 * boundary field, Eq. 25, with the outflow constant of Eq. 22).  The residual,
 * JVP and VJP read the copy, so the caller's array may be freed after the
 * stream reaches this call.  CFV_ERR_SIZE if n != 6N^2. */
cfv_status cfv_set_inner_br(cfv_ctx* ctx, const double* br_dev, int64_t n, hipStream_t s);

/* Copy the inner-boundary B_theta map (device array of n = 6N^2 values, the
 * order of the B_r map) used by the large-E law (inner_mode = 1): the
 * Dirichlet value of B_theta on each inner face, which a potential-field
 * model supplies (Eq. 21).  Zero until set; a constant of the operator (no
 * derivative is taken with respect to it). */
cfv_status cfv_set_inner_btheta(cfv_ctx* ctx, const double* bth_dev, int64_t n, hipStream_t s);

/* Geometry as the kernels see it (device outputs): cell centroids xc[3c+d],
 * volumes vol[c], and per (cell, local face) the face centroid xf[(6c+f)*3+d]
 * and the vector area S outward from the cell (the face owner's numbers). */
cfv_status cfv_geometry(cfv_ctx* ctx, double* xc, double* vol, double* xf, double* S, hipStream_t s);

/* ----------------------------------------------------------- hot path --
 * R = R(U, B_r), the finite-volume residual of ideal MHD with hyperbolic
 * divergence cleaning (Section 2.1, Eqs. 14-17 in the mu = 1 form, plus the
 * psi equation with speed c_h): ghost states on the inner boundary from the
 * B_r map (Section 3.2, Eq. 25 or Eqs. 20-24 by inner_mode) and on the outer
 * boundary (Table 2 laws, Section 4.1), primitives, a least-squares gradient
 * over the six face neighbours with the Barth-Jespersen limiter (limiter =
 * 1), the reconstructed face states, the Rusanov flux of every face evaluated
 * once in its canonical orientation, and the gravity source at the centroid.
 * U, R: device [9][ncells] (caller-owned, must not overlap).  Asynchronous on
 * s; a face state with non-positive (or NaN) density or pressure sets the
 * context's non-physical flag (cfv_status_flags). */
cfv_status cfv_residual(cfv_ctx* ctx, const double* U, double* R, hipStream_t s);
/* Jv = J_U v + J_b dbr, the Jacobian-vector product of the residual: the
 * linearisation the implicit (Newton-Krylov) pseudo-time step of Section 2.1
 * solves with.  v, Jv: device [9][ncells]; dbr: device 6N^2 (may be NULL: no
 * map direction); when R is not NULL the residual is written too.  Exact
 * forward linearisation (the residual's arithmetic on value-tangent pairs);
 * branches (limiter choice, |v_n|, speed picks) follow the primal values.
 * Asynchronous; sets the non-physical flag as cfv_residual. */
cfv_status cfv_jvp(cfv_ctx* ctx, const double* U, const double* v, const double* dbr, double* Jv, double* R,
                   hipStream_t s);
/* gU = J_U^T w and (when gbr is not NULL) gbr = J_b^T w (6N^2 values): the
 * adjoint of the Section 2.1 residual linearisation, for transposed solves
 * of the implicit step and the sensitivity of an outer-boundary objective to
 * the magnetogram B_r map (Section 3.2).  w, gU: device [9][ncells].  A
 * hand-written reverse pass, the exact transpose of cfv_jvp's operator
 * (same branches).  Deterministic: no floating-point atomics.  Asynchronous;
 * uses the context's workspace. */
cfv_status cfv_vjp(cfv_ctx* ctx, const double* U, const double* w, double* gU, double* gbr, hipStream_t s);
/* Backward-Euler diagonal of the implicit pseudo-time step with a local
 * time step set by the CFL number (Sections 2.1 and 4.1): diag[c] = V_c/dt_c
 * = sum over the six faces of s_f |S_f| / cfl, s_f the Rusanov speed of the
 * face (max of |v_n| + c_f on both reconstructed sides and c_h).  diag:
 * device [ncells].  CFV_ERR_ARG unless cfl > 0.  Asynchronous. */
cfv_status cfv_local_dt(cfv_ctx* ctx, const double* U, double cfl, double* diag, hipStream_t s);

/* Non-physical state check (the face-state positivity condition of the
 * reconstruction: no fix-up is applied, the computation goes on and the
 * condition is reported).  The residual, JVP and VJP kernels OR bit 0 into a
 * per-context device word whenever a reconstructed face state or a ghost
 * state has density or pressure that is not positive (NaN included); the
 * word accumulates over calls (also inside cfv_be_step and cfv_steady) until
 * read.  This call synchronises s, returns the word in *flags (host,
 * nullable) and clears it; it returns CFV_ERR_NONPHYSICAL when bit 0 was
 * set, CFV_OK otherwise.  The flag does not change any output. */
cfv_status cfv_status_flags(cfv_ctx* ctx, int32_t* flags, hipStream_t s);

/* -------------------------------------------------------- E-field --
 * The ideal-MHD electric field E = -V x B (Section 2.2), the diagnostic the
 * paper reads for the quality of an inner boundary law (Section 3.1: its
 * azimuthal part should stay small).  At every cell centroid E is projected
 * on the unit vectors r, theta, phi there (Eqs. 20-21; on the polar axis the
 * meridian phi = 0 is taken).  E3 (device, nullable) receives the field as 3
 * rows of ncells: E_r, E_theta, E_phi.  stats8 (device, 8 doubles) receives
 * max_c |E_r|, |E_theta|, |E_phi|, |E| and then the volume-weighted RMS of
 * the same four, sqrt(sum_c V_c E^2 / sum_c V_c).  Fixed reduction order
 * (deterministic).  U is the conservative state, 9 rows of ncells. */
cfv_status cfv_efield(cfv_ctx* ctx, const double* U, double* E3, double* stats8_dev, hipStream_t s);
/* The E-free state (Section 3.1, the first remedy: V0 x B0 = 0): U_out is U
 * with each cell's velocity replaced by its component along B,
 * (V . B / |B|^2) B, and the total energy recomputed from the unchanged
 * density, field and pressure; psi is kept; a cell with B = 0 is copied.
 * U_out may equal U (in place); other overlaps are not allowed. */
cfv_status cfv_efree_state(cfv_ctx* ctx, const double* U, double* U_out, hipStream_t s);

/* --------------------------------------------------------- reductions --
 * out9[v] = sqrt(sum_c (a - b)^2) per variable (b may be NULL): the Eq. 2
 * residual monitor before the log10 (Section 2.1).  a, b: device
 * [9][ncells]; out9: device, 9 doubles.  Fixed reduction order
 * (deterministic).  Asynchronous. */
cfv_status cfv_norms(cfv_ctx* ctx, const double* a, const double* b, double* out9_dev, hipStream_t s);
/* out[i] = <V_i, w> for k vectors V_i stored back to back (9*ncells each,
 * device; 1 <= k <= 32): the Gram-Schmidt projections of the GMRES solve of
 * the implicit step (Section 2.1).  out: device, k doubles.  Fixed
 * reduction order.  Asynchronous. */
cfv_status cfv_dots(cfv_ctx* ctx, const double* V, int32_t k, const double* w, double* out_dev, hipStream_t s);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the dot
 * products of cfv_dots without a context, out[i] = <V_i, w> for k vectors V_i
 * of n entries each stored back to back (device), w (device, n), out
 * (device, k).  Nothing is allocated: the partial sums live in a static
 * device array of 32 x 1024 doubles (256 KiB, held by each device the library
 * runs on until the process ends), so 1 <= k <= 32 (CFV_ERR_ARG otherwise,
 * before any device work).  The same kernels and launch shape as cfv_dots:
 * the results are bitwise those of cfv_dots.  Calls that overlap on one
 * device share that array and race: order them on one stream.
 * Asynchronous. */
cfv_status cfv_dots_noalloc(int64_t n, const double* V, int32_t k, const double* w, double* out, hipStream_t s);
/* y = a*x + b*y over n device values (a, b scalars from the host): the
 * vector update of the Krylov solve and of the pseudo-time step (Section
 * 2.1).  Asynchronous. */
cfv_status cfv_axpby(cfv_ctx* ctx, int64_t n, double a, const double* x, double b, double* y, hipStream_t s);

/* ---------------------------------------------------- implicit solver --
 * Solve (diag + J) x = rhs (transpose = 0) or (diag + J^T) x = rhs
 * (transpose = 1), J = dR/dU at U applied matrix-free through the JVP or the
 * VJP, diag[ncells] a per-cell diagonal applied to all 9 variables: GMRES(m)
 * from x = 0 with modified Gram-Schmidt, restarted up to max_restarts times,
 * stopping when |rhs - A x| <= rtol |rhs| (rtol = 0 runs all iterations).
 * hist (host, nullable, hist_len entries) receives |r_j|/|rhs| after every
 * iteration; iters and final_rel (host, nullable) the iteration count and
 * the last relative residual.  x must not alias rhs.  The Arnoldi vectors,
 * dot products and updates stay on the device; the stream is synchronised
 * once per iteration to bring the Hessenberg column to the host, where the
 * Givens least squares is solved.  The Krylov workspace ((m+1) state
 * vectors) is owned by the context and grown on first use.
 * This is the linear solve of the implicit backward-Euler pseudo-time step
 * of Section 2.1. */
cfv_status cfv_solve(cfv_ctx* ctx, const double* U, const double* diag, const double* rhs, int32_t transpose,
                     int32_t m, int32_t max_restarts, double rtol, double* x, double* hist, int32_t hist_len,
                     int32_t* iters, double* final_rel, hipStream_t s);
/* One backward-Euler pseudo-time step (Section 2.1, with the local CFL time
 * step of Section 4.1): U_new = U + x with (V/dt + J) x = -R(U), V/dt from
 * cfv_local_dt at the given cfl, solved by cfv_solve.  U, U_new: device
 * [9][ncells]; U_new must not alias U.  Synchronises s (through cfv_solve).
 * Returns CFV_ERR_NONPHYSICAL, with U_new undefined, when the residual of U
 * or a Krylov scalar is not finite (cfv_solve); non-positive face states
 * only set the context's flag word (cfv_status_flags). */
cfv_status cfv_be_step(cfv_ctx* ctx, const double* U, double cfl, int32_t m, int32_t max_restarts, double rtol,
                       double* U_new, double* hist, int32_t hist_len, int32_t* iters, double* final_rel,
                       hipStream_t s);

/* ------------------------------------------------------ steady march --
 * The Eq. 2 monitor on the physical quantities: out9 (device) receives, per
 * primitive variable (rho, V_x, V_y, V_z, B_x, B_y, B_z, p, psi), the 2-norm
 * over the cells of the change between the states a and b,
 * sqrt(sum_c (a_c - b_c)^2), before the log10.  Deterministic. */
cfv_status cfv_monitor(cfv_ctx* ctx, const double* a, const double* b, double* out9_dev, hipStream_t s);

/* Pseudo-time march to a steady state (Sections 2.1 and 4.1). */
typedef struct {
  double cfl0;          /* CFL of the first step (the paper starts at 2) */
  double cfl_max;       /* cap (128 in the paper's CFL law; up to 1000 or more) */
  int32_t every;        /* steps between doublings of the CFL (>= 1) */
  int32_t max_iters;    /* at most this many steps (>= 0) */
  int32_t monitor;      /* primitive variable of the stopping rule, 0..8 (1 = V_x) */
  double target;        /* stop once log10 of its Eq. 2 value is below this */
  int32_t m;            /* GMRES(m) per step, 1..200 */
  int32_t max_restarts; /* restarts of the linear solve per step */
  double rtol;          /* relative tolerance of the linear solve (0: all iterations) */
} cfv_steady_cfg;

/* Backward-Euler steps (cfv_be_step) from the state U (device, updated in
 * place) with CFL_i = min(cfl0 2^floor(i / every), cfl_max) at step i, until
 * log10 of the Eq. 2 monitor (cfv_monitor between the states before and after
 * a step) of variable `monitor` falls below target, or max_iters steps.
 * hist (host, nullable, 9 max_iters) receives the nine log10 monitor values
 * of every step, cfl_hist (host, nullable, max_iters) the CFL used, iters the
 * number of steps taken.  The stream is synchronised once per step for the
 * monitor (and once per GMRES iteration inside the solve).  A second state
 * buffer is owned by the context (allocated on first use).  If a step's
 * solve is not finite (cfv_be_step returns CFV_ERR_NONPHYSICAL; its monitors
 * are recorded as NaN) or a step produces a non-finite monitor value, the
 * march stops, U keeps the state before that step, the step is counted in
 * iters and recorded in hist, and CFV_ERR_NONPHYSICAL is returned.
 * Non-positive face states met on the way are left in the context's flag
 * word (cfv_status_flags). */
cfv_status cfv_steady(cfv_ctx* ctx, double* U, const cfv_steady_cfg* cfg, double* hist, double* cfl_hist,
                      int32_t* iters, hipStream_t s);

/* ------------------------------------------------- second derivatives --
 * Directional derivatives of the linearisations, for the second-order terms
 * of the adjoint of the implicit step map (the Newton linearisation of
 * Section 2.1 differentiated once more).  Both take a central difference of
 * two exact first-derivative evaluations at +-h along the direction, with
 * one scalar h = eps / max_e |d_e| / (|u_e| + 1e-3 max|u_var(e)|): every
 * entry moves by at most eps relative to its own size (or to a thousandth of
 * its variable's largest magnitude).  This is the one approximate piece of
 * the sensitivity; h_used (host, nullable) returns h.  Both synchronise the
 * stream twice (the step is chosen on the host) and use a context-owned
 * workspace of two state vectors, allocated on first use.
 *
 * gU2 = d/de [J_U(U + e x)^T w] and, when gbr2 is not NULL,
 * gbr2 = d/de [J_b(U + e x)^T w] (6N^2 values), at e = 0. */
cfv_status cfv_vjp_dir(cfv_ctx* ctx, const double* U, const double* w, const double* x, double eps, double* gU2,
                       double* gbr2, double* h_used, hipStream_t s);
/* Jv2 = d/de [J_U(U + e dU, b + e dbr) v] at e = 0 (dbr may be NULL: the map
 * held by the context is not moved). */
cfv_status cfv_jvp_dir(cfv_ctx* ctx, const double* U, const double* v, const double* dU, const double* dbr, double eps,
                       double* Jv2, double* h_used, hipStream_t s);

/* ------------------------------------------------------------ ensemble --
 * Many independent instances (different grids, B_r maps and states; the
 * magnetogram-driven ensembles the model is meant for) evaluated by one
 * persistent launch per pass.  The work items are (instance, column tile,
 * chunk of chunk_layers layers); each instance's outputs are bitwise those of
 * cfv_residual / cfv_jvp on its own context (the outputs do not depend on the
 * chunk length, see cfv_set_chunk_layers).  The contexts keep owning
 * their grid tables, B_r map and gradient workspaces, so one context may
 * appear in only one ensemble run at a time, and no two runs of ensembles
 * sharing a context may overlap. */
typedef struct {
  int32_t queue;          /* 0: static split of the item list (each XCD takes a
                             contiguous eighth); 1: device work counter */
  int32_t blocks_per_cu;  /* persistent workgroups per compute unit, 1..16 */
  int32_t order;          /* 0: instance order; 1: largest items first */
  int32_t chunk_layers;   /* radial layers per work item, 1..4096; 0: 16 */
} cfv_tuning;
/* ctxs: host array of n contexts on the current device (not owned). */
cfv_status cfv_ensemble_create(cfv_ctx* const* ctxs, int32_t n, const cfv_tuning* t, cfv_ensemble** out);
void cfv_ensemble_destroy(cfv_ensemble* e);
/* Change the schedule (drops a captured graph; a new chunk length rebuilds
 * the item lists, synchronously). */
cfv_status cfv_ensemble_set_tuning(cfv_ensemble* e, const cfv_tuning* t);
/* GMRES preconditioner of the batched backward-Euler step, as
 * cfv_set_preconditioner (0 none, 1 Jacobi by V/dt); it takes effect at the
 * next cfv_ensemble_bind_be_step (a bound step must be bound again). */
cfv_status cfv_ensemble_set_preconditioner(cfv_ensemble* e, int32_t kind);
/* Number of work items and the workgroups a launch uses (host outputs). */
cfv_status cfv_ensemble_items(const cfv_ensemble* e, int64_t* total, int32_t* blocks);
/* Bind the per-instance device buffers (host arrays of n device pointers,
 * copied into a device descriptor table; synchronous).  With v not NULL the
 * run is the JVP: Jv[q] = J_U v[q] (+ J_b dbr[q] when dbr is not NULL), and
 * R[q] too when R is not NULL.  With v NULL it is the residual: R required,
 * Jv and dbr NULL.  Drops a captured graph. */
cfv_status cfv_ensemble_bind(cfv_ensemble* e, const double* const* U, const double* const* v,
                             const double* const* dbr, double* const* R, double* const* Jv);
/* Bind a backward-Euler step of every instance (the ensemble form of
 * cfv_be_step with max_restarts = 0 and rtol = 0): U_new[q] = U[q] + x_q with
 * (V/dt + J) x_q = -R(U[q]) solved by GMRES(m) from x = 0 with modified
 * Gram-Schmidt, all instances in lockstep.  Every scalar of the solve (norms,
 * Gram-Schmidt coefficients, Givens rotations, the least-squares solve) stays
 * on the device, so a run needs no host synchronisation and can be captured.
 * hist (device, nullable, n x m) receives each instance's relative residual
 * after every iteration (an instance that breaks down or converges exactly
 * repeats its last value).  The Krylov workspace ((m + 2) state vectors per
 * instance) is owned by the ensemble.  U_new[q] must not alias U[q].  Drops a
 * captured graph; cfv_ensemble_run / _graph_capture then run the step. */
cfv_status cfv_ensemble_bind_be_step(cfv_ensemble* e, const double* const* U, double* const* U_new, double cfl,
                                     int32_t m, double* hist);
/* Run what is bound on stream s: the residual / JVP (two persistent
 * launches) or the backward-Euler step. */
cfv_status cfv_ensemble_run(cfv_ensemble* e, hipStream_t s);
/* Bind (no map directions) and run. */
cfv_status cfv_ensemble_residual_jvp(cfv_ensemble* e, const double* const* U, const double* const* v,
                                     double* const* R, double* const* Jv, hipStream_t s);
/* Capture one run of what is bound into a HIP graph (s must be a created
 * stream, not the null stream) and replay it.  The graph holds kernel nodes
 * only (the queue counters are cleared by a kernel, not a memset). */
cfv_status cfv_ensemble_graph_capture(cfv_ensemble* e, hipStream_t s);
cfv_status cfv_ensemble_graph_launch(cfv_ensemble* e, hipStream_t s);
/* Per-instance status words of the ensemble's runs (an ensemble keeps its
 * own, separate from its contexts'): bit 0 as cfv_status_flags (a
 * non-positive or NaN face density or pressure), bit 1 a backward-Euler step
 * whose residual norm was not finite.  Synchronises s, writes n words to
 * flags (host, nullable), clears them, and returns CFV_ERR_NONPHYSICAL when
 * any instance has a bit set. */
cfv_status cfv_ensemble_status_flags(cfv_ensemble* e, int32_t* flags, hipStream_t s);
/* Per-kernel event timing of eager runs, as cfv_timing_enable / _read. */
cfv_status cfv_ensemble_timing_enable(cfv_ensemble* e, int32_t on);
cfv_status cfv_ensemble_timing_read(cfv_ensemble* e, int32_t max, char* names, double* total_ms, int64_t* count,
                                    int32_t* n);

/* Batched march to a steady state (Sections 2.1 and 4.1) of every instance
 * of the ensemble: lockstep backward-Euler steps with GMRES(m) (the step of
 * cfv_ensemble_bind_be_step, captured in a graph when s is a created stream
 * and captured again whenever the CFL law changes the CFL), the Eq. 2
 * monitor of each instance after each step (cfv_monitor), and the CFL law
 * and stopping rule of cfv_steady (cfg->max_restarts and cfg->rtol are not
 * used: the lockstep step runs its m iterations).  An instance stops once
 * its monitored variable is below target: later steps of the others still
 * compute it (the graph is shared) but its state is no longer updated.
 * U (device, per instance, updated in place) and U_work (device, per
 * instance, the step's output) are 9 ncells each and must not alias.
 * hist (host, nullable, n x max_iters x 9) receives the log10 monitors, NaN
 * after an instance stopped; steps (host, nullable, n) the steps each
 * instance took; iters the lockstep steps run.  An instance whose step has a
 * non-finite residual norm (bit 1 of its flag word, cfv_ensemble_status_flags)
 * or gives a non-finite monitor keeps its previous state and stops; the call
 * then returns CFV_ERR_NONPHYSICAL after the others finish.  The flag words
 * are cleared when the march starts; bit 0 (non-positive face states) is left
 * for the caller.  The ensemble's
 * binding is replaced by the step binding. */
cfv_status cfv_ensemble_steady(cfv_ensemble* e, double* const* U, double* const* U_work, const cfv_steady_cfg* cfg,
                               double* hist, int32_t* steps, int32_t* iters, hipStream_t s);

/* ------------------------------------------------------------ profiling --
 * While enabled, every kernel launch of the context is bracketed by a pair of
 * HIP events on its launch stream.  cfv_timing_read synchronises on the
 * recorded events and returns, per kernel name (names: max * 32 chars), the
 * total milliseconds and the launch count since the previous read, then
 * clears the record (n = number of names written). */
cfv_status cfv_timing_enable(cfv_ctx* ctx, int32_t on);
/* Work decomposition of the context's own launches: every march (the fused
 * residual march, the dual JVP march, the VJP's gradient march) splits each
 * column tile's Nr layers into chunks of kc layers (1..4096), one work item
 * each.  kc = 0 (the default) lets each march balance its items over the
 * device's compute units: of the chunk counts, the one with the fewest
 * rounds of items times layers marched per item.  A chunk also marches the
 * layers on either side of it, so longer chunks move fewer bytes, shorter
 * ones give more work items on small grids.  Every output is bitwise the
 * same for every kc: each face flux is evaluated once from the same states,
 * and each cell sums its faces in a fixed order. */
cfv_status cfv_set_chunk_layers(cfv_ctx* ctx, int32_t kc);
/* Preconditioner of the context's GMRES solves (cfv_solve, and through it
 * cfv_be_step and cfv_steady): kind 0 none (the default; the step of
 * Section 2.1 as read here), 1 Jacobi: right preconditioning by the solve's
 * own diagonal, (diag + J) D^-1 y = rhs with x = D^-1 y and D = diag per cell
 * (for the backward-Euler step V/dt, proportional under the local time step
 * to the diagonal of V/dt plus the first-order flux Jacobian).  The history
 * still reports |rhs - (diag + J) x| / |rhs|.  With kind 1 every diag entry
 * must be positive (a zero gives non-finite iterates, which the solve
 * reports as CFV_ERR_NONPHYSICAL).  The batched ensemble step takes its own
 * setting (cfv_ensemble_set_preconditioner). */
cfv_status cfv_set_preconditioner(cfv_ctx* ctx, int32_t kind);
cfv_status cfv_timing_read(cfv_ctx* ctx, int32_t max, char* names, double* total_ms, int64_t* count, int32_t* n);

#ifdef __cplusplus
}
#endif
#endif /* CFV_H */
