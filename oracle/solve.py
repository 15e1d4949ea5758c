"""Derivatives, pseudo-time step and monitors (oracle; test infrastructure).

* ``jvp``: J_U v + J_b dbr, the exact directional derivative of the residual
  (forward-mode automatic differentiation of ``mhd.residual``).  Branches
  (min/max picks, |v_n|, the clamp under the square root) follow the values.
* ``vjp``: J_U^T w and J_b^T w by reverse mode on the same function.
* ``local_dt``: the backward-Euler diagonal V_c/dt_c = sum_f s_f |S_f| / CFL,
  i.e. dt_c = CFL V_c / sum_f s_f |S_f| with s_f the Rusanov speed.
* ``eq2``: the residual monitor of Eq. 2, log10 sqrt(sum_i (a_i^t - a_i^{t+1})^2),
  per variable.
* ``gmres``: unrestarted GMRES(m), x0 = 0, modified Gram-Schmidt, Givens
  least squares, for the implicit step (D + J) x = -R (Section 2.1: backward
  Euler with large CFL).
* ``cfl_law``, ``eq2_prim`` and ``steady``: the march to a steady state,
  backward-Euler steps under the CFL law of Section 4.1 with the Eq. 2
  monitor of the primitive quantities and its stopping threshold.
* ``layer_objective`` and ``step_map_sensitivity``: an objective on the state
  after n implicit steps with a fixed diagonal, and its exact gradient with
  respect to the inner B_r map, by reverse mode through the unrolled steps
  with the Jacobian formed densely (small grids only).
"""
from __future__ import annotations

import math

import torch

from . import mhd
from .grid import Grid

DT = torch.float64


def jvp(grid: Grid, U, br, prm, v, dbr=None, cells=None):
    if dbr is None:
        dbr = torch.zeros_like(br)

    def f(U_, br_):
        return mhd.residual(grid, U_, br_, prm, cells)

    R, Jv = torch.func.jvp(f, (U, br), (v, dbr))
    return Jv, R


def vjp(grid: Grid, U, br, prm, w, cells=None):
    """Returns (gU (9, ncells), gbr (6N^2,)) = (J_U^T w, J_b^T w).

    With ``cells``, w holds the weights of those cells only (9, len(cells))."""
    U_ = U.detach().clone().requires_grad_(True)
    b_ = br.detach().clone().requires_grad_(True)
    R = mhd.residual(grid, U_, b_, prm, cells)
    gU, gb = torch.autograd.grad((R * w).sum(), (U_, b_), allow_unused=True)
    if gb is None:
        gb = torch.zeros_like(br)
    return gU, gb


def face_speeds(grid: Grid, U, br, prm, cells=None):
    """Per target cell: Rusanov speeds s (n, 6) and face areas |S| (n, 6)."""
    _, (s, area) = mhd.residual(grid, U, br, prm, cells, return_speeds=True)
    return s, area


def local_dt_diag(grid: Grid, U, br, prm, cfl, cells=None):
    """V_c / dt_c = (sum over faces of s_f |S_f|) / CFL."""
    s, area = face_speeds(grid, U, br, prm, cells)
    return (s * area).sum(1) / cfl


def eq2(a, b):
    """Eq. 2 per variable: log10 of the 2-norm of a - b over cells."""
    d = (a - b)
    return torch.log10(torch.sqrt((d * d).sum(-1)))


def gmres(matvec, rhs, m: int = 30, tol: float = 0.0, precond=None):
    """Unrestarted GMRES(m) from x0 = 0 with modified Gram-Schmidt.

    With precond (a function applying M^-1), right preconditioning: GMRES
    runs on the operator A M^-1 and returns x = M^-1 y; the residual of
    A x = rhs is the same as that of A M^-1 y = rhs.

    Returns x and the list of relative residual norms |r_j| / |rhs| after
    each iteration j = 1..m (from the Givens-rotated least-squares system)."""
    if precond is not None:
        y, hist = gmres(lambda v: matvec(precond(v)), rhs, m, tol)
        return precond(y), hist
    beta = torch.linalg.norm(rhs)
    Vs = [rhs / beta]
    H = torch.zeros(m + 1, m, dtype=DT)
    cs = torch.zeros(m, dtype=DT)
    sn = torch.zeros(m, dtype=DT)
    gvec = torch.zeros(m + 1, dtype=DT)
    gvec[0] = beta
    hist = []
    k_done = 0
    for j in range(m):
        w = matvec(Vs[j])
        for i in range(j + 1):
            H[i, j] = (w * Vs[i]).sum()
            w = w - H[i, j] * Vs[i]
        H[j + 1, j] = torch.linalg.norm(w)
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        den = math.hypot(float(H[j, j]), float(H[j + 1, j]))
        cs[j] = H[j, j] / den
        sn[j] = H[j + 1, j] / den
        H[j, j] = den
        H[j + 1, j] = 0.0
        gvec[j + 1] = -sn[j] * gvec[j]
        gvec[j] = cs[j] * gvec[j]
        hist.append(float(abs(gvec[j + 1]) / beta))
        k_done = j + 1
        if float(H[j + 1, j]) == 0.0 and j + 1 < m:
            pass
        nrm = torch.linalg.norm(w)
        if nrm == 0 or hist[-1] <= tol:
            break
        Vs.append(w / nrm)
    y = torch.linalg.solve_triangular(H[:k_done, :k_done], gvec[:k_done, None], upper=True)[:, 0]
    x = torch.zeros_like(rhs)
    for i in range(k_done):
        x = x + y[i] * Vs[i]
    return x, hist


def be_step(grid: Grid, U, br, prm, cfl: float = 1e3, m: int = 30, diag=None, jacobi: bool = False):
    """One backward-Euler pseudo-time step: (D + J) x = -R, U <- U + x;
    jacobi: GMRES right-preconditioned by D (one value per cell)."""
    R = mhd.residual(grid, U, br, prm)
    if diag is None:
        diag = local_dt_diag(grid, U, br, prm, cfl)

    def A(x):
        Jx, _ = jvp(grid, U, br, prm, x)
        return diag[None, :] * x + Jx

    x, hist = gmres(A, -R, m, precond=(lambda v: v / diag[None, :]) if jacobi else None)
    return U + x, hist, R


def cfl_law(it: int, cfl0: float = 2.0, cfl_max: float = 128.0, every: int = 200) -> float:
    """CFL of pseudo-time iteration it (from 0): cfl0 doubled after every
    `every` iterations and capped at cfl_max (Section 4.1: from 2, doubling
    every few hundred iterations, up to 128; Section 2.1: up to 1000 or more)."""
    cfl = cfl0
    for _ in range(it // every):
        if cfl >= cfl_max:
            break
        cfl *= 2.0
    return min(cfl, cfl_max)


def eq2_prim(Ua, Ub, gamma):
    """Eq. 2 on the physical quantities: per primitive variable (rho, V, B,
    p, psi), log10 sqrt(sum over cells of (a^t - a^{t+1})^2)."""
    Pa = mhd.cons_to_prim(Ua.transpose(0, 1), gamma).transpose(0, 1)
    Pb = mhd.cons_to_prim(Ub.transpose(0, 1), gamma).transpose(0, 1)
    return eq2(Pa, Pb)


def steady(grid: Grid, U, br, prm, iters: int, cfl0: float = 2.0, cfl_max: float = 128.0, every: int = 200,
           m: int = 30, monitor: int = 1, target: float = -math.inf):
    """Pseudo-time marching to a steady state (Sections 2.1, 4.1): backward-
    Euler steps at the CFL of ``cfl_law``; after each step the Eq. 2 monitor
    of the primitives between the old and new state is recorded, and the
    march stops once the monitored variable (default 1, V_x) is below
    target, or after iters steps.  Returns (U, monitor history (n, 9),
    CFL per step)."""
    hist, cfls = [], []
    for it in range(iters):
        cfl = cfl_law(it, cfl0, cfl_max, every)
        Un, _, _ = be_step(grid, U, br, prm, cfl, m)
        res = eq2_prim(U, Un, prm.gamma)
        hist.append(res)
        cfls.append(cfl)
        U = Un
        if float(res[monitor]) < target:
            break
    return U, torch.stack(hist), cfls


def layer_objective(grid: Grid, layer=None):
    """lam with L = <lam, U>: the mean over the 6N^2 cells of one radial layer
    (default the outermost) of the momentum (rho v) projected on r_hat at the
    cell's upper (r+) face centroid."""
    k = grid.Nr - 1 if layer is None else int(layer)
    cols = torch.arange(grid.nb)
    p, rest = cols // (grid.N * grid.N), cols % (grid.N * grid.N)
    cells = grid.encode(p, torch.full_like(p, k), rest // grid.N, rest % grid.N)
    _, _, xf, _ = grid.cell_geometry(cells)
    xo = xf[:, 1]
    rh = xo / torch.linalg.norm(xo, dim=-1, keepdim=True)
    lam = torch.zeros(9, grid.ncells, dtype=DT)
    lam[1:4, cells] = rh.T / grid.nb
    return lam


def step_map_sensitivity(grid: Grid, U0, br, prm, D0, nsteps: int, lam, want_grad: bool = True):
    """L = <lam, U_n> after n steps of U <- U - (D0 + J(U, b))^{-1} R(U, b) from U0,
    with D0 a fixed per-cell diagonal (the implicit step of Section 2.1 with
    exact solves, V/dt held at its initial value), and dL/db.

    The Jacobian is formed densely by reverse mode, each step solves the dense
    system, and the gradient is reverse mode through everything: residuals,
    Jacobians (second derivatives included) and solves.  Returns (L, dL/db)
    (dL/db is None when want_grad is False)."""
    n = 9 * grid.ncells
    D = torch.as_tensor(D0, dtype=DT).detach()
    b = br.detach().clone().requires_grad_(want_grad)
    U = U0.detach().clone()
    for _ in range(nsteps):
        def f(u):
            return mhd.residual(grid, u, b, prm)
        R = f(U)
        J = torch.autograd.functional.jacobian(f, U, create_graph=want_grad, vectorize=True)
        A = J.reshape(n, n) + torch.diag(D.repeat(9))
        x = torch.linalg.solve(A, -R.reshape(n))
        U = U + x.reshape(9, grid.ncells)
    L = (lam * U).sum()
    if not want_grad:
        return float(L), None
    gb, = torch.autograd.grad(L, b)
    return float(L.detach()), gb
