"""Magnetogram sensitivity: gradient of an outer-boundary objective with
respect to the inner-boundary B_r map after n implicit pseudo-time steps.

Step map (the backward-Euler pseudo-time step of Section 2.1, with tight
linear solves so that it is differentiable):

    U_{n+1} = U_n + x_n,   (D0 + J(U_n, b)) x_n = -R(U_n, b),

with D0 = V/dt frozen at the initial state (cfv_local_dt at U_0), b the B_r
map.  Objective: L = mean over the outer layer of rho v . r_hat at the outer
face centroid, L = <lam, U_N> with lam fixed (it is linear in U).

Adjoint (reverse sweep, with mu = A_n^-T lam_{n+1}, A_n = D0 + J_n):

    lam_n = lam_{n+1} - J_n^T mu - H_n^T mu,   g_b -= R_b^T mu + K_n^T mu,

where H_n^T mu and K_n^T mu are the derivatives of (J_n^T mu, R_b^T mu) along
x_n (cfv_vjp_dir: a central difference of two exact VJPs, the one approximate
piece).  States are recomputed from checkpoints every `every` steps (each
segment is recomputed once and kept while it is swept).

Tangent (forward sweep along a map direction db, an independent check of the
adjoint through the JVP kernels):

    dU_{n+1} = dU_n - A_n^-1 (J_n dU_n + R_b db + d/de[J(U_n + e dU_n, b + e db)] x_n),

and dL = <lam, dU_N> must equal <g_b, db>.

The CFL must keep every solve tight, since the adjoint is exact only for an
exact step: unpreconditioned restarted GMRES(40) reaches 1e-12 within about
seven cycles at CFL 0.05 on a 12-layer grid and at CFL 1 on a 4-layer one,
but stalls near 1e-3 at CFL 2 on the 12-layer grid.  A small CFL also limits
how far a B_r change travels in 20 steps (a few cells), so the objective can
be taken on an inner layer (`layer`) when the outer one is out of reach.

Every vector operation runs in the library (residual, JVP/VJP, GMRES,
reductions); this module only orchestrates the calls.
"""
from __future__ import annotations

import torch

from .binding import Context


def outer_objective_weights(ctx: Context, layer: int | None = None) -> torch.Tensor:
    """lam with L = <lam, U>: the mean over the cells of one radial layer
    (default the outermost) of (rho v) . r_hat at their upper face centroid."""
    g = ctx.grid
    N, Nr = g.N, g.Nr
    k = Nr - 1 if layer is None else int(layer)
    if not 0 <= k < Nr:
        raise ValueError(f"layer {k} outside [0, {Nr})")
    xc, vol, xf, S = ctx.geometry()
    lam = torch.zeros(9, g.ncells, dtype=torch.float64, device=xc.device)
    cols = torch.arange(6 * N * N, device=xc.device)
    p = cols // (N * N)
    cells = (p * Nr + k) * N * N + cols % (N * N)
    xo = xf[cells, 1]                                   # outer face centroids
    rh = xo / torch.linalg.norm(xo, dim=-1, keepdim=True)
    w = 1.0 / cols.numel()
    for d in range(3):
        lam[1 + d, cells] = w * rh[:, d]
    return lam


class Sensitivity:
    def __init__(self, ctx: Context, U0: torch.Tensor, cfl: float = 0.05, nsteps: int = 20, every: int = 5,
                 m: int = 40, max_restarts: int = 12, rtol: float = 1e-12, eps: float = 1e-6,
                 layer: int | None = None):
        if nsteps < 1 or every < 1:
            raise ValueError("need nsteps >= 1 and every >= 1")
        self.ctx, self.U0 = ctx, U0
        self.nsteps, self.every = nsteps, every
        self.m, self.max_restarts, self.rtol, self.eps = m, max_restarts, rtol, eps
        self.D0 = ctx.local_dt(U0, cfl)
        self.lam_L = outer_objective_weights(ctx, layer)
        self.max_rel = 0.0

    def _solve(self, U, rhs, transpose):
        x, hist = self.ctx.solve(U, self.D0, rhs, transpose=transpose, m=self.m, max_restarts=self.max_restarts,
                                 rtol=self.rtol)
        if len(hist):
            self.max_rel = max(self.max_rel, float(hist[-1]))
        return x

    def _step(self, U):
        """(U_{n+1}, x_n) with (D0 + J) x_n = -R(U_n)."""
        R = self.ctx.residual(U)
        self.ctx.axpby(0.0, R, -1.0, R)
        x = self._solve(U, R, False)
        Un = U.clone()
        self.ctx.axpby(1.0, x, 1.0, Un)
        return Un, x

    def _objective(self, U) -> float:
        return float(self.ctx.dots(self.lam_L.reshape(1, -1), U.reshape(-1))[0])

    def forward(self, br: torch.Tensor):
        """Run the steps with map br; returns (L, checkpoints)."""
        self.ctx.set_inner_br(br)
        U = self.U0.clone()
        ckpt = {0: U}
        for n in range(self.nsteps):
            U, _ = self._step(U)
            if (n + 1) % self.every == 0:
                ckpt[n + 1] = U
        return self._objective(U), ckpt

    def objective(self, br: torch.Tensor) -> float:
        return self.forward(br)[0]

    def gradient(self, br: torch.Tensor):
        """dL/dbr by the adjoint sweep; returns (L, g_b)."""
        ctx = self.ctx
        L, ckpt = self.forward(br)
        lam = self.lam_L.clone()
        gb = torch.zeros_like(br)
        for s0 in reversed(range(0, self.nsteps, self.every)):
            s1 = min(s0 + self.every, self.nsteps)
            # recompute the segment's states and steps once
            states, steps = [ckpt[s0]], []
            U = ckpt[s0]
            for _ in range(s0, s1):
                U, x = self._step(U)
                states.append(U)
                steps.append(x)
            for n in reversed(range(s0, s1)):
                Un, xn = states[n - s0], steps[n - s0]
                mu = self._solve(Un, lam, True)
                gU, gbr = ctx.vjp(Un, mu)
                gU2, gbr2, _ = ctx.vjp_dir(Un, mu, xn, self.eps)
                for a in (gU, gU2):
                    ctx.axpby(-1.0, a, 1.0, lam)
                for a in (gbr, gbr2):
                    ctx.axpby(-1.0, a, 1.0, gb)
        return L, gb

    def tangent(self, br: torch.Tensor, db: torch.Tensor):
        """Directional derivative dL along db by the forward tangent sweep; returns (L, dL)."""
        ctx = self.ctx
        ctx.set_inner_br(br)
        U = self.U0.clone()
        dU = torch.zeros_like(U)
        for _ in range(self.nsteps):
            Un, x = self._step(U)
            t = ctx.jvp(U, dU, dbr=db)
            t2, _ = ctx.jvp_dir(U, x, dU, dbr=db, eps=self.eps)
            ctx.axpby(1.0, t2, 1.0, t)
            dx = self._solve(U, t, False)
            ctx.axpby(-1.0, dx, 1.0, dU)
            U = Un
        return self._objective(U), self._objective(dU)

    def tangents(self, br: torch.Tensor, dbs, log=None):
        """dL along each map direction of dbs by forward tangent sweeps that
        share one forward trajectory (its solves done once); returns (L, [dL]).
        log: optional callable given a line after every step."""
        ctx = self.ctx
        ctx.set_inner_br(br)
        U = self.U0.clone()
        dUs = [torch.zeros_like(U) for _ in dbs]
        for n in range(self.nsteps):
            if log is not None:
                log(f"tangent sweeps: step {n + 1} of {self.nsteps}")
            Un, x = self._step(U)
            for dU, db in zip(dUs, dbs):
                t = ctx.jvp(U, dU, dbr=db)
                t2, _ = ctx.jvp_dir(U, x, dU, dbr=db, eps=self.eps)
                ctx.axpby(1.0, t2, 1.0, t)
                dx = self._solve(U, t, False)
                ctx.axpby(-1.0, dx, 1.0, dU)
            U = Un
        return self._objective(U), [self._objective(dU) for dU in dUs]
