"""Small helpers shared by the tests (no residual arithmetic)."""
import math

import numpy as np
import torch


def rel_err_per_var(a, b):
    """max_c |a - b| / max_c |b| per variable (rows)."""
    a = torch.as_tensor(a, dtype=torch.float64)
    b = torch.as_tensor(b, dtype=torch.float64)
    num = (a - b).abs().amax(dim=-1)
    den = b.abs().amax(dim=-1).clamp_min(1e-300)
    return num / den


def polytropic_parker(r, gamma, G, rc, rho_c):
    """Transonic polytropic wind through the critical point (rc, rho_c):
    Bernoulli 1/2 v^2 + gamma/(gamma-1) K rho^(gamma-1) - G/r = const and
    rho v r^2 = const, solved by bisection on each branch."""
    vc2 = G / (2 * rc)
    Kp = vc2 / (gamma * rho_c ** (gamma - 1))
    Mdot = rho_c * math.sqrt(vc2) * rc ** 2
    EB = 0.5 * vc2 + vc2 / (gamma - 1) - G / rc
    r = np.asarray(r, dtype=np.float64)
    vs = (gamma * Kp * (Mdot / r ** 2) ** (gamma - 1)) ** (1 / (gamma + 1))
    sub = r < rc
    lo = np.where(sub, 1e-12, vs)
    hi = np.where(sub, vs, 1e3)
    for _ in range(300):
        mid = 0.5 * (lo + hi)
        fm = 0.5 * mid * mid + gamma / (gamma - 1) * Kp * (Mdot / (mid * r * r)) ** (gamma - 1) - G / r - EB
        up = np.where(sub, fm > 0, fm < 0)
        lo = np.where(up, mid, lo)
        hi = np.where(up, hi, mid)
    v = 0.5 * (lo + hi)
    rho = Mdot / (v * r * r)
    return v, rho, Kp * rho ** gamma


def perturbed_parker(N=4, Nr=6, gam=1.05, amp=1e-3, seed=1):
    """Transonic polytropic wind with a radial monopole field (an exact steady
    state of the equations) at the cell centroids, perturbed by uniform noise
    of relative size amp: (oracle grid, U (9, ncells), inner B_r map)."""
    import coronal_inputs as ci
    from oracle import constants as K
    from oracle.grid import Grid
    g = Grid(N, Nr, ci.radial_nodes(Nr))
    xc, _, _, _ = g.cell_geometry(torch.arange(g.ncells))
    r = xc.norm(dim=-1)
    rh = xc / r[:, None]
    v, rho, p = (torch.tensor(a) for a in polytropic_parker(r.numpy(), gam, K.G, 3.0, 0.05))
    P = torch.zeros(g.ncells, 9, dtype=torch.float64)
    P[:, 0], P[:, 1:4], P[:, 7] = rho, v[:, None] * rh, p
    P[:, 4:7] = 0.5 * rh / r[:, None] ** 2
    gen = torch.Generator().manual_seed(seed)
    P[:, :8] *= 1 + amp * (2 * torch.rand(g.ncells, 8, generator=gen, dtype=torch.float64) - 1)
    U = torch.empty(9, g.ncells, dtype=torch.float64)
    U[0] = P[:, 0]
    U[1:4] = (P[:, 0:1] * P[:, 1:4]).T
    U[4:7] = P[:, 4:7].T
    U[7] = P[:, 7] / (gam - 1) + 0.5 * P[:, 0] * (P[:, 1:4] ** 2).sum(1) + 0.5 * (P[:, 4:7] ** 2).sum(1)
    U[8] = 0.0
    return g, U, torch.full((g.nb,), 0.5, dtype=torch.float64)
