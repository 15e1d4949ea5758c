"""Pins of the oracle's assembled residual: invariants, exact steady states,
symmetry and convergence (CPU only)."""
import math

import numpy as np
import pytest
import torch

import coronal_inputs as ci
from helpers import polytropic_parker
from oracle import constants as K
from oracle import mhd
from oracle.grid import Grid

DT = torch.float64


def grid_and_geom(N, Nr, radial="log"):
    g = Grid(N, Nr, ci.radial_nodes(Nr, radial))
    cells = torch.arange(g.ncells)
    xc, V, xf, S = g.cell_geometry(cells)
    return g, cells, xc, V, xf, S


def cons(P, gamma):
    return mhd.prim_to_cons(P, gamma).T.contiguous()


def test_free_stream_preservation():
    """A uniform state has zero interior residual without gravity (outer
    Table 2 case 1 keeps the outer ghosts uniform)."""
    g, cells, xc, V, xf, S = grid_and_geom(6, 8)
    P = torch.tensor([0.7, 0.3, -0.2, 0.1, 0.4, 0.25, -0.5, 0.9, 0.0], dtype=DT).expand(g.ncells, 9)
    U = cons(P, 1.05)
    br = torch.zeros(g.nb, dtype=DT)
    for lim in (0, 1):
        prm = mhd.Params.table2(1, G=0.0, limiter=lim)
        R = mhd.residual(g, U, br, prm)
        _, k, _, _ = g.decode(cells)
        inner = (k >= 2) & (k <= g.Nr - 3)
        Fmax = mhd.physical_flux(P[:1], torch.tensor([[1.0, 0, 0]], dtype=DT), 1.05, 1.0).abs().max()
        scale = float(Fmax * S.norm(dim=-1).max())
        assert float(R[:, inner].abs().max()) < 1e-13 * scale


@pytest.mark.parametrize("inner_mode", [0, 1])
def test_discrete_conservation_telescopes_to_boundary_fluxes(inner_mode):
    """Without gravity, sum over all cells of R equals the sum of the
    boundary-face fluxes: interior fluxes cancel pairwise (low-E and large-E
    inner boundaries)."""
    inst = ci.make_instance(4, 6, "log", lmax=0, seed=5)
    g = Grid(inst.N, inst.Nr, inst.r_nodes)
    U, br = torch.tensor(inst.U), torch.tensor(inst.br)
    prm = mhd.Params(G=0.0, inner_mode=inner_mode, inner_btheta=torch.tensor(ci.btheta_map(inst.N)))
    R = mhd.residual(g, U, br, prm)
    st = mhd._Stencil(g, torch.arange(g.ncells))
    fs = mhd.face_states(g, U, br, prm, torch.arange(g.ncells), st)
    F, _ = mhd.rusanov(fs["PL"], fs["PR"], fs["S"], prm)
    bnd = fs["other"] >= g.ncells
    Fb = (F * bnd[..., None]).sum((0, 1))
    total = R.sum(1)
    scale = F.abs().sum((0, 1))
    assert float(((total - Fb).abs() / scale).max()) < 1e-13


def test_dipole_divergence_converges_second_order():
    """v = 0, psi = 0, uniform rho and p: the psi residual / c_h^2 is the
    discrete divergence of the dipole field; it vanishes at O(h^2)."""
    errs = []
    for N in (8, 16, 32):
        g, cells, xc, V, xf, S = grid_and_geom(N, 2 * N)
        _, k, _, _ = g.decode(cells)
        inner = (k >= 2) & (k <= g.Nr - 3)
        P = torch.zeros(g.ncells, 9, dtype=DT)
        P[:, 0] = 1.0
        P[:, 7] = 1.0
        r = xc.norm(dim=-1, keepdim=True)
        rh = xc / r
        P[:, 4:7] = (3 * rh[:, 2:3] * rh - torch.tensor([0.0, 0, 1], dtype=DT)) / r ** 3
        R = mhd.residual(g, cons(P, 1.05), torch.zeros(g.nb, dtype=DT), mhd.Params(G=0.0, limiter=0, c_h=0.5))
        div = (R[8] / 0.25) / V
        rel = (div.abs() * V ** (1 / 3) / P[:, 4:7].norm(dim=-1))[inner]
        errs.append(float(rel.max()))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def test_hydrostatic_monopole_is_steady_to_truncation():
    """Polytropic hydrostatic atmosphere + radial monopole field (force-free)
    is an exact steady state; its interior residual falls at ~O(h^2) in the
    mean relative to the pressure force on a face."""
    means = []
    gam, Kp = 5.0 / 3.0, 1.0
    for N in (8, 16):
        g, cells, xc, V, xf, S = grid_and_geom(N, 2 * N)
        _, k, _, _ = g.decode(cells)
        inner = (k >= 2) & (k <= g.Nr - 3)
        r = xc.norm(dim=-1)
        C = gam / (gam - 1) * Kp - K.G
        rho = ((K.G / r + C) * (gam - 1) / (gam * Kp)) ** (1 / (gam - 1))
        P = torch.zeros(g.ncells, 9, dtype=DT)
        P[:, 0] = rho
        P[:, 7] = Kp * rho ** gam
        P[:, 4:7] = 0.5 * xc / r[:, None] ** 3
        R = mhd.residual(g, cons(P, gam), torch.zeros(g.nb, dtype=DT), mhd.Params(gamma=gam))
        sc = P[:, 7] * S.norm(dim=-1).max(1).values
        means.append([float((R[0].abs() / sc)[inner].mean()), float((R[1:4].norm(dim=0) / sc)[inner].mean()),
                      float((R[7].abs() / sc)[inner].mean())])
    for a, b in zip(means[0], means[1]):
        assert a / b > 3.5


def test_parker_wind_monopole_is_steady_to_truncation():
    """Transonic polytropic Parker wind with a radial monopole field (v || B,
    so E = -v x B = 0) is an exact steady state of the equations."""
    maxs = []
    gam = 1.05
    for N in (8, 16):
        g, cells, xc, V, xf, S = grid_and_geom(N, 2 * N)
        _, k, _, _ = g.decode(cells)
        inner = (k >= 2) & (k <= g.Nr - 3)
        r = xc.norm(dim=-1)
        rh = xc / r[:, None]
        v, rho, p = (torch.tensor(a) for a in polytropic_parker(r.numpy(), gam, K.G, 3.0, 0.05))
        P = torch.zeros(g.ncells, 9, dtype=DT)
        P[:, 0] = rho
        P[:, 1:4] = v[:, None] * rh
        P[:, 7] = p
        P[:, 4:7] = 0.5 * rh / r[:, None] ** 2
        R = mhd.residual(g, cons(P, gam), torch.zeros(g.nb, dtype=DT), mhd.Params(gamma=gam))
        sc = (p + rho * v * v) * S.norm(dim=-1).max(1).values
        maxs.append([float((R[a].abs() / sc)[inner].max()) for a in (0, 7)] +
                    [float((R[1:4].norm(dim=0) / sc)[inner].max())])
    for a, b in zip(maxs[0], maxs[1]):
        assert a / b > 3.0


def test_residual_commutes_with_rotation_about_z():
    """R(rot U) = rot R(U) for a rotated state and map (P0->P1->P2->P3)."""
    inst = ci.make_instance(4, 5, "log", lmax=3, seed=9)
    g = Grid(inst.N, inst.Nr, inst.r_nodes)
    N = g.N
    U, br = torch.tensor(inst.U), torch.tensor(inst.br)
    rot = torch.tensor([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]], dtype=DT)
    cells = torch.arange(g.ncells)
    p, k, j, i = g.decode(cells)
    p2 = torch.where(p < 4, (p + 1) % 4, p)
    i2 = torch.where(p == 4, N - 1 - j, torch.where(p == 5, j, i))
    j2 = torch.where(p == 4, i, torch.where(p == 5, N - 1 - i, j))
    img = g.encode(p2, k, j2, i2)

    def rotate(A):
        B = A.clone()
        B[1:4] = rot @ A[1:4]
        B[4:7] = rot @ A[4:7]
        out = torch.empty_like(A)
        out[:, img] = B
        return out

    col = torch.arange(g.nb)
    cp, cj, ci_ = col // (N * N), (col // N) % N, col % N
    cp2 = torch.where(cp < 4, (cp + 1) % 4, cp)
    ci2 = torch.where(cp == 4, N - 1 - cj, torch.where(cp == 5, cj, ci_))
    cj2 = torch.where(cp == 4, ci_, torch.where(cp == 5, N - 1 - ci_, cj))
    br2 = torch.empty_like(br)
    br2[(cp2 * N + cj2) * N + ci2] = br
    prm = mhd.Params()
    R = mhd.residual(g, U, br, prm)
    R2 = mhd.residual(g, rotate(U), br2, prm)
    err = (R2 - rotate(R)).abs().amax(1) / R.abs().amax(1)
    assert float(err.max()) < 1e-10


def test_subset_evaluation_equals_full_grid():
    inst = ci.workload("tiny")
    g = Grid(inst.N, inst.Nr, inst.r_nodes)
    U, br = torch.tensor(inst.U), torch.tensor(inst.br)
    R = mhd.residual(g, U, br, mhd.Params())
    sub = torch.tensor([0, 7, 63, 64, 1000, 1023, 2048, 4095, 5000, 6143])
    Rs = mhd.residual(g, U, br, mhd.Params(), cells=sub)
    assert torch.equal(Rs, R[:, sub])


def test_outer_law_difference_scales_with_ghost_distance():
    """On the extended grid with a thin last layer (Section 4.4), the outer
    ghost lies edge/2 beyond the boundary, so two Table 2 laws (cases 1 and
    9, the most different) give ghosts that differ to first order in edge:
    the residual difference in the last layer halves with edge, and no cell
    beyond the stencil's reach of the boundary sees the law at all."""
    N, Nr = 4, 6
    d_last = []
    for edge in (0.02, 0.01, 0.005):
        r = ci.radial_nodes(Nr, "bcind", edge=edge)
        U = torch.from_numpy(ci.to_conservative(ci.primitive_state(N, Nr, r, 5)))
        br = torch.from_numpy(ci.br_map(N, 3, 5))
        g = Grid(N, Nr, r)
        d = (mhd.residual(g, U, br, mhd.Params.table2(1)) -
             mhd.residual(g, U, br, mhd.Params.table2(9))).abs().reshape(9, 6, Nr, N, N)
        assert float(d[:, :, :Nr - 2].max()) == 0.0
        d_last.append(float(d[:, :, Nr - 1].max()))
    assert d_last[0] / d_last[1] == pytest.approx(2.0, rel=0.05)
    assert d_last[1] / d_last[2] == pytest.approx(2.0, rel=0.05)
