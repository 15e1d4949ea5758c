"""Pins of the oracle's E-field diagnostic and E-free initial state
(Sections 2.2 and 3.1) against closed forms and invariants (CPU only)."""
import math

import pytest
import torch

from oracle import mhd
from oracle.grid import Grid
import coronal_inputs as ci

DT = torch.float64


def grid_and_frame(N=6, Nr=3):
    g = Grid(N, Nr, ci.radial_nodes(Nr))
    xc, V, _, _ = g.cell_geometry(torch.arange(g.ncells))
    r = torch.linalg.norm(xc, dim=-1)
    rc = torch.sqrt(xc[:, 0] ** 2 + xc[:, 1] ** 2)
    # the spherical frame written out from the angles (not from the oracle)
    th, ph = torch.acos(xc[:, 2] / r), torch.atan2(xc[:, 1], xc[:, 0])
    rh = torch.stack([torch.sin(th) * torch.cos(ph), torch.sin(th) * torch.sin(ph), torch.cos(th)], -1)
    thh = torch.stack([torch.cos(th) * torch.cos(ph), torch.cos(th) * torch.sin(ph), -torch.sin(th)], -1)
    phh = torch.stack([-torch.sin(ph), torch.cos(ph), torch.zeros_like(ph)], -1)
    assert (rc > 1e-6 * r).all()  # even N: no centroid on the polar axis
    return g, xc, V, r, th, rh, thh, phh


def conservative(rho, v, B, etot=50.0, psi=0.0):
    """U (9, n) from rho, velocity and field; the energy does not enter E."""
    n = rho.numel()
    return torch.cat([rho[None], (rho[:, None] * v).T, B.T, torch.full((1, n), etot, dtype=DT),
                      torch.full((1, n), psi, dtype=DT)], dim=0)


def test_radial_outflow_across_spherical_field():
    # V = V_r r-hat, B = B_r r-hat + B_t theta-hat + B_p phi-hat:
    # -V x B = V_r B_p theta-hat - V_r B_t phi-hat, no radial part
    g, xc, V, r, th, rh, thh, phh = grid_and_frame()
    gen = torch.Generator().manual_seed(11)
    n = g.ncells
    Vr, Br, Bt, Bp = (torch.rand(n, generator=gen, dtype=DT) - 0.3 for _ in range(4))
    rho = 0.5 + torch.rand(n, generator=gen, dtype=DT)
    v = Vr[:, None] * rh
    B = Br[:, None] * rh + Bt[:, None] * thh + Bp[:, None] * phh
    E, mx, rms = mhd.efield(g, conservative(rho, v, B), mhd.Params())
    assert E.shape == (3, n)
    assert torch.allclose(E[0], torch.zeros(n, dtype=DT), atol=1e-14)
    assert torch.allclose(E[1], Vr * Bp, rtol=1e-12, atol=1e-15)
    assert torch.allclose(E[2], -Vr * Bt, rtol=1e-12, atol=1e-15)
    # statistics by brute force over the cells
    mag = torch.sqrt((Vr * Bp) ** 2 + (Vr * Bt) ** 2)
    want_max = [max(abs(float(x)) for x in comp) for comp in (E[0], Vr * Bp, -Vr * Bt, mag)]
    for a, b in zip(mx.tolist(), want_max):
        assert a == pytest.approx(b, rel=1e-12, abs=1e-14)
    vtot = sum(float(x) for x in V)
    for q, comp in enumerate((Vr * Bp, -Vr * Bt, mag)):
        want = math.sqrt(sum(float(V[c]) * float(comp[c]) ** 2 for c in range(n)) / vtot)
        assert float(rms[q + 1]) == pytest.approx(want, rel=1e-12)


def test_rigid_rotation_in_axial_field():
    # V = Omega z-hat x x, B = B0 z-hat: -V x B = -Omega B0 (x - z z-hat), so
    # E_r = -Omega B0 r sin^2(theta), E_theta = -Omega B0 r sin cos, E_phi = 0
    g, xc, V, r, th, rh, thh, phh = grid_and_frame(N=4, Nr=2)
    Om, B0 = 0.7, -1.3
    n = g.ncells
    v = Om * torch.stack([-xc[:, 1], xc[:, 0], torch.zeros(n, dtype=DT)], -1)
    B = torch.tensor([0.0, 0.0, B0], dtype=DT).expand(n, 3)
    E, mx, rms = mhd.efield(g, conservative(torch.ones(n, dtype=DT), v, B), mhd.Params())
    s, c = torch.sin(th), torch.cos(th)
    assert torch.allclose(E[0], -Om * B0 * r * s * s, rtol=1e-12, atol=1e-13)
    assert torch.allclose(E[1], -Om * B0 * r * s * c, rtol=1e-12, atol=1e-13)
    assert torch.allclose(E[2], torch.zeros(n, dtype=DT), atol=1e-13)
    assert float(mx[3]) == pytest.approx(float((abs(Om * B0) * r * s).max()), rel=1e-12)


def test_rms_is_volume_weighted():
    g, xc, V, r, th, rh, thh, phh = grid_and_frame(N=4, Nr=2)
    n = g.ncells
    v = torch.zeros(n, 3, dtype=DT)
    B = torch.zeros(n, 3, dtype=DT)
    c0 = 7
    v[c0] = rh[c0] * 2.0
    B[c0] = phh[c0] * 3.0  # E = 6 theta-hat in cell c0 only
    E, mx, rms = mhd.efield(g, conservative(torch.ones(n, dtype=DT), v, B), mhd.Params())
    w = math.sqrt(float(V[c0]) / float(V.sum()))
    assert float(mx[1]) == pytest.approx(6.0, rel=1e-13) and float(mx[3]) == pytest.approx(6.0, rel=1e-13)
    assert float(rms[1]) == pytest.approx(6.0 * w, rel=1e-12)
    assert float(rms[3]) == pytest.approx(6.0 * w, rel=1e-12)
    assert float(mx[0]) < 1e-14 and float(mx[2]) < 1e-14


def test_efield_orthogonal_to_velocity_and_field():
    inst = ci.make_instance(5, 3, seed=5)
    g = Grid(inst.N, inst.Nr, inst.r_nodes)
    prm = mhd.Params()
    U = torch.from_numpy(inst.U)
    E, _, _ = mhd.efield(g, U, prm)
    P = mhd.cons_to_prim(U.T, prm.gamma)
    rh, thh, phh = mhd.spherical_basis(g.cell_geometry(torch.arange(g.ncells))[0])
    Ec = E[0][:, None] * rh + E[1][:, None] * thh + E[2][:, None] * phh
    scale = torch.linalg.norm(P[:, 1:4], dim=-1) * torch.linalg.norm(P[:, 4:7], dim=-1)
    assert ((Ec * P[:, 1:4]).sum(-1).abs() <= 1e-12 * scale * torch.linalg.norm(P[:, 1:4], dim=-1)).all()
    assert ((Ec * P[:, 4:7]).sum(-1).abs() <= 1e-12 * scale * torch.linalg.norm(P[:, 4:7], dim=-1)).all()
    # |E| = |V| |B| sin(angle)
    cosang = (P[:, 1:4] * P[:, 4:7]).sum(-1) / scale
    mag = torch.linalg.norm(E, dim=0)
    assert torch.allclose(mag, scale * torch.sqrt(1 - cosang ** 2), rtol=1e-8, atol=1e-14)


def test_efree_state_removes_the_electric_field():
    inst = ci.make_instance(5, 3, seed=8)
    g = Grid(inst.N, inst.Nr, inst.r_nodes)
    prm = mhd.Params()
    U = torch.from_numpy(inst.U).clone()
    # cell 3 without field: rho = 1, V = (0.2, 0, 0), B = 0
    U[:7, 3] = torch.tensor([1.0, 0.2, 0.0, 0.0, 0.0, 0.0, 0.0], dtype=DT)
    U0 = mhd.efree_state(U, prm)
    P = mhd.cons_to_prim(U.T, prm.gamma)
    P0 = mhd.cons_to_prim(U0.T, prm.gamma)
    # density, field, pressure and psi kept
    for q in (0, 4, 5, 6, 7, 8):
        assert torch.allclose(P0[:, q], P[:, q], rtol=1e-12, atol=1e-13 * float(P[:, q].abs().max()))
    v, v0, B = P[:, 1:4], P0[:, 1:4], P[:, 4:7]
    # V0 x B = 0 and V0 . B = V . B
    assert torch.linalg.cross(v0, B).abs().max() <= 1e-13 * float((v.norm(dim=-1) * B.norm(dim=-1)).max())
    assert torch.allclose((v0 * B).sum(-1), (v * B).sum(-1), rtol=1e-12, atol=1e-15)
    # the cell with no field is left alone
    assert torch.equal(v0[3], v[3])
    _, mx, _ = mhd.efield(g, U0, prm)
    _, mx_before, _ = mhd.efield(g, U, prm)
    assert float(mx[3]) <= 1e-12 * float(mx_before[3])
    # idempotent, and a state already free of E is unchanged
    U00 = mhd.efree_state(U0, prm)
    assert torch.allclose(U00, U0, rtol=1e-13, atol=1e-15)


def test_efree_state_of_the_paper_dipole_keeps_parallel_outflow():
    # radial wind across a dipole: V0 = V_r (B_r / |B|^2) B, so V0_r = V_r B_r^2/|B|^2
    # and V0_theta = V_r B_r B_theta / |B|^2 (the form the low-E law imposes at the boundary)
    g, xc, V, r, th, rh, thh, phh = grid_and_frame(N=4, Nr=2)
    n = g.ncells
    Vr = torch.full((n,), 0.05, dtype=DT)
    Bd = torch.from_numpy(ci.dipole_field(xc.numpy()))
    U = conservative(torch.ones(n, dtype=DT), Vr[:, None] * rh, Bd)
    P0 = mhd.cons_to_prim(mhd.efree_state(U, mhd.Params()).T, mhd.Params().gamma)
    Br = (Bd * rh).sum(-1)
    Bt = (Bd * thh).sum(-1)
    B2 = (Bd * Bd).sum(-1)
    assert torch.allclose((P0[:, 1:4] * rh).sum(-1), Vr * Br * Br / B2, rtol=1e-12, atol=1e-16)
    assert torch.allclose((P0[:, 1:4] * thh).sum(-1), Vr * Br * Bt / B2, rtol=1e-12, atol=1e-16)
    assert torch.allclose((P0[:, 1:4] * phh).sum(-1), torch.zeros(n, dtype=DT), atol=1e-16)


def test_efree_energy_is_independent_of_gamma():
    # p is kept while V changes: the new energy is E - rho (|V|^2 - |V0|^2) / 2
    inst = ci.make_instance(4, 3, seed=9)
    U = torch.from_numpy(inst.U)
    a = mhd.efree_state(U, mhd.Params(gamma=5.0 / 3.0))
    b = mhd.efree_state(U, mhd.Params(gamma=1.05))
    assert torch.allclose(a, b, rtol=1e-13, atol=1e-15)
    P = mhd.cons_to_prim(U.T, 1.05)
    P0 = mhd.cons_to_prim(a.T, 1.05)
    want = U[7] - 0.5 * P[:, 0] * ((P[:, 1:4] ** 2).sum(-1) - (P0[:, 1:4] ** 2).sum(-1))
    assert torch.allclose(a[7], want, rtol=1e-12, atol=1e-15)
