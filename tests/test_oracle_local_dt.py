"""Pins of the oracle's local pseudo-time step (CPU only).

Section 2.1 marches in pseudo-time with a local time step set by a CFL
number; the reading is dt_c = CFL V_c / sum_f s_f |S_f| with s_f the Rusanov
speed max(|v_n| + c_f over both sides, c_h) of face f, so the backward-Euler
diagonal is V_c / dt_c = sum_f s_f |S_f| / CFL.  On uniform states both
sides of an interior face carry the cell state, and s_f has closed forms:
the sound speed a = sqrt(gamma p / rho) without a field, |v . n| + a with a
flow, max(a, b) for a field along the normal and sqrt(a^2 + b^2) across it
(b = |B| / sqrt(rho), the Alfven speed).  A dropped area factor, a sum over
owned faces only, or CFL multiplying instead of dividing fails these.
"""
import math

import torch

from oracle import mhd, solve
from oracle.grid import Grid

DT = torch.float64


def uniform_state(g, rho, v, B, p, gamma):
    U = torch.zeros(9, g.ncells, dtype=DT)
    v = torch.tensor(v, dtype=DT)
    B = torch.tensor(B, dtype=DT)
    U[0] = rho
    U[1:4] = (rho * v)[:, None]
    U[4:7] = B[:, None]
    U[7] = p / (gamma - 1) + 0.5 * rho * float(v @ v) + 0.5 * float(B @ B)
    return U


def interior_cells(g):
    """Cells whose face neighbours have no boundary face: their gradients
    vanish on a uniform state, so both sides of each face are uniform."""
    cells = torch.arange(g.ncells)
    _, k, _, _ = g.decode(cells)
    return cells[(k >= 2) & (k <= g.Nr - 3)]


def test_local_dt_at_rest_is_sound_speed_times_total_area():
    gam = 5.0 / 3.0
    g = Grid(4, 6, torch.linspace(1.0, 3.0, 7, dtype=DT))
    prm = mhd.Params(gamma=gam, G=0.0)
    rho, p = 1.3, 2.0
    a = math.sqrt(gam * p / rho)
    assert a > prm.c_h
    U = uniform_state(g, rho, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), p, gam)
    br = torch.zeros(g.nb, dtype=DT)
    cells = interior_cells(g)
    cfl = 7.0
    d = solve.local_dt_diag(g, U, br, prm, cfl, cells=cells)
    _, _, _, S = g.cell_geometry(cells)
    area = torch.linalg.norm(S, dim=-1).sum(-1)          # all six faces
    expect = a * area / cfl
    assert torch.allclose(d, expect, rtol=1e-13, atol=0.0)
    # the per-face speeds themselves, on every face of these cells
    s, ar = solve.face_speeds(g, U, br, prm, cells=cells)
    assert torch.allclose(s, torch.full_like(s, a), rtol=1e-14, atol=0.0)
    assert torch.allclose(ar, torch.linalg.norm(S, dim=-1), rtol=1e-14, atol=0.0)
    # dt itself: CFL times the volume over the summed speed-area product
    _, V, _, _ = g.cell_geometry(cells)
    dt = V / d
    assert torch.allclose(dt, cfl * V / (a * area), rtol=1e-13, atol=0.0)


def test_local_dt_with_flow_adds_normal_velocity_and_scales_inversely_with_cfl():
    gam = 1.4
    g = Grid(3, 6, torch.linspace(1.0, 2.5, 7, dtype=DT))
    prm = mhd.Params(gamma=gam, G=0.0)
    rho, p = 0.8, 1.5
    v = (0.3, -0.2, 0.45)
    a = math.sqrt(gam * p / rho)
    U = uniform_state(g, rho, v, (0.0, 0.0, 0.0), p, gam)
    br = torch.zeros(g.nb, dtype=DT)
    cells = interior_cells(g)
    _, _, _, S = g.cell_geometry(cells)
    vv = torch.tensor(v, dtype=DT)
    expect = ((S @ vv).abs() + a * torch.linalg.norm(S, dim=-1)).sum(-1)
    d1 = solve.local_dt_diag(g, U, br, prm, 1.0, cells=cells)
    assert torch.allclose(d1, expect, rtol=1e-13, atol=0.0)
    d4 = solve.local_dt_diag(g, U, br, prm, 4.0, cells=cells)
    assert torch.allclose(d4 * 4.0, d1, rtol=1e-15, atol=0.0)


def test_fast_speed_along_and_across_the_field_on_radial_faces():
    """Odd N: the centre column of panel 0 points along +x, so its radial
    faces have normal x-hat (to rounding) by the panel's mirror symmetry."""
    gam = 5.0 / 3.0
    g = Grid(5, 6, torch.linspace(1.0, 2.0, 7, dtype=DT))
    prm = mhd.Params(gamma=gam, G=0.0)
    rho, p = 1.0, 2.0
    a = math.sqrt(gam * p / rho)
    B0 = 3.0
    b = B0 / math.sqrt(rho)
    br = torch.zeros(g.nb, dtype=DT)
    c = int(g.encode(0, 2, 2, 2))
    cells = torch.tensor([c])
    _, _, xf, S = g.cell_geometry(cells)
    n = S[0, 1] / torch.linalg.norm(S[0, 1])
    assert float((n - torch.tensor([1.0, 0.0, 0.0], dtype=DT)).abs().max()) < 1e-15
    for B, expect in (((B0, 0.0, 0.0), max(a, b)), ((0.0, 0.0, B0), math.sqrt(a * a + b * b))):
        U = uniform_state(g, rho, (0.0, 0.0, 0.0), B, p, gam)
        s, _ = solve.face_speeds(g, U, br, prm, cells=cells)
        assert abs(float(s[0, 0]) - expect) <= 1e-12 * expect
        assert abs(float(s[0, 1]) - expect) <= 1e-12 * expect


def test_local_dt_floor_is_the_cleaning_speed():
    """A cold, field-free state at rest: every face speed is c_h."""
    gam = 1.05
    g = Grid(3, 6, torch.linspace(1.0, 2.0, 7, dtype=DT))
    prm = mhd.Params(gamma=gam, G=0.0)
    U = uniform_state(g, 1.0, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), 1e-6, gam)
    br = torch.zeros(g.nb, dtype=DT)
    cells = interior_cells(g)
    s, _ = solve.face_speeds(g, U, br, prm, cells=cells)
    assert torch.equal(s, torch.full_like(s, prm.c_h))
