"""Pins of the oracle's pointwise physics against what the paper and the
mathematics fix (CPU only)."""
import math

import numpy as np
import pytest
import torch

from conftest import read_golden
from oracle import constants as K
from oracle import mhd
import coronal_inputs as ci

DT = torch.float64


def test_constants_from_printed_reference_values():
    gold = read_golden("paper_values.txt")
    assert K.RHO_REF == gold["rho_ref_kg_m3"] and K.B_REF == gold["B_ref_T"]
    assert K.VR_STAR_SI == gold["vr_star_m_s"] and K.C_H == gold["cleaning_constant"]
    vref = gold["B_ref_T"] / math.sqrt(4e-7 * math.pi * gold["rho_ref_kg_m3"])
    assert abs(vref - 4.80241e5) / 4.80241e5 < 2e-6
    # Eq. 22: V_r* = 1935.07 / (B_ref / sqrt(mu0 rho_ref))
    assert abs(K.VR_STAR - 4.029370e-3) < 5e-10
    assert abs(mhd.Params().outer_exp[0] - gold["outer_density_exponent"]) == 0


def test_table2_presets_match_paper_table():
    import os
    rows = []
    here = os.path.dirname(__file__)
    for line in open(os.path.join(here, "golden", "table2_outer_bc.txt")):
        line = line.split("#", 1)[0].split()
        if line:
            rows.append(line)
    assert len(rows) == 9
    for r in rows:
        case = int(r[0])
        prm = mhd.Params.table2(case)
        rho, br, bt, bp, vr, vt, vp, p, psi = r[1:]
        e = prm.outer_exp
        assert (e[0], e[1], e[2], e[3], e[5], e[6], e[7]) == tuple(
            float(x) for x in (rho, br, bt, bp, vt, vp, p))
        assert prm.outer_vr_mass == (vr == "mass")
        if vr != "mass":
            assert e[4] == float(vr)
        assert prm.outer_psi_zero == (psi == "B0")


def random_prims(n, seed=0):
    g = torch.Generator().manual_seed(seed)
    P = torch.randn(n, 9, generator=g, dtype=DT)
    P[:, 0] = 0.5 + torch.rand(n, generator=g, dtype=DT)
    P[:, 7] = 0.2 + torch.rand(n, generator=g, dtype=DT)
    return P


def textbook_speeds(P, n, gamma, c_h):
    rho, v, B, p = P[0], P[1:4], P[4:7], P[7]
    vn = float(v @ n)
    a2 = gamma * float(p) / float(rho)
    b2 = float(B @ B) / float(rho)
    ca2 = float(B @ n) ** 2 / float(rho)
    root = math.sqrt((a2 + b2) ** 2 - 4 * a2 * ca2)
    cf = math.sqrt(0.5 * (a2 + b2 + root))
    cs = math.sqrt(max(0.0, 0.5 * (a2 + b2 - root)))
    ca = math.sqrt(ca2)
    return sorted([vn - cf, vn - ca, vn - cs, vn, vn + cs, vn + ca, vn + cf, -c_h, c_h])


@pytest.mark.parametrize("seed", range(4))
def test_flux_jacobian_eigenvalues_are_mhd_glm_wave_speeds(seed):
    """The eigenvalues of d(F.n)/dU are the ideal-MHD fast, Alfven, slow and
    entropy speeds v_n +- c and the cleaning speeds +- c_h; the Rusanov speed
    is the largest |eigenvalue|.  A dropped or mis-signed flux term moves them."""
    gamma, c_h = 5.0 / 3.0, 0.7
    P = random_prims(1, seed)[0]
    g = torch.Generator().manual_seed(100 + seed)
    n = torch.randn(3, generator=g, dtype=DT)
    n = n / n.norm()
    U = mhd.prim_to_cons(P, gamma)

    def f(Uc):
        return mhd.physical_flux(mhd.cons_to_prim(Uc, gamma), n, gamma, c_h)

    J = torch.autograd.functional.jacobian(f, U)
    ev = np.sort(np.linalg.eigvals(J.numpy()).real)
    ref = np.array(textbook_speeds(P, n, gamma, c_h))
    assert np.allclose(ev, ref, atol=1e-9, rtol=1e-9)
    lam = float(torch.abs(P[1:4] @ n) + mhd.fast_speed(P, n, gamma))
    assert abs(lam - max(abs(ev[0]), abs(ev[-1]))) < 1e-9


def test_rusanov_consistency_antisymmetry_and_euler_limit():
    prm = mhd.Params(gamma=1.4, c_h=0.8)
    P = random_prims(16, 7)
    S = torch.randn(16, 3, dtype=DT, generator=torch.Generator().manual_seed(3))
    F, _ = mhd.rusanov(P, P, S, prm)
    Fp = mhd.physical_flux(P, S / S.norm(dim=-1, keepdim=True), prm.gamma, prm.c_h) * S.norm(dim=-1, keepdim=True)
    assert torch.allclose(F, Fp, rtol=1e-15, atol=1e-15)
    PR = random_prims(16, 8)
    F1, _ = mhd.rusanov(P, PR, S, prm)
    F2, _ = mhd.rusanov(PR, P, -S, prm)
    assert torch.equal(F1, -F2)
    # B = 0, psi = 0: the hydrodynamic (Euler) flux of a textbook
    Pe = P.clone()
    Pe[:, 4:9] = 0
    n = S / S.norm(dim=-1, keepdim=True)
    Fe = mhd.physical_flux(Pe, n, prm.gamma, prm.c_h)
    rho, v, p = Pe[:, 0], Pe[:, 1:4], Pe[:, 7]
    un = (v * n).sum(-1)
    E = p / (prm.gamma - 1) + 0.5 * rho * (v * v).sum(-1)
    ref = torch.cat([(rho * un)[:, None], rho[:, None] * v * un[:, None] + p[:, None] * n,
                     torch.zeros(16, 3, dtype=DT), ((E + p) * un)[:, None], torch.zeros(16, 1, dtype=DT)], 1)
    assert torch.allclose(Fe, ref, rtol=1e-14, atol=1e-14)


def test_flux_rotation_equivariance():
    prm = mhd.Params(gamma=1.4, c_h=0.8)
    P = random_prims(8, 9)
    n = torch.randn(8, 3, dtype=DT, generator=torch.Generator().manual_seed(4))
    n = n / n.norm(dim=-1, keepdim=True)
    Q, _ = torch.linalg.qr(torch.randn(3, 3, dtype=DT, generator=torch.Generator().manual_seed(5)))
    Pr = P.clone()
    for a, b in ((1, 4), (4, 7)):
        Pr[:, a:b] = P[:, a:b] @ Q.T
    F = mhd.physical_flux(P, n, prm.gamma, prm.c_h)
    Fr = mhd.physical_flux(Pr, n @ Q.T, prm.gamma, prm.c_h)
    for a, b in ((1, 4), (4, 7)):
        F[:, a:b] = F[:, a:b] @ Q.T
    assert torch.allclose(F, Fr, rtol=1e-13, atol=1e-13)


def test_prim_cons_roundtrip():
    P = random_prims(32, 11)
    back = mhd.cons_to_prim(mhd.prim_to_cons(P, 1.05), 1.05)
    assert torch.allclose(back, P, rtol=1e-10, atol=1e-12)


def test_spherical_basis_reproduces_eqs_20_21():
    x = torch.randn(64, 3, dtype=DT, generator=torch.Generator().manual_seed(1))
    B = torch.randn(64, 3, dtype=DT, generator=torch.Generator().manual_seed(2))
    rh, th, ph = mhd.spherical_basis(x)
    X, Y, Z = x.unbind(-1)
    r = x.norm(dim=-1)
    rho = torch.sqrt(X * X + Y * Y)
    Br = X / r * B[:, 0] + Y / r * B[:, 1] + Z / r * B[:, 2]                    # Eq. 20
    Bth = X * Z / (rho * r) * B[:, 0] + Y * Z / (rho * r) * B[:, 1] - rho / r * B[:, 2]   # Eq. 21
    assert torch.allclose((B * rh).sum(-1), Br, rtol=1e-13, atol=1e-13)
    assert torch.allclose((B * th).sum(-1), Bth, rtol=1e-13, atol=1e-13)
    assert torch.allclose(torch.linalg.cross(rh, th), ph, atol=1e-14)


def test_spherical_basis_on_the_polar_axis_is_the_phi0_limit():
    """Reading: on the axis theta-hat, phi-hat are the limits along phi = 0."""
    eps = 1e-9
    for z in (3.0, -2.0):
        x = torch.tensor([[0.0, 0.0, z], [eps, 0.0, z]], dtype=DT)
        # rounding-level offsets from the axis count as on it
        xa = torch.tensor([[3e-17, -2e-17, z], [0.0, 0.0, z]], dtype=DT)
        ra, ta, pa = mhd.spherical_basis(xa)
        assert torch.equal(ta[0], ta[1]) and torch.equal(pa[0], pa[1])
        rh, th, ph = mhd.spherical_basis(x)
        assert torch.allclose(th[0], th[1], atol=1e-8) and torch.allclose(ph[0], ph[1], atol=1e-8)
        assert torch.allclose(torch.linalg.cross(rh[0], th[0]), ph[0], atol=1e-15)


def boundary_face_sample(n=50, seed=0, radius=1.0):
    g = torch.Generator().manual_seed(seed)
    xf = torch.randn(n, 3, dtype=DT, generator=g)
    xf = radius * xf / xf.norm(dim=-1, keepdim=True)
    return xf, g


def test_inner_low_e_ghost_eq25_and_dirichlet_laws():
    prm = mhd.Params()
    xf, g = boundary_face_sample(80, 3)
    PI = random_prims(80, 12)
    br = torch.randn(80, dtype=DT, generator=g)
    PG = mhd.inner_ghost(PI, xf, br, prm)
    Vb = 0.5 * (PG[:, 1:4] + PI[:, 1:4])
    Bb = 0.5 * (PG[:, 4:7] + PI[:, 4:7])
    rh = xf / xf.norm(dim=-1, keepdim=True)
    cross = torch.linalg.cross(Vb, Bb).norm(dim=-1)
    # Eq. 25 to rounding (the face average carries the rounding of 2 V_b - V_I)
    scale = (Vb.norm(dim=-1) + PI[:, 1:4].norm(dim=-1)) * Bb.norm(dim=-1)
    assert float((cross / scale).max()) < 1e-15
    assert torch.allclose((Bb * rh).sum(-1), br, rtol=1e-14, atol=1e-15)         # B_r = map
    t_I = PI[:, 4:7] - (PI[:, 4:7] * rh).sum(-1, keepdim=True) * rh
    t_G = PG[:, 4:7] - (PG[:, 4:7] * rh).sum(-1, keepdim=True) * rh
    assert torch.allclose(t_I, t_G, rtol=1e-13, atol=1e-14)                      # Neumann
    vr = (Vb * rh).sum(-1)
    assert bool((vr >= 0).all())
    err = (vr - prm.vr_star * br ** 2 / (Bb * Bb).sum(-1)).abs()
    assert bool((err <= 1e-13 * vr.abs() + 1e-15 * PI[:, 1:4].norm(dim=-1)).all())
    assert torch.allclose(0.5 * (PG[:, 0] + PI[:, 0]), torch.full((80,), prm.rho_b, dtype=DT), rtol=1e-15)
    assert torch.allclose(0.5 * (PG[:, 7] + PI[:, 7]), torch.full((80,), prm.rho_b * prm.T_b, dtype=DT), rtol=1e-14)
    assert torch.equal(PG[:, 8], -PI[:, 8])


def test_inner_large_e_ghost_removes_poloidal_flux():
    """Large-E law (Eqs. 20-24), checked through properties of the face
    average: B_r and B_theta take the imposed values, B_phi is Neumann, the
    velocity lies along the poloidal field (B_r, B_theta) with no azimuthal
    part and radial part V_r* B_r^2/B_pol^2, so its electric field V x B_b is
    -V_par B_phi (B_r theta-hat - B_theta r-hat) and vanishes only without
    B_phi; rho, p and psi as the low-E law."""
    prm = mhd.Params()
    xf, g = boundary_face_sample(80, 5)
    PI = random_prims(80, 14)
    br = torch.randn(80, dtype=DT, generator=g)
    bth = torch.randn(80, dtype=DT, generator=g)
    PG = mhd.inner_ghost_large_e(PI, xf, br, bth, prm)
    Vb = 0.5 * (PG[:, 1:4] + PI[:, 1:4])
    Bb = 0.5 * (PG[:, 4:7] + PI[:, 4:7])
    rh, th, ph = mhd.spherical_basis(xf)
    comp = lambda a, b: (a * b).sum(-1)
    tol = lambda x: 1e-13 * (x.abs() + PI[:, 1:7].norm(dim=-1))
    assert bool(((comp(Bb, rh) - br).abs() <= tol(br)).all())
    assert bool(((comp(Bb, th) - bth).abs() <= tol(bth)).all())
    assert bool(((comp(PG[:, 4:7], ph) - comp(PI[:, 4:7], ph)).abs() <= tol(comp(PI[:, 4:7], ph))).all())
    vphi = comp(Vb, ph)
    assert float(vphi.abs().max()) <= 1e-13 * float(PI[:, 1:4].abs().max())
    # along the poloidal field: V_r B_theta - V_theta B_r = 0
    vr, vt = comp(Vb, rh), comp(Vb, th)
    assert bool(((vr * bth - vt * br).abs() <= 1e-13 * (vr.abs() + vt.abs() + PI[:, 1:4].norm(dim=-1))
                 * (br.abs() + bth.abs())).all())
    pol2 = br ** 2 + bth ** 2
    assert bool(((vr - prm.vr_star * br ** 2 / pol2).abs() <= tol(vr)).all())
    assert bool((vr >= -1e-15).all())
    # the boundary electric field comes from B_phi alone
    E = torch.linalg.cross(Vb, Bb)
    vpar = prm.vr_star * br / pol2
    E_expect = -(vpar * comp(Bb, ph))[:, None] * (br[:, None] * th - bth[:, None] * rh)
    # (the face average carries the rounding of 2 V_b - V_I, relative to |V_I|)
    scale = (Vb.norm(dim=-1) + PI[:, 1:4].norm(dim=-1)) * Bb.norm(dim=-1)
    assert bool(((E - E_expect).norm(dim=-1) <= 1e-14 * scale).all())
    assert torch.allclose(0.5 * (PG[:, 0] + PI[:, 0]), torch.full((80,), prm.rho_b, dtype=DT), rtol=1e-15)
    assert torch.allclose(0.5 * (PG[:, 7] + PI[:, 7]), torch.full((80,), prm.rho_b * prm.T_b, dtype=DT), rtol=1e-14)
    assert torch.equal(PG[:, 8], -PI[:, 8])


def test_large_e_equals_low_e_without_azimuthal_field():
    """With no interior B_phi and the imposed B_theta equal to the interior
    one, the boundary field is poloidal, so the large-E velocity (along the
    poloidal field) and the low-E velocity (along B_b) coincide."""
    prm = mhd.Params()
    xf, g = boundary_face_sample(60, 8)
    PI = random_prims(60, 15)
    rh, th, ph = mhd.spherical_basis(xf)
    B = PI[:, 4:7]
    PI[:, 4:7] = B - (B * ph).sum(-1, keepdim=True) * ph
    br = torch.randn(60, dtype=DT, generator=g)
    bth = (PI[:, 4:7] * th).sum(-1)
    a = mhd.inner_ghost_large_e(PI, xf, br, bth, prm)
    b = mhd.inner_ghost(PI, xf, br, prm)
    assert float(((a - b).abs() / (b.abs() + 1e-12)).max()) < 1e-12


def test_btheta_map_is_the_dipole_polar_component():
    """The B_theta input of the large-E boundary for the dipole: B_eq sin(theta)
    at r = 1 (standard dipole, B_r = 2 B_eq cos(theta))."""
    for N in (4, 5):
        d = ci.nominal_directions(N).reshape(-1, 3)
        th = np.arccos(np.clip(d[:, 2], -1, 1))
        assert np.allclose(ci.btheta_map(N), ci.GAUSS * np.sin(th), rtol=1e-12, atol=1e-15)
        assert np.allclose(ci.br_map(N, 0, 0), 2 * ci.GAUSS * np.cos(th), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("case", range(1, 10))
def test_outer_ghost_table2_laws(case):
    """Each Table 2 law in its 'quantity * r^e = cst' form (Eqs. 26-31)."""
    prm = mhd.Params.table2(case)
    xf, g = boundary_face_sample(60, case, radius=21.5)
    rh = xf / xf.norm(dim=-1, keepdim=True)
    xI = xf * (1 - 0.02 * torch.rand(60, 1, dtype=DT, generator=g)) + 0.01 * torch.randn(60, 3, dtype=DT, generator=g)
    xG = xf + (xf - xI)
    PI = random_prims(60, 20 + case)
    PG = mhd.outer_ghost(PI, xI, xG, xf, prm)
    rI, rG = xI.norm(dim=-1), xG.norm(dim=-1)
    rh_, th, ph = mhd.spherical_basis(xf)
    comp = lambda P, a, basis: (P[:, a:a + 3] * basis).sum(-1)
    e = prm.outer_exp

    def law(qI, qG, ex):
        assert torch.allclose(qG * rG ** ex, qI * rI ** ex, rtol=1e-13, atol=1e-15)

    law(PI[:, 0], PG[:, 0], e[0])
    law(comp(PI, 4, rh_), comp(PG, 4, rh_), e[1])
    law(comp(PI, 4, th), comp(PG, 4, th), e[2])
    law(comp(PI, 4, ph), comp(PG, 4, ph), e[3])
    if prm.outer_vr_mass:
        law(comp(PI, 1, rh_) * PI[:, 0], comp(PG, 1, rh_) * PG[:, 0], 2.0)
    else:
        law(comp(PI, 1, rh_), comp(PG, 1, rh_), e[4])
    law(comp(PI, 1, th), comp(PG, 1, th), e[5])
    law(comp(PI, 1, ph), comp(PG, 1, ph), e[6])
    law(PI[:, 7], PG[:, 7], e[7])
    if prm.outer_psi_zero:
        assert torch.equal(PG[:, 8] + PI[:, 8], torch.zeros(60, dtype=DT))
    else:
        assert torch.equal(PG[:, 8], PI[:, 8])


def test_lsq_gradient_exact_for_linear_fields():
    g = torch.Generator().manual_seed(5)
    dx = torch.randn(40, 6, 3, dtype=DT, generator=g)
    A = torch.randn(40, 9, 3, dtype=DT, generator=g)
    dq = torch.einsum("nva,nfa->nfv", A, dx)
    gr = mhd.lsq_gradient(dx, dq)
    assert torch.allclose(gr, A, rtol=1e-12, atol=1e-12)


def test_barth_jespersen_bounds_face_values():
    g = torch.Generator().manual_seed(6)
    n = 500
    qc = torch.randn(n, 9, dtype=DT, generator=g)
    qn = qc[:, None] + torch.randn(n, 6, 9, dtype=DT, generator=g)
    grad = 3 * torch.randn(n, 9, 3, dtype=DT, generator=g)
    dxf = torch.randn(n, 6, 3, dtype=DT, generator=g)
    phi = mhd.barth_jespersen(qc, qn, grad, dxf)
    assert bool(((phi >= 0) & (phi <= 1)).all())
    qf = qc[:, None, :] + phi[:, None, :] * torch.einsum("nva,nfa->nfv", grad, dxf)
    qmax = torch.maximum(qc, qn.amax(1))
    qmin = torch.minimum(qc, qn.amin(1))
    tol = 1e-13 * (1 + qc.abs())
    assert bool((qf <= qmax[:, None] + tol[:, None]).all())
    assert bool((qf >= qmin[:, None] - tol[:, None]).all())
    # no limiting needed (the cell is strictly inside its neighbours' range
    # and the extrapolation is tiny) -> phi == 1
    qn2 = qn.clone()
    qn2[:, 0] = qc + 1.0
    qn2[:, 1] = qc - 1.0
    small = mhd.barth_jespersen(qc, qn2, 1e-9 * grad, 1e-9 * dxf)
    assert torch.equal(small, torch.ones_like(small))
    # the limiter is active: some face reaches an extreme exactly
    act = phi < 1
    assert bool(act.any())
    _assert_limited_faces_reach_an_extreme(qc, qn, grad, dxf, phi)


def _assert_limited_faces_reach_an_extreme(qc, qn, grad, dxf, phi):
    """Barth-Jespersen takes the largest factor that keeps every face value
    inside the neighbourhood's range: wherever phi < 1, some face value sits
    on the bound on its side of q_c (q_max where the extrapolation rises,
    q_min where it falls).  With the bounds themselves checked separately,
    this fixes phi; an over-limited factor leaves every face short of both."""
    d2 = torch.einsum("nva,nfa->nfv", grad, dxf)                # (n, 6, 9)
    qf = qc[:, None, :] + phi[:, None, :] * d2
    qmax = torch.maximum(qc, qn.amax(1))[:, None, :]
    qmin = torch.minimum(qc, qn.amin(1))[:, None, :]
    ext = torch.where(d2 > 0, qmax, qmin)
    scale = (qmax - qmin).clamp_min(1e-300)
    hit = ((qf - ext).abs() <= 1e-13 * scale) & (d2 != 0)
    act = phi < 1
    assert bool(hit.any(1)[act].all())
    # and where phi == 1 no face needed limiting: all within the bounds
    assert bool(((qf <= qmax + 1e-13 * scale) & (qf >= qmin - 1e-13 * scale)).all())


def test_barth_jespersen_is_maximal_on_a_shell_stencil():
    """The same property on the gradients and neighbour values of a real
    stencil (the tiny workload's state, every cell and variable)."""
    from oracle.grid import Grid
    inst = ci.make_instance(4, 6, "geometric", lmax=0, seed=11)
    g = Grid(inst.N, inst.Nr, inst.r_nodes)
    U = torch.from_numpy(inst.U)
    br = torch.from_numpy(inst.br)
    cells = torch.arange(g.ncells)
    st = mhd._Stencil(g, cells)
    fs = mhd.face_states(g, U, br, mhd.Params(), cells, st)
    phi = fs["phi"]
    assert bool((phi < 1).any())
    _assert_limited_faces_reach_an_extreme(fs["qc"], fs["qn"], fs["g"], fs["dxf"], phi)


def test_gravity_and_source():
    x = torch.tensor([[2.0, 0.0, 0.0], [0.0, 0.0, -4.0]], dtype=DT)
    gr = mhd.gravity(x, 0.5)
    assert torch.allclose(gr, torch.tensor([[-0.125, 0, 0], [0, 0, 0.5 / 16]], dtype=DT))
    U = torch.tensor([[2.0, 1.0, 0.0, 0.0, 0, 0, 0, 5.0, 0.0]] * 2, dtype=DT)
    S = mhd.source(U, x, 0.5)
    assert torch.allclose(S[0], torch.tensor([0, -0.25, 0, 0, 0, 0, 0, -0.125, 0], dtype=DT))
