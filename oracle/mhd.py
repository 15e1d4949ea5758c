"""Finite-volume ideal-MHD residual with divergence cleaning (oracle).

TEST INFRASTRUCTURE: imported only by the tests, the smoke check and the
bench's CPU-baseline leg.

What is computed (paper Section 2.1 and Eqs. 14-17, Sections 3.2 and 4.1):

* State per cell, conservative: U = (rho, rho v, B, E, psi) with
  E = p/(gamma-1) + rho|v|^2/2 + |B|^2/2 (magnetic units with mu = 1, so the
  printed B^2/8pi and B B/4pi factors read as B^2/2 and B B).
* Primitives P = (rho, v, B, p, psi) are reconstructed.
* Inner boundary "low E" (Section 3.2, Eq. 25): B_r Dirichlet from the
  magnetogram, B_theta and B_phi Neumann, the boundary velocity parallel to
  the boundary field so that V_b x B_b = 0, with radial part V_r* B_r^2/|B|^2
  (V_r* of Eq. 22), rho and p Dirichlet, psi_b = 0 (Section 3.3).
* Inner boundary "large E" (Section 3.2, Eqs. 20-24, the Wind-Predict law,
  selected by inner_mode = 1): B_r and B_theta Dirichlet (the magnetogram
  and an imposed B_theta map, which a potential-field model supplies),
  B_phi Neumann, V = V_par (B_r, B_theta, 0) with V_par = V_r* B_r / B_pol^2.
* Outer boundary: Table 2 ghost laws in r and rho, per variable exponents.
* Second-order reconstruction: unweighted least squares gradient over the six
  face neighbours (ghosts at mirrored centres), optional Barth-Jespersen
  limiter, linear extrapolation to the face centroid.
* Rusanov flux of the MHD + GLM physical flux; gravity source rho g and
  g . rho v with g = -G x/|x|^3 at the cell centroid.
* R_c = sum over faces of the outward numerical flux times |S| minus
  V_c S(U_c): the integrated residual, so dU/dt = -R/V.

* Diagnostics (Sections 2.2 and 3.1): the ideal-MHD electric field
  E = -V x B at the cell centroids in spherical components, its per-component
  maximum and volume-weighted RMS, and the E-free state whose velocity keeps
  only its component along B (V0 x B = 0, the paper's first remedy).

The function ``residual`` evaluates R on any subset of cells; it gathers the
distance-2 stencil it needs.  It is one vectorised code path for both the full
grid and sampled cells.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import constants as K
from .grid import Grid

DT = torch.float64

# Table 2 cases as (exponents, V_r law, psi law).  Exponent e means G = I (rI/rG)^e.
# Order of exponents: rho, B_r, B_theta, B_phi, V_r, V_theta, V_phi, p.
# V_r law "mass" means V_r r^2 rho = const; psi law "B0" means psi_b = 0.
TABLE2 = {
    1: ((0, 0, 0, 0, 0, 0, 0, 0), "const", "B0"),
    2: ((2, 0, 0, 0, 0, 0, 0, 2), "const", "B0"),
    3: ((2, 2, 0, 0, 0, 0, 0, 2), "const", "B0"),
    4: ((2, 2, 0, 1, 0, 0, 0, 2), "const", "B0"),
    5: ((2, 2, 0, 1, 0, 0, 0, 2), "const", "G=I"),
    6: ((2, 2, 0, 1, 0, 0, 1, 2), "mass", "B0"),
    7: ((2, 2, 0, 0, 0, 0, 1, 2), "mass", "B0"),
    8: ((2, 0, 0, 0, 0, 0, 1, 2), "mass", "B0"),
    9: ((3, 2, 0, 1, 0, 0, 1, 3), "mass", "B0"),
}


@dataclass
class Params:
    gamma: float = K.GAMMA
    c_h: float = K.C_H
    G: float = K.G
    vr_star: float = K.VR_STAR
    rho_b: float = K.RHO_B
    T_b: float = K.T_B
    limiter: int = 1
    # outer ghost exponents (rho, B_r, B_th, B_ph, V_r, V_th, V_ph, p):
    # Table 2 case 6 with rho and p at the 2.5 law of Section 4.2.
    outer_exp: tuple = (2.5, 2.0, 0.0, 1.0, 0.0, 0.0, 1.0, 2.5)
    outer_vr_mass: bool = True
    outer_psi_zero: bool = True
    # inner boundary: 0 low-E (Eq. 25), 1 large-E (Eqs. 20-24) with the
    # imposed B_theta map inner_btheta (6 N^2, order (p, j, i))
    inner_mode: int = 0
    inner_btheta: torch.Tensor | None = None

    @staticmethod
    def table2(case: int, **kw) -> "Params":
        e, vr, psi = TABLE2[case]
        return Params(outer_exp=tuple(float(x) for x in e), outer_vr_mass=(vr == "mass"),
                      outer_psi_zero=(psi == "B0"), **kw)


# ----------------------------------------------------------------------------
# pointwise physics
# ----------------------------------------------------------------------------

def dot(a, b):
    return (a * b).sum(-1)


def pick_min(a, b):
    """min(a, b) that returns a on ties (derivative follows the pick)."""
    return torch.where(a <= b, a, b)


def pick_max(a, b):
    return torch.where(a >= b, a, b)


def cons_to_prim(U, gamma):
    """U (..., 9) conservative -> P (..., 9) primitive."""
    rho = U[..., 0]
    v = U[..., 1:4] / rho[..., None]
    B = U[..., 4:7]
    p = (gamma - 1.0) * (U[..., 7] - 0.5 * rho * dot(v, v) - 0.5 * dot(B, B))
    return torch.cat([rho[..., None], v, B, p[..., None], U[..., 8:9]], dim=-1)


def prim_to_cons(P, gamma):
    rho = P[..., 0]
    v = P[..., 1:4]
    B = P[..., 4:7]
    E = P[..., 7] / (gamma - 1.0) + 0.5 * rho * dot(v, v) + 0.5 * dot(B, B)
    return torch.cat([rho[..., None], rho[..., None] * v, B, E[..., None], P[..., 8:9]], dim=-1)


def physical_flux(P, n, gamma, c_h):
    """Normal flux F(U).n of ideal MHD with GLM cleaning, for unit n."""
    rho, v, B, p, psi = P[..., 0], P[..., 1:4], P[..., 4:7], P[..., 7], P[..., 8]
    vn = dot(v, n)
    Bn = dot(B, n)
    B2 = dot(B, B)
    pT = p + 0.5 * B2
    E = p / (gamma - 1.0) + 0.5 * rho * dot(v, v) + 0.5 * B2
    f_mass = rho * vn
    f_mom = rho[..., None] * v * vn[..., None] + pT[..., None] * n - B * Bn[..., None]
    f_B = vn[..., None] * B - Bn[..., None] * v + psi[..., None] * n
    f_E = (E + pT) * vn - Bn * dot(v, B)
    f_psi = c_h * c_h * Bn
    return torch.cat([f_mass[..., None], f_mom, f_B, f_E[..., None], f_psi[..., None]], dim=-1)


def fast_speed(P, n, gamma):
    rho, B, p = P[..., 0], P[..., 4:7], P[..., 7]
    a2 = gamma * p / rho
    b2 = dot(B, B) / rho
    bn2 = dot(B, n) ** 2 / rho
    disc = (a2 + b2) ** 2 - 4.0 * a2 * bn2
    disc = torch.where(disc > 0.0, disc, torch.zeros_like(disc))
    return torch.sqrt(0.5 * (a2 + b2 + torch.sqrt(disc)))


def rusanov(PL, PR, S, prm: Params):
    """Numerical flux through a face of vector area S, oriented L -> R."""
    area = torch.linalg.norm(S, dim=-1)
    n = S / area[..., None]
    FL = physical_flux(PL, n, prm.gamma, prm.c_h)
    FR = physical_flux(PR, n, prm.gamma, prm.c_h)
    lamL = torch.abs(dot(PL[..., 1:4], n)) + fast_speed(PL, n, prm.gamma)
    lamR = torch.abs(dot(PR[..., 1:4], n)) + fast_speed(PR, n, prm.gamma)
    s = pick_max(lamL, lamR)
    s = pick_max(s, torch.full_like(s, prm.c_h))
    UL = prim_to_cons(PL, prm.gamma)
    UR = prim_to_cons(PR, prm.gamma)
    return (0.5 * (FL + FR) - 0.5 * s[..., None] * (UR - UL)) * area[..., None], s


def spherical_basis(x):
    """r-hat, theta-hat, phi-hat at x (..., 3), as in Eqs. 20-21.

    On the polar axis theta-hat and phi-hat are undefined; within a relative
    distance 1e-12 of it (where they would be set by rounding) the limit along
    the meridian phi = 0 is taken: theta-hat = (sign z, 0, 0), phi-hat = (0, 1, 0)."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    r = torch.linalg.norm(x, dim=-1)
    rc = torch.sqrt(X * X + Y * Y)
    axis = rc <= 1e-12 * r
    rcs = torch.where(axis, torch.ones_like(rc), rc)
    rhat = x / r[..., None]
    that = torch.stack([X * Z / (rcs * r), Y * Z / (rcs * r), -rc / r], dim=-1)
    phat = torch.stack([-Y / rcs, X / rcs, torch.zeros_like(X)], dim=-1)
    zero = torch.zeros_like(X)
    that_ax = torch.stack([torch.where(Z >= 0, torch.ones_like(Z), -torch.ones_like(Z)), zero, zero], dim=-1)
    phat_ax = torch.stack([zero, torch.ones_like(X), zero], dim=-1)
    that = torch.where(axis[..., None], that_ax, that)
    phat = torch.where(axis[..., None], phat_ax, phat)
    return rhat, that, phat


def inner_ghost(PI, xf, br, prm: Params):
    """Low-E inner ghost state (Section 3.2, Eq. 25).

    The boundary value b of a Dirichlet variable is the face average, so the
    ghost is G = 2b - I.  B_r takes the map value, B_theta and B_phi keep the
    interior values (Neumann), and the boundary velocity is along B_b with
    radial part V_r* B_r^2/|B_b|^2.  psi_b = 0.
    """
    rhat, that, phat = spherical_basis(xf)
    B = PI[..., 4:7]
    Bth = dot(B, that)
    Bph = dot(B, phat)
    Bb = br[..., None] * rhat + Bth[..., None] * that + Bph[..., None] * phat
    Bb2 = dot(Bb, Bb)
    Vb = (prm.vr_star * br / torch.where(Bb2 > 1e-30, Bb2, torch.full_like(Bb2, 1e-30)))[..., None] * Bb
    rho = 2.0 * prm.rho_b - PI[..., 0]
    v = 2.0 * Vb - PI[..., 1:4]
    Bg = 2.0 * Bb - B
    p = 2.0 * prm.rho_b * prm.T_b - PI[..., 7]
    psi = -PI[..., 8]
    return torch.cat([rho[..., None], v, Bg, p[..., None], psi[..., None]], dim=-1)


def inner_ghost_large_e(PI, xf, br, bth, prm: Params):
    """Large-E inner ghost state (Section 3.2, Eqs. 20-24: the Wind-Predict
    boundary).

    B_r takes the map value and B_theta the imposed value (Dirichlet: face
    average), B_phi keeps the interior value (Neumann).  The velocity removes
    the poloidal flux: with B_pol^2 = B_r^2 + B_theta^2 and
    V_par = V_r* B_r / B_pol^2, V_r = V_par B_r, V_theta = V_par B_theta,
    V_phi = 0 (Dirichlet).  rho, p and psi as in the low-E law.
    """
    rhat, that, phat = spherical_basis(xf)
    B = PI[..., 4:7]
    Bph = dot(B, phat)
    Bb = br[..., None] * rhat + bth[..., None] * that + Bph[..., None] * phat
    Bpol2 = br * br + bth * bth
    Vpar = prm.vr_star * br / torch.where(Bpol2 > 1e-30, Bpol2, torch.full_like(Bpol2, 1e-30))
    Vb = (Vpar * br)[..., None] * rhat + (Vpar * bth)[..., None] * that
    rho = 2.0 * prm.rho_b - PI[..., 0]
    v = 2.0 * Vb - PI[..., 1:4]
    Bg = 2.0 * Bb - B
    p = 2.0 * prm.rho_b * prm.T_b - PI[..., 7]
    psi = -PI[..., 8]
    return torch.cat([rho[..., None], v, Bg, p[..., None], psi[..., None]], dim=-1)


def outer_ghost(PI, xI, xG, xf, prm: Params):
    """Outer ghost state by the Table 2 laws: G = I (r_I/r_G)^e per variable,
    in the spherical components at the face centroid; V_r by V_r r^2 rho =
    const when selected; psi by psi_b = 0 (G = -I) or G = I."""
    e = prm.outer_exp
    rI = torch.linalg.norm(xI, dim=-1)
    rG = torch.linalg.norm(xG, dim=-1)
    q = rI / rG
    rhat, that, phat = spherical_basis(xf)
    v, B = PI[..., 1:4], PI[..., 4:7]
    rho = PI[..., 0] * q ** e[0]
    Br = dot(B, rhat) * q ** e[1]
    Bt = dot(B, that) * q ** e[2]
    Bp = dot(B, phat) * q ** e[3]
    if prm.outer_vr_mass:
        Vr = dot(v, rhat) * (rI * rI * PI[..., 0]) / (rG * rG * rho)
    else:
        Vr = dot(v, rhat) * q ** e[4]
    Vt = dot(v, that) * q ** e[5]
    Vp = dot(v, phat) * q ** e[6]
    p = PI[..., 7] * q ** e[7]
    psi = -PI[..., 8] if prm.outer_psi_zero else PI[..., 8]
    vG = Vr[..., None] * rhat + Vt[..., None] * that + Vp[..., None] * phat
    BG = Br[..., None] * rhat + Bt[..., None] * that + Bp[..., None] * phat
    return torch.cat([rho[..., None], vG, BG, p[..., None], psi[..., None]], dim=-1)


def lsq_gradient(dx, dq):
    """Unweighted least-squares gradient: solve (sum dx dx^T) g = sum dx dq.

    dx (n, 6, 3) neighbour offsets, dq (n, 6, 9) value differences.
    Returns g (n, 9, 3)."""
    M = torch.einsum("nfa,nfb->nab", dx, dx)
    rhs = torch.einsum("nfa,nfv->nav", dx, dq)
    return torch.linalg.solve(M, rhs).transpose(1, 2)


def barth_jespersen(qc, qn, g, dxf):
    """Barth-Jespersen factor per variable (n, 9).

    qc (n, 9), qn (n, 6, 9), g (n, 9, 3), dxf (n, 6, 3) = x_f - x_c.
    Extremes over the cell and its six neighbours; per face the ratio that
    keeps the face value inside them, capped at 1; the minimum over faces.
    Ties keep the earlier candidate (the cell first, then faces in order)."""
    qmax, qmin = qc, qc
    for f in range(6):
        qmax = pick_max(qmax, qn[:, f])
        qmin = pick_min(qmin, qn[:, f])
    one = torch.ones_like(qc)
    phi = one
    for f in range(6):
        d2 = (g * dxf[:, f, None, :]).sum(-1)
        num = torch.where(d2 > 0.0, qmax - qc, qmin - qc)
        den = torch.where(d2 != 0.0, d2, one)
        phif = torch.where(d2 != 0.0, pick_min(one, num / den), one)
        phi = pick_min(phi, phif)
    return phi


def gravity(x, G):
    r = torch.linalg.norm(x, dim=-1)
    return -G * x / (r * r * r)[..., None]


def source(U, x, G):
    """Gravity source S(U) = (0, rho g, 0, g . rho v, 0) at the centroid x."""
    g = gravity(x, G)
    z = torch.zeros_like(U[..., 0:1])
    return torch.cat([z, U[..., 0:1] * g, z, z, z, dot(g, U[..., 1:4])[..., None], z], dim=-1)


# ----------------------------------------------------------------------------
# stencil gathering and the residual
# ----------------------------------------------------------------------------

class _Stencil:
    """Everything about the cells within distance 2 of a target set."""

    def __init__(self, grid: Grid, T: torch.Tensor):
        nc = grid.ncells
        self.grid = grid
        self.T = T
        nbT = grid.neighbours(T)
        self.D1 = torch.unique(torch.cat([T, nbT[nbT < nc]]))
        self.nb1 = grid.neighbours(self.D1)                    # (n1, 6)
        self.D2 = torch.unique(torch.cat([self.D1, self.nb1[self.nb1 < nc]]))
        self.nb2 = grid.neighbours(self.D2)                    # (n2, 6)
        self.ghosts = torch.unique(self.nb1[self.nb1 >= nc])
        xc, V, xf, S = grid.cell_geometry(self.D2)
        self.xc, self.V, self.xf, self.S = xc, V, xf, S
        self.gcell, self.glf, self.gouter, self.gcol = grid.ghost_cell(self.ghosts)
        self.xg = grid.ghost_centres(self.ghosts)
        # owner (canonical L) and the owner's local face for each (D2 cell, face)
        cells2 = self.D2[:, None].expand_as(self.nb2)
        is_g = self.nb2 >= nc
        owner_self = is_g | (self.nb2 > cells2)
        self.owner_self = owner_self
        # reverse local face: position of the cell in its neighbour's list
        nbc = torch.where(is_g, cells2, self.nb2)
        rev = self._reverse(nbc, cells2)
        self.rev = torch.where(is_g, torch.arange(6).expand_as(self.nb2), rev)

    def _reverse(self, nbc, cells2):
        # neighbours of the neighbour: nbc may lie outside D2 only for faces
        # of cells outside D1, which the residual never uses; map those to 0.
        inside = torch.isin(nbc, self.D2)
        pos = torch.searchsorted(self.D2, nbc).clamp(max=self.D2.numel() - 1)
        nn = self.nb2[pos]                                          # (n2, 6, 6)
        hit = nn == cells2[..., None]
        rev = hit.long().argmax(-1)
        return torch.where(inside, rev, torch.zeros_like(rev))

    def loc(self, cells):
        return torch.searchsorted(self.D2, cells)

    def gloc(self, gids):
        return torch.searchsorted(self.ghosts, gids)

    def face_geometry(self, lc: torch.Tensor, lf: torch.Tensor):
        """Canonical centroid and vector area of face lf of D2-local cell lc,
        and the sign (+1 when the cell owns the face)."""
        own = self.owner_self[lc, lf]
        nb = self.nb2[lc, lf]
        olc = torch.where(own, lc, self.loc(torch.where(own, self.D2[lc], nb)))
        olf = torch.where(own, lf, self.rev[lc, lf])
        sign = torch.where(own, 1.0, -1.0).to(DT)
        return self.xf[olc, olf], self.S[olc, olf], sign, olc, olf


def face_states(grid: Grid, U: torch.Tensor, br: torch.Tensor, prm: Params,
                cells: torch.Tensor, st: _Stencil):
    """Reconstructed states on both sides of every face of the target cells.

    Returns a dict with, per (target cell, local face): PL, PR (n, 6, 9) in the
    face's canonical orientation (owner on the left), its vector area S and
    centroid xf (owner's), and sign (+1 when the target cell owns the face).
    Also the unlimited gradients g, limiter factors phi of the D1 cells."""
    nc = grid.ncells
    Ut = U.transpose(0, 1)
    P2 = cons_to_prim(Ut[st.D2], prm.gamma)                  # (n2, 9)

    # ghost primitives
    lI = st.loc(st.gcell)
    PI = P2[lI]
    ar = torch.arange(st.ghosts.numel())
    xfb = st.xf[lI, st.glf]
    inner = ~st.gouter
    PG = torch.zeros(st.ghosts.numel(), 9, dtype=U.dtype)
    if bool(inner.any()):
        if prm.inner_mode == 1:
            bth = torch.as_tensor(prm.inner_btheta, dtype=U.dtype)
            PGi = inner_ghost_large_e(PI[inner], xfb[inner], br[st.gcol[inner]], bth[st.gcol[inner]], prm)
        else:
            PGi = inner_ghost(PI[inner], xfb[inner], br[st.gcol[inner]], prm)
        PG = PG.index_put((ar[inner],), PGi)
    if bool(st.gouter.any()):
        PG = PG.index_put((ar[st.gouter],), outer_ghost(PI[st.gouter], st.xc[lI[st.gouter]],
                                                        st.xg[st.gouter], xfb[st.gouter], prm))

    # value / centre tables: D2 cells then ghosts
    n2 = st.D2.numel()
    vals = torch.cat([P2, PG], dim=0)
    cent = torch.cat([st.xc, st.xg], dim=0)

    def tab(ids):
        gl = st.gloc(ids.clamp(min=nc)).clamp(max=max(st.ghosts.numel() - 1, 0))
        return torch.where(ids >= nc, n2 + gl, st.loc(ids.clamp(max=nc - 1)).clamp(max=n2 - 1))

    # gradients and limiter on the D1 cells
    l1 = st.loc(st.D1)
    t1 = tab(st.nb1)                                         # (n1, 6)
    qc = P2[l1]
    qn = vals[t1]                                            # (n1, 6, 9)
    dx = cent[t1] - st.xc[l1][:, None, :]
    g = lsq_gradient(dx, qn - qc[:, None, :])                # (n1, 9, 3)
    lf6 = torch.arange(6).expand(l1.numel(), 6)
    xf1, _, _, _, _ = st.face_geometry(l1[:, None].expand(-1, 6), lf6)
    dxf = xf1 - st.xc[l1][:, None, :]
    if prm.limiter:
        phi = barth_jespersen(qc, qn, g, dxf)
    else:
        phi = torch.ones_like(qc)
    Glim = g * phi[..., None]
    Gfull = torch.zeros(n2, 9, 3, dtype=U.dtype).index_put((l1,), Glim)

    # faces of the target cells in canonical orientation
    lt = st.loc(st.T)
    nT = lt.numel()
    lc = lt[:, None].expand(-1, 6)
    lf = torch.arange(6).expand(nT, 6)
    xf, S, sign, olc, olf = st.face_geometry(lc, lf)
    other = st.nb2[olc, olf]                                 # R-side id
    og = other >= nc
    PL = P2[olc] + (Gfull[olc] * (xf - st.xc[olc])[..., None, :]).sum(-1)
    lo = torch.where(og, olc, st.loc(other.clamp(max=nc - 1)).clamp(max=n2 - 1))
    PRc = P2[lo] + (Gfull[lo] * (xf - st.xc[lo])[..., None, :]).sum(-1)
    PRg = vals[tab(other)]
    PR = torch.where(og[..., None], PRg, PRc)
    return dict(PL=PL, PR=PR, S=S, xf=xf, sign=sign, other=other, g=g, phi=phi,
                D1=st.D1, PG=PG, ghosts=st.ghosts, qn=qn, qc=qc, dxf=dxf)


def residual(grid: Grid, U: torch.Tensor, br: torch.Tensor, prm: Params,
             cells: torch.Tensor | None = None, _stencil: _Stencil | None = None,
             return_speeds: bool = False):
    """Integrated residual R (9, len(cells)) of the state U (9, ncells).

    br (6 N^2,) is the inner-boundary B_r map in (p, j, i) order.  Every face
    flux is evaluated in the face's canonical orientation and added with +1
    to its owner and -1 to the other cell."""
    nc = grid.ncells
    if cells is None:
        cells = torch.arange(nc)
    st = _stencil if _stencil is not None else _Stencil(grid, cells)
    fs = face_states(grid, U, br, prm, cells, st)
    F, s = rusanov(fs["PL"], fs["PR"], fs["S"], prm)        # (nT, 6, 9)
    flux_sum = (F * fs["sign"][..., None]).sum(1)
    lt = st.loc(st.T)
    R = flux_sum - st.V[lt][:, None] * source(U.transpose(0, 1)[st.T], st.xc[lt], prm.G)
    if return_speeds:
        return R.transpose(0, 1), (s, torch.linalg.norm(fs["S"], dim=-1))
    return R.transpose(0, 1)


def efield(grid, U, prm: Params, cells=None):
    """Electric field of ideal MHD, E = -V x B (Section 2.2, Eqs. E1-E2), at
    the cell centroids in spherical components (E_r, E_theta, E_phi) (3,
    ncells), and the volume-weighted statistics the paper reads: per
    component and for |E|, the maximum and the root mean square
    sqrt(sum_c V_c E^2 / sum_c V_c); returns (E, max4, rms4).  With cells
    given, U holds those cells' states (9, len(cells)) and the statistics
    are over them."""
    if cells is None:
        cells = torch.arange(grid.ncells)
    xc, V, _, _ = grid.cell_geometry(cells)
    P = cons_to_prim(U.transpose(0, 1), prm.gamma)
    E = -torch.linalg.cross(P[:, 1:4], P[:, 4:7])
    rh, th, ph = spherical_basis(xc)
    Es = torch.stack([dot(E, rh), dot(E, th), dot(E, ph)], dim=0)
    mag = torch.linalg.norm(E, dim=-1)
    comps = torch.cat([Es, mag[None]], dim=0)
    mx = comps.abs().amax(dim=1)
    rms = torch.sqrt((comps ** 2 * V[None]).sum(1) / V.sum())
    return Es, mx, rms


def efree_state(U, prm: Params):
    """The E-free initial state of Section 3.1 (fix 1): the velocity keeps
    only its component along B, V0 = (V . B) B / |B|^2 (unchanged where B = 0),
    so that V0 x B = 0; rho, B, p and psi are kept (E is recomputed)."""
    P = cons_to_prim(U.transpose(0, 1), prm.gamma)
    v, B = P[:, 1:4], P[:, 4:7]
    B2 = dot(B, B)
    par = torch.where(B2 > 0, dot(v, B) / torch.where(B2 > 0, B2, torch.ones_like(B2)), torch.zeros_like(B2))
    v0 = torch.where((B2 > 0)[:, None], par[:, None] * B, v)
    P0 = torch.cat([P[:, :1], v0, P[:, 4:]], dim=1)
    return prim_to_cons(P0, prm.gamma).transpose(0, 1)
