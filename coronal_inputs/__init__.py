"""Seeded synthetic workloads for the coronal finite-volume residual.

This module only *makes inputs*: radial node arrays, a noisy isothermal Parker
wind with a dipole field, a synthetic inner-boundary B_r map, and random
directions.  It holds none of the residual's arithmetic (no cell geometry, no
fluxes, no boundary laws) and it is used, unchanged, by both the HIP path and
the CPU oracle so that the two sides see bit-identical inputs.

The fields are sampled at *nominal* cell positions: radius (r_k + r_{k+1})/2
and the direction of the gnomonic map at the cell's mid angles.  These are not
the finite-volume cell centroids, and need not be: they only place realistic
values in each cell.

Cell order is c = ((p*Nr + k)*N + j)*N + i; the B_r map order is (p*N + j)*N + i.
The state layout is SoA conservative [rho, rho*v (3), B (3), E, psi][cell].

Workload recipes (the paper measures no public dataset; these stand in for its
dipole and magnetogram-driven runs, Sections 3 and 5):
  * tiny   : 6 x 8x8 x 16 cells, radial ratio 1.2, dipole B_r map.
  * medium : 6 x 48x48 x 120 cells, log-uniform radii, dipole + l<=15 map.
  * large  : 6 x 96x96 x 240 cells, log-uniform radii, dipole + l<=31 map.
  * ensemble: 64 instances, N in {16,24,32,48} x Nr in {40,60,80,120} x 4.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# --- physical reference values (Section 2.1) and nominal solar constants ------
RHO_REF = 1.67e-13          # kg m^-3
B_REF = 2.2e-4              # T
MU0 = 4.0e-7 * math.pi
GM_SUN = 1.32712440018e20   # m^3 s^-2 (nominal)
R_SUN = 6.957e8             # m (nominal)
K_B = 1.380649e-23
M_P = 1.67262192369e-27
MU_MOL = 0.6
T_CORONA = 1.5e6            # K, isothermal wind temperature
GAUSS = 1.0e-4 / B_REF      # 1 G in units of B_REF

V_REF = B_REF / math.sqrt(MU0 * RHO_REF)
G_GRAV = GM_SUN / (R_SUN * V_REF ** 2)
T_WIND = K_B * T_CORONA / (MU_MOL * M_P * V_REF ** 2)   # p/rho of the wind
GAMMA = 1.05

BASE_SEED = 220904481


@dataclass(frozen=True)
class Workload:
    name: str
    N: int
    Nr: int
    radial: str          # "geometric" or "log"
    ratio: float         # for geometric spacing
    lmax: int            # 0: dipole-only B_r map
    seed: int


WORKLOADS = {
    "tiny": Workload("tiny", 8, 16, "geometric", 1.2, 0, BASE_SEED),
    "medium": Workload("medium", 48, 120, "log", 0.0, 15, BASE_SEED + 1000),
    "large": Workload("large", 96, 240, "log", 0.0, 31, BASE_SEED + 2000),
}


def radial_nodes(Nr: int, radial: str = "log", ratio: float = 1.2,
                 r0: float = 1.0, r1: float = 21.5, r_ext: float = 25.0, edge: float = 0.01) -> np.ndarray:
    """Nr+1 strictly increasing radii from r0 to r1 ("geometric", "log"), or
    from r0 to r_ext with a last layer of width edge ("bcind")."""
    if radial == "geometric":
        dr0 = (r1 - r0) * (ratio - 1.0) / (ratio ** Nr - 1.0)
        r = np.empty(Nr + 1)
        r[0] = r0
        dr = dr0
        for k in range(Nr):
            r[k + 1] = r[k] + dr
            dr *= ratio
        r[-1] = r1
        return r
    if radial == "log":
        r = r0 * (r1 / r0) ** (np.arange(Nr + 1) / Nr)
        r[0], r[-1] = r0, r1
        return r
    if radial == "bcind":
        # the extended grid of the outer-boundary study: log spacing out to
        # r_ext - edge, then one very thin last layer of width edge, so the
        # outer ghost centre sits edge/2 beyond the boundary (r1 is ignored)
        if Nr < 2:
            raise ValueError("the extended grid needs at least two layers")
        r = np.empty(Nr + 1)
        r[:Nr] = r0 * ((r_ext - edge) / r0) ** (np.arange(Nr) / (Nr - 1))
        r[0], r[Nr - 1], r[Nr] = r0, r_ext - edge, r_ext
        return r
    raise ValueError(radial)


def _panel_point(p: int, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    one = np.ones_like(a)
    table = {
        0: (one, a, b), 1: (-a, one, b), 2: (-one, -a, b),
        3: (a, -one, b), 4: (-b, a, one), 5: (b, a, -one),
    }
    x, y, z = table[p]
    d = np.stack([x, y, z], axis=-1)
    return d / np.linalg.norm(d, axis=-1, keepdims=True)


def nominal_directions(N: int) -> np.ndarray:
    """(6, N, N, 3) unit directions at the cell mid angles, order [p, j, i]."""
    mid = -math.pi / 4 + (np.arange(N) + 0.5) * (math.pi / 2) / N
    bb, aa = np.meshgrid(np.tan(mid), np.tan(mid), indexing="ij")  # [j, i]
    return np.stack([_panel_point(p, aa, bb) for p in range(6)])


def parker_isothermal(r: np.ndarray, cs2: float = T_WIND, G: float = G_GRAV):
    """Transonic isothermal Parker wind: speed v(r) and density with rho(1)=1.

    Solves u^2 - ln u^2 = 4 ln(r/rc) + 4 rc/r - 3 (u = v/cs, rc = G/(2 cs^2))
    on the branch that is subsonic inside rc and supersonic outside, by
    bisection in log u.
    """
    r = np.asarray(r, dtype=np.float64)
    cs = math.sqrt(cs2)
    rc = G / (2.0 * cs2)
    rhs = 4.0 * np.log(r / rc) + 4.0 * rc / r - 3.0
    sub = r < rc
    lo = np.where(sub, -60.0, 0.0)      # bracket in ln u
    hi = np.where(sub, 0.0, 10.0)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        u2 = np.exp(2.0 * mid)
        f = u2 - 2.0 * mid - rhs
        # f decreases in u on the subsonic branch, increases on the supersonic
        go_up = np.where(sub, f > 0.0, f < 0.0)
        lo = np.where(go_up, mid, lo)
        hi = np.where(go_up, hi, mid)
    u = np.exp(0.5 * (lo + hi))
    v = u * cs
    v1 = float(parker_speed_at_one(cs2, G))
    rho = (v1 / v) / r ** 2
    return v, rho


def parker_speed_at_one(cs2: float = T_WIND, G: float = G_GRAV) -> float:
    cs = math.sqrt(cs2)
    rc = G / (2.0 * cs2)
    rhs = 4.0 * math.log(1.0 / rc) + 4.0 * rc - 3.0
    lo, hi = -60.0, 0.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        f = math.exp(2 * mid) - 2 * mid - rhs
        if f > 0.0:
            lo = mid
        else:
            hi = mid
    return math.exp(0.5 * (lo + hi)) * cs


def dipole_field(x: np.ndarray, b_eq: float = GAUSS) -> np.ndarray:
    """Dipole along +z with |B| = b_eq at the equator of r = 1."""
    r = np.linalg.norm(x, axis=-1, keepdims=True)
    rhat = x / r
    zhat = np.array([0.0, 0.0, 1.0])
    mr = rhat[..., 2:3]
    return b_eq * (3.0 * mr * rhat - zhat) / r ** 3


def real_harmonics(lmax: int, theta: np.ndarray, phi: np.ndarray):
    """Real orthonormal Y_lm for l = 1..lmax, m = -l..l (order l up, m up).

    Fully normalised associated Legendre functions by the standard stable
    recurrences (no Condon-Shortley phase); Y_lm = sqrt(2) Pbar_l^m cos(m phi)
    for m > 0, sqrt(2) Pbar_l^|m| sin(|m| phi) for m < 0, Pbar_l^0 for m = 0."""
    x = np.cos(theta)
    sx = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    P = {}
    pmm = np.full_like(x, math.sqrt(1.0 / (4.0 * math.pi)))
    for m in range(lmax + 1):
        if m > 0:
            pmm = math.sqrt((2.0 * m + 1.0) / (2.0 * m)) * sx * pmm
        P[(m, m)] = pmm
        if m + 1 <= lmax:
            P[(m + 1, m)] = math.sqrt(2.0 * m + 3.0) * x * pmm
        for l in range(m + 2, lmax + 1):
            a = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
            b = math.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
            P[(l, m)] = a * (x * P[(l - 1, m)] - b * P[(l - 2, m)])
    out = []
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            if m > 0:
                out.append(math.sqrt(2.0) * P[(l, m)] * np.cos(m * phi))
            elif m < 0:
                out.append(math.sqrt(2.0) * P[(l, -m)] * np.sin(-m * phi))
            else:
                out.append(P[(l, 0)])
    return np.stack(out) if out else np.zeros((0,) + np.shape(theta))


def br_map(N: int, lmax: int, seed: int, peak_gauss: float = 5.0) -> np.ndarray:
    """Inner-boundary B_r map, order (p, j, i), nondimensional.

    Dipole B_r (2 G at the poles) plus, when lmax > 0, random real harmonics
    with amplitude l^-1.5 * N(0,1), scaled so that max |B_r| = peak_gauss.
    """
    d = nominal_directions(N).reshape(-1, 3)
    dip = dipole_field(d)
    br_dip = np.sum(dip * d, axis=-1)
    if lmax <= 0:
        return br_dip
    theta = np.arccos(np.clip(d[:, 2], -1.0, 1.0))
    phi = np.arctan2(d[:, 1], d[:, 0])
    Y = real_harmonics(lmax, theta, phi)
    rng = np.random.default_rng(seed + 11)
    amps = []
    for l in range(1, lmax + 1):
        amps.extend([l ** -1.5] * (2 * l + 1))
    coef = np.asarray(amps) * rng.standard_normal(len(amps))
    h = coef @ Y
    target = peak_gauss * GAUSS
    lo, hi = 0.0, 1.0
    while np.max(np.abs(br_dip + hi * h)) < target:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.max(np.abs(br_dip + mid * h)) < target:
            lo = mid
        else:
            hi = mid
    return br_dip + 0.5 * (lo + hi) * h


def btheta_map(N: int) -> np.ndarray:
    """Inner-boundary B_theta of the dipole at the same directions as br_map,
    order (p, j, i), nondimensional: the B_theta a potential-field model gives
    for a dipole source.  theta-hat = (x z/(rho r), y z/(rho r), -rho/r) with
    rho = sqrt(x^2 + y^2); on the polar axis its phi = 0 limit,
    (cos theta, 0, -sin theta)."""
    d = nominal_directions(N).reshape(-1, 3)
    B = dipole_field(d)
    rho = np.sqrt(d[:, 0] ** 2 + d[:, 1] ** 2)
    axis = rho <= 1e-12
    rs = np.where(axis, 1.0, rho)
    th = np.stack([d[:, 0] * d[:, 2] / rs, d[:, 1] * d[:, 2] / rs, -rho], axis=-1)
    th[axis] = np.stack([d[axis, 2], np.zeros(int(axis.sum())), np.zeros(int(axis.sum()))], axis=-1)
    return np.sum(B * th, axis=-1)


def primitive_state(N: int, Nr: int, r_nodes: np.ndarray, seed: int,
                    noise: float = 0.01) -> np.ndarray:
    """(9, ncells) primitives [rho, v(3), B(3), p, psi] of the noisy wind."""
    d = nominal_directions(N)                      # [p, j, i, 3]
    rmid = 0.5 * (r_nodes[:-1] + r_nodes[1:])       # [k]
    v, rho = parker_isothermal(rmid)
    x = rmid[None, :, None, None, None] * d[:, None]          # [p,k,j,i,3]
    vel = v[None, :, None, None, None] * d[:, None]
    B = dipole_field(x)
    rho_c = np.broadcast_to(rho[None, :, None, None], x.shape[:-1])
    prim = np.zeros((9,) + x.shape[:-1])
    prim[0] = rho_c
    prim[1:4] = np.moveaxis(vel * np.ones_like(x), -1, 0)
    prim[4:7] = np.moveaxis(B, -1, 0)
    prim[7] = T_WIND * rho_c
    prim = prim.reshape(9, -1)
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, size=(8, prim.shape[1]))
    prim[:8] *= 1.0 + noise * u
    return prim


def to_conservative(prim: np.ndarray, gamma: float = GAMMA) -> np.ndarray:
    """Express the generated primitives as the SoA conservative state."""
    rho, v, B, p, psi = prim[0], prim[1:4], prim[4:7], prim[7], prim[8]
    U = np.empty_like(prim)
    U[0] = rho
    U[1:4] = rho * v
    U[4:7] = B
    U[7] = p / (gamma - 1.0) + 0.5 * rho * np.sum(v * v, axis=0) + 0.5 * np.sum(B * B, axis=0)
    U[8] = psi
    return U


def direction(ncells: int, seed: int, scale: np.ndarray | None = None) -> np.ndarray:
    """Seeded N(0,1) direction (9, ncells), optionally scaled elementwise."""
    rng = np.random.default_rng(seed + 7)
    v = rng.standard_normal((9, ncells))
    if scale is not None:
        v *= scale
    return v


def scaled_direction(U: np.ndarray, seed: int) -> np.ndarray:
    """N(0,1) * (|U| + 1e-6 * max_c |U_var|): a direction sized like the state."""
    floor = 1e-6 * np.max(np.abs(U), axis=1, keepdims=True)
    return direction(U.shape[1], seed, np.abs(U) + floor)


def br_direction(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed + 13)
    return rng.standard_normal(n) * GAUSS


@dataclass
class Instance:
    N: int
    Nr: int
    r_nodes: np.ndarray
    U: np.ndarray       # (9, ncells) conservative
    br: np.ndarray      # (6 N^2,)
    seed: int

    @property
    def ncells(self) -> int:
        return 6 * self.N * self.N * self.Nr


def make_instance(N: int, Nr: int, radial: str = "log", ratio: float = 1.2,
                  lmax: int = 0, seed: int = BASE_SEED, noise: float = 0.01) -> Instance:
    r = radial_nodes(Nr, radial, ratio)
    prim = primitive_state(N, Nr, r, seed, noise)
    return Instance(N, Nr, r, to_conservative(prim), br_map(N, lmax, seed), seed)


def workload(name: str) -> Instance:
    w = WORKLOADS[name]
    return make_instance(w.N, w.Nr, w.radial, w.ratio, w.lmax, w.seed)


def ensemble_specs(n: int = 64, seed: int = BASE_SEED + 4000):
    """Uneven instance shapes: N x Nr full factorial, repeated, shuffled."""
    shapes = [(N, Nr) for N in (16, 24, 32, 48) for Nr in (40, 60, 80, 120)]
    reps = (n + len(shapes) - 1) // len(shapes)
    specs = (shapes * reps)[:n]
    order = np.random.default_rng(seed).permutation(n)
    return [(specs[o][0], specs[o][1], seed + 1 + idx) for idx, o in enumerate(order)]


def ensemble_instances(n: int = 64, lmax: int = 15):
    """The ensemble's instances: each a log-spaced shell with its own seeded
    state and magnetogram (as the 1.66M-cell workload, at its own size)."""
    return [make_instance(N, Nr, "log", lmax=lmax, seed=s) for N, Nr, s in ensemble_specs(n)]
