"""Nondimensional parameters of the coronal model (product defaults).

Reference values of the paper's Eq. 1: rho_ref = 1.67e-13 kg/m^3 and
B_ref = 2.2e-4 T; the reference speed is the Alfven speed B_ref/sqrt(mu0
rho_ref) (the form in Eq. 22's denominator; it evaluates to 4.80e5 m/s).
The inner-boundary outflow V_r* = 1935.07 m/s / V_ref (Eq. 22).  The
cleaning speed is 1 (Section 3.3).  The outer law defaults to Table 2
case 6 with rho and p extrapolated as r^-2.5 (Section 4.2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

_RHO_REF = 1.67e-13
_B_REF = 2.2e-4
_V_REF = _B_REF / math.sqrt(4.0e-7 * math.pi * _RHO_REF)
_GM_SUN = 1.32712440018e20
_R_SUN = 6.957e8
_KB_OVER_MP = 1.380649e-23 / 1.67262192369e-27

# Table 2 (Section 4.1): powers e in G = I (r_I/r_G)^e for
# (rho, B_r, B_theta, B_phi, V_r, V_theta, V_phi, p), V_r mass law, psi_b = 0.
OUTER_CASES = {
    1: ((0, 0, 0, 0, 0, 0, 0, 0), False, True),
    2: ((2, 0, 0, 0, 0, 0, 0, 2), False, True),
    3: ((2, 2, 0, 0, 0, 0, 0, 2), False, True),
    4: ((2, 2, 0, 1, 0, 0, 0, 2), False, True),
    5: ((2, 2, 0, 1, 0, 0, 0, 2), False, False),
    6: ((2, 2, 0, 1, 0, 0, 1, 2), True, True),
    7: ((2, 2, 0, 0, 0, 0, 1, 2), True, True),
    8: ((2, 0, 0, 0, 0, 0, 1, 2), True, True),
    9: ((3, 2, 0, 1, 0, 0, 1, 3), True, True),
}


@dataclass
class Params:
    gamma: float = 1.05
    c_h: float = 1.0
    G: float = _GM_SUN / (_R_SUN * _V_REF ** 2)
    vr_star: float = 1935.07 / _V_REF
    rho_b: float = 1.0
    T_b: float = _KB_OVER_MP * 1.5e6 / (0.6 * _V_REF ** 2)
    limiter: int = 1
    inner_mode: int = 0      # 0: low-E inner boundary; 1: large-E (needs Context.set_inner_btheta)
    outer_exp: tuple = (2.5, 2.0, 0.0, 1.0, 0.0, 0.0, 1.0, 2.5)
    outer_vr_mass: bool = True
    outer_psi_zero: bool = True

    @classmethod
    def outer_case(cls, case: int, **kw) -> "Params":
        e, mass, psi0 = OUTER_CASES[case]
        return cls(outer_exp=tuple(float(x) for x in e), outer_vr_mass=mass, outer_psi_zero=psi0, **kw)


V_REF = _V_REF
