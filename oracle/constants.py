"""Nondimensional constants (oracle; test infrastructure).

Reference density and field are the paper's Eq. 1 values; the reference speed
is the Alfven speed B_ref / sqrt(mu0 rho_ref), the form spelled out in Eq. 22's
denominator.  (The paper quotes 4.5e5 m/s for it in Section 2.1; evaluating the
formula gives 4.80e5 m/s, and the formula is what the oracle uses.)  Lengths
are in solar radii.
"""
import math

RHO_REF = 1.67e-13            # kg/m^3, Eq. 1
B_REF = 2.2e-4                # T, Eq. 1
MU0 = 4.0e-7 * math.pi
V_REF = B_REF / math.sqrt(MU0 * RHO_REF)

VR_STAR_SI = 1935.07          # m/s, prescribed inner radial outflow, Eq. 22
VR_STAR = VR_STAR_SI / V_REF  # nondimensional, Eq. 22

# Nominal solar values (the paper states none): GM_sun and R_sun.
GM_SUN = 1.32712440018e20
R_SUN = 6.957e8
G = GM_SUN / (R_SUN * V_REF * V_REF)   # gravity constant in g = -G x/|x|^3

# Inner-boundary temperature 1.5 MK as p/rho, with mean molecular weight 0.6.
K_B = 1.380649e-23
M_P = 1.67262192369e-27
T_B = K_B * 1.5e6 / (0.6 * M_P * V_REF * V_REF)
RHO_B = 1.0

GAMMA = 1.05          # polytropic index (not printed in the paper)
C_H = 1.0             # divergence-cleaning constant, Section 3.3 default
