"""MI355X-native FP64 finite-volume coronal MHD residual, JVP and VJP.

The hot path of the implicit coronal model of Brchnelova et al. ("To E or not
to E: Numerical Nuances of Global Coronal Models"): the ideal-MHD residual
with divergence cleaning on a spherical shell, its ghost-cell boundary laws,
its exact Jacobian-vector product and its adjoint, written as HIP kernels
for gfx950 behind a C ABI (include/cfv.h) and bound here with ctypes.
"""
from .params import Params, OUTER_CASES, V_REF  # noqa: F401
from .binding import CfvError, CfvNonPhysical, Context, Ensemble, Grid, Tuning, lib  # noqa: F401
from .autograd import MHDResidual, residual  # noqa: F401
