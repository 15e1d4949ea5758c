"""CPU oracle for the coronal finite-volume MHD residual (TEST INFRASTRUCTURE).

This package is the plain, slow, obviously-correct reference that the HIP path
is checked against.  It is test infrastructure only: it may be imported by the
tests, by the smoke check and by the bench's CPU-baseline leg, and by nothing
else.  The product library never calls it and has no fallback to it.

It is written from the paper (Brchnelova et al., "To E or not to E: Numerical
Nuances of Global Coronal Models") and shares no code with the HIP path:

* ``constants``: reference values (Eq. 1) and the inner-boundary outflow
  constant (Eq. 22), in the nondimensional units of Section 2.1.
* ``grid``: the cubed-sphere hexahedral shell, its geometry from the cell
  vertices, and connectivity derived *geometrically* by point location.
* ``mhd``: ideal MHD with hyperbolic divergence cleaning (Eqs. 14-17 and
  Section 2.1), second-order finite-volume reconstruction, the low-E inner
  boundary (Eq. 25, Section 3.2) and the outer ghost laws (Table 2).
* ``solve``: local pseudo-time step, the Eq. 2 residual monitor, GMRES and the
  backward-Euler step (Section 2.1), and the exact B_r-map gradient of an
  objective after several implicit steps (dense, small grids).

Everything is float64 PyTorch CPU code, vectorised over cells and faces with
no blocking or fusion.  Forward-mode derivatives (JVP) use torch.func.jvp and
reverse-mode (VJP) uses torch.autograd on the same residual function.
"""
