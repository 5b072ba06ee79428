"""CPU oracle for the nodal DG right-hand side — TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 NumPy implementation of what the GPU path computes, written
from the method's definitions (nodal DG on affine tetrahedra, Hesthaven &
Warburton 2008, cited by the paper's introduction for its DG layout; Euler
equations and explicit Runge-Kutta time stepping, the paper's Sec. 5.2 vortex
benchmark).  The paper prints none of the DG formulas, so every formula here is
a reading of the textbook method; each module names the reading it follows.

Only the test-suite, the smoke entry and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library (no kernels,
headers, tables or constant generators); both sides are fed the same arrays
from the seeded input generator, which holds none of the method's arithmetic.

Modules:
  reference_element  nodes (warp & blend), Lagrange operators Dr/Ds/Dt, mass,
                     face mass, LIFT, Fmask
  mesh               affine geometry, face normals/areas, face-node connectivity
  hex                tensor-product hexahedra: LGL nodes, 1-D operators, factored
                     lift, Euler RHS on periodic rectilinear grids, and the
                     overintegrated (Gauss-point) weak form
  shock              on the hexahedra: modal smoothness indicator, artificial
                     viscosity (BR1), positivity-preserving limiter
  euler              strong-form Euler RHS with a local Lax-Friedrichs flux
  lsrk               five-stage, fourth-order low-storage Runge-Kutta
  precision          FP32 / split-BF16 contraction emulation and error bounds
  thermo             mixture thermodynamics, temperature Newton, Arrhenius sources
  mlp                learned temperature guess (forward, backward, Adam)
  ns                 reacting Navier-Stokes right-hand side with BR1 viscous terms
"""
