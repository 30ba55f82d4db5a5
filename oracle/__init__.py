"""FP64 NumPy oracle for the WaterLily-style incompressible Navier-Stokes step.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised CPU statement of what the GPU library computes.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
it; the product path never does.  It shares no code with the HIP library and
imports nothing from it.

Paper: Weymouth & Font, "WaterLily.jl: A differentiable fluid simulator in
Julia with fast heterogeneous execution" (arXiv 2304.08159).  The paper states
the method in one paragraph (Sec. 2 "Computational approach") and one code
snippet (the pressure-gradient loop in Sec. 2).  Every constant it leaves open
is fixed by a named reading that both the oracle and the GPU follow; each
module's docstring lists the readings it implements.

Conventions (all modules):
  * arrays are indexed a[x, y] (2D) or a[x, y, z] (3D): axis i is direction i;
  * grid spacing 1; cell I spans [I, I+1) componentwise, centre I + 1/2;
  * the velocity component u_i(I) lives on the LOWER i-face of cell I
    (position I + 1/2 - delta_i/2), which is what the gradient loop
    u[I,i] -= coeff[I,i]*(p[I]-p[I-del(i)]) of Sec. 2 implies;
  * p, sigma (the projection right-hand side) are cell-centred.

Modules:
  grid      boundary codes, shifts, level sizes
  geometry  signed-distance body -> BDIM moments and Poisson coefficients
  poisson   matrix-free operator, damped-Jacobi V-cycle GMG, min-norm coarse
  momentum  CFL time step, third-order upwind-biased flux, BDIM blend, BCs
  step      divergence, projection, Heun time step (the simstep! analogue)

Functions whose result no independent check fixes say "parity unpinned" in
their docstring.
"""

from . import grid, geometry, poisson, momentum, step  # noqa: F401
