"""FP64 CPU oracle for the PCEXP / DG-Euler hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy/SciPy implementation of what the HIP path computes, written from the
paper (Li, Luo, Wang, Ju, "An exponential time-integrator scheme for steady
and unsteady inviscid flows", arXiv 1801.06300).  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never does.  It shares no code with the HIP path: the two
meet only through the seeded inputs of the ``workloads`` package.

Functions accept complex arrays wherever the complex-step derivative needs
them.  Each module cites the section / equation of the paper it follows.

Readings where the paper leaves the choice open (no value in the paper fixes
them); each is pinned by the property that defines it rather than by a
number from the paper:
  * the Gaussian quadrature rule (conical-product Gauss-Jacobi, q = p+1):
    exact integrals of monomials up to its degree;
  * the Roe flux without entropy fix: consistency, antisymmetry, Roe's
    property against the exact flux Jacobian, supersonic upwinding;
  * the local Lax-Friedrichs flux: consistency, antisymmetry, dissipation
    speed equal to the largest eigenvalue magnitude of the flux Jacobians;
  * the slip-wall and Riemann-invariant far-field ghost states: the mirror
    relations, and the characteristic invariants, entropy and tangential
    velocity recovered from the far-field ghost state.
"""
