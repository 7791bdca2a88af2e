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

Parity-unpinned readings (no value in the paper fixes them; they are pinned
only by free-stream, conservation and oracle/GPU agreement):
  * the Gaussian quadrature rule (conical-product Gauss-Jacobi, q = p+1);
  * the Roe flux without entropy fix and the local Lax-Friedrichs flux;
  * the slip-wall and Riemann-invariant far-field ghost states.
"""
