"""CPU oracle for the entropy-split SBP-SAT discretization (TEST INFRASTRUCTURE).

This package is a plain, slow, double-precision reference written from the
paper (Worku & Zingg, "Entropy-split multidimensional summation-by-parts
discretization of the Euler and compressible Navier-Stokes equations").
It exists only to check the HIP implementation: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the HIP path; the only common module is
the seeded input generator ``paper_2305_07181_amd.workloads``.

Modules
  operators  reference-element diagonal-E SBP operators (Def. 1, Sec. 2.1)
  geometry   physical operators, metrics and facet matching (Sec. 2.1)
  physics    pointwise Euler/NS quantities (Sec. 2.2-3, 4, 4.5, 5)
  residual   entropy-split, Hadamard-form residuals and SATs (Sec. 4, 5, 6.2)
  rrk        relaxation RK4 time step (Sec. 6.1)

Parity status per function is recorded in each module header.
"""
