"""Plain, slow, FP64 CPU oracle for the implicit SPH radiation-diffusion step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (the only common module is the seeded input generator ``synth``, which
holds none of the method's arithmetic).

Paper: Bassett, Owen & Brunner, "Efficient smoothed particle radiation
hydrodynamics I: Thermal radiative transfer" (arXiv:2001.11606).

Every function follows the plain definition of what the method computes:

* ``kernels``    -- the SPH kernels and their radial derivatives (Sec. 2.3,
                    kernel normalisation and the Wendland C4 equation) and the
                    cubic B-spline used by the synthetic workloads;
* ``neighbors``  -- the pair predicate and brute-force / cell-list searches;
* ``operator``   -- frozen per-step data (Fleck factor, Sec. 2.2; flux limiter,
                    Sec. 2.1; volume V = m/rho, Sec. 2.3), the Brookshaw second
                    derivative assembled as a sparse matrix (Sec. 2.3-2.4, the
                    diffusion-solve equation of Sec. 3.2) and the right-hand side;
* ``linsolve``   -- dense and Jacobi-preconditioned CG solves of that system;
* ``material``   -- the per-particle Newton solve of the material equation
                    (Sec. 3.2);
* ``step``       -- Algorithm 1 (nonlinear elimination outer loop), the
                    convergence test (Sec. 2.2) and the energy sums (Sec. 2.5);
* ``timestep``   -- the adaptive time-step controller (Sec. 3.3).

Parity pins: see ``tests/test_oracle_*.py``.  The AMG preconditioner of the GPU
path has no oracle counterpart (the paper fixes no AMG parameters; only the
solution of the linear system is unique) -- parity unpinned for AMG internals.
"""
from . import kernels, neighbors, operator, linsolve, material, step, timestep  # noqa: F401
