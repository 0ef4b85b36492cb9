"""CPU FP64 oracle for the blended-shell Stokes hot path (arXiv 2506.04157).

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call,
link or execute anything in this directory; only ``tests/``, the smoke check
in ``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` use it.

The oracle is written from the paper's text, in plain numpy/scipy, FP64:

* ``mesh``        macro meshes (unit cube, icosahedral shell), structured
                  refinement, P1/P2 node sets, blending map (Sec. 4.1).
* ``quadrature``  reference-tetrahedron quadrature rules.
* ``fem``         element-by-element assembly of A, B, C, M_{1/eta} and the
                  buoyancy right-hand side into global sparse matrices
                  (Sec. 5.1, the definitions of A, B, C, f).
* ``system``      boundary/pressure constraints and a direct solve of the
                  resulting square system (Sec. 5.1, eqs. SaddlePointStructure-
                  Dirichlet and InnerSaddlePointSystem).
* ``solvers``     assembled-matrix references for the solver components:
                  Chebyshev smoother, grid transfers, V-cycle, CG, BFBT,
                  symmetric Uzawa, FGMRES (Sec. 5.2).
* ``adjoint``     assembled gradient of J = 1/2 |u - u_obs|^2 with respect to
                  nodal log-viscosity and temperature.

It shares no code with the HIP path.  Pins that tie it to the paper and to
mathematics (closed forms, invariants, printed DoF counts, convergence rates)
live in ``tests/test_oracle_*.py``.
"""
